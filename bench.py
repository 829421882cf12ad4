"""Benchmark of the two-species multirange lattice Boltzmann step on one MI355X.

Workload: a 4096 x 4096 lattice, moving bounce-back walls at +-0.02 (Couette
shear), random 50/50 emulsion start (rho 1.0 / 0.1 per site, seed 1) with the
linear Couette velocity, symmetric couplings G^a = -9.0, G^r = 8.1 (both
species), G_AB = 0.405, rho0 = 0.83, tau = 1.  A step is one full time step of
both species: pseudo-potential, belt-1/two-belt forces, BGK collision,
streaming, walls and the FP64 wall-stress accumulation.  Populations are FP32;
the headline `value` runs them two steps per pass ("f32x2": one kernel keeps
step t's populations on chip and runs step t+1 behind it, bitwise the result
of single steps, so each population crosses HBM once per two updates); the
single-step kernel ("f32"), FP16- and BF16-deviation storage and the moment
form ("mom32": at tau = 1 six moments per site, 48 bytes per update) are timed
beside it.  Each variant's `frac` is the HBM floor of its launches (each
population or moment read once and written once per launch: 144 B per update
for FP32 one step per pass, 72 B two steps per pass) over the launch time;
`effective_gbs` states the one-step bytes (144 B for FP32) at the same
throughput.  The roofline object is the headline variant's.

Prints one JSON line.  `roofline.achieved` is the floor bytes of one launch
divided by the device time per launch, from HIP events recorded on the
lattice's stream around the timed steps; `roofline.traffic` is the HBM bytes
of a launch that rocprofv3's FETCH_SIZE / WRITE_SIZE counters measured on the
current kernel source (null once the source has changed).  `hbm` adds the rate
of that traffic and the live rate of a plain streaming copy on the same GPU.
Each variant carries its error against the FP64 step at the benchmark's own
length and the record of the 5000-step workload length.  `cpu_baseline` is
the FP64 oracle on all host threads, with a single-thread rate beside it.

Before each variant's warm-up, the same step kernel runs for half a second on
a separate lattice of the same size, storage and initial state (clock ramp),
the warm-up steps queued right behind it: the first tens of launches after
even a few tens of milliseconds of idle GPU run 10-20 % slow, and a ramp on
other data (uniform densities) left the 16-bit forms' first launches slow.

The launch shape comes from the project's autotuner (timed before the timed
region; cached in paper_1004_5058_amd/tuning.json).  A second leg measures
flow-curve points per hour on the batched 48-lattice ensemble (10 000 steps
each) against a plain one-lattice-at-a-time loop; a third leg counts
stress-controlled flow-curve points per hour with and without the surrogate.
With --surrogate-check-size the stress-controlled leg runs again on the knee
refinement's checking lattices (1024 x 512, 10 000 steps).
With --knee, a network trained on 2000 ensemble lattices proposes flow-curve
refinements near the yield stress, each checked by a 1024x512 lattice run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--variants f32x2,f32,f16x2,bf16x2,f16dev,bf16dev,mom32] [--size 4096] [--no-flowcurve]
       [--no-tune] [--no-surrogate] [--no-errors] [--ramp SECONDS] [--surrogate-check-size] [--knee]
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Variants timed on the 4096^2 workload: storage, time steps per kernel pass,
# the per-update bytes of one step per pass in that storage (18 population
# loads + 18 stores; the moment form 6 + 6 moments) and the HBM bytes an
# update must move in the variant as run (two steps per pass: each population
# is read and written once per two updates, so half).  The roofline object
# uses the latter: the bytes the kernel cannot avoid, per launch, over the
# launch's duration.
VARIANTS = {
    "f32x2": dict(storage="f32", per_pass=2, bytes_per_lup=144, floor_per_lup=72),
    "f32": dict(storage="f32", per_pass=1, bytes_per_lup=144, floor_per_lup=144),
    "f16x2": dict(storage="f16dev", per_pass=2, bytes_per_lup=72, floor_per_lup=36),
    "bf16x2": dict(storage="bf16dev", per_pass=2, bytes_per_lup=72, floor_per_lup=36),
    "f16dev": dict(storage="f16dev", per_pass=1, bytes_per_lup=72, floor_per_lup=72),
    "bf16dev": dict(storage="bf16dev", per_pass=1, bytes_per_lup=72, floor_per_lup=72),
    "mom32": dict(storage="mom32", per_pass=1, bytes_per_lup=48, floor_per_lup=48),
}
DEFAULT_VARIANTS = "f32x2,f32,f16x2,bf16x2,f16dev,bf16dev,mom32"
# Before each variant's W warm-up steps the same step kernel runs for this
# long on a separate lattice of the same size and storage: the GPU lowers its
# clocks while the host sets a lattice up (about a second per 4096^2 lattice),
# and the first 10-40 launches after that run 3-8 % slower than the steady
# state (a streaming copy as the warm-up recovers only part of it).  The
# benchmarked lattice itself takes exactly W untimed and K timed steps.
CLOCK_RAMP_S = 0.5


def variant_storage(v):
    return VARIANTS[v]["storage"]


def kernel_source_hash():
    """Hash of the step kernels' source code, comments and layout removed (a
    comment edit leaves the committed counters valid; a code change does not)."""
    import re
    h = hashlib.sha256()
    for name in ("lb_kernels.hip", "lb_device.hpp"):
        with open(os.path.join(ROOT, "paper_1004_5058_amd", "csrc", name), encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_counters(workload, variant):
    """The committed rocprofv3 counter summary of a variant's step kernel
    (HBM bytes per launch, VALU busy share), if it was taken on the current
    kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/{variant}")
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e


def measured_traffic(workload, variant):
    """HBM bytes per kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    e = measured_counters(workload, variant)
    return None if e is None else e.get("bytes_per_launch")


def stated_precision(workload):
    """Errors of each storage form against the FP64 step at the workload's
    stated length (5000 steps), from the committed long-run record."""
    path = os.path.join(ROOT, "profiles", "precision_couette_emulsion_4096x4096_5000steps.json")
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def ramp_lattice(variant, n, tune_cache=None, u=0.02, fields=None):
    """A separate n x n lattice for the clock ramp: same kernel, launch shape
    and bytes per step as the variant, and with `fields` (rho_a, rho_b, ux, uy)
    the same initial state as the timed lattice (the clocks the GPU settles at
    depend on the data it computes on: after a ramp on uniform densities the
    16-bit forms ran their first timed launches up to 5 % slow); without,
    uniform densities (cheap to set up)."""
    import numpy as np
    from paper_1004_5058_amd import inputs, lb
    vd = VARIANTS[variant]
    if fields is None:
        ra = np.full((n, n), 0.55)
        fields = (ra, ra, None, None)
    lat = lb.Lattice(n, n, *fields, u_top=u, u_bot=-u, storage=vd["storage"], profile=False,
                     **inputs.COUPLINGS)
    if tune_cache is not None:
        lat.autotune(tune_cache, steps=10)
    if lat.launch()["steps_per_pass"] != vd["per_pass"]:
        lat.set_fusion(vd["per_pass"])
    return lat


def run_ramp(lat, seconds, then=None):
    """Steps the ramp lattice for `seconds`; `then` (the next work) is queued
    right behind its last steps, so the GPU does not idle in between (even a
    few tens of milliseconds idle let the clocks fall: the next 20-40
    launches then run 10-20 % slow).  Returns the ramp steps taken."""
    import torch
    done = 0
    t0 = time.perf_counter()
    while True:
        lat.step(64)
        done += 64
        if time.perf_counter() - t0 >= seconds:
            break
        torch.cuda.synchronize()
    if then is not None:
        then()
    torch.cuda.synchronize()
    return done


def gpu_run(variant, n, steps, warmup, u=0.02, seed=1, tune_cache=None, ramp_s=0.0):
    import torch
    from paper_1004_5058_amd import inputs, lb
    vd = VARIANTS[variant]
    ra, rb = inputs.emulsion(n, n, seed=seed)
    ux, uy = inputs.couette(n, n, u, -u)
    lat = lb.Lattice(n, n, ra, rb, ux, uy, u_top=u, u_bot=-u, storage=vd["storage"], profile=False,
                     **inputs.COUPLINGS)
    if tune_cache is not None:
        lat.autotune(tune_cache, steps=10)
    # the tuner may pick either; each variant states its own steps per pass
    # (a tuned fused tile height and width are kept)
    if lat.launch()["steps_per_pass"] != vd["per_pass"]:
        lat.set_fusion(vd["per_pass"])
    shape = lat.launch()
    if vd["per_pass"] == 2:
        shape["lanes"], shape["columns"] = lat.fusion_tile()
    # clock ramp on a separate lattice from the same initial state, the
    # warm-up steps queued right behind it; the ramp lattice is freed only
    # after the timed region (freeing synchronises the device)
    ramp = ramp_lattice(variant, n, tune_cache=tune_cache, u=u, fields=(ra, rb, ux, uy)) if ramp_s > 0 else None
    del ra, rb, ux, uy
    try:
        if ramp is not None:
            ramp_steps = run_ramp(ramp, ramp_s, then=lambda: lat.step(warmup))
        else:
            ramp_steps = 0
            lat.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the timed region: `steps` steps bracketed by HIP events on the
        # lattice's own stream (lb_time_steps), which give the device time per step
        ms_kernel = lat.time_steps(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        if ramp is not None:
            ramp.close()
            del ramp
    sb, st, ns = lat.stress()
    fields = lat.fields()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    lups = float(n) * n
    return dict(ms_per_step=1e3 * wall / steps, mlups=lups * steps / wall / 1e6,
                ms_kernel=ms_kernel, stress=[sb, st], nsamples=ns, shape=shape, fields=fields, ramp_steps=ramp_steps)


def errors_vs_f64(run, ref):
    """Density error relative to the largest density, momentum error on the
    scale rho c_S, and relative error of the mean wall stress."""
    import numpy as np
    ra, rb, ux, uy = ref["fields"]
    a, b, vx, vy = run["fields"]
    scale_r = max(ra.max(), rb.max())
    scale_j = (ra + rb).max() / np.sqrt(3.0)
    e_rho = max(np.abs(a - ra).max(), np.abs(b - rb).max()) / scale_r
    e_j = max(np.abs(vx * (a + b) - ux * (ra + rb)).max(), np.abs(vy * (a + b) - uy * (ra + rb)).max()) / scale_j
    s_ref = 0.5 * (ref["stress"][0] + ref["stress"][1])
    s = 0.5 * (run["stress"][0] + run["stress"][1])
    return dict(rho=float(f"{e_rho:.3e}"), j=float(f"{e_j:.3e}"), stress=float(f"{abs(s - s_ref) / abs(s_ref):.3e}"))


def gpu_run_f64(n, steps, u=0.02, seed=1):
    """The FP64 population step over `steps` steps (one step per pass): the
    reference of the variants' error figures.  Its 4096^2 windows match the
    oracle to <= 1e-15 (tests/test_gpu_fullsize.py)."""
    import torch
    from paper_1004_5058_amd import inputs, lb
    ra, rb = inputs.emulsion(n, n, seed=seed)
    ux, uy = inputs.couette(n, n, u, -u)
    lat = lb.Lattice(n, n, ra, rb, ux, uy, u_top=u, u_bot=-u, storage="f64", profile=False, **inputs.COUPLINGS)
    del ra, rb, ux, uy
    lat.step(steps)
    sb, st, _ = lat.stress()
    fields = lat.fields()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return dict(stress=[sb, st], fields=fields)


def flowcurve_rates(steps, n_lat=48, seed=100, tune_cache=None):
    """Flow-curve points per hour on the batched ensemble (48 lattices, heights
    256..1024, width 2H, U log-uniform in [1e-4, 5e-2], G^r in [7.5, 8.5]):
    one persistent step kernel per time step for the whole batch, replayed as
    HIP graphs, against the plain loop (one lattice at a time, one launch per
    step, no graph, each lattice size in its own tuned shape).  Both produce
    the same per-lattice stresses.  The batch is
    also run in the moment form (tau = 1); its stresses are compared with the
    FP32 population batch."""
    from paper_1004_5058_amd import flowcurve, inputs, lb
    draws = inputs.ensemble(n_lat, seed=seed)
    specs = flowcurve.lattice_specs(draws, inputs.COUPLINGS)
    sites = sum(s["nx"] * s["ny"] for s in specs)
    b = lb.Batch(specs, storage="f32", profile=True)
    if tune_cache is not None:
        # tuned before the timed run; the run applies the cached entry
        b.autotune(tune_cache, steps=10)
    shape = b.launch()
    b.close()
    rows_b, wall_b = flowcurve.run_batched(specs, steps, tune_cache=tune_cache)
    print(f"# flow curve: batched {n_lat} lattices x {steps} steps in {wall_b:.2f} s", file=sys.stderr, flush=True)
    rows_p, wall_p = flowcurve.run_plain(specs, steps, tune_cache=tune_cache)
    print(f"# flow curve: plain loop in {wall_p:.2f} s", file=sys.stderr, flush=True)
    agree = max(abs(a["sigma"] - c["sigma"]) / max(abs(c["sigma"]), 1e-300) for a, c in zip(rows_b, rows_p))
    # the same ensemble in the moment form (tau = 1), batched, tuned shape
    b = lb.Batch(specs, storage="mom32", profile=True)
    if tune_cache is not None:
        b.autotune(tune_cache, steps=10)
    tm = b.launch()
    b.close()
    rows_m, wall_m = flowcurve.run_batched(specs, steps, storage="mom32", tune_cache=tune_cache)
    print(f"# flow curve: batched moment form in {wall_m:.2f} s", file=sys.stderr, flush=True)
    agree_m = max(abs(a["sigma"] - c["sigma"]) / max(abs(c["sigma"]), 1e-300) for a, c in zip(rows_m, rows_b))
    # The Herschel-Bulkley flow curve: the same sizes and wall speeds at one
    # fixed coupling set (the parity workload's, G^r = 8.1), batched
    fixed = [dict(d, g_aa2=inputs.COUPLINGS["g_aa2"], g_bb2=inputs.COUPLINGS["g_bb2"]) for d in draws]
    specs_f = flowcurve.lattice_specs(fixed, inputs.COUPLINGS)
    rows_f, wall_f = flowcurve.run_batched(specs_f, steps, tune_cache=tune_cache)
    print(f"# flow curve: fixed-coupling batch in {wall_f:.2f} s", file=sys.stderr, flush=True)
    curve = flowcurve.hb_curve(rows_f)
    curve.update(couplings=dict(g_a=inputs.COUPLINGS["g_aa1"], g_r=inputs.COUPLINGS["g_aa2"],
                                g_ab=inputs.COUPLINGS["g_ab"]),
                 wall_s=round(wall_f, 3),
                 points_S_sigma=[[float(f"{r['S']:.6e}"), float(f"{r['S_bulk']:.6e}"), float(f"{r['sigma']:.6e}")]
                                 for r in sorted(rows_f, key=lambda r: r["S"])])
    return dict(lattices=n_lat, steps=steps, sites=sites, hb_flow_curve=curve,
                batched_mom_points_per_hour=round(n_lat * 3600.0 / wall_m, 1), batched_mom_s=round(wall_m, 3),
                batched_mom_mlups=round(sites * steps / wall_m / 1e6, 1),
                mom_vs_f32_max_sigma_rel=float(f"{agree_m:.3e}"),
                mom_note="moment-form stresses differ from the FP32 population batch by this much "
                         "(two FP32 trajectories of chaotic emulsions after 10^4 steps): not the 1 % bar",
                mom_launch_shape={k: tm[k] for k in ("bx", "ly", "grid")},
                batched_points_per_hour=round(n_lat * 3600.0 / wall_b, 1),
                plain_points_per_hour=round(n_lat * 3600.0 / wall_p, 1),
                batched_s=round(wall_b, 3), plain_s=round(wall_p, 3),
                batched_mlups=round(sites * steps / wall_b / 1e6, 1),
                plain_mlups=round(sites * steps / wall_p / 1e6, 1),
                speedup=round(wall_p / wall_b, 3), max_sigma_mismatch=agree, launch_shape=shape)


def surrogate_rates(n_cases=10, k=4, storage="f32", plain=True, size=None):
    """Stress-controlled flow-curve points per hour: the shear rate at which a
    fixed-coupling lattice reaches a target wall stress, accepted when a
    lattice run is within 1 % (every accepted point is a lattice result).  A
    stream of two batches of cases (A, then B): batched k-section (k lattice
    runs per case and round, one launch per step for all of them), and batched
    with the surrogate, whose network the HIP kernels train on batch A's
    lattice runs (no separate ensemble; the training is charged) and which
    places batch B's runs.  The plain per-run loop (bisection, one lattice run
    at a time) serves batch B for reference.  size: None for the 256 x 128,
    20 000-step task; "check" for the knee refinement's checking lattices
    (1024 x 512, 10 000 steps, wall speeds 0.005-0.06, the cases' rates 4e-5
    to 1.6e-4) with batch A's search shared by both streams and no plain loop."""
    from paper_1004_5058_amd import surrogate
    G = surrogate.GAIN
    if size == "check":
        nx, ny, steps, seed, u = 1024, 512, 10000, G["seed"], (0.005, 0.06)
        s_cases = (4e-5, 1.6e-4)
        plain = False
    else:
        nx, ny, steps, seed, u = G["nx"], G["ny"], G["steps"], G["seed"], G["u"]
        s_cases = (1.5e-4, 6e-4)
    S_lo, S_hi = 2 * u[0] / ny, 2 * u[1] / ny

    def lattice(batched):
        return lambda pts: surrogate.lattice_stresses(pts, nx, ny, steps, seed, storage=storage, batched=batched)
    cases_a = surrogate.draw_points(n_cases, 31, s_cases, (-9.2, -9.05), (7.9, 8.05), max_sum=-0.98)
    cases_b = surrogate.draw_points(n_cases, 47, s_cases, (-9.2, -9.05), (7.9, 8.05), max_sum=-0.98)
    targets = lattice(True)(cases_a + cases_b)
    ta, tb = targets[:n_cases], targets[n_cases:]
    out = dict(lattice=f"{nx}x{ny}", storage=storage, steps=steps, cases_per_batch=n_cases, runs_per_round=k,
               rate_range=[S_lo, S_hi])
    r, sa_k, sb_k = surrogate.stream_points(cases_a, ta, cases_b, tb, lattice(True), S_lo, S_hi, k=k)
    out["batched"] = r
    print(f"# stress-controlled points ({storage}, {nx}x{ny}), batched k-section: {r}", file=sys.stderr, flush=True)
    surr = surrogate.FlowSurrogate(max_rows=2048, seed=0)
    reuse = (sa_k, r["A"]["rounds"], r["A"]["wall_s"]) if size == "check" else None
    r, _, sb_n = surrogate.stream_points(cases_a, ta, cases_b, tb, lattice(True), S_lo, S_hi, k=k,
                                         use_network=True, surr=surr, batch_a=reuse)
    # the network's error on batch B's lattice runs (after the fact)
    import numpy as np
    err = [abs(float(surr.predict(g1, g2, np.exp(x))[0]) - sig) / abs(sig)
           for s, (g1, g2, _) in zip(sb_n, cases_b) for x, _, sig in s.points]
    r["network_rel_err_on_B_runs"] = dict(median=float(f"{np.median(err):.3e}"),
                                          p90=float(f"{np.quantile(err, 0.9):.3e}"))
    if reuse is not None:
        r["A_reused"] = "batch A's k-section search and time shared with the k-section stream"
    out["batched_surrogate"] = r
    print(f"# stress-controlled points ({storage}, {nx}x{ny}), batched with the surrogate: {r}", file=sys.stderr,
          flush=True)
    if plain:
        t0 = time.perf_counter()
        ss = [surrogate.RootSearch(t, S_lo, S_hi, k=1) for t in tb]
        for s, (g1, g2, _) in zip(ss, cases_b):
            surrogate.search_batched([s], lambda todo: lattice(False)([(g1, g2, S) for _, S in todo]))
        wall = time.perf_counter() - t0
        ok = sum(s.result is not None for s in ss)
        out["plain_batch_B"] = dict(lattice_runs=sum(s.runs for s in ss), accepted=ok, wall_s=round(wall, 2),
                                    points_per_hour=round(ok * 3600.0 / wall, 1))
        print(f"# stress-controlled points ({storage}), plain loop on batch B: {out['plain_batch_B']}",
              file=sys.stderr, flush=True)
    return out


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, steps=7, u=0.02, seed=1):
    """The FP64 oracle on the same 4096^2 workload, a bounded number of steps,
    built -O3 -march=native for this host (no contraction: the same results)."""
    from oracle import oracle as O
    from paper_1004_5058_amd import inputs
    O.use_native_build()
    ra, rb = inputs.emulsion(n, n, seed=seed)
    ux, uy = inputs.couette(n, n, u, -u)
    p = O.OracleParams(nx=n, ny=n, walls=True, u_top=u, u_bot=-u, **inputs.COUPLINGS)
    f = O.init(p, ra, rb, ux, uy)
    del ra, rb, ux, uy
    t0 = time.perf_counter()
    f, _, _ = O.run(p, f, steps)
    dt = time.perf_counter() - t0
    return dict(value=round(float(n) * n * steps / dt / 1e6, 3), unit="MLUPS", cores=O.threads(), kind="oracle",
                cpu=cpu_model(), build="gcc -O3 -march=native -ffp-contract=off -fopenmp",
                sample=f"{steps} FP64 oracle steps of the full {n}x{n} lattice ({dt:.1f} s)")


_SINGLE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_1004_5058_amd import inputs
O.use_native_build()
n, steps, u = int(sys.argv[2]), int(sys.argv[3]), 0.02
ra, rb = inputs.emulsion(n, n, seed=1)
ux, uy = inputs.couette(n, n, u, -u)
p = O.OracleParams(nx=n, ny=n, walls=True, u_top=u, u_bot=-u, **inputs.COUPLINGS)
f = O.init(p, ra, rb, ux, uy)
t0 = time.perf_counter()
O.run(p, f, steps)
dt = time.perf_counter() - t0
print(json.dumps({"value": round(n * n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.threads(),
                  "sample": f"{steps} FP64 oracle steps of a {n}x{n} lattice of the same recipe ({dt:.1f} s)"}))
"""


def cpu_single_thread(n=1024, steps=3):
    """The oracle on one thread, in a child process (OMP_NUM_THREADS=1; the
    child never touches the GPU)."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _SINGLE_THREAD, ROOT, str(n), str(steps)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--variants", default=DEFAULT_VARIANTS,
                    help="comma-separated, the first is the headline: " + ", ".join(VARIANTS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ramp", type=float, default=CLOCK_RAMP_S,
                    help="seconds of the same step kernel on a separate lattice before each variant's warm-up "
                         "steps (0: none)")
    ap.add_argument("--no-errors", action="store_true", help="skip the FP64 reference run of the error figures")
    ap.add_argument("--no-flowcurve", action="store_true", help="skip the batched-vs-plain flow-curve leg")
    ap.add_argument("--flow-steps", type=int, default=10000)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the stress-controlled surrogate leg")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape instead of the autotuner")
    ap.add_argument("--surrogate-check-size", action="store_true",
                    help="add the surrogate leg at the knee refinement's checking size (1024x512, 10 000 steps)")
    ap.add_argument("--knee", action="store_true",
                    help="add the knee-refinement leg: a network trained on 2000 ensemble lattices proposes "
                         "refinements near the yield stress, each checked by a 1024x512 lattice run (minutes)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1004_5058_amd", "tuning.json"))
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU and the library drives one GPU per process; --gpus {a.gpus} "
              "is not supported (sharding by y-slabs with halo rows, or whole lattices per GPU, is designed but not "
              "built).", file=sys.stderr)
        sys.exit(2)
    variants = [v for v in a.variants.split(",") if v]
    for v in variants:
        if v not in VARIANTS:
            print(f"bench.py: unknown variant {v} (known: {', '.join(VARIANTS)})", file=sys.stderr)
            sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.calib_copy:
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    n = a.size
    workload = f"couette_emulsion_{n}x{n}"
    tune = None if a.no_tune else a.tune_cache
    res = {}
    for v in variants:
        res[v] = gpu_run(v, n, a.steps, a.warmup, tune_cache=tune, ramp_s=a.ramp)
        print(f"# {v}: {res[v]['mlups']:.0f} MLUPS, kernel {res[v]['ms_kernel']:.4f} ms/step", file=sys.stderr,
              flush=True)
    ref = None
    if not a.no_errors:
        # the FP64 population step over the same number of steps: the
        # reference of every variant's error figures
        ref = gpu_run_f64(n, a.steps + a.warmup)
    torch.cuda.empty_cache()
    head = variants[0]
    r = res[head]
    vd = VARIANTS[head]
    lups = float(n) * n
    ms_launch = r["ms_kernel"] * vd["per_pass"]
    bytes_launch = vd["floor_per_lup"] * vd["per_pass"] * lups
    achieved = bytes_launch / (ms_launch * 1e-3) / 1e9
    traffic = measured_traffic(workload, head)
    line = {
        "metric": "MLUPS (2-species)",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if vd["storage"] in ("f32", "mom32") else vd["storage"],
        "data": "synthetic (seeded emulsion start, linear Couette velocity)",
        "config": {"workload": workload, "nx": n, "ny": n, "storage": vd["storage"],
                   "steps_per_pass": vd["per_pass"], "walls": "bounce-back +-0.02",
                   "tau": 1.0, "rho0": 0.83, "G": [-9.0, 8.1, -9.0, 8.1, 0.405]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_launch": bytes_launch, "steps_per_launch": vd["per_pass"],
                     "ms_per_launch": round(ms_launch, 5),
                     "effective_gbs": round(vd["bytes_per_lup"] * lups / (r["ms_kernel"] * 1e-3) / 1e9, 1),
                     "valu_busy": (measured_counters(workload, head) or {}).get("valu_busy")},
        "variants": {},
        "clock_ramp": (f"{a.ramp:g} s of the same step kernel on a separate {n}x{n} lattice of the same storage "
                       "and initial state "
                       f"({r['ramp_steps']} steps), the {a.warmup} warm-up steps queued right behind it") if a.ramp > 0
        else None,
    }
    for v in variants:
        d = VARIANTS[v]
        rv = res[v]
        fl = d["floor_per_lup"] * lups / (rv["ms_kernel"] * 1e-3) / 1e9
        line["variants"][v] = {
            "mlups": round(rv["mlups"], 1), "ms_kernel": round(rv["ms_kernel"], 5), "launch_shape": rv["shape"],
            "storage": d["storage"], "steps_per_pass": d["per_pass"],
            "floor_bytes_per_lup": d["floor_per_lup"], "gbs": round(fl, 1), "frac": round(fl / HBM_PEAK_GBS, 4),
            "bytes_per_lup_one_step": d["bytes_per_lup"],
            "effective_gbs": round(d["bytes_per_lup"] * lups / (rv["ms_kernel"] * 1e-3) / 1e9, 1),
            "sigma_bot_top": [float(f"{x:.7e}") for x in rv["stress"]]}
        mc = measured_counters(workload, v)
        if mc is not None:
            # counters of the committed profile on this kernel source: HBM bytes
            # per launch over this run's launch time, and the VALU busy share
            line["variants"][v]["measured_gbs"] = round(
                mc["bytes_per_launch"] / (rv["ms_kernel"] * d["per_pass"] * 1e-3) / 1e9, 1)
            line["variants"][v]["valu_busy"] = mc.get("valu_busy")
        if ref is not None:
            line["variants"][v]["err_vs_f64"] = dict(errors_vs_f64(rv, ref), steps=a.steps + a.warmup)
    stated = stated_precision(workload)
    if stated is not None:
        line["precision_at_5000_steps"] = stated
    for v in variants:
        del res[v]["fields"]
    from paper_1004_5058_amd import lb
    cp = lb.copy_peak()
    measured = None if traffic is None else traffic / (ms_launch * 1e-3) / 1e9
    line["hbm"] = {"measured_gbs": None if measured is None else round(measured, 1),
                   "measured_frac_of_peak": None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                   "measured_frac_of_copy_peak": None if measured is None else round(measured / cp, 4),
                   "copy_peak_gbs": round(cp, 1), "achieved_frac_of_copy_peak": round(achieved / cp, 4),
                   "copy": "library streaming copy, 16 B per lane, 2 GiB read + 2 GiB written"}
    if not a.no_flowcurve:
        try:
            line["flowcurve"] = flowcurve_rates(a.flow_steps, tune_cache=tune)
            print(f"# flow curve: {line['flowcurve']}", file=sys.stderr, flush=True)
        except Exception as e:  # reported, never hidden
            line["flowcurve"] = {"error": repr(e)}
    if not a.no_flowcurve and not a.no_surrogate:
        try:
            line["surrogate"] = surrogate_rates()
        except Exception as e:  # reported, never hidden
            line["surrogate"] = {"error": repr(e)}
    if a.surrogate_check_size:
        try:
            line["surrogate_check_size"] = surrogate_rates(size="check")
        except Exception as e:  # reported, never hidden
            line["surrogate_check_size"] = {"error": repr(e)}
    if a.knee:
        from paper_1004_5058_amd import surrogate
        try:
            kr = surrogate.knee_refinement(
                couplings=((-9.0, 8.1), (-9.2, 8.0), (-8.8, 7.7)),
                log=lambda m: print(f"# knee refinement: {m}", file=sys.stderr, flush=True))
            for c in kr["curves"]:
                c.pop("network_curve", None)      # 400 samples per curve: not for the one-line record
            line["knee_refinement"] = kr
        except Exception as e:  # reported, never hidden
            line["knee_refinement"] = {"error": repr(e)}
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n)
        line["cpu_baseline"]["single_thread"] = cpu_single_thread()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
