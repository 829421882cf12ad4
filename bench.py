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
beside it.  Each variant's `frac` uses the algorithmic bytes of one update in
its storage (144 for FP32); f32x2 also reports its own floor (72 B per update).
The roofline object is the headline variant's.

Prints one JSON line.  `roofline.achieved` is the algorithmic HBM traffic of a
step (18 population loads + 18 stores per site) divided by the device time per
step, from HIP events recorded on the lattice's stream around the timed steps.  `hbm` adds
the rate of the measured traffic (rocprofv3 counters, when taken on the
current kernel source) and the live rate of a plain streaming copy on the same
GPU.  `cpu_baseline` is the FP64 oracle on all host threads, with a
single-thread rate beside it.

The launch shape comes from the project's autotuner (timed before the timed
region; cached in paper_1004_5058_amd/tuning.json).  A second leg measures
flow-curve points per hour on the batched 48-lattice ensemble (10 000 steps
each) against a plain one-lattice-at-a-time loop; a third leg counts
stress-controlled flow-curve points per hour with and without the surrogate.
With --knee, a network trained on 2000 ensemble lattices proposes flow-curve
refinements near the yield stress, each checked by a 1024x512 lattice run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--variants f32x2,f32,f16dev,bf16dev,mom32] [--size 4096] [--no-flowcurve] [--no-tune]
       [--no-surrogate] [--knee]
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
# Algorithmic HBM bytes per 2-species lattice update: 18 population loads and
# 18 stores in the storage format (the moment form: 6 + 6 moments).  "f32x2"
# is FP32 storage run two steps per pass (lb_set_fusion); its roofline figure
# keeps the per-update 144 B, while each population actually crosses HBM once
# per two updates (FLOOR_PER_LUP).
BYTES_PER_LUP = {"f64": 288, "f32": 144, "f32x2": 144, "f16dev": 72, "bf16dev": 72, "mom32": 48, "mom64": 96}
FLOOR_PER_LUP = {"f32x2": 72}
STEPS_PER_LAUNCH = {"f32x2": 2}


def variant_storage(v):
    return "f32" if v == "f32x2" else v


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("lb_kernels.hip", "lb_device.hpp"):
        with open(os.path.join(ROOT, "paper_1004_5058_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage):
    """HBM bytes per kernel launch (a launch advances STEPS_PER_LAUNCH steps)
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/{storage}")
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch", e.get("bytes_per_step"))


def gpu_run(variant, n, steps, warmup, u=0.02, seed=1, tune_cache=None):
    import torch
    from paper_1004_5058_amd import inputs, lb
    ra, rb = inputs.emulsion(n, n, seed=seed)
    ux, uy = inputs.couette(n, n, u, -u)
    lat = lb.Lattice(n, n, ra, rb, ux, uy, u_top=u, u_bot=-u, storage=variant_storage(variant), profile=False,
                     **inputs.COUPLINGS)
    del ra, rb, ux, uy
    if tune_cache is not None:
        lat.autotune(tune_cache, steps=10)
    if variant_storage(variant) == "f32":
        # the tuner may pick either; each variant states its own steps per pass
        # (a tuned fused tile height is kept)
        want = STEPS_PER_LAUNCH.get(variant, 1)
        if lat.launch()["steps_per_pass"] != want:
            lat.set_fusion(want)
    shape = lat.launch()
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the timed region: `steps` steps bracketed by HIP events on the lattice's
    # own stream (lb_time_steps), which give the device time per step
    ms_kernel = lat.time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sb, st, ns = lat.stress()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    lups = float(n) * n
    return dict(ms_per_step=1e3 * wall / steps, mlups=lups * steps / wall / 1e6,
                ms_kernel=ms_kernel, stress=[sb, st], nsamples=ns,
                shape=shape)


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
        b.autotune(tune_cache, steps=3)
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
        b.autotune(tune_cache, steps=3)
    tm = b.launch()
    b.close()
    rows_m, wall_m = flowcurve.run_batched(specs, steps, storage="mom32", tune_cache=tune_cache)
    print(f"# flow curve: batched moment form in {wall_m:.2f} s", file=sys.stderr, flush=True)
    agree_m = max(abs(a["sigma"] - c["sigma"]) / max(abs(c["sigma"]), 1e-300) for a, c in zip(rows_m, rows_b))
    return dict(lattices=n_lat, steps=steps, sites=sites,
                batched_mom_points_per_hour=round(n_lat * 3600.0 / wall_m, 1), batched_mom_s=round(wall_m, 3),
                batched_mom_mlups=round(sites * steps / wall_m / 1e6, 1),
                mom_vs_f32_max_sigma_rel=float(f"{agree_m:.3e}"),
                mom_launch_shape={k: tm[k] for k in ("bx", "ly", "grid")},
                batched_points_per_hour=round(n_lat * 3600.0 / wall_b, 1),
                plain_points_per_hour=round(n_lat * 3600.0 / wall_p, 1),
                batched_s=round(wall_b, 3), plain_s=round(wall_p, 3),
                batched_mlups=round(sites * steps / wall_b / 1e6, 1),
                plain_mlups=round(sites * steps / wall_p / 1e6, 1),
                speedup=round(wall_p / wall_b, 3), max_sigma_mismatch=agree, launch_shape=shape)


def surrogate_rates(n_train=512, n_cases=10, storage="f32", plain=True):
    """Stress-controlled flow-curve points per hour: the shear rate at which a
    fixed-coupling lattice reaches a target wall stress, accepted when a
    lattice run is within 1 % (a lattice run checks every point).  Three ways:
    the plain loop (bisection, one lattice run at a time), batched bisection
    (one launch per step for all open cases), and batched with the surrogate
    (network trained by the HIP kernels on a batched ensemble; the ensemble
    and the training are charged to it).  `storage` is the lattice storage of
    every run (the training ensemble, the targets and the solvers)."""
    from paper_1004_5058_amd import surrogate
    G = surrogate.GAIN
    nx, ny, steps, seed = G["nx"], G["ny"], G["steps"], G["seed"]
    S_lo, S_hi = 2 * G["u"][0] / ny, 2 * G["u"][1] / ny

    def lattice(batched):
        return lambda pts: surrogate.lattice_stresses(pts, nx, ny, steps, seed, storage=storage, batched=batched)
    t0 = time.perf_counter()
    pts = surrogate.draw_points(n_train, 300, (S_lo, S_hi), G["g1"], G["g2"])
    sig = lattice(True)(pts)
    rows = [dict(g_aa1=g1, g_aa2=g2, S=S, sigma=v) for (g1, g2, S), v in zip(pts, sig)]
    surr = surrogate.FlowSurrogate(max_rows=1024, seed=0)
    surr.fit(rows, iters=4000, lr=3e-3)
    t_train = time.perf_counter() - t0
    cases = surrogate.draw_points(n_cases, 31, (1.5e-4, 6e-4), (-9.2, -9.05), (7.9, 8.05), max_sum=-0.98)
    targets = lattice(True)(cases)
    out = dict(lattice=f"{nx}x{ny}", storage=storage, steps=steps, cases=n_cases, train_lattices=n_train,
               train_s=round(t_train, 2))
    legs = ((("plain", "bisect", False),) if plain else ()) + (("batched", "bisect", True),
                                                              ("batched_surrogate", "surrogate", True))
    for name, method, batched in legs:
        t0 = time.perf_counter()
        solvers, rounds = surrogate.stress_controlled_points(cases, targets, method, lattice(batched), S_lo, S_hi,
                                                             surr=surr)
        wall = time.perf_counter() - t0
        if method == "surrogate":
            wall_all = wall + t_train
        else:
            wall_all = wall
        ok = sum(s.result is not None for s in solvers)
        out[name] = dict(lattice_runs=sum(s.runs for s in solvers), accepted=ok, wall_s=round(wall_all, 2),
                         points_per_hour=round(ok * 3600.0 / wall_all, 1))
        if method == "surrogate":
            out[name]["wall_s_without_training"] = round(wall, 2)
        print(f"# stress-controlled points ({storage}), {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def cpu_baseline(n, steps=7, u=0.02, seed=1):
    """The FP64 oracle on the same 4096^2 workload, a bounded number of steps."""
    from oracle import oracle as O
    from paper_1004_5058_amd import inputs
    ra, rb = inputs.emulsion(n, n, seed=seed)
    ux, uy = inputs.couette(n, n, u, -u)
    p = O.OracleParams(nx=n, ny=n, walls=True, u_top=u, u_bot=-u, **inputs.COUPLINGS)
    f = O.init(p, ra, rb, ux, uy)
    del ra, rb, ux, uy
    t0 = time.perf_counter()
    f, _, _ = O.run(p, f, steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(float(n) * n * steps / dt / 1e6, 3), unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{steps} FP64 oracle steps of the full {n}x{n} lattice ({dt:.1f} s)")


_SINGLE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_1004_5058_amd import inputs
n, steps, u = int(sys.argv[2]), int(sys.argv[3]), 0.02
ra, rb = inputs.emulsion(n, n, seed=1)
ux, uy = inputs.couette(n, n, u, -u)
p = O.OracleParams(nx=n, ny=n, walls=True, u_top=u, u_bot=-u, **inputs.COUPLINGS)
f = O.init(p, ra, rb, ux, uy)
t0 = time.perf_counter()
O.run(p, f, steps)
dt = time.perf_counter() - t0
print(json.dumps({"value": round(n * n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1,
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
    ap.add_argument("--variants", default="f32x2,f32,f16dev,bf16dev,mom32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-flowcurve", action="store_true", help="skip the batched-vs-plain flow-curve leg")
    ap.add_argument("--flow-steps", type=int, default=10000)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the stress-controlled surrogate leg")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape instead of the autotuner")
    ap.add_argument("--knee", action="store_true",
                    help="add the knee-refinement leg: a network trained on 2000 ensemble lattices proposes "
                         "refinements near the yield stress, each checked by a 1024x512 lattice run (minutes)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1004_5058_amd", "tuning.json"))
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the library drives one GPU per process; --gpus {a.gpus} is not supported "
              "(sharding by y-slabs with halo rows, or whole lattices per GPU, is not implemented).",
              file=sys.stderr)
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
    variants = [v for v in a.variants.split(",") if v]
    res = {}
    for v in variants:
        res[v] = gpu_run(v, n, a.steps, a.warmup, tune_cache=None if a.no_tune else a.tune_cache)
        print(f"# {v}: {res[v]['mlups']:.0f} MLUPS, kernel {res[v]['ms_kernel']:.4f} ms/step", file=sys.stderr,
              flush=True)
    head = variants[0]
    r = res[head]
    bytes_step = BYTES_PER_LUP[head] * float(n) * n
    achieved = bytes_step / (r["ms_kernel"] * 1e-3) / 1e9
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
        "dtype": variant_storage(head),
        "data": "synthetic (seeded emulsion start, linear Couette velocity)",
        "config": {"workload": workload, "nx": n, "ny": n, "storage": variant_storage(head),
                   "steps_per_pass": STEPS_PER_LAUNCH.get(head, 1), "walls": "bounce-back +-0.02",
                   "tau": 1.0, "rho0": 0.83, "G": [-9.0, 8.1, -9.0, 8.1, 0.405]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "variants": {v: {"mlups": round(res[v]["mlups"], 1), "ms_kernel": round(res[v]["ms_kernel"], 5),
                         "launch_shape": res[v]["shape"],
                         "alg_gbs": round(BYTES_PER_LUP[v] * float(n) * n / (res[v]["ms_kernel"] * 1e-3) / 1e9, 1),
                         "bytes_per_lup": BYTES_PER_LUP[v],
                         "sigma_bot_top": [float(f"{x:.7e}") for x in res[v]["stress"]]} for v in variants},
    }
    for v in variants:
        line["variants"][v]["frac"] = round(line["variants"][v]["alg_gbs"] / HBM_PEAK_GBS, 4)
        if v in FLOOR_PER_LUP:
            fl = FLOOR_PER_LUP[v] * float(n) * n / (res[v]["ms_kernel"] * 1e-3) / 1e9
            line["variants"][v]["floor_bytes_per_lup"] = FLOOR_PER_LUP[v]
            line["variants"][v]["floor_gbs"] = round(fl, 1)
            line["variants"][v]["frac_of_floor"] = round(fl / HBM_PEAK_GBS, 4)
    from paper_1004_5058_amd import lb
    cp = lb.copy_peak()
    per_launch = STEPS_PER_LAUNCH.get(head, 1)
    measured = None if traffic is None else traffic / (per_launch * r["ms_kernel"] * 1e-3) / 1e9
    line["hbm"] = {"measured_gbs": None if measured is None else round(measured, 1),
                   "measured_frac_of_peak": None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                   "measured_frac_of_copy_peak": None if measured is None else round(measured / cp, 4),
                   "steps_per_launch": per_launch,
                   "copy_peak_gbs": round(cp, 1), "frac_of_copy_peak": round(achieved / cp, 4),
                   "copy": "library streaming copy, 16 B per lane, 2 GiB read + 2 GiB written"}
    if not a.no_flowcurve:
        try:
            line["flowcurve"] = flowcurve_rates(a.flow_steps, tune_cache=None if a.no_tune else a.tune_cache)
            print(f"# flow curve: {line['flowcurve']}", file=sys.stderr, flush=True)
        except Exception as e:  # reported, never hidden
            line["flowcurve"] = {"error": repr(e)}
    if not a.no_flowcurve and not a.no_surrogate:
        try:
            line["surrogate"] = surrogate_rates()
        except Exception as e:  # reported, never hidden
            line["surrogate"] = {"error": repr(e)}
    if a.knee:
        from paper_1004_5058_amd import surrogate
        try:
            line["knee_refinement"] = surrogate.knee_refinement(
                couplings=((-9.0, 8.1), (-9.2, 8.0), (-8.8, 7.7)),
                log=lambda m: print(f"# knee refinement: {m}", file=sys.stderr, flush=True))
        except Exception as e:  # reported, never hidden
            line["knee_refinement"] = {"error": repr(e)}
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n)
        line["cpu_baseline"]["single_thread"] = cpu_single_thread()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
