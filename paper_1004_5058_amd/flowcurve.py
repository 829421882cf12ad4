"""Flow curves sigma(S) from batched Couette lattices, and the Herschel-Bulkley
fit sigma = sigma_Y + B S^beta (section "Numerical Results": the yield stress,
the master curve and the exponent fit).

Shear rate.  Each lattice is sheared between walls at +U and -U a distance
ny apart: the nominal rate is S = 2U/ny.  The measured bulk rate S_bulk is the
least-squares slope of the time-averaged line profile U(y) over the central
half of the channel (the paper measures S = dU/dy of the time-averaged
profile).  The stress is the time-averaged wall shear stress, the mean of the
two walls; their difference is reported as a steadiness check.

The fit (host, FP64) is variable projection: on a grid of beta in (0, 2] the
pair (sigma_Y, B) is the linear least-squares solution with sigma_Y >= 0; the
best grid point is polished by Gauss-Newton on all three parameters.
"""
import time

import numpy as np


def hb_fit(S, sigma, beta_grid=None, polish=True):
    """Fit sigma = sigma_Y + B S^beta to points with S > 0.

    Returns dict(sigma_y, B, beta, rss)."""
    S = np.asarray(S, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    keep = S > 0
    S, sigma = S[keep], sigma[keep]
    if S.size < 3:
        raise ValueError("need at least three points with S > 0")
    if beta_grid is None:
        beta_grid = np.linspace(0.01, 2.0, 400)
    logS = np.log(S)

    def solve(beta):
        p = np.exp(beta * logS)
        A = np.column_stack([np.ones_like(p), p])
        coef, *_ = np.linalg.lstsq(A, sigma, rcond=None)
        sy, B = coef
        if sy < 0:                        # constrained: sigma_Y = 0
            sy = 0.0
            B = float(p @ sigma / (p @ p))
        r = sigma - sy - B * p
        return float(r @ r), float(sy), float(B)

    best = None
    for beta in beta_grid:
        rss, sy, B = solve(beta)
        if best is None or rss < best[0]:
            best = (rss, sy, B, float(beta))
    rss, sy, B, beta = best
    if polish:
        x = np.array([sy, B, beta])
        for _ in range(50):
            p = np.exp(x[2] * logS)
            r = sigma - x[0] - x[1] * p
            J = np.column_stack([np.ones_like(p), p, x[1] * p * logS])
            step, *_ = np.linalg.lstsq(J, r, rcond=None)
            xn = x + step
            if xn[0] < 0:
                xn[0] = 0.0
            pn = np.exp(xn[2] * logS)
            rn = sigma - xn[0] - xn[1] * pn
            if rn @ rn <= r @ r:
                x = xn
                if np.max(np.abs(step) / (np.abs(x) + 1e-300)) < 1e-13:
                    break
            else:
                break
        p = np.exp(x[2] * logS)
        r = sigma - x[0] - x[1] * p
        if r @ r <= rss:
            sy, B, beta, rss = float(x[0]), float(x[1]), float(x[2]), float(r @ r)
    return dict(sigma_y=sy, B=B, beta=beta, rss=rss)


def hb_curve(rows):
    """Herschel-Bulkley fits of one fixed-coupling flow curve (rows of
    run_batched / run_plain): sigma against the nominal rate S = 2U/ny and
    against the bulk rate S_bulk of the time-averaged profile (the paper's
    measured dU/dy; points with S_bulk <= 0 are dropped), with the spread of
    S_bulk / S and the largest relative difference of the two walls' stresses
    (zero in a steady state)."""
    S = np.array([r["S"] for r in rows], dtype=np.float64)
    Sb = np.array([r["S_bulk"] for r in rows], dtype=np.float64)
    sig = np.array([r["sigma"] for r in rows], dtype=np.float64)
    steady = np.array([r["steady"] for r in rows], dtype=np.float64)
    out = dict(points=int(S.size), nominal=hb_fit(S, sig))
    ok = Sb > 0
    out["bulk"] = hb_fit(Sb[ok], sig[ok]) if int(ok.sum()) >= 3 else None
    out["bulk_points"] = int(ok.sum())
    ratio = Sb / S
    out["S_bulk_over_S"] = dict(median=float(np.median(ratio)), min=float(ratio.min()), max=float(ratio.max()))
    out["wall_mismatch_max"] = float(steady.max())
    out["wall_mismatch_median"] = float(np.median(steady))
    return out


def bulk_rate(profile):
    """Least-squares slope of U(y) over the central half of the channel."""
    ny = len(profile)
    a, b = ny // 4, ny - ny // 4
    y = np.arange(a, b, dtype=np.float64)
    return float(np.polyfit(y, np.asarray(profile[a:b], dtype=np.float64), 1)[0])


def lattice_specs(draws, couplings, init="emulsion"):
    """Build lb.Batch specs from ensemble draws (inputs.ensemble)."""
    from . import inputs
    specs = []
    for d in draws:
        nx, ny, u = d["nx"], d["ny"], d["u_wall"]
        if init == "emulsion":
            ra, rb = inputs.emulsion(nx, ny, seed=d["seed"])
        else:
            ra, rb = inputs.noise(nx, ny, seed=d["seed"])
        ux, uy = inputs.couette(nx, ny, u, -u)
        c = dict(couplings)
        for k in ("g_aa1", "g_aa2", "g_bb1", "g_bb2"):
            if k in d:
                c[k] = d[k]
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=ux, uy=uy, u_top=u, u_bot=-u, **c))
    return specs


def run_batched(specs, steps, storage="f32", average_from=None, bx=0, ly=0, grid=0, graph=32, tune_cache=None):
    """Advance all lattices together (one step kernel per time step, HIP
    graphs); average the stress and profile over the last steps - average_from
    steps (default: the second half).  With tune_cache, the batch takes its
    launch shape and steps per pass from the autotuner (a cached entry is
    applied without timing; tune beforehand to keep tuning out of the run),
    else the given shape."""
    import torch
    from . import lb
    if average_from is None:
        average_from = steps // 2
    t0 = time.perf_counter()
    b = lb.Batch(specs, storage=storage, profile=True)
    if tune_cache is not None:
        b.autotune(tune_cache, steps=10)
    elif bx or ly or grid:
        b.set_launch(bx, ly, grid)
    b.set_graph(graph)
    b.step(average_from)
    b.stress_reset()
    b.step(steps - average_from)
    sb, st, n = b.stress()
    rows = []
    for k, s in enumerate(specs):
        prof, _ = b.profile(k)
        sig = 0.5 * (sb[k] + st[k])
        rows.append(dict(nx=s["nx"], ny=s["ny"], u_wall=s["u_top"], S=2 * s["u_top"] / s["ny"],
                         S_bulk=bulk_rate(prof), sigma=sig, sigma_bot=sb[k], sigma_top=st[k],
                         steady=abs(sb[k] - st[k]) / max(abs(sig), 1e-300),
                         g_aa1=s["g_aa1"], g_aa2=s["g_aa2"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    return rows, wall


def run_plain(specs, steps, storage="f32", average_from=None, tune_cache=None):
    """The same runs one lattice at a time, one kernel launch per step (or
    per two steps where the tuner picked that), no graph: the baseline the
    batched path is measured against.  With tune_cache, every lattice size is
    autotuned once before the timed loop (results cached in that JSON file)
    and each lattice applies the cached entry of its size (shape and steps
    per pass; no timing); otherwise the library's default shape."""
    import torch
    from . import lb
    if average_from is None:
        average_from = steps // 2

    def kwargs(s):
        return {k: v for k, v in s.items() if k not in ("nx", "ny", "rho_a", "rho_b", "ux", "uy")}

    if tune_cache is not None:
        tuned = set()
        for s in specs:
            key = (s["nx"], s["ny"])
            if key in tuned:
                continue
            lat = lb.Lattice(s["nx"], s["ny"], s["rho_a"], s["rho_b"], s["ux"], s["uy"], storage=storage,
                             profile=True, **kwargs(s))
            lat.set_graph(0)
            lat.autotune(tune_cache, steps=10)
            lat.close()
            tuned.add(key)
    t0 = time.perf_counter()
    rows = []
    for s in specs:
        lat = lb.Lattice(s["nx"], s["ny"], s["rho_a"], s["rho_b"], s["ux"], s["uy"], storage=storage,
                         profile=True, **kwargs(s))
        lat.set_graph(0)
        if tune_cache is not None:
            lat.autotune(tune_cache, steps=10)      # the cached entry of this size
        lat.step(average_from)
        lat.stress_reset()
        lat.step(steps - average_from)
        sb, st, _ = lat.stress()
        prof, _ = lat.profile()
        sig = 0.5 * (sb + st)
        rows.append(dict(nx=s["nx"], ny=s["ny"], u_wall=s["u_top"], S=2 * s["u_top"] / s["ny"],
                         S_bulk=bulk_rate(prof), sigma=sig, sigma_bot=sb, sigma_top=st,
                         steady=abs(sb - st) / max(abs(sig), 1e-300), g_aa1=s["g_aa1"], g_aa2=s["g_aa2"]))
        lat.close()
    torch.cuda.synchronize()
    return rows, time.perf_counter() - t0
