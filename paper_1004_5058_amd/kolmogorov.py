"""The paper's own driving protocol (section "Numerical Results").

A fully periodic L x L box; the two species start from sinusoidal density
modulations rho_A = 0.61 (1 + 0.1 sin(k_in y)), rho_B = 0.61 (1 + 0.01 sin(k_in y)),
k_in = 64 pi / L, at rest; an external body force along x, F_x(y) = F0 sin(k_f y)
with k_f = 2 pi / L, drives the flow.  F0 is set so that a Newtonian fluid of the
same density and viscosity would settle into the Kolmogorov flow
u_x = U0 sin(k_f y): F0 = rho nu k_f^2 U0, nu = (tau - 1/2) / 3.

Observables (host analysis of what the kernels return):
- the line-averaged speed U_x(y, t) = (1/L) sum_x u_x(x, y, t) (`lb_line_profile`);
- the response R(t) = Uhat(t) / U0 with Uhat = (2/L) sum_y U_x(y, t) sin(k_f y); R = 1
  for the laminar Newtonian flow, R < 1 measures the slowing down;
- the time-averaged profile U(y) (the FP64 profile accumulators of the step);
- the stress from the momentum balance d_y P_xy = F_x.  With a periodic stress of
  zero mean, P_xy(y) = -(F0 / k_f) cos(k_f y); the paper's scatter pairs |P_xy(y)|
  with the local shear |dU/dy| of the time-averaged profile, and fits
  sigma = sigma_Y + B S^beta to it (Fig. 4).
"""
import time

import numpy as np

from . import flowcurve, inputs

# The paper's coupling set (footnote of "Numerical Results"): asymmetric A/B,
# A-B repulsion on belt 1 only, tau = 1; rho0 is the swept parameter.
PAPER_COUPLINGS = dict(tau=1.0, g_aa1=-9.0, g_aa2=8.1, g_bb1=-8.0, g_bb2=7.1, g_ab=0.045)


def wavenumber(L):
    return 2.0 * np.pi / L


def forcing_amplitude(U0, L, tau, rho):
    """F0 = rho nu k_f^2 U0: the amplitude whose laminar response is U0 sin(k_f y)."""
    nu = (tau - 0.5) / 3.0
    return rho * nu * wavenumber(L) ** 2 * U0


def response(profile, U0):
    """R = (2/L) sum_y U_x(y) sin(k_f y) / U0 for a line-averaged profile."""
    U = np.asarray(profile, dtype=np.float64)
    L = U.size
    y = np.arange(L, dtype=np.float64)
    return float(2.0 / L * np.dot(U, np.sin(wavenumber(L) * y)) / U0)


def stress_profile(F0, L):
    """P_xy(y) = -(F0/k_f) cos(k_f y): the zero-mean periodic solution of d_y P_xy = F_x."""
    y = np.arange(L, dtype=np.float64)
    k = wavenumber(L)
    return -(F0 / k) * np.cos(k * y)


def shear_profile(profile):
    """dU/dy of a periodic profile by central differences."""
    U = np.asarray(profile, dtype=np.float64)
    return 0.5 * (np.roll(U, -1) - np.roll(U, 1))


def scatter(profile, F0):
    """(|S(y)|, |P_xy(y)|) pairs of the paper's stress/shear scatter."""
    U = np.asarray(profile, dtype=np.float64)
    return np.abs(shear_profile(U)), np.abs(stress_profile(F0, U.size))


def initial_densities(L, nx=None, init="paper", seed=1):
    """init = "paper": the paper's start, rho_A = 0.61 (1 + 0.1 sin(k_in y)),
    rho_B = 0.61 (1 + 0.01 sin(k_in y)); "emulsion": the seeded demixed start
    of the sheared workloads (per site (1.0, 0.1) or (0.1, 1.0))."""
    nx = L if nx is None else nx
    if init == "emulsion":
        return inputs.emulsion(nx, L, seed=seed)
    if init != "paper":
        raise ValueError(f"unknown start {init!r}")
    k_in = 64.0 * np.pi / L
    return inputs.sinusoid_y(nx, L, 0.61, 0.1, k_in), inputs.sinusoid_y(nx, L, 0.61, 0.01, k_in)


def lattice_kwargs(L, rho0, U0, couplings=None, rho=1.22):
    """Parameters of one protocol lattice (periodic in y, body force on)."""
    c = dict(PAPER_COUPLINGS if couplings is None else couplings)
    tau = c.get("tau", 1.0)
    return dict(c, rho0=rho0, walls=False, fx_amp=forcing_amplitude(U0, L, tau, rho), fx_k=wavenumber(L))


def run(L=512, rho0=0.83, U0=0.1, steps=100000, sample_every=1000, average_from=None, storage="f32",
        couplings=None, device="cuda:0", init="paper", log=None, tune=True):
    """Run the protocol on one lattice.  Returns R(t) samples, the profile
    averaged over [average_from, steps), the stress/shear scatter and its
    Herschel-Bulkley fit (None when fewer than three flowing points).  With
    tune, the autotuner picks the launch shape and, for FP32, the steps per
    pass before the run (the results do not depend on either)."""
    from . import lb
    if average_from is None:
        average_from = steps // 2
    ra, rb = initial_densities(L, init=init)
    kw = lattice_kwargs(L, rho0, U0, couplings, rho=float(np.mean(ra + rb)))
    F0 = kw["fx_amp"]
    lat = lb.Lattice(L, L, ra, rb, None, None, device=device, storage=storage, profile=True, **kw)
    if tune:
        lat.autotune(None, steps=5)
    t0 = time.perf_counter()
    ts, Rs = [], []
    t = 0
    averaging = False
    while t < steps:
        if not averaging and t >= average_from:
            lat.stress_reset()
            averaging = True
        n = min(sample_every, steps - t)
        if not averaging:
            n = min(n, average_from - t)
        lat.step(n)
        t += n
        Rs.append(response(lat.line_profile(), U0))
        ts.append(t)
        if log:
            log(f"t={t} R={Rs[-1]:.4f}")
    if not averaging:
        lat.stress_reset()
    prof, nsamp = lat.profile()
    wall = time.perf_counter() - t0
    lat.close()
    S, P = scatter(prof, F0)
    flowing = S > 1e-3 * max(S.max(), 1e-300)
    fit = None
    if np.count_nonzero(flowing) >= 3:
        try:
            fit = flowcurve.hb_fit(S[flowing], P[flowing])
        except ValueError:
            fit = None
    return dict(L=L, rho0=rho0, U0=U0, F0=F0, steps=steps, t=np.array(ts), R=np.array(Rs), profile=prof,
                samples=nsamp, R_mean=response(prof, U0) if nsamp else float("nan"), S=S, sigma=P,
                sigma0=F0 / wavenumber(L), fit=fit, wall_s=wall, mlups=L * L * steps / wall * 1e-6)


def sweep(rho0_list, L=512, U0=0.1, steps=100000, sample_every=1000, average_from=None, storage="f32",
          couplings=None, device="cuda:0", tune=True, init="paper", log=None):
    """The protocol at several rho0 at once: one lattice per rho0 in one batch
    (one launch per step for all of them).  Returns one result dict per rho0
    (as `run`) plus the batch's wall time."""
    from . import lb
    if average_from is None:
        average_from = steps // 2
    ra, rb = initial_densities(L, init=init)
    kws = [lattice_kwargs(L, r0, U0, couplings, rho=float(np.mean(ra + rb))) for r0 in rho0_list]
    specs = [dict(nx=L, ny=L, rho_a=ra, rho_b=rb, ux=None, uy=None, **kw) for kw in kws]
    b = lb.Batch(specs, device=device, storage=storage, profile=True)
    if tune:
        b.autotune(None, steps=5)
    t0 = time.perf_counter()
    n = len(specs)
    ts, Rs = [], [[] for _ in range(n)]
    t = 0
    averaging = False
    while t < steps:
        if not averaging and t >= average_from:
            b.stress_reset()
            averaging = True
        m = min(sample_every, steps - t)
        if not averaging:
            m = min(m, average_from - t)
        b.step(m)
        t += m
        ts.append(t)
        for k in range(n):
            Rs[k].append(response(b.line_profile(k), U0))
        if log:
            log(f"t={t} R=" + " ".join(f"{R[-1]:.4f}" for R in Rs))
    if not averaging:
        b.stress_reset()
    wall = time.perf_counter() - t0
    out = []
    for k, (r0, kw) in enumerate(zip(rho0_list, kws)):
        prof, nsamp = b.profile(k)
        F0 = kw["fx_amp"]
        S, P = scatter(prof, F0)
        flowing = S > 1e-3 * max(S.max(), 1e-300)
        fit = None
        if np.count_nonzero(flowing) >= 3:
            try:
                fit = flowcurve.hb_fit(S[flowing], P[flowing])
            except ValueError:
                fit = None
        out.append(dict(L=L, rho0=r0, U0=U0, F0=F0, steps=steps, t=np.array(ts), R=np.array(Rs[k]),
                        profile=prof, samples=nsamp, R_mean=response(prof, U0) if nsamp else float("nan"),
                        S=S, sigma=P, sigma0=F0 / wavenumber(L), fit=fit))
    b.close()
    return out, wall


def vft_fit(rho0, inv_R, rho_c_grid=None):
    """Fit 1/R = A exp(B / (rho_c - rho0)) (section "Numerical Results", Fig. 5):
    for each rho_c above the data, ln(1/R) is linear in 1/(rho_c - rho0), so
    (ln A, B) is a linear least-squares solve; the best rho_c on the grid is
    then refined by golden-section search.  Returns dict(A, B, rho_c, rss)."""
    x = np.asarray(rho0, dtype=np.float64)
    z = np.log(np.asarray(inv_R, dtype=np.float64))
    if x.size < 3:
        raise ValueError("need at least three points")
    lo = x.max() + 1e-6
    if rho_c_grid is None:
        rho_c_grid = lo + np.logspace(-5, 0, 400)

    def solve(rc):
        A = np.column_stack([np.ones_like(x), 1.0 / (rc - x)])
        coef, *_ = np.linalg.lstsq(A, z, rcond=None)
        r = z - A @ coef
        return float(r @ r), coef

    best = min(rho_c_grid, key=lambda rc: solve(rc)[0])
    i = int(np.searchsorted(rho_c_grid, best))
    a = rho_c_grid[max(i - 1, 0)]
    b = rho_c_grid[min(i + 1, len(rho_c_grid) - 1)]
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    for _ in range(200):
        if solve(c)[0] < solve(d)[0]:
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    rc = 0.5 * (a + b)
    rss, coef = solve(rc)
    return dict(A=float(np.exp(coef[0])), B=float(coef[1]), rho_c=float(rc), rss=rss)
