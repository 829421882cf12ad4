"""Seeded synthetic inputs shared by the HIP path, its tests and the benchmark.

This module holds no lattice-Boltzmann arithmetic: it only draws initial
density and velocity fields (float64, shape (ny, nx)) and the ensemble
parameters, from numpy's PCG64 generator with a fixed seed, so that both the
GPU library and the CPU oracle start from byte-identical arrays.

Workload recipes (the paper itself runs a 512x512 periodic box; these are the
synthetic stand-ins of the same model):
  noise     rho_s = mean + U(-amp, amp), i.i.d. per site and species
  emulsion  per site a fair coin picks (rho_A, rho_B) = (major, minor) or
            (minor, major)
  couette   u_x(y) = u_bot + (u_top - u_bot) (y + 1/2) / ny, u_y = 0: the linear
            profile between walls at y = -1/2 and y = ny - 1/2
"""
import numpy as np


def noise(nx, ny, seed, mean=0.5, amp=0.01):
    rng = np.random.default_rng(seed)
    ra = mean + rng.uniform(-amp, amp, size=(ny, nx))
    rb = mean + rng.uniform(-amp, amp, size=(ny, nx))
    return ra, rb


def emulsion(nx, ny, seed, major=1.0, minor=0.1):
    rng = np.random.default_rng(seed)
    coin = rng.integers(0, 2, size=(ny, nx)).astype(bool)
    ra = np.where(coin, major, minor).astype(np.float64)
    rb = np.where(coin, minor, major).astype(np.float64)
    return ra, rb


def couette(nx, ny, u_top, u_bot):
    y = (np.arange(ny, dtype=np.float64) + 0.5) / ny
    ux = np.repeat((u_bot + (u_top - u_bot) * y)[:, None], nx, axis=1)
    return ux, np.zeros((ny, nx))


def sinusoid_y(nx, ny, mean, amp, k):
    """rho(y) = mean (1 + amp sin(k y)), constant along x."""
    y = np.arange(ny, dtype=np.float64)
    return np.repeat((mean * (1.0 + amp * np.sin(k * y)))[:, None], nx, axis=1)


# Coupling set of the hot-path workloads: symmetric A/B, belt-1 attraction,
# two-belt repulsion, belt-1 A-B repulsion, psi reference density 0.83.
COUPLINGS = dict(tau=1.0, rho0=0.83, g_aa1=-9.0, g_aa2=8.1, g_bb1=-9.0, g_bb2=8.1, g_ab=0.405)


def ensemble(n=48, seed=100, heights=(256, 384, 512, 768, 1024),
             u_range=(1e-4, 5e-2), g2_range=(7.5, 8.5), g1_range=None):
    """Parameter draws of the batched flow-curve ensemble.

    Each lattice: height H from `heights`, width 2H, wall speed U log-uniform
    in u_range (top +U, bottom -U), G^r_AA = G^r_BB uniform in g2_range and,
    if g1_range is given, G^a_AA = G^a_BB uniform in it.  Returns a list of
    dicts with the lattice's own init seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        h = int(rng.choice(heights))
        u = float(np.exp(rng.uniform(np.log(u_range[0]), np.log(u_range[1]))))
        g2 = float(rng.uniform(*g2_range))
        g1 = float(rng.uniform(*g1_range)) if g1_range else COUPLINGS["g_aa1"]
        out.append(dict(nx=2 * h, ny=h, u_wall=u, g_aa2=g2, g_bb2=g2,
                        g_aa1=g1, g_bb1=g1, seed=seed + k))
    return out
