"""Flow-curve surrogate: an MLP (HIP training/inference kernels, include/mlp.h)
mapping (G^a, G^r, log S) to the time-averaged wall stress of a Couette
lattice, trained on points from batched lattice runs, used to propose where
to refine a fixed-coupling flow curve near the yield stress.  Lattice runs
check every proposal and stay the judge of the surrogate's error.

The network regresses s = asinh(sigma / SIGMA_UNIT): close to log for
stresses well above SIGMA_UNIT and linear through zero, so small and
fluctuating stresses at low shear rate stay representable.
"""
import time

import numpy as np

from . import flowcurve, inputs

SIGMA_UNIT = 1e-7


def to_target(sigma):
    return np.arcsinh(np.asarray(sigma, dtype=np.float64) / SIGMA_UNIT)


def from_target(s):
    return SIGMA_UNIT * np.sinh(np.asarray(s, dtype=np.float64))


def features(g1, g2, S):
    return np.column_stack([np.asarray(g1, float), np.asarray(g2, float), np.log(np.asarray(S, float))])


def ensemble_points(n, steps, seed=100, heights=(256, 384, 512, 768, 1024), u_range=(1e-4, 5e-2),
                    g1_range=(-9.5, -8.5), g2_range=(7.5, 8.5), per_batch=48, storage="f32", log=None):
    """n lattice runs drawn like the batched flow-curve ensemble (plus G^a
    draws), advanced `per_batch` at a time through the batched step."""
    rows, wall = [], 0.0
    k = 0
    while k < n:
        m = min(per_batch, n - k)
        draws = inputs.ensemble(m, seed=seed + k, heights=heights, u_range=u_range, g2_range=g2_range,
                                g1_range=g1_range)
        specs = flowcurve.lattice_specs(draws, inputs.COUPLINGS)
        r, w = flowcurve.run_batched(specs, steps, storage=storage)
        rows += r
        wall += w
        k += m
        if log:
            log(f"ensemble: {k}/{n} points, {wall:.1f} s")
    return rows, wall


def _glorot(seed):
    """Glorot-uniform initial parameters in the mlp.h layout (biases zero)."""
    rng = np.random.default_rng(seed)
    H = 64

    def g(fo, fi):
        a = np.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))
    return np.concatenate([g(H, 3).ravel(), np.zeros(H), g(H, H).ravel(), np.zeros(H), g(1, H)[0],
                           [0.0]]).astype(np.float32)


class FlowSurrogate:
    """MLP surrogate of sigma(G^a, G^r, S) on the GPU kernels."""

    def __init__(self, max_rows=8192, seed=0, device="cuda:0"):
        from .mlp import MLP
        self.net = MLP(max_rows=max_rows, device=device)
        self.seed = seed
        self.trained = 0

    def fit(self, rows, iters=4000, lr=3e-3):
        X = features([r["g_aa1"] for r in rows], [r["g_aa2"] for r in rows], [r["S"] for r in rows])
        y = to_target([r["sigma"] for r in rows])
        self.net.set_params(_glorot(self.seed))
        sd = X.std(0)
        sd[sd == 0] = 1.0
        self.net.set_norm(X.mean(0), sd, float(y.mean()), float(max(y.std(), 1e-12)))
        self.net.set_data(X, y)
        t0 = time.perf_counter()
        loss = self.net.train(iters, lr)
        self.trained = len(rows)
        return loss, time.perf_counter() - t0

    def predict(self, g1, g2, S):
        S = np.atleast_1d(np.asarray(S, float))
        g1 = np.broadcast_to(g1, S.shape)
        g2 = np.broadcast_to(g2, S.shape)
        return from_target(self.net.infer(features(g1, g2, S)))

    def knee(self, g1, g2, S_lo, S_hi, n=400):
        """Shear rate where the fitted Herschel-Bulkley power term equals the
        yield stress (the crossover from yield-dominated to flow-dominated
        stress) on the surrogate's flow curve, and the fit itself."""
        S = np.logspace(np.log10(S_lo), np.log10(S_hi), n)
        fit = flowcurve.hb_fit(S, self.predict(g1, g2, S))
        if fit["sigma_y"] <= 0 or fit["B"] <= 0:
            return float(np.sqrt(S_lo * S_hi)), fit
        sk = (fit["sigma_y"] / fit["B"]) ** (1.0 / fit["beta"])
        return float(np.clip(sk, S_lo, S_hi)), fit

    def propose(self, g1, g2, S_lo, S_hi, k=6, width=1.0):
        """k shear rates log-spaced within +-width decades of the knee."""
        sk, fit = self.knee(g1, g2, S_lo, S_hi)
        lo = max(S_lo, sk * 10 ** (-width))
        hi = min(S_hi, sk * 10 ** width)
        return np.logspace(np.log10(lo), np.log10(hi), k), fit


def lb_flow_points(S_list, g1, g2, steps, ny=512, nx=1024, seed=500, storage="f32"):
    """Fixed-coupling lattice runs at the given nominal shear rates (walls at
    +-S ny / 2), batched; returns rows and wall time."""
    draws = []
    for k, S in enumerate(S_list):
        draws.append(dict(nx=nx, ny=ny, u_wall=float(S) * ny / 2.0, g_aa1=g1, g_bb1=g1, g_aa2=g2, g_bb2=g2,
                          seed=seed + k))
    specs = flowcurve.lattice_specs(draws, inputs.COUPLINGS)
    return flowcurve.run_batched(specs, steps, storage=storage)
