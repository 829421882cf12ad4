"""Flow-curve surrogate: an MLP (HIP training/inference kernels, include/mlp.h)
mapping (G^a, G^r, log S) to the time-averaged wall stress of a Couette
lattice, trained on points from batched lattice runs, used to propose where
to refine a fixed-coupling flow curve near the yield stress.  Lattice runs
check every proposal and remain the reference for the surrogate's error.

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
        stress) on the surrogate's flow curve, and the fit itself.  A curve
        without a yield stress (below 1e-9 of its largest stress: round-off of
        the fit) has no knee; the middle of the range is returned."""
        S = np.logspace(np.log10(S_lo), np.log10(S_hi), n)
        sig = self.predict(g1, g2, S)
        fit = flowcurve.hb_fit(S, sig)
        if fit["sigma_y"] <= 1e-9 * float(np.max(np.abs(sig))) or fit["B"] <= 0:
            return float(np.sqrt(S_lo * S_hi)), fit
        sk = (fit["sigma_y"] / fit["B"]) ** (1.0 / fit["beta"])
        return float(np.clip(sk, S_lo, S_hi)), fit

    def curve(self, g1, g2):
        """The network's curve x = log S -> asinh target at fixed couplings."""
        return lambda x: to_target(self.predict(g1, g2, np.exp(np.asarray(x, dtype=np.float64))))

    def root(self, g1, g2, sigma_target, S_lo, S_hi, n=512):
        """The network's shear rate for sigma_target on [S_lo, S_hi] (grid
        point nearest in asinh space) and its local slope dt/dlog S there."""
        x = np.linspace(np.log(S_lo), np.log(S_hi), n)
        t = to_target(self.predict(g1, g2, np.exp(x)))
        k = int(np.argmin(np.abs(t - to_target(sigma_target))))
        a, b = max(k - 2, 0), min(k + 2, n - 1)
        slope = (t[b] - t[a]) / (x[b] - x[a])
        return float(x[k]), float(slope)

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



def knee_refinement(n_train=2000, steps=10000, couplings=((-9.0, 8.1),), k=6, width=1.0, train_storage="mom32",
                    check_nx=1024, check_ny=512, heights=(256, 384, 512, 768, 1024), seed=100, iters=4000,
                    lr=3e-3, tol=0.01, log=None):
    """Refinement of fixed-coupling flow curves near the yield stress, proposed
    by a network trained on the batched ensemble and checked by lattice runs.

    n_train lattices drawn like the batched flow-curve ensemble (heights,
    width 2H, wall speeds log-uniform in [1e-4, 5e-2], G^r and G^a uniform)
    run `steps` steps in batches (storage `train_storage`; the moment form is
    exact at tau = 1); every tenth row is held out, the rest train the network.
    For each (G^a, G^r) in `couplings` the network's flow curve over the
    ensemble's range of nominal rates is fitted (Herschel-Bulkley), k rates
    log-spaced within +-width decades of its knee are proposed, and each is
    checked by a check_nx x check_ny population-form (FP32) lattice run of the
    same length.  A proposal is accepted when the network's stress is within
    tol of the lattice's.  Returns the errors, counts and wall times."""
    t0 = time.perf_counter()
    rows, t_ens = ensemble_points(n_train, steps, seed=seed, heights=heights, storage=train_storage, log=log)
    train = [r for i, r in enumerate(rows) if i % 10]
    held = rows[::10]
    surr = FlowSurrogate(max_rows=max(len(train), 1), seed=0)
    loss, t_fit = surr.fit(train, iters=iters, lr=lr)
    g1h = np.array([r["g_aa1"] for r in held])
    g2h = np.array([r["g_aa2"] for r in held])
    Sh = np.array([r["S"] for r in held])
    sh = np.array([r["sigma"] for r in held])
    e_held = np.abs(surr.predict(g1h, g2h, Sh) - sh) / np.maximum(np.abs(sh), 1e-300)
    # the same error of the constant predictor (the training rows' median stress)
    e_const = np.abs(np.median([r["sigma"] for r in train]) - sh) / np.maximum(np.abs(sh), 1e-300)
    # the fit to the training rows in the network's own target space
    yt = to_target([r["sigma"] for r in train])
    pt = to_target(surr.predict(np.array([r["g_aa1"] for r in train]), np.array([r["g_aa2"] for r in train]),
                                np.array([r["S"] for r in train])))
    S_all = np.array([r["S"] for r in rows])
    S_lo, S_hi = float(S_all.min()), float(S_all.max())
    curves, t_chk, accepted, total = [], 0.0, 0, 0
    for c, (g1, g2) in enumerate(couplings):
        S_prop, fit = surr.propose(g1, g2, S_lo, S_hi, k=k, width=width)
        pred = surr.predict(g1, g2, S_prop)
        S_grid = np.logspace(np.log10(S_lo), np.log10(S_hi), 400)      # the curve knee() fits
        check_seed = seed + 10000 + 100 * c
        lb_rows, w = lb_flow_points(S_prop, g1, g2, steps, ny=check_ny, nx=check_nx, seed=check_seed)
        t_chk += w
        lbs = np.array([r["sigma"] for r in lb_rows])
        err = np.abs(pred - lbs) / np.maximum(np.abs(lbs), 1e-300)
        ok = int(np.sum(err <= tol))
        accepted += ok
        total += len(S_prop)
        curves.append(dict(g_aa1=g1, g_aa2=g2, knee_S=float(surr.knee(g1, g2, S_lo, S_hi)[0]),
                           hb_network=fit, S=[float(x) for x in S_prop], sigma_network=[float(x) for x in pred],
                           sigma_lattice=[float(x) for x in lbs], rel_err=[float(x) for x in err],
                           accepted=ok, hb_lattice=flowcurve.hb_fit(S_prop, lbs) if len(S_prop) >= 3 else None,
                           check_seed=check_seed,
                           network_curve=dict(S=[float(x) for x in S_grid],
                                              sigma=[float(x) for x in surr.predict(g1, g2, S_grid)])))
        if log:
            log(f"coupling ({g1}, {g2}): knee {curves[-1]['knee_S']:.3e}, errors "
                + ", ".join(f"{x:.3f}" for x in err))
    wall = time.perf_counter() - t0
    return dict(train_lattices=len(train), held_out=len(held), steps=steps, train_storage=train_storage,
                check_lattice=f"{check_nx}x{check_ny}", S_range=[S_lo, S_hi], train_loss=float(loss),
                held_out_rel_err_median=float(np.median(e_held)), held_out_rel_err_p90=float(np.quantile(e_held, 0.9)),
                held_out_rel_err_const_median=float(np.median(e_const)),
                train_target_mse=float(np.mean((pt - yt) ** 2)), train_target_var=float(np.var(yt)),
                ensemble_s=round(t_ens, 2), train_s=round(t_fit, 2), check_s=round(t_chk, 2), wall_s=round(wall, 2),
                proposals=total, accepted=accepted, points_per_hour=round(accepted * 3600.0 / wall, 1),
                curves=curves)


class RateSolver:
    """Stress-controlled point: the shear rate S in [S_lo, S_hi] at which a
    lattice's time-averaged wall stress equals sigma_target, to a relative
    tolerance tol, found from lattice runs only (every accepted point is a
    lattice result; no method accepts a predicted stress).

    Works in x = log S and t = asinh(sigma / SIGMA_UNIT), where a power-law
    flow curve is close to a straight line.  method:
      "bisect"   bisection of the bracket;
      "secant"   safeguarded secant: starts at the bracket's midpoint with
                 the Newtonian slope dt/dx = 1, then uses the slope through
                 the last two lattice points (the previous slope if that is
                 not positive); a step leaving the bracket, or one taken
                 when three runs have not halved the bracket, is replaced
                 by bisection;
      "surrogate" starts at the network's root; after each lattice run it
                 moves to the root of the network's curve shifted by that
                 run's residual (t_lattice - t_network at the run's S), so
                 the network supplies the shape of the curve and the
                 lattice its level; same bracket and stall safeguards.
                 model(x array) -> t array is the network's curve at the
                 case's couplings.
    A bracket narrower than min_width in log S with no accepted point means
    the flow curve jumps across the target there (a discontinuous branch
    change): the solver stops with jump = True and no result.
    Driven by propose() -> S or None (done) and update(sigma)."""

    def __init__(self, sigma_target, S_lo, S_hi, method="secant", x0=None, slope0=1.0, tol=0.01,
                 max_runs=40, min_width=1e-3, model=None):
        self.target = float(sigma_target)
        self.tt = float(to_target(sigma_target))
        self.lo, self.hi = np.log(S_lo), np.log(S_hi)
        self.method = method
        self.x = 0.5 * (self.lo + self.hi) if x0 is None else float(np.clip(x0, self.lo, self.hi))
        self.slope = float(slope0)
        self.tol = tol
        self.max_runs = max_runs
        self.runs = 0
        self.prev = None
        self.min_width = min_width
        self.model = model
        if method == "surrogate" and model is None:
            raise ValueError("the surrogate method needs the network's curve")
        self.widths = [self.hi - self.lo]
        self.result = None          # (S, sigma) once accepted
        self.jump = False

    def propose(self):
        if self.result is not None or self.jump or self.runs >= self.max_runs:
            return None
        return float(np.exp(self.x))

    def update(self, sigma):
        self.runs += 1
        x, t = self.x, float(to_target(sigma))
        if abs(sigma - self.target) <= self.tol * abs(self.target):
            self.result = (float(np.exp(x)), float(sigma))
            return
        if t < self.tt:
            self.lo = max(self.lo, x)
        else:
            self.hi = min(self.hi, x)
        if self.hi - self.lo < self.min_width:
            self.jump = True
            return
        mid = 0.5 * (self.lo + self.hi)
        self.widths.append(self.hi - self.lo)
        # secant steps that have not halved the bracket over three runs
        # (a kink or a jump between the points) give way to bisection
        stalled = len(self.widths) > 3 and self.widths[-1] > 0.5 * self.widths[-4]
        if self.method == "bisect" or stalled:
            self.x = mid
            self.prev = (x, t)
            return
        if self.method == "surrogate":
            self.prev = (x, t)
            self.x = self._shifted_root(x, t, mid)
            return
        if self.prev is not None and self.prev[0] != x:
            s = (t - self.prev[1]) / (x - self.prev[0])
            if s > 0:
                self.slope = s
        self.prev = (x, t)
        xn = x + (self.tt - t) / self.slope if self.slope > 0 else mid
        self.x = xn if self.lo < xn < self.hi else mid

    def _shifted_root(self, x, t, mid, n=257):
        """Root inside the bracket of model(x') + (t - model(x)) = target,
        linearly interpolated between grid points; the midpoint if the
        shifted curve does not cross the target inside the bracket."""
        c = t - float(self.model(np.array([x]))[0])
        g = np.linspace(self.lo, self.hi, n)[1:-1]
        r = np.asarray(self.model(g), dtype=np.float64) + c - self.tt
        cross = np.nonzero(np.signbit(r[:-1]) != np.signbit(r[1:]))[0]
        if cross.size == 0:
            return mid
        k = cross[np.argmin(np.abs(g[cross] - x))]       # the crossing nearest the last run
        return float(g[k] - r[k] * (g[k + 1] - g[k]) / (r[k + 1] - r[k]))


def solve_batched(solvers, lb_eval_many):
    """Advance solvers in lockstep: each round gathers every open solver's
    proposal and runs them as one lattice batch.  lb_eval_many(list of
    (solver index, S)) -> list of sigma.  Returns the number of rounds."""
    rounds = 0
    while True:
        todo = [(k, s.propose()) for k, s in enumerate(solvers)]
        todo = [(k, S) for k, S in todo if S is not None]
        if not todo:
            return rounds
        sig = lb_eval_many(todo)
        for (k, _), v in zip(todo, sig):
            solvers[k].update(v)
        rounds += 1


def lattice_stresses(points, nx, ny, steps, seed, storage="f32", batched=True):
    """Time-averaged wall stress of fixed-coupling Couette lattices at
    (g1, g2, S) points, all started from the same seeded emulsion: one batch
    (one launch per step for all lattices), or one lattice at a time (the
    plain loop)."""
    draws = [dict(nx=nx, ny=ny, u_wall=S * ny / 2.0, g_aa1=g1, g_bb1=g1, g_aa2=g2, g_bb2=g2, seed=seed)
             for g1, g2, S in points]
    specs = flowcurve.lattice_specs(draws, inputs.COUPLINGS)
    if batched:
        rows, _ = flowcurve.run_batched(specs, steps, storage=storage)
    else:
        rows, _ = flowcurve.run_plain(specs, steps, storage=storage)
    return [r["sigma"] for r in rows]


def stress_controlled_points(cases, targets, method, lb_eval_many, S_lo, S_hi, surr=None, tol=0.01):
    """Run one solver per case (g1, g2, _) towards its target stress, in
    lockstep rounds through lb_eval_many; returns (solvers, rounds)."""
    solvers = []
    for (g1, g2, _), t in zip(cases, targets):
        x0, sl, model = None, 1.0, None
        if method == "surrogate":
            x0, sl = surr.root(g1, g2, t, S_lo, S_hi)
            model = surr.curve(g1, g2)
        solvers.append(RateSolver(t, S_lo, S_hi, method=method, x0=x0, slope0=sl, tol=tol, model=model))
    rounds = solve_batched(solvers, lambda todo: lb_eval_many([(cases[k][0], cases[k][1], S) for k, S in todo]))
    return solvers, rounds


class RootSearch:
    """Stress-controlled point with k lattice runs per round: the shear rate
    in [S_lo, S_hi] at which a lattice's time-averaged wall stress equals
    sigma_target to a relative tolerance tol, from lattice runs only (the
    accepted point is the lattice run closest to the target among those
    within tolerance).

    Works in x = log S and t = asinh(sigma / SIGMA_UNIT).  The bracket
    [lo, hi] holds the target's crossing: after each round it is narrowed to
    the first pair of neighbouring results (lattice runs inside it, sorted in
    x, with the bracket ends) that straddle the target.  placement:
      "ksect"  k rates dividing the bracket into k + 1 equal parts (k = 1:
               bisection);
      "model"  k rates centred on a model's root, spread by h: at first the
               root of model(x) = target with h = h0; after lattice results,
               the root of the model shifted onto the nearest result
               (model(x) + t_lattice - model(x_lattice)) with h halved each
               round and never wider than the bracket allows.  model(x array)
               -> t array is the network's curve at the case's couplings.
    A bracket narrower than min_width with no accepted run means the flow
    curve jumps across the target there: the search stops (jump = True)."""

    def __init__(self, sigma_target, S_lo, S_hi, k=4, placement="ksect", model=None, h0=0.1, tol=0.01,
                 min_width=1e-3, max_rounds=12):
        self.target = float(sigma_target)
        self.tt = float(to_target(sigma_target))
        self.lo, self.hi = float(np.log(S_lo)), float(np.log(S_hi))
        self.k = int(k)
        self.placement = placement
        if placement == "model" and model is None:
            raise ValueError("model placement needs the network's curve")
        self.model = model
        self.h = float(h0)
        self.tol = tol
        self.min_width = min_width
        self.max_rounds = max_rounds
        self.rounds = 0
        self.runs = 0
        self.points = []            # (x, t, sigma) of every lattice run
        self.result = None          # (S, sigma) once accepted
        self.jump = False
        self._pending = None

    def done(self):
        return self.result is not None or self.jump or self.rounds >= self.max_rounds

    def _model_root(self, c=0.0):
        """Root of model(x) + c = target inside the bracket (grid, linear
        interpolation), the crossing nearest the bracket's centre; None if none."""
        g = np.linspace(self.lo, self.hi, 257)
        r = np.asarray(self.model(g), dtype=np.float64) + c - self.tt
        cross = np.nonzero(np.signbit(r[:-1]) != np.signbit(r[1:]))[0]
        if cross.size == 0:
            return None
        mid = 0.5 * (self.lo + self.hi)
        q = cross[np.argmin(np.abs(g[cross] - mid))]
        return float(g[q] - r[q] * (g[q + 1] - g[q]) / (r[q + 1] - r[q]))

    def propose(self):
        """The k rates of this round, or None when done."""
        if self.done():
            return None
        w = self.hi - self.lo
        if self.placement == "ksect":
            xs = [self.lo + w * (i + 1) / (self.k + 1) for i in range(self.k)]
        else:
            if self.points:
                # shift the model onto the lattice result nearest the bracket's centre
                mid = 0.5 * (self.lo + self.hi)
                xn, tn, _ = min(self.points, key=lambda p: abs(p[0] - mid))
                c = tn - float(self.model(np.array([xn]))[0])
                centre = self._model_root(c)
            else:
                centre = self._model_root()
            if centre is None:
                centre = 0.5 * (self.lo + self.hi)
            h = min(self.h, w / (self.k + 1))
            xs = [centre + h * (i - 0.5 * (self.k - 1)) for i in range(self.k)]
            # inside the bracket: shift the pattern, else spread it over the bracket
            if xs[0] <= self.lo or xs[-1] >= self.hi:
                shift = max(self.lo + 0.5 * h - xs[0], min(0.0, self.hi - 0.5 * h - xs[-1]))
                xs = [x + shift for x in xs]
                if xs[0] <= self.lo or xs[-1] >= self.hi:
                    xs = [self.lo + w * (i + 1) / (self.k + 1) for i in range(self.k)]
            self.h *= 0.5
        self._pending = xs
        return [float(np.exp(x)) for x in xs]

    def update(self, sigmas):
        xs = self._pending
        self._pending = None
        self.rounds += 1
        self.runs += len(sigmas)
        ok = []
        for x, s in zip(xs, sigmas):
            self.points.append((x, float(to_target(s)), float(s)))
            if abs(s - self.target) <= self.tol * abs(self.target):
                ok.append((abs(s - self.target), x, float(s)))
        if ok:
            _, x, s = min(ok)
            self.result = (float(np.exp(x)), s)
            return
        # narrow the bracket to the first straddling neighbours
        inside = sorted((x, t) for x, t, _ in self.points if self.lo < x < self.hi)
        seq = [(self.lo, -np.inf)] + inside + [(self.hi, np.inf)]
        for (xa, ta), (xb, tb) in zip(seq[:-1], seq[1:]):
            if ta < self.tt <= tb:
                self.lo, self.hi = xa, xb
                break
        if self.hi - self.lo < self.min_width:
            self.jump = True


def search_batched(searches, lb_eval_many):
    """Advance searches in lockstep rounds: each round gathers every open
    search's k rates and runs them as one lattice batch.  lb_eval_many(list of
    (search index, S)) -> list of sigma.  Returns the number of rounds."""
    rounds = 0
    while True:
        todo = []
        for k, s in enumerate(searches):
            p = s.propose()
            if p is not None:
                todo.append((k, p))
        if not todo:
            return rounds
        flat = [(k, S) for k, p in todo for S in p]
        sig = lb_eval_many(flat)
        o = 0
        for k, p in todo:
            searches[k].update(sig[o:o + len(p)])
            o += len(p)
        rounds += 1


def rows_of(searches, cases):
    """Training rows (couplings, S, sigma) of every lattice run of searches."""
    rows = []
    for s, (g1, g2, _) in zip(searches, cases):
        rows += [dict(g_aa1=g1, g_aa2=g2, S=float(np.exp(x)), sigma=sig) for x, _, sig in s.points]
    return rows


def stream_points(cases_a, targets_a, cases_b, targets_b, lattice, S_lo, S_hi, k=4, use_network=False,
                  surr=None, iters=4000, lr=3e-3, h0=0.1, log=None, batch_a=None):
    """Stress-controlled points for a stream of two batches of cases, batched:
    batch A by k-section; batch B by k-section, or, with use_network, by
    network placement, the network (surr, a FlowSurrogate) trained by the HIP
    kernels on every lattice run of batch A (the runs the stream has made
    anyway; no separate training ensemble).  lattice(list of (g1, g2, S)) ->
    list of sigma.  Returns a report with wall times (training included),
    lattice runs, rounds and accepted points per batch.  batch_a: the
    (solvers, rounds, wall seconds) of an earlier run of batch A with the
    same arguments (the returned solvers and the report's A rounds and wall
    time), reused instead of searching batch A again: its lattice runs are
    deterministic, and reusing them charges the stream batch A's time as
    measured then."""
    import time as _t

    def run(cases, targets, placement, model_of=None):
        t0 = _t.perf_counter()
        ss = []
        for (g1, g2, _), t in zip(cases, targets):
            ss.append(RootSearch(t, S_lo, S_hi, k=k, placement=placement,
                                 model=model_of(g1, g2) if model_of else None, h0=h0))
        rounds = search_batched(ss, lambda todo: lattice([(cases[j][0], cases[j][1], S) for j, S in todo]))
        return ss, rounds, _t.perf_counter() - t0

    out = {}
    sa, ra, wa = batch_a if batch_a is not None else run(cases_a, targets_a, "ksect")
    out["A"] = _summary(sa, ra, wa)
    t_train = 0.0
    if use_network:
        t0 = _t.perf_counter()
        rows = rows_of(sa, cases_a)
        surr.fit(rows, iters=iters, lr=lr)
        t_train = _t.perf_counter() - t0
        out["train"] = dict(rows=len(rows), wall_s=round(t_train, 3))
        sb, rb, wb = run(cases_b, targets_b, "model", model_of=surr.curve)
    else:
        sb, rb, wb = run(cases_b, targets_b, "ksect")
    out["B"] = _summary(sb, rb, wb)
    acc = out["A"]["accepted"] + out["B"]["accepted"]
    wall = wa + t_train + wb
    out.update(accepted=acc, lattice_runs=out["A"]["lattice_runs"] + out["B"]["lattice_runs"],
               wall_s=round(wall, 3), points_per_hour=round(acc * 3600.0 / wall, 1))
    for s, t in zip(sa + sb, list(targets_a) + list(targets_b)):
        if s.result is not None:
            assert abs(s.result[1] - t) <= s.tol * abs(t)
    if log:
        log(out)
    return out, sa, sb


def _summary(ss, rounds, wall):
    return dict(cases=len(ss), accepted=sum(s.result is not None for s in ss), jumps=sum(s.jump for s in ss),
                lattice_runs=sum(s.runs for s in ss), rounds=rounds, wall_s=round(wall, 3),
                status="".join("a" if s.result is not None else ("j" if s.jump else "c") for s in ss))


# The stress-controlled setting the surrogate is trained and judged in: 256 x 128
# Couette lattices, 20000 steps, common seeded start, couplings straddling the
# edge of the emulsion region, wall speeds 6e-3 .. 6e-2.
GAIN = dict(nx=256, ny=128, steps=20000, seed=7, g1=(-9.2, -9.0), g2=(7.9, 8.1), u=(6e-3, 6e-2))


def draw_points(n, seed, s_range, g1_range, g2_range, max_sum=None):
    """(g1, g2, S) draws: couplings uniform, S log-uniform; with max_sum,
    draws above G^a + G^r = max_sum are moved onto it (the emulsion side)."""
    rng = np.random.default_rng(seed)
    g1 = rng.uniform(*g1_range, n)
    g2 = rng.uniform(*g2_range, n)
    if max_sum is not None:
        over = g1 + g2 > max_sum
        g2[over] -= (g1 + g2 - max_sum)[over]
    S = np.exp(rng.uniform(np.log(s_range[0]), np.log(s_range[1]), n))
    return list(zip(g1.tolist(), g2.tolist(), S.tolist()))
