"""Stress-controlled rate search (host logic) on analytic Herschel-Bulkley
flow curves: every method accepts only points within tolerance of the curve
it queries, bisection needs the number of halvings its bracket implies, and a
start from the exact root with the exact slope needs one run."""
import numpy as np
import pytest

from paper_1004_5058_amd.surrogate import RateSolver, solve_batched, to_target

S_LO, S_HI = 1e-4, 1e-3


def hb(S, sy=2e-5, B=4e-3, beta=0.5):
    return sy + B * np.asarray(S) ** beta


def _run(solvers, curve):
    calls = []

    def many(todo):
        calls.append(len(todo))
        return [curve(S) for _, S in todo]
    rounds = solve_batched(solvers, many)
    return rounds, calls


@pytest.mark.parametrize("method", ["bisect", "secant", "surrogate"])
def test_accepted_points_meet_tolerance(method):
    targets = hb(np.array([1.3e-4, 2.7e-4, 6.1e-4, 9.5e-4]))
    solvers = []
    for t in targets:
        x0, sl = None, 1.0
        model = None
        if method == "surrogate":               # a model 5 % off in stress
            S = np.logspace(-4, -3, 2001)
            k = np.argmin(np.abs(1.05 * hb(S) - t))
            x0, sl = np.log(S[k]), 0.45
            model = lambda x: to_target(1.05 * hb(np.exp(x)))
        solvers.append(RateSolver(t, S_LO, S_HI, method=method, x0=x0, slope0=sl, tol=0.01, model=model))
    rounds, calls = _run(solvers, hb)
    for s, t in zip(solvers, targets):
        assert s.result is not None
        S, sig = s.result
        assert abs(sig - t) <= 0.01 * t and sig == hb(S)
    assert rounds == max(s.runs for s in solvers)
    assert sum(calls) == sum(s.runs for s in solvers)


def test_exact_model_needs_one_run():
    t = hb(3.3e-4)
    x = np.log(3.3e-4)
    sl = float((to_target(hb(np.exp(x + 1e-6))) - to_target(hb(np.exp(x - 1e-6)))) / 2e-6)
    s = RateSolver(t, S_LO, S_HI, method="surrogate", x0=x, slope0=sl, model=lambda x: to_target(hb(np.exp(x))))
    _run([s], hb)
    assert s.runs == 1


def test_shifted_model_step_corrects_a_level_error():
    """A model with the right shape and a 20 % level error: one run gives the
    offset, the shifted model's root is then the true root (two runs)."""
    model = lambda x: to_target(1.2 * hb(np.exp(x), sy=0.0))
    curve = lambda S: hb(S, sy=0.0)
    for S_true in (1.2e-4, 3e-4, 8e-4):
        t = curve(S_true)
        xs = np.linspace(np.log(S_LO), np.log(S_HI), 4001)
        x0 = xs[np.argmin(np.abs(model(xs) - to_target(t)))]
        s = RateSolver(t, S_LO, S_HI, method="surrogate", x0=x0, model=model)
        _run([s], curve)
        assert s.result is not None and s.runs <= 2


def test_bisection_count_matches_bracket():
    """With sigma ~ S (Newtonian), a 1 % stress window is a 1 % window in S:
    bisection stops within ceil(log2(ln(S_hi/S_lo) / 0.01)) + 1 halvings."""
    lin = lambda S: (1 / 6) * np.asarray(S)
    rng = np.random.default_rng(0)
    bound = int(np.ceil(np.log2(np.log(S_HI / S_LO) / 0.01))) + 1
    for S_true in np.exp(rng.uniform(np.log(S_LO), np.log(S_HI), 20)):
        s = RateSolver(lin(S_true), S_LO, S_HI, method="bisect")
        _run([s], lin)
        assert s.result is not None and s.runs <= bound
        s2 = RateSolver(lin(S_true), S_LO, S_HI, method="secant")
        _run([s2], lin)
        assert s2.runs <= 2               # the Newtonian start slope is exact


def test_non_monotone_curve_still_accepts_a_root():
    """A curve with a dip keeps its bracket logic: the solver lands on some
    point within tolerance, never outside [S_lo, S_hi]."""
    wiggly = lambda S: hb(S) * (1 + 0.08 * np.sin(40 * np.log(S)))
    for method in ("bisect", "secant"):
        for S_true in (1.5e-4, 4e-4, 8e-4):
            s = RateSolver(wiggly(S_true), S_LO, S_HI, method=method)
            _run([s], wiggly)
            assert s.result is not None
            assert S_LO <= s.result[0] <= S_HI


def test_jump_across_target_stops():
    """A curve that steps over the target (no point within tolerance) ends
    with jump set: bisection after log2(bracket / min_width) runs, the secant
    within three runs per halving."""
    step = lambda S: np.where(np.asarray(S) < 3e-4, 1e-5, 1e-4)
    for method in ("bisect", "secant"):
        s = RateSolver(3e-5, S_LO, S_HI, method=method)
        _run([s], step)
        assert s.result is None and s.jump
        halvings = int(np.ceil(np.log2(np.log(S_HI / S_LO) / 1e-3)))
        assert s.runs <= (halvings + 2 if method == "bisect" else 3 * halvings)


# ------------------------------------------------ k lattice runs per round ---

from paper_1004_5058_amd.surrogate import RootSearch, search_batched, stream_points  # noqa: E402


def _search(searches, curve):
    calls = []

    def many(todo):
        calls.append(len(todo))
        return [curve(S) for _, S in todo]
    return search_batched(searches, many), calls


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_ksection_accepts_within_tolerance_in_the_rounds_its_bracket_implies(k):
    """k-section shrinks the bracket (k + 1)-fold per round: on a continuous
    curve the accepted run is within tolerance and the round count is at most
    what the bracket reduction to the tolerance's width in log S implies."""
    targets = hb(np.array([1.3e-4, 2.7e-4, 6.1e-4, 9.5e-4]))
    ss = [RootSearch(t, S_LO, S_HI, k=k) for t in targets]
    rounds, calls = _search(ss, hb)
    for s, t in zip(ss, targets):
        assert s.result is not None and abs(s.result[1] - t) <= 0.01 * t and s.result[1] == hb(s.result[0])
        assert s.runs == k * s.rounds
    # dt/dx >= 0.3 here, so any run within 0.01 / 0.3 in x of the root is accepted
    need = int(np.ceil(np.log(np.log(S_HI / S_LO) / (2 * 0.01 / 0.3)) / np.log(k + 1))) + 1
    assert rounds <= need
    assert sum(calls) == sum(s.runs for s in ss)


def test_model_placement_exact_model_accepts_in_one_round():
    t = hb(3.3e-4)
    s = RootSearch(t, S_LO, S_HI, k=4, placement="model", model=lambda x: to_target(hb(np.exp(x))), h0=0.05)
    _search([s], hb)
    assert s.rounds == 1 and s.result is not None


def test_model_placement_with_a_level_error():
    """A model with the right shape and a 20 % level error: the first round
    (around its wrong root) gives the offset, the shifted model's root is then
    the true root: two rounds at most."""
    targets = hb(np.array([1.7e-4, 4.4e-4, 8.0e-4]))
    ss = [RootSearch(t, S_LO, S_HI, k=4, placement="model", model=lambda x: to_target(1.2 * hb(np.exp(x))),
                     h0=0.05) for t in targets]
    _search(ss, hb)
    for s, t in zip(ss, targets):
        assert s.result is not None and s.rounds <= 2 and abs(s.result[1] - t) <= 0.01 * t


def test_jump_across_the_target_stops_the_search():
    """A curve that jumps over the target: no run can be within 1 %; the
    bracket closes on the jump and the search reports it."""
    def jumpy(S):
        S = np.asarray(S)
        return np.where(S < 4e-4, hb(S), 1.5 * hb(S))
    t = 1.2 * hb(4e-4)
    for placement, model in (("ksect", None), ("model", lambda x: to_target(hb(np.exp(x))))):
        s = RootSearch(t, S_LO, S_HI, k=4, placement=placement, model=model)
        _search([s], jumpy)
        assert s.result is None and s.jump and s.rounds < s.max_rounds
        assert abs(np.exp(s.lo) - 4e-4) / 4e-4 < 2e-3


def test_stream_trains_on_its_own_runs_and_counts_everything():
    """stream_points: batch A by k-section, the network fitted on exactly A's
    lattice runs, batch B placed by it; every lattice call is counted and the
    wall time includes the training."""
    cases_a = [(-9.1, 8.0, 0.0)] * 3
    cases_b = [(-9.1, 8.0, 0.0)] * 2
    ta = list(hb(np.array([1.5e-4, 3.0e-4, 7.0e-4])))
    tb = list(hb(np.array([2.2e-4, 5.5e-4])))
    seen = []

    def lattice(pts):
        seen.extend(pts)
        return [float(hb(S)) for _, _, S in pts]

    class Fake:
        def fit(self, rows, iters, lr):
            self.rows = rows
            return 0.0, 0.0

        def curve(self, g1, g2):
            return lambda x: to_target(1.05 * hb(np.exp(np.asarray(x))))
    surr = Fake()
    out, sa, sb = stream_points(cases_a, ta, cases_b, tb, lattice, S_LO, S_HI, k=4, use_network=True, surr=surr)
    assert len(surr.rows) == sum(s.runs for s in sa) == out["A"]["lattice_runs"]
    assert out["lattice_runs"] == len(seen) and out["accepted"] == 5
    assert out["B"]["rounds"] <= 2 and out["train"]["rows"] == len(surr.rows)
