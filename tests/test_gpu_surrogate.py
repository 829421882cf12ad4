"""What the trained surrogate gains: stress-controlled flow-curve points.

Each case asks for the shear rate at which a fixed-coupling Couette lattice
reaches a target time-averaged wall stress (to 1 %).  Three solvers take
lattice runs until one is within tolerance, so a lattice run checks every
accepted point: bisection, a safeguarded secant without the network, and a
search that starts at the network's root and then follows the network's
curve shifted onto each lattice result.  The network is trained by the HIP
kernels on a batched lattice ensemble over the couplings and rates; its gain
is the number of lattice runs saved per accepted point.

Every lattice starts from the same seeded emulsion (common random numbers),
so the measured stress is one deterministic function of (G, S) for all
solvers and for the training data.  The training couplings straddle the edge
of the emulsion region (G^a + G^r near -0.9; beyond it the mixture dissolves
and the fluid is Newtonian); the gain cases lie inside it (G^a + G^r below
-0.98), where the flow curve is shear thinning and continuous.  Lattice
256 x 128, 20000 steps, stress averaged over the second half.  A solver that
fails (run cap, or a jump across the target) is charged its runs."""
import time

import numpy as np
import pytest

from gpu_common import need_gpu
from paper_1004_5058_amd import surrogate

pytestmark = pytest.mark.gpu

_G = surrogate.GAIN
NX, NY, STEPS, SEED = _G["nx"], _G["ny"], _G["steps"], _G["seed"]
G1, G2 = _G["g1"], _G["g2"]
U = _G["u"]
S_LO, S_HI = 2 * U[0] / NY, 2 * U[1] / NY


def _lb(points):
    """Lattice stress at (g1, g2, S) points, one batch."""
    return surrogate.lattice_stresses(points, NX, NY, STEPS, SEED)


def _draw(n, seed, s_range=(S_LO, S_HI), g1_range=G1, g2_range=G2, max_sum=None):
    return surrogate.draw_points(n, seed, s_range, g1_range, g2_range, max_sum)


@pytest.fixture(scope="module")
def trained():
    need_gpu()
    pts = _draw(512, seed=300)
    t0 = time.perf_counter()
    sig = _lb(pts)
    t_ens = time.perf_counter() - t0
    rows = [dict(g_aa1=g1, g_aa2=g2, S=S, sigma=s) for (g1, g2, S), s in zip(pts, sig)]
    surr = surrogate.FlowSurrogate(max_rows=1024, seed=0)
    loss, t_fit = surr.fit(rows, iters=4000, lr=3e-3)
    print(f"\nensemble: {len(rows)} lattices {NX}x{NY}x{STEPS} in {t_ens:.1f} s; "
          f"training loss {loss:.3e} in {t_fit:.1f} s")
    return surr


def test_surrogate_on_held_out_lattices(trained):
    pts = _draw(64, seed=900)
    sig = np.array(_lb(pts))
    pred = np.array([trained.predict(g1, g2, S)[0] for g1, g2, S in pts])
    rel = np.abs(pred - sig) / np.abs(sig)
    print(f"held-out relative stress error: median {np.median(rel):.3f}, "
          f"90% {np.quantile(rel, 0.9):.3f}, max {rel.max():.3f}")
    assert np.median(rel) < 0.15


def test_surrogate_saves_lattice_runs(trained):
    cases = _draw(10, seed=31, s_range=(1.5e-4, 6e-4), g1_range=(-9.2, -9.05), g2_range=(7.9, 8.05),
                  max_sum=-0.98)
    targets = _lb(cases)
    report = {}
    for method in ("bisect", "secant", "surrogate"):
        t0 = time.perf_counter()
        solvers, rounds = surrogate.stress_controlled_points(cases, targets, method, _lb, S_LO, S_HI,
                                                            surr=trained)
        wall = time.perf_counter() - t0
        runs = [s.runs for s in solvers]
        ok = sum(s.result is not None for s in solvers)
        status = "".join("a" if s.result is not None else ("j" if s.jump else "c") for s in solvers)
        report[method] = (sum(runs), ok, status)
        print(f"{method:9s}: {sum(runs):3d} lattice runs {runs}, {ok}/{len(solvers)} accepted [{status}] "
              f"(a accepted, j jump, c run cap), {rounds} batched rounds, {wall:.1f} s, "
              f"{sum(runs) / max(ok, 1):.2f} runs per accepted point")
        for s, t in zip(solvers, targets):
            if s.result is not None:
                assert abs(s.result[1] - t) <= 0.01 * abs(t)
    per = {m: r / max(ok, 1) for m, (r, ok, _) in report.items()}
    # A case that is not accepted is a jump of the fixed-seed flow curve across
    # its target (a droplet break-up), where no method can reach 1 %; which
    # cases straddle a jump moves with the FP32 rounding of these chaotic
    # emulsions.  What the method controls: no case runs out of its run
    # budget, and most cases are accepted.
    assert "c" not in report["surrogate"][2]
    assert report["surrogate"][1] >= len(cases) // 2
    assert per["surrogate"] < per["secant"] and per["surrogate"] < per["bisect"]
    assert report["surrogate"][0] < report["secant"][0] and report["surrogate"][0] < report["bisect"][0]
