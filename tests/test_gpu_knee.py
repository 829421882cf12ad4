"""The knee-refinement path end to end on a reduced ensemble: batched
lattices (heights 256 and 384, 2000 steps, moment form) train the network,
which proposes rates around the Herschel-Bulkley knee of two fixed-coupling
curves; each proposal is checked by a 1024 x 512 population-form lattice run
of the same length.  The full-size run (2000 training lattices of all five
heights, 10 000 steps) is the benchmark's --knee leg.

What a broken path fails here: the knee and the proposals are recomputed from
the network's own sampled curve (Herschel-Bulkley fit, knee where the power
term equals the yield stress, rates log-spaced over a decade each side,
clipped to the ensemble's range); the checking stress of a proposal is
recomputed by an independent single-lattice run, bit for bit; the trained
network must explain most of the variance of its own training targets.  (On
held-out rows it does not beat the constant predictor at this reduced size:
the ensemble's stress is not a function of the network's inputs, see the
benchmark's knee leg; that is printed, not asserted.)"""
import numpy as np
import pytest

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu
K, STEPS, SEED = 4, 2000, 100


@pytest.fixture(scope="module")
def knee():
    need_gpu()
    from paper_1004_5058_amd import surrogate
    r = surrogate.knee_refinement(n_train=96, steps=STEPS, couplings=((-9.0, 8.1), (-9.3, 8.0)), k=K,
                                  heights=(256, 384), seed=SEED, log=print)
    print(f"\nreduced knee refinement: {r['accepted']}/{r['proposals']} within 1 %, held-out median error "
          f"{r['held_out_rel_err_median']:.3f} (constant predictor {r['held_out_rel_err_const_median']:.3f}), "
          f"wall {r['wall_s']} s")
    return r


def test_bookkeeping(knee):
    r = knee
    assert r["train_lattices"] == 86 and r["held_out"] == 10 and r["check_lattice"] == "1024x512"
    assert np.isfinite(r["train_loss"]) and np.isfinite(r["held_out_rel_err_median"])
    for c in r["curves"]:
        lat = np.array(c["sigma_lattice"])
        assert np.all(np.isfinite(lat))
        err = np.abs(np.array(c["sigma_network"]) - lat) / np.abs(lat)
        np.testing.assert_allclose(err, c["rel_err"], rtol=1e-12)
        assert c["accepted"] == int(np.sum(err <= 0.01))
    assert r["accepted"] == sum(c["accepted"] for c in r["curves"]) and r["proposals"] == 2 * K


def test_proposals_follow_the_network_knee(knee):
    from paper_1004_5058_amd import flowcurve
    S_lo, S_hi = knee["S_range"]
    assert 0 < S_lo < S_hi
    for c in knee["curves"]:
        Sg, sg = np.array(c["network_curve"]["S"]), np.array(c["network_curve"]["sigma"])
        assert Sg[0] == pytest.approx(S_lo, rel=1e-12) and Sg[-1] == pytest.approx(S_hi, rel=1e-12)
        fit = flowcurve.hb_fit(Sg, sg)
        for key in ("sigma_y", "B", "beta"):
            assert fit[key] == pytest.approx(c["hb_network"][key], rel=1e-9, abs=1e-300)
        if fit["sigma_y"] > 1e-9 * np.abs(sg).max() and fit["B"] > 0:
            sk = float(np.clip((fit["sigma_y"] / fit["B"]) ** (1.0 / fit["beta"]), S_lo, S_hi))
        else:
            sk = float(np.sqrt(S_lo * S_hi))
        assert c["knee_S"] == pytest.approx(sk, rel=1e-9)
        want = np.logspace(np.log10(max(S_lo, sk / 10)), np.log10(min(S_hi, sk * 10)), K)
        np.testing.assert_allclose(c["S"], want, rtol=1e-12)


def test_checking_run_is_an_independent_lattice_result(knee):
    """The first proposal of the first curve, run again as one lattice (not a
    batch), gives the recorded checking stress bit for bit."""
    from paper_1004_5058_amd import flowcurve, inputs, lb
    c = knee["curves"][0]
    S0 = c["S"][0]
    d = dict(nx=1024, ny=512, u_wall=float(S0) * 512 / 2.0, g_aa1=c["g_aa1"], g_bb1=c["g_aa1"],
             g_aa2=c["g_aa2"], g_bb2=c["g_aa2"], seed=c["check_seed"])
    s = flowcurve.lattice_specs([d], inputs.COUPLINGS)[0]
    kw = {k: v for k, v in s.items() if k not in ("nx", "ny", "rho_a", "rho_b", "ux", "uy")}
    lat = lb.Lattice(s["nx"], s["ny"], s["rho_a"], s["rho_b"], s["ux"], s["uy"], storage="f32", **kw)
    try:
        lat.step(STEPS // 2)
        lat.stress_reset()
        lat.step(STEPS - STEPS // 2)
        sb, st, n = lat.stress()
    finally:
        lat.close()
    assert n == STEPS - STEPS // 2
    assert 0.5 * (sb + st) == c["sigma_lattice"][0]


def test_network_fits_its_training_rows(knee):
    """A broken training step (no update, wrong gradient sign, unscaled
    targets) leaves the training error at or above the targets' variance."""
    print(f"\ntraining rows: target MSE {knee['train_target_mse']:.4g}, variance {knee['train_target_var']:.4g}")
    assert knee["train_target_var"] > 0
    assert knee["train_target_mse"] < 0.5 * knee["train_target_var"]
