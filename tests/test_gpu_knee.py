"""The knee-refinement path end to end on a reduced ensemble: batched
lattices (heights 256 and 384, 2000 steps, moment form) train the network,
which proposes rates around the Herschel-Bulkley knee of two fixed-coupling
curves; each proposal is checked by a 1024 x 512 population-form lattice run
of the same length.  The full-size run (2000 training lattices of all five
heights, 10 000 steps) is the benchmark's --knee leg."""
import numpy as np
import pytest

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def test_knee_refinement_reduced():
    need_gpu()
    from paper_1004_5058_amd import surrogate
    r = surrogate.knee_refinement(n_train=96, steps=2000, couplings=((-9.0, 8.1), (-9.3, 8.0)), k=4,
                                  heights=(256, 384), log=print)
    assert r["train_lattices"] == 86 and r["held_out"] == 10 and r["check_lattice"] == "1024x512"
    assert np.isfinite(r["train_loss"]) and np.isfinite(r["held_out_rel_err_median"])
    S_lo, S_hi = r["S_range"]
    assert 0 < S_lo < S_hi
    for c in r["curves"]:
        S = np.array(c["S"])
        assert len(S) == 4 and np.all(np.diff(np.log(S)) > 0)
        assert S[0] >= S_lo * (1 - 1e-12) and S[-1] <= S_hi * (1 + 1e-12)
        assert S[0] >= c["knee_S"] / 10 * (1 - 1e-9) and S[-1] <= c["knee_S"] * 10 * (1 + 1e-9)
        lat = np.array(c["sigma_lattice"])
        assert np.all(np.isfinite(lat))
        err = np.abs(np.array(c["sigma_network"]) - lat) / np.abs(lat)
        np.testing.assert_allclose(err, c["rel_err"], rtol=1e-12)
        assert c["accepted"] == int(np.sum(err <= 0.01))
    assert r["accepted"] == sum(c["accepted"] for c in r["curves"]) and r["proposals"] == 8
    print(f"\nreduced knee refinement: {r['accepted']}/{r['proposals']} within 1 %, held-out median error "
          f"{r['held_out_rel_err_median']:.3f}, wall {r['wall_s']} s")
