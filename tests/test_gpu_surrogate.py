"""What the trained surrogate gains: stress-controlled flow-curve points.

Each case asks for the shear rate at which a fixed-coupling Couette lattice
(256 x 128, 20000 steps, stress averaged over the second half, every lattice
started from the same seeded emulsion so that the stress is one deterministic
function of (G, S)) reaches a target wall stress to 1 %.  Every round runs k
lattices per open case as one batch; an accepted point is always a lattice
result.  A stream of two batches of cases: batch A by k-section; batch B by
k-section (the method without the network) or placed by the network, which
the HIP kernels train on batch A's own lattice runs (no separate training
ensemble).

The bar for the network: on batch B it accepts at least as many cases as
k-section does on the same cases, in no more rounds and with fewer lattice
runs, and no case exhausts its rounds.  Cases the network's search does not
accept are jumps of the fixed-seed flow curve across the target (droplet
break-up), which stop any method."""
import numpy as np
import pytest

from gpu_common import need_gpu
from paper_1004_5058_amd import surrogate

pytestmark = pytest.mark.gpu

_G = surrogate.GAIN
NX, NY, STEPS, SEED = _G["nx"], _G["ny"], _G["steps"], _G["seed"]
S_LO, S_HI = 2 * _G["u"][0] / NY, 2 * _G["u"][1] / NY
K = 4


def _lb(points):
    return surrogate.lattice_stresses(points, NX, NY, STEPS, SEED)


def _cases(seed, n=10):
    return surrogate.draw_points(n, seed, (1.5e-4, 6e-4), (-9.2, -9.05), (7.9, 8.05), max_sum=-0.98)


@pytest.fixture(scope="module")
def streams():
    need_gpu()
    ca, cb = _cases(31), _cases(47)
    targets = _lb(ca + cb)
    ta, tb = targets[:len(ca)], targets[len(ca):]
    ks, _, _ = surrogate.stream_points(ca, ta, cb, tb, _lb, S_LO, S_HI, k=K)
    surr = surrogate.FlowSurrogate(max_rows=2048, seed=0)
    net, sa, sb = surrogate.stream_points(ca, ta, cb, tb, _lb, S_LO, S_HI, k=K, use_network=True, surr=surr)
    for name, r in (("k-section", ks), ("network", net)):
        print(f"\n{name}: A {r['A']}\n{'':10s} B {r['B']}\n{'':10s} total {r['accepted']} accepted, "
              f"{r['lattice_runs']} runs, {r['wall_s']} s, {r['points_per_hour']} points/h")
    return ks, net, surr, cb, sb


def test_network_trained_on_batch_a_runs_only(streams):
    ks, net, surr, _, _ = streams
    assert net["train"]["rows"] == net["A"]["lattice_runs"] == ks["A"]["lattice_runs"]
    assert surr.trained == net["train"]["rows"]
    assert net["A"] == {**ks["A"], "wall_s": net["A"]["wall_s"]}      # batch A: the same search


def test_network_gains_on_batch_b(streams):
    ks, net, _, _, _ = streams
    kb, nb = ks["B"], net["B"]
    assert "c" not in nb["status"] and "c" not in kb["status"]
    assert nb["accepted"] >= kb["accepted"]
    assert nb["rounds"] <= kb["rounds"]
    assert nb["lattice_runs"] < kb["lattice_runs"]


def test_network_error_on_batch_b_runs(streams):
    """Held-out accuracy: the network's stress at batch B's lattice runs (new
    couplings and rates) against those runs."""
    _, _, surr, cb, sb = streams
    err = np.array([abs(float(surr.predict(g1, g2, np.exp(x))[0]) - sig) / abs(sig)
                    for s, (g1, g2, _) in zip(sb, cb) for x, _, sig in s.points])
    print(f"network error on batch B's runs: median {np.median(err):.3f}, 90% {np.quantile(err, 0.9):.3f}")
    assert np.median(err) < 0.15
