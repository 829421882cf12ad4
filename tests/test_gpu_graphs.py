"""Graph replays, each one checked: lattices that step through captured HIP
graphs (8 steps per graph, one replay per step call) match twins that launch
every step directly, bit for bit after every replay, with the library's own
eager work between the replays (population and field reads, FP64 sums, a
stress reset) and the synchronisations those imply.  FP32 with one and two
steps per pass, FP16 deviation, the moment form, and a batch of uneven
lattices."""
import numpy as np
import pytest

from gpu_common import gpu_lattice, need_gpu
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu
REPLAYS = 6


@pytest.mark.parametrize("storage,per_pass", [("f32", 1), ("f32", 2), ("f16dev", 1), ("mom32", 1)])
def test_every_replay_matches_direct_launches(storage, per_pass):
    need_gpu()
    nx, ny, u = 200, 72, 0.02
    ra, rb = inputs.emulsion(nx, ny, seed=21)
    ux, uy = inputs.couette(nx, ny, u, -u)
    lats = []
    for graph in (0, 8):
        lat = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=u, u_bot=-u, storage=storage)
        lat.set_fusion(per_pass)
        lat.set_graph(graph)
        lats.append(lat)
    direct, graphed = lats
    for k in range(REPLAYS):
        for lat in lats:
            lat.step(8)
        np.testing.assert_array_equal(graphed.populations(), direct.populations(), err_msg=f"replay {k}")
        for a, b in zip(graphed.fields(), direct.fields()):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(np.asarray(graphed.sums()), np.asarray(direct.sums()))
        assert graphed.stress() == direct.stress()
        if k == 2:
            for lat in lats:
                lat.stress_reset()
    assert graphed.time() == direct.time() == 8 * REPLAYS
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("per_pass", [1, 2])
def test_every_batch_replay_matches_direct_launches(per_pass):
    need_gpu()
    from paper_1004_5058_amd import lb
    specs = []
    for k, (nx, ny) in enumerate([(256, 128), (100, 37), (512, 64)]):
        ra, rb = inputs.emulsion(nx, ny, seed=30 + k)
        u = 0.01 * (k + 1)
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, u_top=u, u_bot=-u,
                          g_aa2=7.9 + 0.1 * k))
    batches = []
    for graph in (0, 8):
        b = lb.Batch(specs, storage="f32", profile=True)
        b.set_fusion(per_pass)
        b.set_graph(graph)
        batches.append(b)
    direct, graphed = batches
    for k in range(REPLAYS):
        for b in batches:
            b.step(8)
        for i in range(len(specs)):
            for x, y in zip(graphed.fields(i), direct.fields(i)):
                np.testing.assert_array_equal(x, y, err_msg=f"replay {k}, lattice {i}")
            np.testing.assert_array_equal(graphed.profile(i)[0], direct.profile(i)[0])
        for x, y in zip(graphed.stress(), direct.stress()):
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
        if k == 2:
            for b in batches:
                b.stress_reset()
    for b in batches:
        b.close()
