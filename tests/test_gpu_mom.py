"""Moment form of the step at tau = 1 (storage "mom64" / "mom32"): six
moments per site instead of 18 populations, the same recurrence as Eq. (1)
with the velocity shift at tau = 1.  Checked against the FP64 oracle (which
steps populations) on fields, exported populations and wall stress, and for
bitwise independence of launch shape, batching and graphs."""
import numpy as np
import pytest

from gpu_common import compare_fields, err_pop, gpu_lattice, need_gpu, oracle_params, oracle_run
from oracle import oracle as O
from paper_1004_5058_amd import inputs, kolmogorov as K

pytestmark = pytest.mark.gpu
TOL = {"mom64": 1e-12, "mom32": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _couette(nx, ny, u=0.03, seed=1):
    ra, rb = inputs.emulsion(nx, ny, seed=seed)
    ux, uy = inputs.couette(nx, ny, u, -u)
    return ra, rb, ux, uy


@pytest.mark.parametrize("storage", ["mom64", "mom32"])
@pytest.mark.parametrize("nx,ny,steps", [(64, 48, 100), (131, 37, 100), (40, 2, 30), (70, 64, 1), (33, 17, 0)])
def test_couette_walls_against_oracle(storage, nx, ny, steps):
    u = 0.03
    ra, rb, ux, uy = _couette(nx, ny, u)
    p = oracle_params(nx, ny, True, u, -u)
    g, sb, st = oracle_run(p, ra, rb, ux, uy, steps)
    lat = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=u, u_bot=-u, storage=storage)
    lat.step(steps)
    tol = TOL[storage]
    e = compare_fields(lat, p, g, tol)
    assert err_pop(lat.populations(), g) <= 10 * tol
    if steps:
        gb, gt, n = lat.stress()
        assert n == steps
        assert abs(gb - sb) <= 10 * tol * abs(sb) and abs(gt - st) <= 10 * tol * abs(st)
    print(f"\n{storage} {nx}x{ny} {steps} steps: {e}")


@pytest.mark.parametrize("storage", ["mom64", "mom32"])
def test_periodic_noise_against_oracle(storage):
    nx, ny = 96, 64
    ra, rb = inputs.noise(nx, ny, seed=0)
    p = oracle_params(nx, ny, False, 0, 0)
    g, _, _ = oracle_run(p, ra, rb, None, None, 200)
    lat = gpu_lattice(nx, ny, ra, rb, walls=False, storage=storage)
    lat.step(200)
    compare_fields(lat, p, g, TOL[storage])
    assert err_pop(lat.populations(), g) <= 10 * TOL[storage]


@pytest.mark.parametrize("storage", ["mom64", "mom32"])
def test_paper_protocol_against_oracle(storage):
    """Body force, paper couplings, sinusoidal start, fully periodic."""
    L, nx = 64, 48
    kw = K.lattice_kwargs(L, 0.83, 0.1)
    ra, rb = K.initial_densities(L, nx)
    p = O.OracleParams(nx=nx, ny=L, **kw)
    g, _, _ = oracle_run(p, ra, rb, None, None, 100)
    lat = gpu_lattice(nx, L, ra, rb, storage=storage, **kw)
    lat.step(100)
    compare_fields(lat, p, g, TOL[storage])
    _, _, oux, _ = O.fields(p, g)
    assert np.max(np.abs(lat.line_profile() - oux.mean(axis=1))) <= TOL[storage]


def test_long_run_mom64_matches_oracle():
    nx, ny, u = 48, 40, 0.05
    ra, rb, ux, uy = _couette(nx, ny, u, seed=3)
    p = oracle_params(nx, ny, True, u, -u)
    g, sb, st = oracle_run(p, ra, rb, ux, uy, 1000)
    lat = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=u, u_bot=-u, storage="mom64")
    lat.step(1000)
    compare_fields(lat, p, g, 1e-11)


@pytest.mark.parametrize("bx,ly", [(64, 1), (64, 3), (128, 7), (256, 16), (256, 1000)])
def test_launch_shape_bitwise(bx, ly):
    nx, ny = 200, 52
    ra, rb, ux, uy = _couette(nx, ny, seed=5)
    ref = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32", profile=True)
    ref.step(9)
    lat = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32", profile=True)
    lat.set_launch(bx, ly)
    lat.step(9)
    np.testing.assert_array_equal(lat.populations(), ref.populations())
    assert lat.stress() == ref.stress()
    # the line profile is summed per tile (tiles overlap by four columns), so
    # its FP64 summation order follows the tile width
    np.testing.assert_allclose(lat.profile()[0], ref.profile()[0], rtol=1e-13, atol=1e-17)


def test_graphs_batch_and_checkpoint_are_bitwise():
    from paper_1004_5058_amd import lb
    nx, ny = 96, 40
    ra, rb, ux, uy = _couette(nx, ny, seed=6)
    direct = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32")
    direct.set_graph(0)
    direct.step(70)
    graph = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32")
    graph.set_graph(8)
    graph.step(70)
    np.testing.assert_array_equal(direct.populations(), graph.populations())
    # checkpoint at t = 30, continue, compare
    a = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32")
    a.step(30)
    buf = a.save()
    b = gpu_lattice(nx, ny, ra, rb, ux, uy, u_top=0.03, u_bot=-0.03, storage="mom32")
    b.load(buf)
    assert b.time() == 30
    b.step(40)
    np.testing.assert_array_equal(b.populations(), direct.populations())
    # batch of uneven lattices
    specs = []
    for k, (w, h) in enumerate([(96, 40), (50, 23), (130, 64)]):
        r1, r2, u1, u2 = _couette(w, h, seed=10 + k)
        specs.append(dict(nx=w, ny=h, rho_a=r1, rho_b=r2, ux=u1, uy=u2, u_top=0.03, u_bot=-0.03,
                          **inputs.COUPLINGS))
    bt = lb.Batch(specs, storage="mom32", profile=False)
    bt.step(25)
    for k, s in enumerate(specs):
        kw = {q: v for q, v in s.items() if q not in ("nx", "ny", "rho_a", "rho_b", "ux", "uy")}
        lat = lb.Lattice(s["nx"], s["ny"], s["rho_a"], s["rho_b"], s["ux"], s["uy"], storage="mom32", **kw)
        lat.step(25)
        for x, y in zip(bt.fields(k), lat.fields()):
            np.testing.assert_array_equal(x, y)
        lat.close()
    bt.close()


def test_conservation_periodic():
    nx, ny = 80, 64
    ra, rb = inputs.emulsion(nx, ny, seed=8)
    lat = gpu_lattice(nx, ny, ra, rb, walls=False, storage="mom64")
    s0 = lat.sums()
    lat.step(50)
    s1 = lat.sums()
    assert abs(s1[0] - s0[0]) < 1e-11 * s0[0] and abs(s1[1] - s0[1]) < 1e-11 * s0[1]
    assert abs(s1[2] - s0[2]) < 1e-10 and abs(s1[3] - s0[3]) < 1e-10


def test_narrowest_tiles_fit_the_item_table():
    """64-lane moment-form tiles collide 60 columns: a 64-wide lattice takes
    two strips, and with one-row segments the batch's item table must hold
    them (it is sized for 60-column tiles)."""
    from paper_1004_5058_amd import lb
    nx, ny, u = 64, 24, 0.01
    ra, rb = inputs.noise(nx, ny, 3)
    p = oracle_params(nx, ny, True, u, -u)
    g, _, _ = oracle_run(p, ra, rb, None, None, 20)
    b = lb.Batch([dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, u_top=u, u_bot=-u)],
                 storage="mom32", profile=False)
    b.set_launch(64, 1, 0)
    b.step(20)

    class _M:
        def fields(self):
            return b.fields(0)
    compare_fields(_M(), p, g, 1e-6)
    b.close()
