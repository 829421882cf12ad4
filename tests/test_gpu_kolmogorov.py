"""The paper's driving on the GPU (section "Numerical Results"): the body force
F_x(y) = F0 sin(k_f y) in the HIP step and the line-averaged profile call,
against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

from gpu_common import compare_fields, err_pop, gpu_lattice, need_gpu, oracle_run
from oracle import oracle as O
from paper_1004_5058_amd import inputs, kolmogorov as K

pytestmark = pytest.mark.gpu

ZERO = dict(g_aa1=0.0, g_aa2=0.0, g_bb1=0.0, g_bb2=0.0, g_ab=0.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _protocol(L, nx, rho0=0.83, U0=0.1, couplings=None):
    kw = K.lattice_kwargs(L, rho0, U0, couplings)     # includes walls=False
    ra, rb = K.initial_densities(L, nx)
    p = O.OracleParams(nx=nx, ny=L, **kw)
    return ra, rb, kw, p


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6)])
@pytest.mark.parametrize("L,nx", [(64, 64), (96, 70), (40, 131)])
def test_protocol_parity(storage, tol, L, nx):
    """Paper couplings, sinusoidal start, body force, fully periodic: fields,
    populations and the line profile after 100 steps."""
    ra, rb, kw, p = _protocol(L, nx)
    g, _, _ = oracle_run(p, ra, rb, None, None, 100)
    lat = gpu_lattice(nx, L, ra, rb, storage=storage, **kw)
    lat.step(100)
    e = compare_fields(lat, p, g, tol)
    assert err_pop(lat.populations(), g) <= 10 * tol
    _, _, oux, _ = O.fields(p, g)
    prof = lat.line_profile()
    ref = oux.mean(axis=1)
    assert np.max(np.abs(prof - ref)) <= 0.5 * tol
    print(f"\nL={L} nx={nx} {storage}: {e}, line profile {np.max(np.abs(prof - ref)):.2e}")


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_momentum_grows_by_the_body_force(storage, tol):
    """Couplings on, periodic: total x momentum gains nx sum_y F_x(y) per step."""
    nx, ny, F0, k = 96, 80, 2e-4, 0.29
    ra, rb = inputs.emulsion(nx, ny, seed=4)
    lat = gpu_lattice(nx, ny, ra, rb, walls=False, storage=storage, fx_amp=F0, fx_k=k, **K.PAPER_COUPLINGS)
    s0 = lat.sums()
    lat.step(20)
    s1 = lat.sums()
    want = 20 * nx * F0 * float(np.sum(np.sin(k * np.arange(ny))))
    assert s1[2] - s0[2] == pytest.approx(want, rel=tol)
    assert abs(s1[3] - s0[3]) < tol * abs(want)


def test_newtonian_kolmogorov_flow_on_gpu():
    """All couplings zero: the steady response equals the oracle's (R = 1 up to
    the lattice's second-order term), from the line profile and from the
    time-averaged profile accumulators."""
    L, nx, U0 = 64, 8, 0.01
    tau = 1.0
    kf = K.wavenumber(L)
    F0 = K.forcing_amplitude(U0, L, tau, 1.22)
    ra = np.full((L, nx), 0.61)
    steps = int(np.ceil(30.0 / ((tau - 0.5) / 3.0 * kf * kf)))
    p = O.OracleParams(nx=nx, ny=L, walls=False, tau=tau, fx_amp=F0, fx_k=kf, **ZERO)
    g, _, _ = oracle_run(p, ra, ra.copy(), None, None, steps)
    _, _, oux, _ = O.fields(p, g)
    R_ref = K.response(oux.mean(axis=1), U0)
    # FP32 bound: storage rounding (~3e-8 per population and step) walks over
    # the relaxation time 1/(nu k^2) ~ 625 steps of this flow, ~sqrt(625) x
    # 3e-8 ~ 7.5e-7 in u, i.e. ~7.5e-5 in R at U0 = 0.01: bound 1e-4.
    for storage, tol in (("f64", 1e-12), ("f32", 1e-4)):
        lat = gpu_lattice(nx, L, ra, ra.copy(), walls=False, storage=storage, profile=True, tau=tau,
                          fx_amp=F0, fx_k=kf, **ZERO)
        lat.step(steps)
        R = K.response(lat.line_profile(), U0)
        lat.stress_reset()
        lat.step(10)
        prof, n = lat.profile()
        assert n == 10
        print(f"\n{storage}: R {R:.8f} (oracle {R_ref:.8f}), time-averaged {K.response(prof, U0):.8f}")
        assert R == pytest.approx(R_ref, abs=tol)
        assert K.response(prof, U0) == pytest.approx(R_ref, abs=3 * tol)
    assert abs(R_ref - 1.0) < 1e-3


def test_batch_with_body_forces_equals_single_lattices():
    """Lattices with different forcing amplitudes and wavenumbers in one batch
    give bitwise the single-lattice results."""
    from paper_1004_5058_amd import lb
    specs = []
    for k, (L, nx, U0) in enumerate([(64, 64, 0.1), (48, 100, 0.05), (32, 20, 0.2)]):
        ra, rb, kw, _ = _protocol(L, nx, U0=U0)
        specs.append(dict(nx=nx, ny=L, rho_a=ra, rho_b=rb, ux=None, uy=None, **kw))
    b = lb.Batch(specs, storage="f32", profile=False)
    b.step(30)
    for k, s in enumerate(specs):
        kw = {q: v for q, v in s.items() if q not in ("nx", "ny", "rho_a", "rho_b", "ux", "uy")}
        lat = lb.Lattice(s["nx"], s["ny"], s["rho_a"], s["rho_b"], None, None, storage="f32", **kw)
        lat.step(30)
        for a, c in zip(b.fields(k), lat.fields()):
            np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(b.line_profile(k), lat.line_profile())
        lat.close()
    b.close()


def test_protocol_driver_runs():
    """The protocol driver at a small size: R(t) samples, a time-averaged
    profile and the stress/shear scatter, all finite."""
    r = K.run(L=64, rho0=0.83, U0=0.1, steps=600, sample_every=200, average_from=300)
    assert list(r["t"]) == [200, 300, 500, 600] and np.all(np.isfinite(r["R"]))
    assert r["samples"] == 300
    assert np.all(np.isfinite(r["profile"])) and np.all(np.isfinite(r["S"]))
    assert r["sigma0"] == pytest.approx(r["F0"] / K.wavenumber(64))
