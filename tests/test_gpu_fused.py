"""Two time steps per pass (lb_set_fusion; FP32, FP16- and BF16-deviation
storage): the fused kernel keeps step t's populations in on-chip memory and
runs step t+1 behind it.  It performs the operations of two single steps on the
same values (the library is built with multiply-add contraction inside
expressions only; every stored value is rounded to the storage format by one
rule that both kernels share, and the ring holds it as HBM would), so populations, wall stresses and step counts must equal the
single-step path bit for bit, with walls or periodic y, body force, any tile
height and block width (128, 192, 256 lanes per step), odd step counts (the
last step runs alone) and graphs of either parity."""
import numpy as np
import pytest

from gpu_common import compare_fields, gpu_lattice, need_gpu, oracle_params, oracle_run
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _pair(nx, ny, storage, walls, body, steps, ly2, graph, seed=5, init="emulsion", lanes=0, tau=None):
    u = 0.02 if walls else 0.0
    ra, rb = (inputs.emulsion(nx, ny, seed=seed) if init == "emulsion" else inputs.noise(nx, ny, seed))
    ux, uy = inputs.couette(nx, ny, u, -u) if walls else (None, None)
    kw = dict(fx_amp=3e-5, fx_k=0.21) if body else {}
    if tau is not None:
        kw["tau"] = tau
    out = []
    for fused in (False, True):
        lat = gpu_lattice(nx, ny, ra, rb, ux, uy, walls=walls, u_top=u, u_bot=-u, storage=storage, **kw)
        lat.set_graph(graph)
        if fused:
            lat.set_fusion_tile(lanes)
            lat.set_fusion(2, ly2)
            if lanes:
                assert lat.fusion_tile() == (lanes, lanes - (6 if storage == "f32" and lanes == 128 else 10))
        lat.step(steps)
        out.append((lat.populations(), lat.stress(), lat.time()))
        lat.close()
    return out


@pytest.mark.parametrize("lanes", [128, 192, 256])
@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("nx,ny,walls,body,ly2", [(600, 300, True, False, 0), (500, 120, False, True, 7),
                                                   (252, 31, True, True, 1), (8, 6, True, False, 64),
                                                   (1000, 40, False, False, 0), (6, 2, False, False, 0),
                                                   (122, 3, True, False, 2), (244, 17, True, True, 0),
                                                   (10, 2, False, True, 0), (300, 53, True, True, 12)])
def test_fused_bitwise_equals_single_steps(storage, nx, ny, walls, body, ly2, lanes):
    (p1, s1, t1), (p2, s2, t2) = _pair(nx, ny, storage, walls, body, 30, ly2, 32, lanes=lanes)
    assert t1 == t2 == 30
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("tau", [0.83, 1.37])
@pytest.mark.parametrize("walls,body", [(True, False), (False, True)])
def test_fused_bitwise_any_tau(storage, tau, walls, body):
    """Away from tau = 1 the relaxation f - omega (f - f^eq) is not f^eq, so
    the rounding of the stored value matters: each stored value is defined
    once (FP16: the post-collision multiply-add rounded once to FP16; values
    bounced at a wall rounded to FP32 first) and both kernels store exactly
    that, with walls (every wall path, both walls moving) or periodic y with
    the body force."""
    (p1, s1, t1), (p2, s2, t2) = _pair(300, 53, storage, walls, body, 30, 12, 32, tau=tau)
    assert t1 == t2 == 30
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
@pytest.mark.parametrize("steps,graph", [(31, 0), (31, 6), (40, 6), (37, 32)])
def test_fused_odd_steps_and_graph_parity(steps, graph, storage):
    """Odd step counts end with one single step; graphs of 6 steps hold three
    fused pairs (an odd number of buffer swaps per replay)."""
    nx = 333
    (p1, s1, t1), (p2, s2, t2) = _pair(nx, 97, storage, True, True, steps, 0, graph)
    assert t1 == t2 == steps
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("nx", [1, 2, 3, 5])
@pytest.mark.parametrize("walls", [True, False])
def test_fused_tiny_widths(storage, nx, walls):
    """Lattices narrower than the stencil: every lane of a tile wraps onto a
    few columns (one column: all lanes hold the same site)."""
    (p1, s1, t1), (p2, s2, t2) = _pair(nx, 7, storage, walls, not walls, 13, 0, 0, init="noise")
    assert t1 == t2 == 13
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("lanes", [128, 192, 256])
def test_fused_odd_width(lanes, storage):
    """Odd nx: the tiles' columns wrap around the periodic x at an odd
    column (16-bit storage takes every column from its own lane: no column
    pairs)."""
    (p1, s1, _), (p2, s2, _) = _pair(257, 64, storage, True, False, 20, 16, 32, lanes=lanes)
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1
    (p1, s1, _), (p2, s2, _) = _pair(9, 11, storage, False, True, 21, 0, 0, lanes=lanes)
    np.testing.assert_array_equal(p2, p1)


@pytest.mark.parametrize("storage,tol", [("f16dev", 6e-5), ("bf16dev", 5e-4)])
def test_fused_16bit_matches_oracle(storage, tol):
    """16-bit deviation storage two steps per pass against the FP64 oracle,
    100 steps (the tolerances of the single-step 16-bit parity tests)."""
    nx, ny, u, steps = 300, 128, 0.01, 100
    ra, rb = inputs.noise(nx, ny, 0)
    p = oracle_params(nx, ny, True, u, -u)
    g, _, _ = oracle_run(p, ra, rb, None, None, steps)
    lat = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage=storage)
    lat.set_fusion(2)
    lat.step(steps)
    e = compare_fields(lat, p, g, tol)
    print(f"\nfused {storage} {nx}x{ny}, {steps} steps: {e}")


def test_fused_matches_oracle():
    nx, ny, u, steps = 300, 128, 0.01, 100
    ra, rb = inputs.noise(nx, ny, 0)
    p = oracle_params(nx, ny, True, u, -u)
    g, sb, st = oracle_run(p, ra, rb, None, None, steps)
    lat = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage="f32")
    lat.set_fusion(2)
    lat.step(steps)
    e = compare_fields(lat, p, g, 1e-6)
    gb, gt, n = lat.stress()
    assert n == steps
    assert abs(gb - sb) / abs(sb) < 1e-5 and abs(gt - st) / abs(st) < 1e-5
    print(f"\nfused FP32 {nx}x{ny}, {steps} steps: {e}")


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
def test_fused_batch_equals_single_steps(storage):
    """A batch of uneven lattices (odd widths among them), each with its own
    walls, wall speed, couplings and tau, two steps per pass against one."""
    from paper_1004_5058_amd import lb
    specs = []
    for k, (nx, ny, walls) in enumerate([(512, 256, True), (301, 77, False), (1024, 130, True), (41, 9, True),
                                         (7, 33, False)]):
        ra, rb = inputs.emulsion(nx, ny, seed=20 + k)
        u = 0.01 * (k + 1) if walls else 0.0
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, walls=walls, u_top=u, u_bot=-u,
                          g_aa2=7.8 + 0.1 * k, tau=0.8 + 0.15 * k))
    res = []
    for fused in (False, True):
        b = lb.Batch(specs, storage=storage, profile=False)
        if fused:
            b.set_fusion(2)
        b.step(24)
        res.append(([b.fields(k) for k in range(len(specs))], b.stress()))
        b.close()
    for a, c in zip(res[0][0], res[1][0]):
        for x, y in zip(a, c):
            np.testing.assert_array_equal(y, x)
    for x, y in zip(res[0][1][:2], res[1][1][:2]):
        np.testing.assert_array_equal(y, x)
    assert res[0][1][2] == res[1][1][2] == 24


def test_fused_refused_where_not_built():
    from paper_1004_5058_amd import lb
    ra, rb = inputs.noise(64, 16, 1)
    for storage, (a, b) in (("f64", (ra, rb)), ("mom32", (ra, rb))):
        lat = gpu_lattice(b.shape[1], 16, a, b, storage=storage)
        with pytest.raises(lb.LBError, match="two steps per pass"):
            lat.set_fusion(2)
        with pytest.raises(lb.LBError, match="lanes"):
            lat.set_fusion_tile(64)
        lat.step(2)           # still steps, one step per pass
        lat.close()


@pytest.mark.parametrize("storage,nx", [("f32", 1024), ("f16dev", 1023)])
def test_autotune_considers_two_steps_per_pass(tmp_path, storage, nx):
    """The tuner also times two steps per pass for an FP32 or 16-bit lattice
    (odd nx included), applies the faster mode, preserves the state (either
    mode is bitwise the single-step result) and records the choice in the
    cache; a profile-enabled lattice of the same key applies the cached entry
    and accumulates its profile."""
    import json
    ny, u = 512, 0.02
    ra, rb = inputs.emulsion(nx, ny, seed=3)
    ref = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage=storage)
    ref.step(10)
    lat = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage=storage)
    lat.step(4)
    cache = str(tmp_path / "tune.json")
    bx, ly, ms = lat.autotune(cache, steps=4)
    assert lat.time() == 4 and ms > 0
    lat.step(6)
    np.testing.assert_array_equal(lat.populations(), ref.populations())
    assert lat.stress() == ref.stress()
    (key, ent), = json.load(open(cache)).items()
    assert ent["fusion"] in (1, 2) and "ly2" in ent and (ent["bx"], ent["ly"]) == (bx, ly)
    c = lat.launch()
    assert (c["bx"], c["ly"], c["steps_per_pass"]) == (bx, ly, ent["fusion"])
    if ent["ly2"]:
        assert c["ly2"] == ent["ly2"]
    print(f"\n{key}: {ent}")
    prof = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage=storage, profile=True)
    assert prof.autotune(cache, steps=4)[:2] == (bx, ly)
    prof.step(4)
    assert prof.time() == 4 and prof.profile()[1] == 4


@pytest.mark.parametrize("nx,ny,walls,body,ly2", [(600, 300, True, False, 0), (500, 120, False, True, 7),
                                                   (252, 31, True, True, 1), (1000, 40, True, False, 16)])
def test_fused_profile_matches_single_steps(nx, ny, walls, body, ly2):
    """With the line profile on, two steps per pass keep populations and wall
    stress bitwise and accumulate the profile from the fused tiles' partial
    sums: equal to the single-step profile to FP64 rounding (the column
    groups of the partial sums differ), across a stress reset and an odd
    step count."""
    res = []
    for per_pass in (1, 2):
        ra, rb = inputs.emulsion(nx, ny, seed=5)
        kw = dict(fx_amp=1e-5, fx_k=2 * np.pi / ny) if body else {}
        lat = gpu_lattice(nx, ny, ra, rb, walls=walls, u_top=0.02 if walls else 0.0,
                          u_bot=-0.02 if walls else 0.0, storage="f32", profile=True, **kw)
        lat.set_fusion(per_pass, ly2)
        lat.step(10)
        lat.stress_reset()
        lat.step(23)
        res.append((lat.populations(), lat.stress(), lat.profile()))
        lat.close()
    (p1, s1, (q1, n1)), (p2, s2, (q2, n2)) = res
    np.testing.assert_array_equal(p2, p1)
    assert s2 == s1 and n1 == n2 == 23
    scale = np.max(np.abs(q1))
    assert scale > 0
    assert np.max(np.abs(q2 - q1)) <= 1e-13 * scale, np.max(np.abs(q2 - q1)) / scale


def test_fused_batch_profile_matches_single_steps():
    from paper_1004_5058_amd import lb
    specs = []
    for k, (nx, ny) in enumerate([(512, 256), (300, 77), (1024, 130)]):
        ra, rb = inputs.emulsion(nx, ny, seed=50 + k)
        u = 0.01 * (k + 1)
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, u_top=u, u_bot=-u))
    res = []
    for per_pass in (1, 2):
        b = lb.Batch(specs, storage="f32", profile=True)
        b.set_fusion(per_pass, 64)
        b.step(26)
        res.append(([b.fields(k) for k in range(len(specs))], b.stress(),
                    [b.profile(k)[0] for k in range(len(specs))]))
        b.close()
    for a, c in zip(res[0][0], res[1][0]):
        for x, y in zip(a, c):
            np.testing.assert_array_equal(y, x)
    for x, y in zip(res[0][1][:2], res[1][1][:2]):
        np.testing.assert_array_equal(y, x)
    for q1, q2 in zip(res[0][2], res[1][2]):
        assert np.max(np.abs(q2 - q1)) <= 1e-13 * np.max(np.abs(q1))


def test_launch_reports_the_configuration_in_effect():
    """lb_get_launch / lbb_get_launch report what set_launch, set_fusion and a
    cached autotune entry left in effect, the automatic fused height resolved."""
    from paper_1004_5058_amd import lb
    ra, rb = inputs.emulsion(600, 300, seed=2)
    lat = gpu_lattice(600, 300, ra, rb, u_top=0.01, u_bot=-0.01, storage="f32")
    lat.set_launch(128, 32)
    c = lat.launch()
    assert (c["bx"], c["ly"], c["steps_per_pass"]) == (128, 32, 1) and 1 <= c["ly2"] <= 300
    lat.set_fusion(2, 40)
    assert lat.launch() == dict(bx=128, ly=32, steps_per_pass=2, ly2=40)
    lat.set_fusion(2, 0)
    c = lat.launch()
    assert c["steps_per_pass"] == 2 and 1 <= c["ly2"] <= 300
    lat.close()
    specs = [dict(nx=300, ny=77, rho_a=ra[:77, :300].copy(), rho_b=rb[:77, :300].copy(), ux=None, uy=None)]
    b = lb.Batch(specs, storage="f32", profile=True)
    b.set_launch(256, 16, 512)
    b.set_fusion(2, 12)
    assert b.launch() == dict(bx=256, ly=16, grid=512, steps_per_pass=2, ly2=12)
    b.close()


@pytest.mark.parametrize("resume_per_pass", [2, 1])
def test_fused_checkpoint_resume(resume_per_pass):
    """A checkpoint taken with two steps per pass (profile on, so the fused
    partial sums are part of it) resumes bitwise, whether the resumed run keeps
    two steps per pass or switches to one: populations, stress and profile
    equal those of the run that continued without the checkpoint."""
    nx, ny = 300, 96
    ra, rb = inputs.emulsion(nx, ny, seed=8)
    a = gpu_lattice(nx, ny, ra, rb, u_top=0.02, u_bot=-0.02, storage="f32", profile=True)
    a.set_fusion(2)
    a.step(30)
    ck = a.save()
    a.set_fusion(resume_per_pass)
    a.step(21)
    b = gpu_lattice(nx, ny, ra, rb, u_top=0.02, u_bot=-0.02, storage="f32", profile=True)
    b.set_fusion(resume_per_pass)
    b.load(ck)
    assert b.time() == 30
    b.step(21)
    np.testing.assert_array_equal(a.populations(), b.populations())
    assert a.stress() == b.stress()
    np.testing.assert_array_equal(a.profile()[0], b.profile()[0])
    a.close()
    b.close()
