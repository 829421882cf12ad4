"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every function include/lb.h declares, and validates parameters before
any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lb.h", "mlp.h")]


def _declared(path):
    if not os.path.exists(path):
        return []
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lb_status|const char\*|int32_t|void)\s+\**(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared(HEADERS[0])
    for n in ("lb_init", "lb_step", "lb_fields", "lb_stress", "lb_state_bytes", "lb_destroy",
              "lbb_init", "lbb_step", "lbb_stress"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1004_5058_amd import lb
    L = lb.load_library()
    missing = [n for h in HEADERS for n in _declared(h) if not hasattr(L, n)]
    assert not missing, missing


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library the binding raises instead of falling back."""
    from paper_1004_5058_amd import lb
    saved = lb._lib
    lb._lib = None
    try:
        with pytest.raises(ImportError):
            lb.load_library(str(tmp_path / "missing.so"))
    finally:
        lb._lib = saved


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(rho0=0.0), "rho0"),
    (dict(g_ab=float("inf")), "non-finite"),
    (dict(storage=7), "storage"),
])
def test_state_bytes_rejects_bad_parameters(kw, msg):
    from paper_1004_5058_amd import lb
    p = lb.make_params(64, 64, **{k: v for k, v in kw.items() if k != "storage"})
    if "storage" in kw:
        p.storage = kw["storage"]
    with pytest.raises(lb.LBError) as e:
        lb.lb_state_bytes(p)
    assert e.value.code == -1 and msg in str(e.value)


def test_state_bytes_rejects_bad_sizes():
    from paper_1004_5058_amd import lb
    for nx, ny in [(0, 8), (8, 1), (70000, 8)]:
        with pytest.raises(lb.LBError):
            lb.lb_state_bytes(lb.make_params(nx, ny))
    # one species' planes above 4 GiB of 32-bit buffer offsets
    with pytest.raises(lb.LBError):
        lb.lb_state_bytes(lb.make_params(16384, 16384, storage="f64"))


@pytest.mark.parametrize("storage,n", [("f64", 7680), ("f32", 10880), ("f16dev", 15424), ("mom32", 13376)])
def test_largest_accepted_lattice(storage, n):
    """The largest square lattice whose planes of one species (nine values,
    six in the moment form) stay below 4 GiB of 32-bit buffer offsets is
    accepted; the next size up (64 more columns and rows) is refused."""
    from paper_1004_5058_amd import lb
    assert lb.lb_state_bytes(lb.make_params(n, n, storage=storage)) > 0
    with pytest.raises(lb.LBError, match="too large"):
        lb.lb_state_bytes(lb.make_params(n + 64, n + 64, storage=storage))


def test_state_bytes_layout_scales_with_storage():
    """Two population buffers of 18 planes; a plane holds ny rows of the
    64-element-aligned pitch and starts one row and 64 elements past the
    previous one (planes never a power of two apart)."""
    from paper_1004_5058_amd import lb
    b64 = lb.lb_state_bytes(lb.make_params(512, 256, storage="f64"))
    b32 = lb.lb_state_bytes(lb.make_params(512, 256, storage="f32"))
    b16 = lb.lb_state_bytes(lb.make_params(512, 256, storage="f16dev"))
    plane = 512 * (256 + 1) + 64
    pop = 2 * 18 * plane
    assert b64 - b32 == pop * 4 and b32 - b16 == pop * 2


def test_init_rejects_bad_inputs_before_device_work():
    """Non-positive or non-finite initial densities and a misaligned or small
    state are refused with LB_EINVAL / LB_ENOMEM without touching a GPU."""
    from paper_1004_5058_amd import lb
    L = lb.load_library()
    p = lb.make_params(8, 8)
    ra = np.full((8, 8), 0.5)
    rb = np.full((8, 8), 0.5)
    h = ctypes.c_void_p()
    need = lb.lb_state_bytes(p)
    fake = ctypes.c_void_p(4096)   # never dereferenced: validation fails first
    bad = ra.copy()
    bad[3, 4] = -0.1
    assert L.lb_init(ctypes.byref(p), fake, need, None, lb._dptr(bad), lb._dptr(rb), None, None,
                     ctypes.byref(h)) == -1
    bad[3, 4] = float("nan")
    assert L.lb_init(ctypes.byref(p), fake, need, None, lb._dptr(bad), lb._dptr(rb), None, None,
                     ctypes.byref(h)) == -1
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(4097), need, None, lb._dptr(ra), lb._dptr(rb),
                     None, None, ctypes.byref(h)) == -1
    assert L.lb_init(ctypes.byref(p), fake, need - 256, None, lb._dptr(ra), lb._dptr(rb), None, None,
                     ctypes.byref(h)) == -2
    assert b"smaller" in L.lb_last_error()
    assert L.lb_step(None, 1) == -1


def test_batch_init_names_the_lattice_and_site_of_a_bad_field():
    """A batch's initial fields are checked on several host threads; the error
    names the lowest-numbered lattice at fault and its first offending site
    (densities before u_x before u_y), and nothing touches a GPU."""
    from paper_1004_5058_amd import lb
    L = lb.load_library()
    shapes = [(8, 8), (16, 12), (40, 24), (12, 10)]
    P = (lb.lb_params * len(shapes))()
    for k, (nx, ny) in enumerate(shapes):
        P[k] = lb.make_params(nx, ny)
    need = ctypes.c_size_t()
    assert L.lbb_state_bytes(P, len(shapes), ctypes.byref(need)) == 0
    fields = {key: [np.full((ny, nx), 0.5 if key.startswith("rho") else 0.01) for nx, ny in shapes]
              for key in ("rho_a", "rho_b", "ux", "uy")}

    def init():
        ptrs = {}
        for key, arrs in fields.items():
            ptrs[key] = (lb._DP * len(shapes))(*[lb._dptr(a) for a in arrs])
        h = ctypes.c_void_p()
        rc = L.lbb_init(P, len(shapes), ctypes.c_void_p(4096), 0, None, ptrs["rho_a"], ptrs["rho_b"],
                        ptrs["ux"], ptrs["uy"], ctypes.byref(h))
        return rc, L.lb_last_error().decode()

    # valid fields: the device-state size check is the first failure
    rc, msg = init()
    assert rc == -2 and "smaller" in msg
    fields["uy"][3][2, 5] = float("inf")
    fields["ux"][2][7, 3] = float("nan")
    fields["rho_b"][2][9, 1] = 0.0
    rc, msg = init()
    assert rc == -1 and "lattice 2" in msg and "non-finite initial ux" in msg and f"site {7 * 40 + 3}" in msg
    fields["rho_a"][2][0, 39] = -1.0
    rc, msg = init()
    assert rc == -1 and "lattice 2" in msg and "density" in msg and "site 39" in msg
    fields["rho_a"][2][0, 39] = 0.5
    fields["ux"][2][7, 3] = 0.0
    rc, msg = init()
    assert rc == -1 and "lattice 2" in msg and "density" in msg and f"site {9 * 40 + 1}" in msg
    fields["rho_b"][2][9, 1] = 0.5
    rc, msg = init()
    assert rc == -1 and "lattice 3" in msg and "non-finite initial uy" in msg and f"site {2 * 12 + 5}" in msg


def test_moment_storage_requires_tau_one():
    """The moment form holds the post-collision state only at tau = 1."""
    from paper_1004_5058_amd import lb
    lb.load_library()
    with pytest.raises(lb.LBError, match="tau = 1"):
        lb.lb_state_bytes(lb.make_params(32, 16, tau=0.8, storage="mom32"))
    assert lb.lb_state_bytes(lb.make_params(32, 16, tau=1.0, storage="mom32")) > 0
    # 6 moments per site instead of 18 populations (each buffer padded to the
    # 32 bytes per site of the FP64 staging: 2 x 32 instead of 2 x 72)
    m = lb.lb_state_bytes(lb.make_params(256, 256, tau=1.0, storage="mom32"))
    f = lb.lb_state_bytes(lb.make_params(256, 256, tau=1.0, storage="f32"))
    assert m < 0.5 * f


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev", "mom32", "mom64"])
@pytest.mark.parametrize("nx,ny", [(64, 48), (128, 20), (131, 37)])
def test_state_buffers_hold_the_fp64_staging(storage, nx, ny):
    """Initial fields and field reads are staged as four FP64 arrays in a state
    buffer, so each of the two buffers holds at least 32 bytes per site (the
    FP32 moment form stores only 24)."""
    from paper_1004_5058_amd import lb
    lb.load_library()
    n = lb.lb_state_bytes(lb.make_params(nx, ny, tau=1.0, storage=storage))
    assert n >= 2 * 32 * nx * ny


def test_last_error_is_per_thread():
    """lb_last_error is thread-local: two threads that fail validation in
    different ways, both before either reads its message, each read their own."""
    import threading
    from paper_1004_5058_amd import lb
    L = lb.load_library()
    gate = threading.Barrier(2)
    out = {}

    def worker(name, kw):
        p = lb.make_params(64, 64, **kw)
        n = ctypes.c_size_t()
        code = L.lb_state_bytes(ctypes.byref(p), ctypes.byref(n))
        gate.wait()                    # both errors are set before either message is read
        out[name] = (code, L.lb_last_error().decode())

    threads = [threading.Thread(target=worker, args=("tau", dict(tau=0.4))),
               threading.Thread(target=worker, args=("rho0", dict(rho0=-1.0)))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=30)
    assert out["tau"][0] == -1 and "tau" in out["tau"][1] and "rho0" not in out["tau"][1]
    assert out["rho0"][0] == -1 and "rho0" in out["rho0"][1] and "tau" not in out["rho0"][1]
