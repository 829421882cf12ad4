"""ctypes binding of the C ABI in include/lb.h (argument marshalling only).

Every computation runs in the HIP library paper_1004_5058_amd/_lib/liblbmi.so.
PyTorch supplies device memory (a uint8 tensor holds the lattice state) and
the stream (torch's current stream on the lattice's device).  Importing this
module without the built library raises: there is no CPU fallback.

Functions carry the C names (lb_init, lb_step, lb_fields, lb_stress, ...);
`Lattice` and `Batch` wrap them for convenience.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbmi.so")

STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3, "mom32": 4, "mom64": 5}
STATUS = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EDEVICE", -4: "LB_ENONFINITE",
          -5: "LB_ESTATE"}


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls_y", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("g_aa1", ctypes.c_double), ("g_aa2", ctypes.c_double),
        ("g_bb1", ctypes.c_double), ("g_bb2", ctypes.c_double), ("g_ab", ctypes.c_double),
        ("u_top", ctypes.c_double), ("u_bot", ctypes.c_double),
        ("rho_ref_a", ctypes.c_double), ("rho_ref_b", ctypes.c_double),
        ("profile", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("fx_amp", ctypes.c_double), ("fx_k", ctypes.c_double),
    ]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def load_library(path=LIB_PATH):
    """Load liblbmi.so (built by paper_1004_5058_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so device memory and streams from torch are valid in its calls
    # (a second runtime instance in the process would not see them).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    st = ctypes.c_int
    P = ctypes.POINTER(lb_params)
    H = ctypes.c_void_p
    DPP = ctypes.POINTER(_DP)
    sig = {
        "lb_state_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "lb_init": [P, _VP, ctypes.c_size_t, _VP, _DP, _DP, _DP, _DP, ctypes.POINTER(H)],
        "lb_step": [H, ctypes.c_int32],
        "lb_set_fusion": [H, ctypes.c_int32, ctypes.c_int32],
        "lbb_set_fusion": [H, ctypes.c_int32, ctypes.c_int32],
        "lb_set_fusion_tile": [H, ctypes.c_int32],
        "lbb_set_fusion_tile": [H, ctypes.c_int32],
        "lb_get_fusion_tile": [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "lbb_get_fusion_tile": [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "lb_get_launch": [H] + [ctypes.POINTER(ctypes.c_int32)] * 4,
        "lbb_get_launch": [H] + [ctypes.POINTER(ctypes.c_int32)] * 5,
        "lb_fields": [H, _DP, _DP, _DP, _DP],
        "lb_fields_device": [H, _VP, _VP, _VP, _VP],
        "lb_populations": [H, _DP],
        "lb_stress": [H, _DP, _DP, ctypes.POINTER(ctypes.c_int64)],
        "lb_stress_reset": [H],
        "lb_profile": [H, _DP, ctypes.POINTER(ctypes.c_int64)],
        "lb_sums": [H, _DP],
        "lb_set_watchdog": [H, ctypes.c_int32],
        "lb_set_launch": [H, ctypes.c_int32, ctypes.c_int32],
        "lb_set_graph": [H, ctypes.c_int32],
        "lb_save": [H, _VP, ctypes.POINTER(ctypes.c_size_t)],
        "lb_load": [H, _VP, ctypes.c_size_t],
        "lb_time": [H, ctypes.POINTER(ctypes.c_int64)],
        "lb_time_steps": [H, ctypes.c_int32, _DP],
        "lb_destroy": [H],
        "lb_autotune": [H, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_int32), _DP],
        "lbb_autotune": [H, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _DP],
        "lb_copy_peak": [_VP, _VP, ctypes.c_size_t, _VP, ctypes.c_int32, _DP],
        "lbb_state_bytes": [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
        "lbb_init": [P, ctypes.c_int32, _VP, ctypes.c_size_t, _VP, DPP, DPP, DPP, DPP, ctypes.POINTER(H)],
        "lbb_step": [H, ctypes.c_int32],
        "lbb_stress": [H, _DP, _DP, ctypes.POINTER(ctypes.c_int64)],
        "lbb_stress_noalloc": [H, _DP, _DP, ctypes.POINTER(ctypes.c_int64)],
        "lbb_stress_reset": [H],
        "lbb_fields": [H, ctypes.c_int32, _DP, _DP, _DP, _DP],
        "lbb_profile": [H, ctypes.c_int32, _DP, ctypes.POINTER(ctypes.c_int64)],
        "lbb_set_launch": [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
        "lbb_set_graph": [H, ctypes.c_int32],
        "lbb_time_steps": [H, ctypes.c_int32, _DP],
        "lbb_destroy": [H],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = st
    L.lb_last_error.argtypes = []
    L.lb_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise LBError(code, _lib.lb_last_error().decode())


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _field(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        raise ValueError(f"field of shape {a.shape}, expected {shape}")
    return a


def make_params(nx, ny, *, tau=1.0, rho0=0.83, g_aa1=-9.0, g_aa2=8.1, g_bb1=-9.0, g_bb2=8.1,
                g_ab=0.405, walls=True, u_top=0.0, u_bot=0.0, storage="f32", rho_ref_a=0.0,
                rho_ref_b=0.0, profile=False, fx_amp=0.0, fx_k=0.0):
    p = lb_params()
    p.nx, p.ny, p.walls_y = int(nx), int(ny), int(bool(walls))
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.tau, p.rho0 = tau, rho0
    p.g_aa1, p.g_aa2, p.g_bb1, p.g_bb2, p.g_ab = g_aa1, g_aa2, g_bb1, g_bb2, g_ab
    p.u_top, p.u_bot = u_top, u_bot
    p.rho_ref_a, p.rho_ref_b = rho_ref_a, rho_ref_b
    p.profile = int(bool(profile))
    p.fx_amp, p.fx_k = fx_amp, fx_k
    return p


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ---------------------------------------------------------- C-named calls --

def lb_state_bytes(p):
    L = load_library()
    n = ctypes.c_size_t()
    _check(L.lb_state_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def lb_init(p, state, stream, rho_a, rho_b, ux=None, uy=None):
    L = load_library()
    shp = (p.ny, p.nx)
    ra, rb = _field(rho_a, shp), _field(rho_b, shp)
    u, v = _field(ux, shp), _field(uy, shp)
    h = ctypes.c_void_p()
    _check(L.lb_init(ctypes.byref(p), ctypes.c_void_p(state.data_ptr()), state.numel(), stream,
                     _dptr(ra), _dptr(rb), _dptr(u), _dptr(v), ctypes.byref(h)))
    return h


def lb_step(h, n):
    _check(_lib.lb_step(h, int(n)))


def lb_fields(h, ny, nx):
    out = [np.empty((ny, nx)) for _ in range(4)]
    _check(_lib.lb_fields(h, *[_dptr(o) for o in out]))
    return tuple(out)


def lb_populations(h, ny, nx):
    f = np.empty((2, 9, ny, nx))
    _check(_lib.lb_populations(h, _dptr(f)))
    return f


def lb_stress(h):
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(_lib.lb_stress(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
    return a.value, b.value, n.value


def lb_stress_reset(h):
    _check(_lib.lb_stress_reset(h))


def lb_profile(h, ny):
    prof = np.empty(ny)
    n = ctypes.c_int64()
    _check(_lib.lb_profile(h, _dptr(prof), ctypes.byref(n)))
    return prof, n.value


def lb_sums(h):
    out = np.zeros(5)
    _check(_lib.lb_sums(h, _dptr(out)))
    return out


def lb_destroy(h):
    if h:
        _check(_lib.lb_destroy(h))


def copy_peak(nbytes=2 ** 31, reps=10, device="cuda:0"):
    """Read+write GB/s of the library's streaming copy kernel on nbytes."""
    torch = _torch()
    L = load_library()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    g = ctypes.c_double()
    _check(L.lb_copy_peak(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                          _stream_handle(torch.device(device)), int(reps), ctypes.byref(g)))
    return g.value


# ------------------------------------------------------------- wrappers ---

class Lattice:
    """One lattice on one GPU.  Fields are float64 numpy arrays (ny, nx)."""

    def __init__(self, nx, ny, rho_a, rho_b, ux=None, uy=None, device="cuda:0", **kw):
        torch = _torch()
        load_library()
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device(device)
        self.params = make_params(nx, ny, **kw)
        nbytes = lb_state_bytes(self.params)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.state.data_ptr() % 256:
            raise RuntimeError("device state not 256-byte aligned")
        self._h = None
        with torch.cuda.device(self.device):
            self._stream = _stream_handle(self.device)
            self._h = lb_init(self.params, self.state, self._stream, rho_a, rho_b, ux, uy)

    def step(self, n=1):
        lb_step(self._h, n)
        return self

    def fields(self):
        """(rho_a, rho_b, ux, uy), synchronising."""
        return lb_fields(self._h, self.ny, self.nx)

    def fields_device(self):
        torch = _torch()
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(4)]
        _check(_lib.lb_fields_device(self._h, *[ctypes.c_void_p(o.data_ptr()) for o in out]))
        return tuple(out)

    def populations(self):
        return lb_populations(self._h, self.ny, self.nx)

    def stress(self):
        """(sigma_bot, sigma_top, nsamples): time averages since init / reset."""
        return lb_stress(self._h)

    def stress_reset(self):
        lb_stress_reset(self._h)

    def profile(self):
        return lb_profile(self._h, self.ny)

    def line_profile(self):
        """Instantaneous U_x(y) = (1/nx) sum_x u_x of the current state."""
        out = np.empty(self.ny)
        _check(_lib.lb_line_profile(self._h, _dptr(out)))
        return out

    def sums(self):
        return lb_sums(self._h)

    def set_watchdog(self, every):
        _check(_lib.lb_set_watchdog(self._h, int(every)))

    def set_launch(self, bx=0, ly=0):
        _check(_lib.lb_set_launch(self._h, int(bx), int(ly)))

    def set_graph(self, steps_per_graph):
        _check(_lib.lb_set_graph(self._h, int(steps_per_graph)))

    def set_fusion(self, steps_per_pass, ly2=0):
        """1 or 2 time steps per pass of the step kernel (2: FP32 or 16-bit
        population storage)."""
        _check(_lib.lb_set_fusion(self._h, int(steps_per_pass), int(ly2)))

    def set_fusion_tile(self, lanes):
        """Lanes per time step of the fused kernel's blocks: 128, 192, 256, or 0 (automatic)."""
        _check(_lib.lb_set_fusion_tile(self._h, int(lanes)))

    def fusion_tile(self):
        """(lanes per step, stored columns per tile) of the fused kernel in effect."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lb_get_fusion_tile(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def launch(self):
        """The launch configuration in effect: dict(bx, ly, steps_per_pass, ly2),
        ly2 the fused tile height with the automatic choice resolved."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(_lib.lb_get_launch(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("bx", "ly", "steps_per_pass", "ly2"), (x.value for x in v)))

    def autotune(self, cache_path=None, steps=20):
        """Pick the fastest launch shape, and for FP32 and 16-bit storage the
        steps per pass and fused block width (state preserved); returns
        (bx, ly, ms per step)."""
        bx, ly, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(_lib.lb_autotune(self._h, path, int(steps), ctypes.byref(bx), ctypes.byref(ly), ctypes.byref(ms)))
        return bx.value, ly.value, ms.value

    def time(self):
        t = ctypes.c_int64()
        _check(_lib.lb_time(self._h, ctypes.byref(t)))
        return t.value

    def time_steps(self, n):
        ms = ctypes.c_double()
        _check(_lib.lb_time_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def save(self):
        n = ctypes.c_size_t()
        _check(_lib.lb_save(self._h, None, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(_lib.lb_save(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib.lb_load(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    def close(self):
        if self._h:
            lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several independent lattices advanced by one step kernel per time step.

    specs: list of dicts with nx, ny, rho_a, rho_b, optional ux, uy and any
    make_params keyword (all share one storage precision)."""

    def __init__(self, specs, device="cuda:0", storage="f32", profile=True):
        torch = _torch()
        L = load_library()
        self.device = torch.device(device)
        n = len(specs)
        self.n = n
        self.shapes = [(int(s["ny"]), int(s["nx"])) for s in specs]
        P = (lb_params * n)()
        keep = []
        for k, s in enumerate(specs):
            kw = {a: b for a, b in s.items() if a not in ("nx", "ny", "rho_a", "rho_b", "ux", "uy", "seed")}
            kw.setdefault("storage", storage)
            kw.setdefault("profile", profile)
            P[k] = make_params(s["nx"], s["ny"], **kw)
        nbytes = ctypes.c_size_t()
        _check(L.lbb_state_bytes(P, n, ctypes.byref(nbytes)))
        self.state = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        arrs = {}
        for key in ("rho_a", "rho_b", "ux", "uy"):
            ptrs = (_DP * n)()
            for k, s in enumerate(specs):
                a = _field(s.get(key), self.shapes[k])
                keep.append(a)
                ptrs[k] = _dptr(a) if a is not None else None
            arrs[key] = ptrs
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._stream = _stream_handle(self.device)
            _check(L.lbb_init(P, n, ctypes.c_void_p(self.state.data_ptr()), self.state.numel(), self._stream,
                              arrs["rho_a"], arrs["rho_b"], arrs["ux"], arrs["uy"], ctypes.byref(self._h)))
        self.params = P

    def step(self, n=1):
        _check(_lib.lbb_step(self._h, int(n)))
        return self

    def stress(self):
        sb = np.zeros(self.n)
        st = np.zeros(self.n)
        ns = ctypes.c_int64()
        _check(_lib.lbb_stress(self._h, _dptr(sb), _dptr(st), ctypes.byref(ns)))
        return sb, st, ns.value

    def stress_noalloc(self):
        """stress() through the entry point that allocates nothing (its
        reduction staged in the library's own device array)."""
        sb = np.zeros(self.n)
        st = np.zeros(self.n)
        ns = ctypes.c_int64()
        torch = _torch()
        with torch.cuda.device(self.device):
            _check(_lib.lbb_stress_noalloc(self._h, _dptr(sb), _dptr(st), ctypes.byref(ns)))
        return sb, st, ns.value

    def stress_reset(self):
        _check(_lib.lbb_stress_reset(self._h))

    def fields(self, k):
        ny, nx = self.shapes[k]
        out = [np.empty((ny, nx)) for _ in range(4)]
        _check(_lib.lbb_fields(self._h, int(k), *[_dptr(o) for o in out]))
        return tuple(out)

    def profile(self, k):
        ny, _ = self.shapes[k]
        prof = np.empty(ny)
        ns = ctypes.c_int64()
        _check(_lib.lbb_profile(self._h, int(k), _dptr(prof), ctypes.byref(ns)))
        return prof, ns.value

    def line_profile(self, k):
        ny, _ = self.shapes[k]
        out = np.empty(ny)
        _check(_lib.lbb_line_profile(self._h, int(k), _dptr(out)))
        return out

    def set_launch(self, bx=0, ly=0, grid=0):
        _check(_lib.lbb_set_launch(self._h, int(bx), int(ly), int(grid)))

    def set_graph(self, steps_per_graph):
        _check(_lib.lbb_set_graph(self._h, int(steps_per_graph)))

    def set_fusion(self, steps_per_pass, ly2=0):
        """1 or 2 time steps per pass of the step kernel (2: FP32 or 16-bit
        population storage)."""
        _check(_lib.lbb_set_fusion(self._h, int(steps_per_pass), int(ly2)))

    def set_fusion_tile(self, lanes):
        """Lanes per time step of the fused kernel's blocks: 128, 192, 256, or 0 (automatic)."""
        _check(_lib.lbb_set_fusion_tile(self._h, int(lanes)))

    def fusion_tile(self):
        """(lanes per step, stored columns per tile) of the fused kernel in effect."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lbb_get_fusion_tile(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def launch(self):
        """The launch configuration in effect: dict(bx, ly, grid, steps_per_pass,
        ly2), ly2 the fused tile height with the automatic choice resolved."""
        v = [ctypes.c_int32() for _ in range(5)]
        _check(_lib.lbb_get_launch(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("bx", "ly", "grid", "steps_per_pass", "ly2"), (x.value for x in v)))

    def time_steps(self, n):
        ms = ctypes.c_double()
        _check(_lib.lbb_time_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def autotune(self, cache_path=None, steps=10):
        """Pick the fastest launch shape and grid, and for FP32 and 16-bit storage
        the steps per pass and fused block width
        (state preserved); returns (bx, ly, grid, ms per step)."""
        bx, ly, grid, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(_lib.lbb_autotune(self._h, path, int(steps), ctypes.byref(bx), ctypes.byref(ly), ctypes.byref(grid),
                                 ctypes.byref(ms)))
        return bx.value, ly.value, grid.value, ms.value

    def close(self):
        if self._h:
            _check(_lib.lbb_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
