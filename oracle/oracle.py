"""NumPy/ctypes front end of the FP64 C oracle (oracle/lb_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the package smoke check and the
benchmark's CPU-baseline leg.  It never imports the HIP library, and the HIP
library never imports it.

Population arrays are float64 with shape (2, 9, ny, nx): species A/B, D2Q9
direction in the order 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1),
5 (1,1), 6 (-1,1), 7 (-1,-1), 8 (1,-1).
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None
_native = False


def use_native_build():
    """Load the copy built with -march=native for this host (the CPU-baseline
    timing); same results bit for bit.  Call before the first oracle call."""
    global _native
    if _lib is not None and not _native:
        raise RuntimeError("the oracle library is already loaded")
    _native = True


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("walls", ctypes.c_int),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("g_att", ctypes.c_double * 2), ("g_rep", ctypes.c_double * 2),
        ("g_ab", ctypes.c_double), ("u_top", ctypes.c_double), ("u_bot", ctypes.c_double),
        ("fx_amp", ctypes.c_double), ("fx_k", ctypes.c_double),
    ]


@dataclass
class OracleParams:
    """Model parameters in the paper's notation (Eq. (1), Eq. (2))."""
    nx: int
    ny: int
    tau: float = 1.0
    rho0: float = 0.83
    g_aa1: float = -9.0   # G^a_AA, belt 1
    g_aa2: float = 8.1    # G^r_AA, belts 1-2
    g_bb1: float = -9.0   # G^a_BB
    g_bb2: float = 8.1    # G^r_BB
    g_ab: float = 0.405   # G^X_AB, belt 1
    walls: bool = True
    u_top: float = 0.0
    u_bot: float = 0.0
    fx_amp: float = 0.0   # body force F_x(y) = fx_amp sin(fx_k y) (section "Numerical Results")
    fx_k: float = 0.0

    def _c(self):
        p = _Params()
        p.nx, p.ny, p.walls = self.nx, self.ny, int(bool(self.walls))
        p.tau, p.rho0 = self.tau, self.rho0
        p.g_att[0], p.g_att[1] = self.g_aa1, self.g_bb1
        p.g_rep[0], p.g_rep[1] = self.g_aa2, self.g_bb2
        p.g_ab, p.u_top, p.u_bot = self.g_ab, self.u_top, self.u_bot
        p.fx_amp, p.fx_k = self.fx_amp, self.fx_k
        return p


def lib():
    global _lib
    if _lib is None:
        path = _build.build(native=_native)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(_Params)
        L.orc_tables.argtypes = [ip, ip, dp, ip]
        L.orc_stencil_weight.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_psi.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_psi.restype = ctypes.c_double
        L.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_force.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.orc_init.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_collide.argtypes = [pp, dp, dp, dp, dp]
        L.orc_stream.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, dp, dp]
        L.orc_run.argtypes = [pp, dp, ctypes.c_int, dp]
        L.orc_sums.argtypes = [pp, dp, dp]
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables():
    L = lib()
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int * 9)()
    L.orc_tables(cx, cy, w, opp)
    return np.array(cx[:]), np.array(cy[:]), np.array(w[:]), np.array(opp[:])


def stencil_weight(cx, cy):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_stencil_weight(int(cx), int(cy), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium(float(rho), float(ux), float(uy), _ptr(out))
    return out


def psi(rho, rho0):
    return lib().orc_psi(float(rho), float(rho0))


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    assert a.shape == shape, (a.shape, shape)
    return a


def init(p: OracleParams, rho_a, rho_b, ux=None, uy=None):
    shp = (p.ny, p.nx)
    f = np.empty((2, 9, p.ny, p.nx))
    ra, rb = _f64(rho_a, shp), _f64(rho_b, shp)
    u = None if ux is None else _f64(ux, shp)
    v = None if uy is None else _f64(uy, shp)
    cp = p._c()
    lib().orc_init(ctypes.byref(cp), _ptr(ra), _ptr(rb), _ptr(u), _ptr(v), _ptr(f))
    return f


def fields(p: OracleParams, f):
    f = _f64(f, (2, 9, p.ny, p.nx))
    out = [np.empty((p.ny, p.nx)) for _ in range(4)]
    cp = p._c()
    lib().orc_fields(ctypes.byref(cp), _ptr(f), *[_ptr(o) for o in out])
    return tuple(out)


def force(p: OracleParams, rho_a, rho_b):
    shp = (p.ny, p.nx)
    ra, rb = _f64(rho_a, shp), _f64(rho_b, shp)
    out = [np.empty(shp) for _ in range(4)]
    cp = p._c()
    lib().orc_force(ctypes.byref(cp), _ptr(ra), _ptr(rb), *[_ptr(o) for o in out])
    return tuple(out)  # FAx, FAy, FBx, FBy


def collide(p: OracleParams, f):
    f = _f64(f, (2, 9, p.ny, p.nx))
    fs = np.empty_like(f)
    ra = np.empty((p.ny, p.nx))
    rb = np.empty((p.ny, p.nx))
    cp = p._c()
    lib().orc_collide(ctypes.byref(cp), _ptr(f), _ptr(fs), _ptr(ra), _ptr(rb))
    return fs, ra, rb


def step(p: OracleParams, f):
    """One step; returns (f_new, (F_bot_x, F_top_x))."""
    f = _f64(f, (2, 9, p.ny, p.nx))
    g = np.empty_like(f)
    wf = np.zeros(2)
    cp = p._c()
    lib().orc_step(ctypes.byref(cp), _ptr(f), _ptr(g), _ptr(wf))
    return g, (wf[0], wf[1])


def run(p: OracleParams, f, nsteps):
    """nsteps steps; returns (f_new, sum_t sigma_bot, sum_t sigma_top)."""
    g = np.array(_f64(f, (2, 9, p.ny, p.nx)), copy=True)
    st = np.zeros(2)
    cp = p._c()
    lib().orc_run(ctypes.byref(cp), _ptr(g), int(nsteps), _ptr(st))
    return g, st[0], st[1]


def sums(p: OracleParams, f):
    f = _f64(f, (2, 9, p.ny, p.nx))
    out = np.zeros(4)
    cp = p._c()
    lib().orc_sums(ctypes.byref(cp), _ptr(f), _ptr(out))
    return out  # mass_A, mass_B, jx, jy


def threads():
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_threads())
