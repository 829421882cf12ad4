"""Shared helpers of the GPU parity tests: run the same seeded inputs through
the HIP library (via its C ABI binding) and through the FP64 oracle, and the
error norms the comparisons use."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1004_5058_amd import inputs

CS = 1.0 / np.sqrt(3.0)


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1004_5058_amd import lb
    lb.load_library()          # raises if the HIP library is missing
    return torch


def couplings(**kw):
    d = dict(inputs.COUPLINGS)
    d.update(kw)
    return d


def oracle_params(nx, ny, walls, u_top, u_bot, **kw):
    c = couplings(**kw)
    return O.OracleParams(nx=nx, ny=ny, walls=walls, u_top=u_top, u_bot=u_bot, **c)


def gpu_lattice(nx, ny, ra, rb, ux=None, uy=None, walls=True, u_top=0.0, u_bot=0.0,
                storage="f64", profile=False, **kw):
    from paper_1004_5058_amd import lb
    return lb.Lattice(nx, ny, ra, rb, ux, uy, walls=walls, u_top=u_top, u_bot=u_bot,
                      storage=storage, profile=profile, **couplings(**kw))


def oracle_run(p, ra, rb, ux, uy, steps):
    f = O.init(p, ra, rb, ux, uy)
    g, sb, st = O.run(p, f, steps)
    return g, sb / max(steps, 1), st / max(steps, 1)


def err_rho(gpu, ref):
    """max |delta rho| / max |rho_ref|."""
    return float(np.max(np.abs(gpu - ref)) / np.max(np.abs(ref)))


def err_j(gpu_u, gpu_rho, ref_u, ref_rho):
    """max |delta j| / (max rho c_S): momentum error on a velocity scale."""
    dj = np.abs(gpu_u * gpu_rho - ref_u * ref_rho)
    return float(np.max(dj) / (np.max(ref_rho) * CS))


def err_pop(gpu, ref):
    return float(np.max(np.abs(gpu - ref)) / np.max(np.abs(ref)))


def compare_fields(lat, p, g, tol):
    """Compare the GPU lattice's fields with oracle populations g; returns the errors."""
    ra, rb, ux, uy = lat.fields()
    oa, ob, oux, ouy = O.fields(p, g)
    e = dict(rho_a=err_rho(ra, oa), rho_b=err_rho(rb, ob),
             jx=err_j(ux, ra + rb, oux, oa + ob), jy=err_j(uy, ra + rb, ouy, oa + ob))
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, f"errors above {tol}: {e}"
    return e
