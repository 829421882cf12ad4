"""A plain C program drives the library through include/lb.h alone (device
state from hipMalloc, the legacy default stream, no torch) and reproduces,
bit for bit, what the Python binding computes for the same lattice: FP32
with two steps per pass over an odd number of steps (fused pairs and a final
single step)."""
import subprocess

import numpy as np
import pytest

from c_abi_client import build_client
from gpu_common import need_gpu
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu


def test_c_client_matches_python_binding(tmp_path):
    need_gpu()
    from paper_1004_5058_amd import lb
    nx, ny, steps, u = 300, 96, 31, 0.02
    ra, rb = inputs.emulsion(nx, ny, seed=12)
    ux, uy = inputs.couette(nx, ny, u, -u)
    np.concatenate([a.ravel() for a in (ra, rb, ux, uy)]).astype(np.float64).tofile(tmp_path / "in.bin")
    exe = build_client(tmp_path)
    r = subprocess.run([exe, str(nx), str(ny), str(steps), "1", "2", repr(u), str(tmp_path / "in.bin"),
                        str(tmp_path / "out.bin")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = (tmp_path / "out.bin").read_bytes()
    n = nx * ny
    got = np.frombuffer(raw[:4 * n * 8], dtype=np.float64).reshape(4, ny, nx)
    sig = np.frombuffer(raw[4 * n * 8:4 * n * 8 + 16], dtype=np.float64)
    ns = int(np.frombuffer(raw[4 * n * 8 + 16:], dtype=np.int64)[0])

    lat = lb.Lattice(nx, ny, ra, rb, ux, uy, u_top=u, u_bot=-u, storage="f32", **inputs.COUPLINGS)
    lat.set_fusion(2)
    lat.step(steps)
    want = lat.fields()
    sb, st, n_py = lat.stress()
    lat.close()
    for a, b in zip(got, want):
        np.testing.assert_array_equal(a, b)
    assert sig[0] == sb and sig[1] == st and ns == n_py == steps
