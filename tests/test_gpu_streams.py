"""Handles on different HIP streams are independent: two lattices created on
two torch streams (default priority), one FP32 with two steps per pass and
one FP16-deviation, step concurrently through their graphs, and each ends
bitwise where it ends when run alone (the library keeps no device state
outside the caller's allocation)."""
import numpy as np
import pytest

from gpu_common import gpu_lattice, need_gpu
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu
SPECS = [(300, 128, 0.01, "f32", 2), (256, 200, 0.02, "f16dev", 1)]


def _make(k):
    nx, ny, u, storage, per_pass = SPECS[k]
    ra, rb = inputs.emulsion(nx, ny, seed=40 + k)
    lat = gpu_lattice(nx, ny, ra, rb, u_top=u, u_bot=-u, storage=storage)
    lat.set_fusion(per_pass)
    return lat


def test_two_streams_step_concurrently():
    need_gpu()
    import torch
    ref = []
    for k in range(2):
        lat = _make(k)
        lat.step(64)
        ref.append((lat.populations(), lat.stress()))
        lat.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    lats = []
    for k in range(2):
        with torch.cuda.stream(streams[k]):
            lats.append(_make(k))
    for _ in range(4):
        for lat in lats:
            lat.step(16)                  # asynchronous, each on its own stream
    torch.cuda.synchronize()
    for k, lat in enumerate(lats):
        np.testing.assert_array_equal(lat.populations(), ref[k][0])
        assert lat.stress() == ref[k][1]
        lat.close()
