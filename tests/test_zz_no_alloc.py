"""The allocation-free entry point (lbb_stress_noalloc): the per-lattice
reduction of lbb_stress staged in the library's own device array instead of
the caller's state.  Through the C ABI it must return lbb_stress's results bit
for bit, on two calls in a row (the second with a smaller batch, so stale
entries of the shared array would show), and refuse batches beyond its
4096-lattice array."""
import numpy as np
import pytest

from gpu_common import need_gpu
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    from paper_1004_5058_amd import lb
    specs = []
    for k, (nx, ny) in enumerate(sizes):
        ra, rb = inputs.emulsion(nx, ny, seed=seed + k)
        u = 0.004 * (k + 1)
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, u_top=u, u_bot=-u,
                          g_aa2=7.9 + 0.05 * k))
    return lb.Batch(specs, storage="f32", profile=False)


def test_noalloc_stress_equals_lbb_stress():
    need_gpu()
    for sizes, steps, seed in (([(256, 128), (300, 77), (128, 256), (64, 40), (512, 96)], 17, 1),
                               ([(96, 64), (200, 50)], 9, 30)):
        b = _batch(sizes, seed)
        try:
            b.step(steps)
            ref = b.stress()
            got = b.stress_noalloc()
            assert got[2] == ref[2] == steps
            np.testing.assert_array_equal(got[0], ref[0])
            np.testing.assert_array_equal(got[1], ref[1])
            assert np.all(ref[0] != 0) and np.all(ref[1] != 0)
            # a second read of the same state, after more steps and a reset
            b.stress_reset()
            b.step(4)
            ref = b.stress()
            got = b.stress_noalloc()
            np.testing.assert_array_equal(got[0], ref[0])
            np.testing.assert_array_equal(got[1], ref[1])
        finally:
            b.close()


def test_noalloc_stress_refuses_batches_beyond_its_array():
    need_gpu()
    from paper_1004_5058_amd import lb
    b = _batch([(4, 2)] * 4097, 500)
    try:
        with pytest.raises(lb.LBError, match="at most 4096"):
            b.stress_noalloc()
        sb, st, n = b.stress()          # the allocating form still serves it
        assert len(sb) == 4097 and n == 0
    finally:
        b.close()
