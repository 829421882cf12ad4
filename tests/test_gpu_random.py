"""Seeded randomized parity sweep: lattice sizes from a single column to
several tiles with ragged tails, periodic or walled, random tau, rho0,
couplings, wall speeds, body force, every storage form and launch shape,
each against the FP64 oracle on the same inputs after 30 steps (fields to the
bound of the storage, populations element by element).  The draws pick the
test configurations only; no model arithmetic happens here.

Bounds: FP64 and the FP64 moment form 1e-12, FP32 and the FP32 moment form
1e-6 (the parity target).  16-bit deviation storage from the noise start
(rho = 0.5 +- 0.01 around rho_ref = 0.5): deviations stay below ~4/9 x 0.02,
half an FP16 ulp there is ~2e-6 per population, so 31 roundings of nine
populations move a density by at most ~5e-4, the FP16 bound; 8x that for
BF16's coarser mantissa.  (Moving walls and tau near 1/2 give the largest
errors of the sweep, ~1.2e-4 in both 16-bit forms.)"""
import numpy as np
import pytest

from gpu_common import compare_fields, err_pop, gpu_lattice, need_gpu, oracle_params, oracle_run
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-6, "f16dev": 5e-4, "bf16dev": 4e-3, "mom64": 1e-12, "mom32": 1e-6}
STORAGES = ("f64", "f32", "f16dev", "bf16dev", "mom64", "mom32")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _draw(seed):
    r = np.random.default_rng(1000 + seed)
    walls = bool(r.integers(2))
    nx = int(r.choice([1, 2, 3, 5])) if seed % 6 == 0 else int(r.integers(6, 300))
    ny = int(r.integers(2, 8)) if seed % 6 == 1 else int(r.integers(8, 160))
    kw = dict(tau=float(r.uniform(0.6, 1.8)), rho0=float(r.uniform(0.7, 0.9)),
              g_aa1=float(r.uniform(-10.0, -7.0)), g_aa2=float(r.uniform(6.0, 9.0)),
              g_bb1=float(r.uniform(-10.0, -7.0)), g_bb2=float(r.uniform(6.0, 9.0)),
              g_ab=float(r.uniform(0.0, 0.5)))
    if r.integers(2):
        kw.update(fx_amp=float(r.uniform(0.0, 1e-4)), fx_k=float(r.uniform(0.0, 1.0)))
    u_top, u_bot = (float(r.uniform(-0.03, 0.03)), float(r.uniform(-0.03, 0.03))) if walls else (0.0, 0.0)
    storage = STORAGES[seed % len(STORAGES)]
    if storage.startswith("mom"):
        kw["tau"] = 1.0          # the moment form holds the state at tau = 1 only
    bx = int(r.choice([64, 128, 256] + ([512] if storage in ("f32", "f16dev", "bf16dev") else [])))
    ly = int(r.integers(1, 200))
    # FP32 and 16-bit storage: two steps per pass in about half of the cases,
    # random fused tile height (16-bit: any nx, odd ones included)
    fuse = storage in ("f32", "f16dev", "bf16dev") and bool(r.integers(2))
    ly2 = int(r.integers(0, 100))
    return nx, ny, walls, u_top, u_bot, kw, storage, bx, ly, fuse, ly2


@pytest.mark.parametrize("seed", range(36))
def test_random_configuration_matches_oracle(seed):
    nx, ny, walls, u_top, u_bot, kw, storage, bx, ly, fuse, ly2 = _draw(seed)
    ra, rb = inputs.noise(nx, ny, seed)
    p = oracle_params(nx, ny, walls, u_top, u_bot, **kw)
    g, _, _ = oracle_run(p, ra, rb, None, None, 30)
    lat = gpu_lattice(nx, ny, ra, rb, walls=walls, u_top=u_top, u_bot=u_bot, storage=storage, **kw)
    lat.set_launch(bx, ly)
    # the fused block width from a generator of its own (the draws above
    # stay those of earlier sweeps): 128, 192 or 256 lanes or automatic
    lanes = int(np.random.default_rng(9000 + seed).choice([0, 128, 192, 256]))
    if fuse:
        lat.set_fusion_tile(lanes)
        lat.set_fusion(2, ly2)
    lat.step(30)
    tol = TOL[storage]
    e = compare_fields(lat, p, g, tol)
    ep = err_pop(lat.populations(), g)
    print(f"\nseed {seed}: {nx}x{ny} walls={walls} {storage}{' fused ly2 %d lanes %d' % (ly2, lanes) if fuse else ''} "
          f"shape {bx}x{ly} tau {kw['tau']:.3f}: "
          f"{max(e.values()):.2e}, populations {ep:.2e}")
    assert ep <= 10 * tol
    lat.close()


class _Member:
    """One lattice of a batch, seen through the fields call the comparisons use."""

    def __init__(self, batch, k):
        self.batch, self.k = batch, k

    def fields(self):
        return self.batch.fields(self.k)


@pytest.mark.parametrize("seed", range(12))
def test_random_batch_matches_oracle(seed):
    """Batches of 2-7 lattices of random sizes, each with its own walls, tau,
    couplings, wall speeds and body force, under a random tile shape,
    persistent grid and graph length: every lattice against its own oracle
    run after 30 steps."""
    import torch
    from paper_1004_5058_amd import lb
    r = np.random.default_rng(5000 + seed)
    storage = ("f64", "f32", "f16dev", "mom32")[seed % 4]
    specs, cases = [], []
    for k in range(int(r.integers(2, 8))):
        nx, ny = int(r.integers(1, 260)), int(r.integers(2, 140))
        walls = bool(r.integers(2))
        kw = dict(tau=1.0 if storage == "mom32" else float(r.uniform(0.6, 1.8)), rho0=float(r.uniform(0.7, 0.9)),
                  g_aa1=float(r.uniform(-10.0, -7.0)), g_aa2=float(r.uniform(6.0, 9.0)),
                  g_bb1=float(r.uniform(-10.0, -7.0)), g_bb2=float(r.uniform(6.0, 9.0)),
                  g_ab=float(r.uniform(0.0, 0.5)))
        if r.integers(2):
            kw.update(fx_amp=float(r.uniform(0.0, 1e-4)), fx_k=float(r.uniform(0.0, 1.0)))
        u_top, u_bot = (float(r.uniform(-0.03, 0.03)), float(r.uniform(-0.03, 0.03))) if walls else (0.0, 0.0)
        ra, rb = inputs.noise(nx, ny, 100 * seed + k)
        specs.append(dict(nx=nx, ny=ny, rho_a=ra, rho_b=rb, ux=None, uy=None, walls=walls, u_top=u_top,
                          u_bot=u_bot, **kw))
        cases.append((oracle_params(nx, ny, walls, u_top, u_bot, **kw), ra, rb))
    bx = int(r.choice([64, 128, 256] + ([512] if storage in ("f32", "f16dev") else [])))
    ly = int(r.integers(1, 150))
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    grid = int(r.choice([0, ncu, 2 * ncu]))
    graph = int(r.choice([0, 2, 8, 32]))
    fuse = storage in ("f32", "f16dev", "bf16dev") and bool(r.integers(2))
    b = lb.Batch(specs, storage=storage, profile=False)
    b.set_launch(bx, ly, grid)
    b.set_graph(graph)
    lanes = int(np.random.default_rng(9500 + seed).choice([0, 128, 192, 256]))
    if fuse:
        b.set_fusion_tile(lanes)
        b.set_fusion(2, int(r.integers(0, 60)))
    b.step(30)
    worst = 0.0
    for k, (p, ra, rb) in enumerate(cases):
        g, _, _ = oracle_run(p, ra, rb, None, None, 30)
        e = compare_fields(_Member(b, k), p, g, TOL[storage])
        worst = max(worst, max(e.values()))
    b.close()
    print(f"\nbatch seed {seed}: {len(specs)} lattices {storage}{' fused lanes %d' % lanes if fuse else ''} shape {bx}x{ly} "
          f"grid {grid} graph {graph}: "
          f"worst {worst:.2e}")
