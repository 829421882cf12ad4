"""The 1024 x 1024 Couette emulsion workload at its full length: wall speed
0.05, 20 000 steps, the wall stress averaged over the second half.

The FP64 oracle would need about half an hour of host time for this run, so
the long-run reference is the GPU's FP64 population step (which matches the
oracle to 1e-12 over 1000 steps) and it is cross-checked by the independent
FP64 moment form (tau = 1).  The flow is not chaotic in this regime (a 1e-7
perturbation of the start moves the averaged stress by ~1e-8, one of 1e-4 by
~3e-5), so the time average is well conditioned and the storage forms can be
compared with it.

Bounds: the two FP64 forms differ only by rounding order: 1e-10 bounds 20 000
steps of ~1e-16 per step with room.  The averaged stress is a small difference
of large momentum fluxes (at wall speed 0.05 it is ~1e-3 of the diagonal
populations whose difference makes it), so the storage rounding of the
populations reaches its relative error amplified; no useful bound follows from
the arithmetic, and the reduced-precision errors are stated (printed; the
measured values are FP32 1.4e-4 at worst, FP16 9e-3) under bounds of a few
times those: FP32 2e-3, FP16 2 %.  BF16 deviation storage does not reach the
1 % accuracy of the flow-curve points on this run (measured 2.4e-2 / 0.13 /
7.9e-2 at the bottom wall / top wall / mean): the test asserts that it misses
it, so that the documented limit of the form stays true."""
import json
import os

import numpy as np
import pytest

from gpu_common import need_gpu
from paper_1004_5058_amd import inputs

pytestmark = pytest.mark.gpu
N, U, STEPS = 1024, 0.05, 20000
BOUND = {"mom64": 1e-10, "f32": 2e-3, "f32x2": 2e-3, "mom32": 2e-3, "f16dev": 2e-2}
# the accuracy a flow-curve point needs (relative error of the mean stress)
POINT_BAR = 1e-2


def _run(storage, fusion=1):
    from paper_1004_5058_amd import lb
    ra, rb = inputs.emulsion(N, N, seed=1)
    ux, uy = inputs.couette(N, N, U, -U)
    lat = lb.Lattice(N, N, ra, rb, ux, uy, u_top=U, u_bot=-U, storage=storage, **inputs.COUPLINGS)
    try:
        if fusion > 1:
            lat.set_fusion(fusion)
        lat.step(STEPS // 2)
        lat.stress_reset()
        lat.step(STEPS // 2)
        sb, st, n = lat.stress()
        assert n == STEPS // 2 and lat.time() == STEPS
        return np.array([sb, st, 0.5 * (sb + st)])
    finally:
        lat.close()


def test_time_averaged_wall_stress_1024_full_length():
    need_gpu()
    ref = _run("f64")
    assert np.all(ref > 0)
    out = {"mom64": _run("mom64"), "f32": _run("f32"), "f32x2": _run("f32", fusion=2), "mom32": _run("mom32"),
           "f16dev": _run("f16dev"), "bf16dev": _run("bf16dev")}
    print(f"\nFP64 reference: sigma_bot {ref[0]:.9e}, sigma_top {ref[1]:.9e}, mean {ref[2]:.9e}")
    for k, v in out.items():
        e = np.abs(v - ref) / np.abs(ref)
        print(f"{k:8s}: relative error bot {e[0]:.2e}, top {e[1]:.2e}, mean {e[2]:.2e} "
              f"(bound {BOUND.get(k, 'none: stated')})")
        if k == "bf16dev":
            assert e[2] > POINT_BAR, "BF16 deviation storage now meets the 1 % bar: update the documented limit"
        else:
            assert np.all(e < BOUND[k]), (k, e)
    # two steps per pass is bitwise the single-step run
    np.testing.assert_array_equal(out["f32x2"], out["f32"])


# The 4096 x 4096 workload at its stated length (wall speed 0.02, 5000 steps):
# fields at the end and the wall stress averaged over the second half, each
# storage form against the GPU's FP64 step (whose full-size windows match the
# oracle, tests/test_gpu_fullsize.py).  Fields, FP32: each population is
# rounded once per step (2^-24 relative); added linearly over 5000 steps that
# is 3e-4 of the largest density (and of the momentum scale).  The averaged
# stress (~6e-6 here, ~1e-4 of the populations it is made from) and the FP16
# form are stated under bounds of a few times the measured values (FP32 stress
# 2e-3, measured 5.3e-4; FP16 5e-2, measured 1.4e-2 fields and 1.3e-2 stress).
# BF16 deviation storage does not hold the droplet interfaces over this run
# (measured: density error 0.24 of the largest density, stress 43 %): the test
# asserts that it misses the 1 % bar of a flow-curve point (the documented
# limit: a short-horizon form).  The 16-bit forms run two steps per pass too;
# those runs must equal the single-step ones bit for bit.  With LB_RESULTS_DIR
# set, the errors are written to precision_couette_emulsion_4096x4096_5000steps.json
# there (the record the benchmark quotes).
N4, U4, STEPS4 = 4096, 0.02, 5000
FIELD_BOUND = {"f32x2": 3e-4, "mom32": 3e-4, "f16dev": 5e-2}
STRESS_BOUND = {"f32x2": 2e-3, "mom32": 2e-3, "f16dev": 5e-2}


def _run4(storage, fusion=1):
    from paper_1004_5058_amd import lb
    ra, rb = inputs.emulsion(N4, N4, seed=1)
    ux, uy = inputs.couette(N4, N4, U4, -U4)
    lat = lb.Lattice(N4, N4, ra, rb, ux, uy, u_top=U4, u_bot=-U4, storage=storage, **inputs.COUPLINGS)
    del ra, rb, ux, uy
    try:
        if fusion > 1:
            lat.set_fusion(fusion)
        lat.step(STEPS4 // 2)
        lat.stress_reset()
        lat.step(STEPS4 // 2)
        sb, st, n = lat.stress()
        assert n == STEPS4 // 2
        a, b, vx, vy = lat.fields()
        return (a, b, vx * (a + b), vy * (a + b)), np.array([sb, st, 0.5 * (sb + st)])
    finally:
        lat.close()


def test_4096_fields_and_stress_full_length():
    need_gpu()
    (ra, rb, jx, jy), sref = _run4("f64")
    scale_r = max(ra.max(), rb.max())
    scale_j = (ra + rb).max() / np.sqrt(3.0)
    print(f"\nFP64 reference after {STEPS4} steps: stress bot {sref[0]:.9e}, top {sref[1]:.9e}")
    errs, runs = {}, {}
    for storage in ("f32x2", "mom32", "f16dev", "f16x2", "bf16dev", "bf16x2"):
        name = {"f32x2": "f32", "f16x2": "f16dev", "bf16x2": "bf16dev"}.get(storage, storage)
        (a, b, x, y), s = _run4(name, fusion=2 if storage.endswith("x2") else 1)
        e_rho = max(np.abs(a - ra).max(), np.abs(b - rb).max()) / scale_r
        e_j = max(np.abs(x - jx).max(), np.abs(y - jy).max()) / scale_j
        e_s = np.abs(s - sref) / np.abs(sref)
        if storage in ("f16x2", "bf16x2"):
            # two steps per pass: bitwise the single-step run of the same storage
            for u, v in zip((a, b, x, y), runs[name][0]):
                np.testing.assert_array_equal(u, v)
            np.testing.assert_array_equal(s, runs[name][1])
        else:
            runs[storage] = ((a, b, x, y), s)
        del a, b, x, y
        errs[storage] = (e_rho, e_j, e_s)
        print(f"{storage:8s}: rho {e_rho:.2e}, j {e_j:.2e} (bound {FIELD_BOUND.get(storage, 'stated')}), stress "
              f"bot {e_s[0]:.2e} top {e_s[1]:.2e} mean {e_s[2]:.2e} (bound {STRESS_BOUND.get(storage, 'stated')})")
    out_dir = os.environ.get("LB_RESULTS_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        rec = {"workload": f"couette_emulsion_{N4}x{N4}", "steps": STEPS4, "wall_speed": U4,
               "reference": "FP64 population step on the GPU (4096^2 windows match the oracle to <= 1e-15)",
               "norms": "rho: max |d rho| / max rho; j: max |d j| / (max rho c_S); stress: relative error of the "
                        "wall stress averaged over the second half (bottom, top, mean)",
               "errors": {k: {"rho": float(f"{v[0]:.3e}"), "j": float(f"{v[1]:.3e}"),
                              "stress_bot_top_mean": [float(f"{x:.3e}") for x in v[2]],
                              "meets_1pct_stress": bool(v[2][2] < 1e-2)} for k, v in errs.items()}}
        with open(os.path.join(out_dir, "precision_couette_emulsion_4096x4096_5000steps.json"), "w") as f:
            json.dump(rec, f, indent=1)
    for storage, (e_rho, e_j, e_s) in errs.items():
        if storage.startswith("bf16"):
            assert e_s[2] > POINT_BAR, "BF16 deviation storage now meets the 1 % bar: update the documented limit"
            continue
        if storage == "f16x2":
            continue          # bitwise the f16dev run, checked above
        assert e_rho < FIELD_BOUND[storage] and e_j < FIELD_BOUND[storage], storage
        assert np.all(e_s < STRESS_BOUND[storage]), storage
