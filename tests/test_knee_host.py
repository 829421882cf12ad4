"""Host logic of the knee proposer (no GPU): on an exact Herschel-Bulkley
curve sigma = sigma_Y + B S^beta the knee, where the power term equals the
yield stress, is S_k = (sigma_Y / B)^(1 / beta); the proposals are k rates
log-spaced within the stated decades of it, clipped to the searched range; a
curve without a yield stress falls back to the middle of the range."""
import numpy as np
import pytest

from paper_1004_5058_amd import surrogate

S_LO, S_HI = 2e-7, 4e-4


def _exact(sy, B, beta):
    s = surrogate.FlowSurrogate.__new__(surrogate.FlowSurrogate)
    s.predict = lambda g1, g2, S: sy + B * np.atleast_1d(np.asarray(S, dtype=np.float64)) ** beta
    return s


@pytest.mark.parametrize("sy,S_k,beta", [(1.5e-4, 1e-5, 0.5), (1.5e-4, 1e-6, 0.25), (5e-5, 1e-4, 0.8)])
def test_knee_of_exact_curve(sy, S_k, beta):
    B = sy / S_k ** beta
    s = _exact(sy, B, beta)
    sk, fit = s.knee(-9.0, 8.1, S_LO, S_HI)
    assert abs(sk - S_k) / S_k < 1e-6
    assert abs(fit["sigma_y"] - sy) / sy < 1e-8 and abs(fit["beta"] - beta) < 1e-8
    S, _ = s.propose(-9.0, 8.1, S_LO, S_HI, k=6, width=1.0)
    lo, hi = max(S_LO, S_k / 10), min(S_HI, S_k * 10)
    assert len(S) == 6
    assert abs(S[0] - lo) / lo < 1e-6 and abs(S[-1] - hi) / hi < 1e-6
    r = np.diff(np.log(S))
    assert np.all(r > 0) and np.ptp(r) < 1e-9


def test_proposals_clipped_to_range():
    sy, beta, S_k = 1e-4, 0.5, 2e-4            # a decade above the knee lies outside the range
    s = _exact(sy, sy / S_k ** beta, beta)
    S, _ = s.propose(0, 0, S_LO, S_HI, k=5, width=1.0)
    assert abs(S[-1] - S_HI) / S_HI < 1e-12 and abs(S[0] - S_k / 10) / (S_k / 10) < 1e-6


def test_newtonian_curve_falls_back_to_middle():
    s = _exact(0.0, 0.18, 1.0)
    sk, fit = s.knee(0, 0, S_LO, S_HI)
    assert fit["sigma_y"] < 1e-15
    assert abs(sk - np.sqrt(S_LO * S_HI)) / sk < 1e-12
