"""Herschel-Bulkley fitter (host analysis): exact recovery of noise-free
synthetic flow curves, the sigma_Y >= 0 constraint, the Newtonian limit, and
robustness to small noise."""
import numpy as np
import pytest

from paper_1004_5058_amd.flowcurve import bulk_rate, hb_fit


@pytest.mark.parametrize("sy,B,beta", [(1.5e-4, 2e-3, 0.25), (1.5e-4, 5e-3, 0.5), (0.0, 0.17, 1.0),
                                       (3e-5, 1e-2, 0.8), (2e-4, 1e-3, 1.6)])
def test_exact_recovery(sy, B, beta):
    S = np.logspace(-7, -3, 30)
    sigma = sy + B * S ** beta
    fit = hb_fit(S, sigma)
    assert fit["beta"] == pytest.approx(beta, rel=1e-6)
    assert fit["B"] == pytest.approx(B, rel=1e-5)
    assert fit["sigma_y"] == pytest.approx(sy, abs=1e-9 * max(sigma))


def test_newtonian_limit_gives_zero_yield():
    """sigma = rho nu S (a Newtonian fluid): beta = 1, sigma_Y = 0."""
    S = np.linspace(1e-6, 1e-4, 20)
    fit = hb_fit(S, (1.0 / 6.0) * S)
    assert fit["beta"] == pytest.approx(1.0, rel=1e-6)
    assert fit["sigma_y"] == pytest.approx(0.0, abs=1e-12)


def test_noisy_recovery():
    rng = np.random.default_rng(0)
    S = np.logspace(-6, -3, 48)
    sigma = 1.5e-4 + 4e-3 * S ** 0.5
    fit = hb_fit(S, sigma * (1 + 2e-3 * rng.standard_normal(S.size)))
    assert fit["beta"] == pytest.approx(0.5, abs=0.05)
    assert fit["sigma_y"] == pytest.approx(1.5e-4, rel=0.05)


def test_rejects_too_few_points():
    with pytest.raises(ValueError):
        hb_fit([1e-4, 2e-4, 0.0], [1.0, 2.0, 3.0])


def test_bulk_rate_of_linear_profile():
    y = np.arange(64)
    assert bulk_rate(0.01 * (y + 0.5) - 0.3) == pytest.approx(0.01, rel=1e-12)
