"""Surrogate network: HIP forward, gradient and Adam training against the FP64
NumPy oracle on identical seeded data and initial parameters."""
import numpy as np
import pytest

from gpu_common import need_gpu
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(-9.5, -8.5, n), rng.uniform(7.5, 8.5, n), rng.uniform(-9, -3, n)])
    y = 1e-4 * (1 + 0.3 * (X[:, 1] - 8) + np.exp(0.5 * (X[:, 2] + 6)) + 0.1 * (X[:, 0] + 9))
    return X.astype(np.float32), y.astype(np.float32)


def _net(X, y, seed=1):
    from paper_1004_5058_amd.mlp import MLP
    net = MLP(max_rows=4096)
    theta = M.init_params(seed).astype(np.float32)
    net.set_params(theta)
    mu, sd = X.mean(0), X.std(0)
    sd = np.where(sd > 0, sd, 1.0).astype(np.float32)
    ysd = float(y.std()) if y.std() > 0 else 1.0
    net.set_norm(mu, sd, float(y.mean()), ysd)
    net.set_data(X, y)
    Xs = (X.astype(np.float64) - mu) / sd
    ys = (y.astype(np.float64) - float(y.mean())) / ysd
    return net, theta.astype(np.float64), Xs, ys


def test_infer_matches_oracle():
    X, y = _data(1000)
    net, theta, Xs, _ = _net(X, y)
    out = net.infer(X)
    ref, _ = M.forward(theta, Xs)
    np.testing.assert_allclose((out - float(y.mean())) / float(y.std()), ref, rtol=0, atol=2e-5)


@pytest.mark.parametrize("n", [1, 37, 2000])
def test_loss_and_gradient_match_oracle(n):
    X, y = _data(n, seed=n)
    net, theta, Xs, ys = _net(X, y)
    loss, g = net.loss_grad()
    lref, gref = M.loss_grad(theta, Xs, ys)
    assert loss == pytest.approx(lref, rel=2e-5, abs=1e-7)
    scale = np.max(np.abs(gref))
    np.testing.assert_allclose(g, gref, rtol=0, atol=2e-5 * scale)


def test_adam_training_tracks_oracle():
    X, y = _data(500, seed=3)
    net, theta, Xs, ys = _net(X, y)
    net.train(25, 3e-3)
    tref, _ = M.train(theta, Xs, ys, 25, 3e-3)
    got = net.get_params().astype(np.float64)
    np.testing.assert_allclose(got, tref, rtol=0, atol=5e-4)


def test_training_reduces_loss_and_generalises():
    X, y = _data(2000, seed=4)
    net, theta, Xs, ys = _net(X, y)
    l0, _ = net.loss_grad()
    net.train(1500, 3e-3)
    l1, _ = net.loss_grad()
    assert l1 < 0.01 * l0
    Xt, yt = _data(300, seed=99)
    pred = net.infer(Xt)
    assert np.max(np.abs(pred - yt)) / np.max(np.abs(yt)) < 0.05


def test_bad_inputs_rejected():
    from paper_1004_5058_amd import lb
    from paper_1004_5058_amd.mlp import MLP
    net = MLP(max_rows=16)
    with pytest.raises(lb.LBError):
        net.set_data(np.zeros((17, 3)), np.zeros(17))
    with pytest.raises(lb.LBError):
        net.set_norm([0, 0, 0], [1, 0, 1], 0.0, 1.0)
    with pytest.raises(lb.LBError):
        net.loss_grad()           # no data yet
