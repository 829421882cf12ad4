"""Pins of the FP64 surrogate-network oracle: gradients against central
finite differences, the closed form of the first Adam step, a network that
reduces to a known function, and loss decrease on a smooth target."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 3))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    return X, y


def test_parameter_count():
    assert M.NPARAM == 4481


def test_gradient_matches_central_differences():
    X, y = _data()
    theta = M.init_params(3)
    theta[M.H * 3:M.H * 4] = 0.1          # non-zero biases exercise every term
    theta[-1] = -0.2
    _, g = M.loss_grad(theta, X, y)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(M.NPARAM, 60, replace=False), [M.NPARAM - 1, 0, 200, 4416]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (M.loss_grad(tp, X, y)[0] - M.loss_grad(tm, X, y)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_first_adam_step_is_signed_lr():
    """At t = 1 the bias-corrected step is lr * g / (|g| + eps): a step of
    size lr against the sign of every non-zero gradient component."""
    theta = np.zeros(M.NPARAM)
    g = np.linspace(-1, 1, M.NPARAM)
    g[M.NPARAM // 2] = 0.0
    t1, m, v = M.adam_step(theta, g, np.zeros(M.NPARAM), np.zeros(M.NPARAM), 1, 0.01)
    nz = g != 0
    np.testing.assert_allclose(t1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    big = np.abs(g) > 1e-3
    np.testing.assert_allclose(t1[big], -0.01 * np.sign(g[big]), rtol=1e-5)
    assert t1[M.NPARAM // 2] == 0.0


def test_forward_reduces_to_a_known_function():
    """Only one path switched on: out = w3 tanh(w2 tanh(w1 x0 + c1) + c2) + c3."""
    W1 = np.zeros((M.H, 3)); W1[5, 0] = 0.7
    b1 = np.zeros(M.H); b1[5] = 0.1
    W2 = np.zeros((M.H, M.H)); W2[9, 5] = -1.3
    b2 = np.zeros(M.H); b2[9] = 0.2
    W3 = np.zeros(M.H); W3[9] = 2.0
    theta = M.pack(W1, b1, W2, b2, W3, 0.3)
    X = np.array([[0.5, 9.0, -9.0], [-1.0, 0.0, 0.0]])
    out, _ = M.forward(theta, X)
    ref = 2.0 * np.tanh(-1.3 * np.tanh(0.7 * X[:, 0] + 0.1) + 0.2) + 0.3
    np.testing.assert_allclose(out, ref, rtol=1e-15)


def test_training_reduces_loss():
    X, y = _data(200)
    theta = M.init_params(0)
    l0, _ = M.loss_grad(theta, X, (y - y.mean()) / y.std())
    theta, l1 = M.train(theta, X, (y - y.mean()) / y.std(), 300, 1e-2)
    assert l1 < 0.2 * l0
