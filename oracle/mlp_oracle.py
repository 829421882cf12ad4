"""Plain FP64 NumPy reference of the surrogate network (3 -> 64 -> 64 -> 1, tanh).

TEST INFRASTRUCTURE ONLY: the GPU training and inference kernels are checked
against it; it shares nothing with them.

The network maps standardised inputs x' = (x - mu_in)/sd_in to a standardised
output; the loss is the mean squared error on y' = (y - mu_out)/sd_out.
Parameter vector (the interface layout, 4481 values):
    W1 (64 x 3, row-major), b1 (64), W2 (64 x 64, row-major: W2[j, k] feeds
    unit j from unit k), b2 (64), W3 (64), b3 (1).
Training is full-batch Adam (Kingma & Ba, 2015) with the usual bias
corrections: m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import numpy as np

H = 64
NPARAM = H * 3 + H + H * H + H + H + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    o = 0
    W1 = theta[o:o + 3 * H].reshape(H, 3); o += 3 * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]]).astype(np.float64)


def init_params(seed):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    def glorot(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))
    return pack(glorot(H, 3), np.zeros(H), glorot(H, H), np.zeros(H), glorot(1, H)[0], 0.0)


def forward(theta, Xs):
    """Standardised inputs (n, 3) -> standardised outputs (n,), and the activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    a1 = np.tanh(Xs @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    return a2 @ W3 + b3, (a1, a2)


def loss_grad(theta, Xs, ys):
    """MSE on standardised data and its gradient by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    n = Xs.shape[0]
    out, (a1, a2) = forward(theta, Xs)
    r = out - ys
    loss = np.mean(r * r)
    d = 2.0 * r / n                       # dL/dout
    gW3 = a2.T @ d
    gb3 = d.sum()
    d2 = np.outer(d, W3) * (1.0 - a2 * a2)  # dL/dz2
    gW2 = d2.T @ a1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - a1 * a1)      # dL/dz1
    gW1 = d1.T @ Xs
    gb1 = d1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, Xs, ys, iters, lr):
    m = np.zeros(NPARAM)
    v = np.zeros(NPARAM)
    loss = None
    for t in range(1, iters + 1):
        loss, g = loss_grad(theta, Xs, ys)
        theta, m, v = adam_step(theta, g, m, v, t, lr)
    return theta, loss
