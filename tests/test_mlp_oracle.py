"""Pins of the predictor network's FP64 oracle: the backward pass against
central finite differences (relative 1e-6), Adam against its closed form on
a quadratic, and training reducing the loss on a separable toy set."""
import numpy as np

from inputs.workloads import mlp_init_params
from oracle.mlp import n_params, forward, loss_and_grad, adam, train

F, H = 12, 32


def _data(N=200, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, F))
    y = (X[:, 0] + 0.5 * X[:, 3] > 0.3).astype(float) * rng.uniform(0.5, 1.0, N)
    return X, y


def test_layout_and_forward_range():
    p = mlp_init_params(F, H, 1).astype(np.float64)
    assert len(p) == n_params(F, H)
    s, _ = forward(p, _data()[0], F, H)
    assert np.all((s > 0) & (s < 1))


def test_gradient_matches_finite_differences():
    X, y = _data(64, 2)
    p = mlp_init_params(F, H, 3).astype(np.float64) * 2.0
    L, g = loss_and_grad(p, X, y, F, H)
    rng = np.random.default_rng(4)
    idx = rng.choice(len(p), 60, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (loss_and_grad(pp, X, y, F, H)[0] - loss_and_grad(pm, X, y, F, H)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-6), (i, fd, g[i])


def test_adam_closed_form_first_step():
    # first step: m_hat = g, v_hat = g^2 -> p - lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    X, y = _data(300, 5)
    p0 = mlp_init_params(F, H, 6).astype(np.float64)
    p, hist = train(p0, X, y, F, H, 300, 1e-2)
    assert hist[-1] < 0.5 * hist[0]
