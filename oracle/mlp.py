"""FP64 reference of the learned constraint predictor's network (test
infrastructure only): a fully connected network

    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  s = sigmoid(w3 . h2 + b3)

on per-coordinate face features x (length F), trained by mean squared error
against the coordinate's participation in the eigenvectors selected by the
adaptive eigenproblems (Sec. 6), with Adam.  The flat parameter layout is
[W1 (H x F, row-major), b1 (H), W2 (H x H, row-major), b2 (H), w3 (H), b3 (1)].

Forward and backward are written out layer by layer; the backward pass is
pinned against central finite differences in the tests.
"""
import numpy as np


def n_params(F, H):
    return H * F + H + H * H + H + H + 1


def unpack(p, F, H):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]; o += 1
    return W1, b1, W2, b2, w3, b3


def forward(p, X, F, H):
    """X: N x F.  Returns s (N) and the cached activations."""
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    z1 = X @ W1.T + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = np.tanh(z2)
    z3 = h2 @ w3 + b3
    s = 1.0 / (1.0 + np.exp(-z3))
    return s, (X, h1, h2, s)


def loss_and_grad(p, X, y, F, H):
    """L = mean_i (s_i - y_i)^2 and dL/dp (flat, same layout)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    s, (X, h1, h2, s) = forward(p, X, F, H)
    N = X.shape[0]
    r = s - y
    L = float(np.mean(r * r))
    d3 = (2.0 / N) * r * s * (1.0 - s)            # dL/dz3
    g_w3 = h2.T @ d3
    g_b3 = d3.sum()
    d2 = np.outer(d3, w3) * (1.0 - h2 * h2)       # dL/dz2
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)              # dL/dz1
    g_W1 = d1.T @ X
    g_b1 = d1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return L, g


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns updated (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(p, X, y, F, H, epochs, lr):
    """Full-batch Adam; returns parameters and the loss history."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hist = []
    for t in range(1, epochs + 1):
        L, g = loss_and_grad(p, X, y, F, H)
        hist.append(L)
        p, m, v = adam(p, g, m, v, t, lr)
    return p, np.array(hist)
