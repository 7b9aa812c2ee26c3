"""FP64 reference of the learned plan chooser's perceptron -- TEST
INFRASTRUCTURE ONLY (see the package header).

The network is y = W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 with
in_dim -> hidden -> hidden -> 1, trained on the mean squared error
(1/B) sum_i (y_i - t_i)^2.  The paper has no learned component: this module
follows the textbook definitions.  The gradient is the chain rule written out
layer by layer; the optimizer is Adam as published by Kingma and Ba (2015,
Algorithm 1: exponential moving averages of the gradient and its square,
bias-corrected, step lr * m_hat / (sqrt(v_hat) + eps)).

Parameter vector order (shared with the library's ABI, not its code):
W1 (in_dim x hidden, row-major), b1, W2 (hidden x hidden), b2, W3 (hidden),
b3.  relu'(z) is taken as 0 at z = 0.

Pinned by tests/test_oracle_mlp.py: a hand-worked forward pass, central
finite differences of the loss, the linear regime's closed form, and the
closed form of Adam's first steps.
"""

from __future__ import annotations

import numpy as np


def param_count(d: int, h: int) -> int:
    return d * h + h + h * h + h + h + 1


def unpack(p: np.ndarray, d: int, h: int):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == param_count(d, h)
    o = 0
    w1 = p[o:o + d * h].reshape(d, h); o += d * h
    b1 = p[o:o + h]; o += h
    w2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    w3 = p[o:o + h]; o += h
    b3 = p[o]
    return w1, b1, w2, b2, w3, b3


def pack(w1, b1, w2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(w1), np.ravel(b1), np.ravel(w2), np.ravel(b2), np.ravel(w3),
                           np.atleast_1d(b3)]).astype(np.float64)


def forward(p, x, d: int, h: int):
    """Returns (y, cache) for inputs x of shape (B, d)."""
    w1, b1, w2, b2, w3, b3 = unpack(p, d, h)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ w1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, d: int, h: int) -> float:
    y, _ = forward(p, x, d, h)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2))


def gradient(p, x, t, d: int, h: int):
    """(flat gradient in parameter order, loss)."""
    w1, b1, w2, b2, w3, b3 = unpack(p, d, h)
    y, (x, z1, h1, z2, h2) = forward(p, x, d, h)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    dy = 2.0 * (y - t) / B                 # dL/dy
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    dh2 = np.outer(dy, w3)                 # dL/dh2
    dz2 = dh2 * (z2 > 0.0)
    g_w2 = h1.T @ dz2
    g_b2 = dz2.sum(axis=0)
    dh1 = dz2 @ w2.T
    dz1 = dh1 * (z1 > 0.0)
    g_w1 = x.T @ dz1
    g_b1 = dz1.sum(axis=0)
    return pack(g_w1, g_b1, g_w2, g_b2, g_w3, g_b3), float(np.mean((y - t) ** 2))


def adam_step(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update at 1-based step `step`; returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def init_params(rng: np.random.Generator, d: int, h: int) -> np.ndarray:
    """He-normal weights and zero biases."""
    w1 = rng.normal(0.0, np.sqrt(2.0 / d), size=(d, h))
    w2 = rng.normal(0.0, np.sqrt(2.0 / h), size=(h, h))
    w3 = rng.normal(0.0, np.sqrt(1.0 / h), size=h)
    return pack(w1, np.zeros(h), w2, np.zeros(h), w3, 0.0)
