"""Pins of the perceptron oracle (oracle/mlp.py) against values fixed by the
mathematics: a forward and backward pass worked by hand, central finite
differences of the loss, the closed form of the network where every ReLU is
active, and the closed form of Adam's first two steps under a constant
gradient (bias correction makes both steps -lr * g / (|g| + eps))."""

import numpy as np
import pytest

from oracle import mlp as M


def hand_params():
    # in_dim 2, hidden 2
    w1 = np.array([[1.0, -1.0], [2.0, 1.0]])
    b1 = np.array([0.0, 0.5])
    w2 = np.array([[1.0, 0.0], [-4.0, 1.0]])
    b2 = np.array([0.0, -1.0])
    w3 = np.array([2.0, 7.0])
    b3 = 0.25
    return M.pack(w1, b1, w2, b2, w3, b3)


def test_forward_by_hand():
    # z1 = [1+2, -1+1] + [0, .5] = [3, .5]; z2 = [3 - 2, .5] + [0, -1] = [1, -.5]
    # h2 = [1, 0]; y = 2 * 1 + 7 * 0 + .25
    y, (x, z1, h1, z2, h2) = M.forward(hand_params(), [[1.0, 1.0]], 2, 2)
    assert np.allclose(z1, [[3.0, 0.5]])
    assert np.allclose(z2, [[1.0, -0.5]])
    assert np.allclose(h2, [[1.0, 0.0]])
    assert y.tolist() == [2.25]


def test_gradient_by_hand():
    # t = .25: loss (2.25 - .25)^2 = 4, dy = 2 * 2 = 4
    g, loss = M.gradient(hand_params(), [[1.0, 1.0]], [0.25], 2, 2)
    assert loss == 4.0
    w1, b1, w2, b2, w3, b3 = M.unpack(g, 2, 2)
    assert w3.tolist() == [4.0, 0.0] and b3 == 4.0
    # dh2 = 4 * [2, 7], masked by z2 > 0 -> dz2 = [8, 0]
    assert w2.tolist() == [[24.0, 0.0], [4.0, 0.0]] and b2.tolist() == [8.0, 0.0]
    # dh1 = dz2 W2^T = [8, -32]; both z1 > 0
    assert w1.tolist() == [[8.0, -32.0], [8.0, -32.0]] and b1.tolist() == [8.0, -32.0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    d, h, b = 5, 7, 6
    p = M.init_params(rng, d, h) + rng.normal(0, 0.1, M.param_count(d, h))
    x = rng.normal(size=(b, d))
    t = rng.normal(size=b)
    g, _ = M.gradient(p, x, t, d, h)
    eps = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        num[i] = (M.loss(p + e, x, t, d, h) - M.loss(p - e, x, t, d, h)) / (2 * eps)
    # no pre-activation sits within eps of a ReLU kink at these draws
    _, (_, z1, _, z2, _) = M.forward(p, x, d, h)
    assert min(np.abs(z1).min(), np.abs(z2).min()) > 1e-4
    assert np.max(np.abs(g - num)) <= 1e-6 * max(1.0, np.max(np.abs(num)))


def test_linear_regime_closed_form():
    rng = np.random.default_rng(4)
    d, h = 4, 3
    w1 = rng.uniform(0.1, 1.0, (d, h))
    w2 = rng.uniform(0.1, 1.0, (h, h))
    w3 = rng.normal(size=h)
    b1 = np.full(h, 10.0)
    b2 = np.full(h, 10.0)
    b3 = -0.5
    x = rng.uniform(0.0, 1.0, (5, d))
    y, _ = M.forward(M.pack(w1, b1, w2, b2, w3, b3), x, d, h)
    # every pre-activation is positive, so the network is affine
    want = x @ (w1 @ w2 @ w3) + (b1 @ w2 @ w3 + b2 @ w3 + b3)
    assert np.allclose(y, want, rtol=1e-12, atol=1e-12)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=9)
    g = rng.normal(size=9)
    lr, eps = 0.01, 1e-8
    m = np.zeros(9)
    v = np.zeros(9)
    p1, m, v = M.adam_step(p0, g, m, v, 1, lr)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    p2, m, v = M.adam_step(p1, g, m, v, 2, lr)
    assert np.allclose(p2, p0 - 2 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
