"""Pins of the warm-start network's FP64 reference: gradient against central
differences, Adam's first step against its closed form, the loss of a zero
network, and a forward pass evaluated by hand."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K


@pytest.mark.parametrize("H,depth", [(32, 1), (32, 3), (64, 2)])
def test_gradient_matches_central_differences(H, depth):
    rng = np.random.default_rng(H + depth)
    p = K.net_init_params(H, depth, seed=7)
    p += 0.05 * rng.normal(size=p.size)          # nonzero biases too
    x = rng.normal(size=(6, 5))
    t = rng.normal(size=(6, 3))
    loss, g = O.mlp_gradient(p, H, depth, x, t)
    y = O.mlp_forward(p, H, depth, x)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-14 * max(1.0, loss)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        fd = (np.mean((O.mlp_forward(pp, H, depth, x) - t) ** 2) -
              np.mean((O.mlp_forward(pm, H, depth, x) - t) ** 2)) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k]))


def test_zero_network_predicts_zero():
    p = np.zeros(O.mlp_num_params(32, 2))
    x = np.ones((4, 5))
    t = np.arange(12.0).reshape(4, 3)
    loss, g = O.mlp_gradient(p, 32, 2, x, t)
    assert np.all(O.mlp_forward(p, 32, 2, x) == 0.0)
    assert abs(loss - np.mean(t ** 2)) < 1e-14


def test_forward_by_hand_one_hidden_layer():
    """depth 1, H = 32 with one active hidden unit: y_j = W1[j,0] s(W0[0].x + b0[0]) + b1[j]."""
    H = 32
    n = O.mlp_num_params(H, 1)
    p = np.zeros(n)
    W0 = p[:5 * H].reshape(H, 5)
    W0[0] = [0.5, -1.0, 0.25, 2.0, 0.0]
    p[5 * H] = 0.1                                  # b0[0]
    off1 = 5 * H + H
    W1 = p[off1:off1 + 3 * H].reshape(3, H)
    W1[:, 0] = [1.0, -2.0, 0.5]
    p[off1 + 3 * H:] = [0.3, 0.0, -0.1]
    x = np.array([[1.0, 0.5, 2.0, -0.25, 7.0]])
    z = 0.5 * 1.0 - 1.0 * 0.5 + 0.25 * 2.0 + 2.0 * -0.25 + 0.1
    s = z / (1 + math.exp(-z))
    exp = np.array([s + 0.3, -2 * s, 0.5 * s - 0.1])
    assert np.abs(O.mlp_forward(p, H, 1, x)[0] - exp).max() < 1e-15


def test_adam_first_step_closed_form():
    """After one step with zero moments: p -= lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = O.mlp_adam(p0, g, np.zeros(50), np.zeros(50), 1e-2, 1)
    assert np.abs(p1 - (p0 - 1e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    assert np.abs(m - 0.1 * g).max() < 1e-16 and np.abs(v - 0.001 * g * g).max() < 1e-16
