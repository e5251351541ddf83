"""Pins of the oracle's surrogate network: gradients against central
differences, the structure (hidden-unit permutation symmetry), the
initialisation statistics, Adam's first-step closed form, and that training
fits a smooth target."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def P0(oracle):
    return oracle.mlp_init(11)


def test_parameter_count(oracle):
    assert oracle.mlp_n_params() == 16 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 8 + 8 == 137992


def test_init_is_he_normal_fp32(oracle, P0):
    for l, (ws, shape, bs) in enumerate(oracle.mlp_slices()):
        W = P0[ws]
        fan_in = shape[1]
        assert np.all(P0[bs] == 0.0)
        assert np.all(W.astype(np.float32).astype(np.float64) == W)
        sd = math.sqrt(2.0 / fan_in)
        n = W.size
        assert abs(W.mean()) < 5 * sd / math.sqrt(n)
        assert abs(W.std() / sd - 1.0) < 5 / math.sqrt(2 * n)
    # a different seed gives different weights
    assert not np.array_equal(oracle.mlp_init(12)[:100], P0[:100])


def test_gradient_matches_central_differences(oracle, P0):
    rng = np.random.default_rng(0)
    P = P0 + rng.normal(size=P0.size) * 0.01     # nonzero biases too
    x = rng.normal(size=(5, 16))
    t = rng.normal(size=(5, 8))
    loss, g = oracle.mlp_loss_grad(P, x, t)
    idx = []
    for ws, shape, bs in oracle.mlp_slices():
        idx += list(rng.integers(ws.start, ws.stop, 6)) + list(rng.integers(bs.start, bs.stop, 3))
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.mlp_loss_grad(Pp, x, t, False)[0] - oracle.mlp_loss_grad(Pm, x, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_hidden_unit_permutation_symmetry(oracle, P0):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 16))
    y0 = oracle.mlp_forward(P0, x)
    P = P0.copy()
    (w1, s1, b1), (w2, s2, b2) = oracle.mlp_slices()[:2]
    perm = rng.permutation(256)
    W1 = P[w1].reshape(s1)[perm]
    B1 = P[b1][perm]
    W2 = P[w2].reshape(s2)[:, perm]
    P[w1], P[b1], P[w2] = W1.ravel(), B1, W2.ravel()
    assert np.allclose(oracle.mlp_forward(P, x), y0, rtol=1e-12, atol=1e-12)


def test_bf16_forward_is_close_to_fp64(oracle, P0):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(64, 16))
    y = oracle.mlp_forward(P0, x)
    yb = oracle.mlp_forward(P0, x, bf16=True)
    assert np.max(np.abs(yb - y)) <= 0.03 * np.max(np.abs(y))
    assert not np.array_equal(yb, y)


def test_adam_first_step_closed_form(oracle):
    # with zero moments the bias-corrected first step is -lr g / (|g| + eps)
    rng = np.random.default_rng(3)
    g = rng.normal(size=1000)
    P = np.zeros(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    oracle.adam_step(P, g, m, v, 1, lr=1e-3, eps=1e-8)
    assert np.allclose(P, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_training_fits_a_smooth_target(oracle, P0):
    rng = np.random.default_rng(4)
    A = rng.normal(size=(16, 8)) * 0.3
    x = rng.normal(size=(128, 16))
    t = np.sin(x @ A)
    P = P0.copy()
    m, v = np.zeros_like(P), np.zeros_like(P)
    l0 = oracle.mlp_loss_grad(P, x, t, False)[0]
    for k in range(1, 61):
        _, g = oracle.mlp_loss_grad(P, x, t)
        oracle.adam_step(P, g, m, v, k, lr=3e-3)
    l1 = oracle.mlp_loss_grad(P, x, t, False)[0]
    assert l1 < 0.1 * l0
