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


def test_gelu_at_known_values_and_against_the_library(oracle):
    # tanh-form GELU: 0 at 0, x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))); its values at +-1 and 2 (the
    # closed form evaluated with Python's libm); x for large x, 0 for very negative x; the derivative 1/2 at 0
    y, dy = oracle.gelu([0.0, 1.0, -1.0, 2.0, 12.0, -12.0])
    assert y[0] == 0.0 and dy[0] == 0.5
    assert abs(y[1] - 0.8411919906082768) < 1e-15
    assert abs(y[2] + 0.15880800939172324) < 1e-15
    assert abs(y[3] - 1.954597694087775) < 1e-15
    assert y[4] == 12.0 and abs(y[5]) < 1e-30
    # against PyTorch's own tanh-form GELU and its autograd derivative, in float64
    torch = pytest.importorskip("torch")
    x = np.linspace(-6.0, 6.0, 241)
    t = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    g = torch.nn.functional.gelu(t, approximate="tanh")
    g.sum().backward()
    y, dy = oracle.gelu(x)
    assert np.max(np.abs(y - g.detach().numpy())) < 1e-15
    assert np.max(np.abs(dy - t.grad.numpy())) < 1e-14


def test_bf16_rounding_is_nearest_even(oracle):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    hi = rng.integers(0, 0x7F7F, 4000, dtype=np.uint32)         # finite bfloat16 patterns
    ties = ((hi << 16) | 0x8000).view(np.float32).astype(np.float64)   # exactly halfway to the next bfloat16
    up = ((hi << 16) | 0x8001).view(np.float32).astype(np.float64)
    down = ((hi << 16) | 0x7FFF).view(np.float32).astype(np.float64)
    got = oracle.to_bf16(ties)
    # ties go to the even bfloat16: up when the kept pattern is odd, down when even
    want = (((hi + (hi & 1)) << 16).astype(np.uint32)).view(np.float32).astype(np.float64)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.to_bf16(up), (((hi + 1) << 16).astype(np.uint32)).view(np.float32).astype(np.float64))
    assert np.array_equal(oracle.to_bf16(down), ((hi << 16).astype(np.uint32)).view(np.float32).astype(np.float64))
    # negative values, random values, the largest finite, infinities: as PyTorch's conversion
    x = np.concatenate([-ties, rng.normal(size=4000) * 10.0 ** rng.uniform(-30, 30, 4000),
                        [3.3895313892515355e38, 3.4e38, np.inf, -np.inf, 0.0, -0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.to_bf16(x), ref)


def test_adam_steps_two_and_three_match_the_library(oracle):
    # three steps with different gradients: moments carried across steps, bias corrections at t = 2, 3
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    P0 = rng.normal(size=500)
    gs = [rng.normal(size=500) * s for s in (1.0, 0.3, 2.0)]
    P, m, v = P0.copy(), np.zeros(500), np.zeros(500)
    p = torch.tensor(P0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t, g in enumerate(gs, 1):
        oracle.adam_step(P, g, m, v, t, lr=1e-3, eps=1e-8)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        assert np.allclose(P, p.detach().numpy(), rtol=1e-13, atol=1e-16), t


def test_bf16_backward_pins(oracle, P0):
    # the backward with BF16 operands: its loss is the BF16 forward's mean squared
    # error, its last bias gradient the unrounded dL/dy summed over rows (closed
    # forms from the forward alone), and every gradient within the BF16 bound of
    # the FP64 backward (itself pinned by central differences)
    rng = np.random.default_rng(12)
    P = P0 + rng.normal(size=P0.size) * 0.01
    x = rng.normal(size=(64, 16))
    t = rng.normal(size=(64, 8))
    lb, gb = oracle.mlp_loss_grad(P, x, t, bf16=True)
    l64, g64 = oracle.mlp_loss_grad(P, x, t)
    yb = oracle.mlp_forward(P, x, bf16=True)
    assert abs(lb - np.mean((yb - t) ** 2)) <= 1e-15 * lb
    b4 = oracle.mlp_slices()[3][2]
    assert np.allclose(gb[b4], 2.0 * np.sum(yb - t, axis=0) / t.size, rtol=1e-12, atol=1e-16)
    for ws, shape, bs in oracle.mlp_slices():
        for sl in (ws, bs):
            assert np.max(np.abs(gb[sl] - g64[sl])) <= 2e-2 * np.max(np.abs(g64[sl]))
    assert not np.array_equal(gb, g64)
