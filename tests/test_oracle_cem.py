"""Pins of the oracle's CE select and refit (Sec. III-B, Alg. 1).

Hand-built populations whose elite sets are obvious, the textbook mean and
covariance (numpy), the library Cholesky, the closed-form variance contraction
of one CE step on a 1-D quadratic, and brute-force convergence to its argmin.
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2512_11571_amd import workloads

SEL_TOP, SEL_ALL_FEAS, SEL_ONE, SEL_TIER1, SEL_NONE = range(5)


def test_cholesky_matches_library(oracle):
    rng = np.random.default_rng(1)
    for D in (1, 3, 12, 16):
        B = rng.normal(size=(D, D))
        A = B @ B.T + D * np.eye(D)
        L, rc = oracle.cholesky(A)
        assert rc == 0
        assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-13, atol=1e-13)
        assert np.all(np.triu(L, 1) == 0)


def test_cholesky_rejects_indefinite(oracle):
    L, rc = oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert rc == 1


def test_factor_cov_degenerate_uses_jitter(oracle):
    # identical elites give S = 0: the floor jitter keeps the factor defined
    L, rc = oracle.factor_cov(np.zeros((3, 3)))
    assert rc == 0 and np.allclose(np.diag(L), math.sqrt(1e-12))
    # a rank-deficient S gets a tiny relative jitter and still factors
    v = np.array([1.0, 2.0, 3.0])
    L, rc = oracle.factor_cov(np.outer(v, v))
    assert rc == 0 and np.allclose(L @ L.T, np.outer(v, v), atol=1e-6)


def test_select_hand_cases(oracle):
    nan = float("nan")
    cost = np.array([5.0, 3.0, nan, 3.0, 1.0, 0.5, 2.0], np.float32)
    tier = np.array([0, 0, 0, 0, 0, 1, 2], np.uint8)
    # feasible = tier 0 and not NaN: idx 4 (1.0), 1 (3.0), 3 (3.0, tie -> higher index later), 0 (5.0)
    idx, mode, counts = oracle.select(cost, tier, 3)
    assert list(idx) == [4, 1, 3] and mode == SEL_TOP
    assert list(counts) == [4, 1, 1, 1]
    idx, mode, _ = oracle.select(cost, tier, 10)
    assert list(idx) == [4, 1, 3, 0] and mode == SEL_ALL_FEAS
    # exactly one feasible
    idx, mode, _ = oracle.select(np.array([2.0, 1.0, 0.5], np.float32), np.array([1, 0, 2], np.uint8), 2)
    assert list(idx) == [1] and mode == SEL_ONE
    # none feasible: all-actions-succeeded plans (tier 1) are used
    idx, mode, _ = oracle.select(np.array([2.0, 1.0, 0.5, 4.0], np.float32), np.array([1, 1, 2, 1], np.uint8), 2)
    assert list(idx) == [1, 0] and mode == SEL_TIER1
    idx, mode, _ = oracle.select(np.array([2.0, 1.0], np.float32), np.array([2, 3], np.uint8), 2)
    assert len(idx) == 0 and mode == SEL_NONE


def test_select_ties_broken_by_index(oracle):
    cost = np.full(64, 1.5, np.float32)
    tier = np.zeros(64, np.uint8)
    idx, _, _ = oracle.select(cost, tier, 8)
    assert list(idx) == list(range(8))
    cost[[40, 7, 63]] = 1.0
    idx, _, _ = oracle.select(cost, tier, 5)
    assert list(idx) == [7, 40, 63, 0, 1]


def test_refit_is_textbook_mle(oracle):
    rng = np.random.default_rng(2)
    Z = rng.normal(size=(100, 5)).astype(np.float32)
    elite = np.array([3, 17, 42, 8, 99, 0, 55], np.int32)
    cov0 = np.eye(5)
    mu, S, L, rc = oracle.refit(Z, elite, SEL_TOP, 1, cov0, np.zeros(5), np.eye(5))
    E = Z[elite].astype(np.float64)
    assert np.allclose(mu, E.mean(0), rtol=1e-14, atol=1e-15)
    assert np.allclose(S, np.cov(E.T, bias=True), rtol=1e-12, atol=1e-15)
    assert np.allclose(L @ L.T, S, atol=1e-9)
    # diagonal mode keeps only the variances
    mu, S, L, rc = oracle.refit(Z, elite, SEL_TOP, 0, cov0, np.zeros(5), np.eye(5))
    assert np.allclose(S, np.diag(E.var(0)), rtol=1e-12, atol=1e-15)
    # a single elite: mean = that row, covariance = (0.1 sigma0)^2
    cov0 = np.diag([0.5, 2.0, 1.0, 1.0, 4.0])
    mu, S, L, rc = oracle.refit(Z, elite[:1], SEL_ONE, 0, cov0, np.zeros(5), np.eye(5))
    assert np.array_equal(mu, Z[3].astype(np.float64))
    assert np.allclose(np.diag(S), 0.01 * np.diag(cov0))
    # nothing selected: theta unchanged
    mu, S, L, rc = oracle.refit(Z, elite[:0], SEL_NONE, 0, cov0, np.ones(5), 2 * np.eye(5))
    assert np.array_equal(mu, np.ones(5)) and np.array_equal(S, 2 * np.eye(5))


def _ce_step_1d(oracle, seed, it, a, mu, sig, N, Ne):
    Z = oracle.sample(seed, it, 0, N, np.array([mu]), np.array([[sig]]))
    cost = ((Z[:, 0].astype(np.float64) - a) ** 2).astype(np.float32)
    idx, mode, _ = oracle.select(cost, np.zeros(N, np.uint8), Ne)
    mu1, S1, L1, _ = oracle.refit(Z, idx, mode, 0, np.array([[sig * sig]]), np.array([mu]), np.array([[sig * sig]]))
    return mu1[0], S1[0, 0]


@pytest.mark.parametrize("frac", [8 / 64, 64 / 1024])
def test_one_ce_step_variance_contraction_closed_form(oracle, frac):
    # cost (z - a)^2 centred at the mean: the elites are the central fraction p
    # of N(a, s^2); their variance ratio is that of a normal truncated to |x| < c,
    # c = Phi^-1(1/2 + p/2): 1 - 2 c phi(c) / (2 Phi(c) - 1).
    N = 1 << 20
    Ne = int(N * frac)
    a, sig = 0.7, 0.3
    c = stats.norm.ppf(0.5 + frac / 2)
    ratio = 1 - 2 * c * stats.norm.pdf(c) / (2 * stats.norm.cdf(c) - 1)
    mu1, var1 = _ce_step_1d(oracle, 5, 0, a, a, sig, N, Ne)
    # a uniform-like elite distribution: var of the sample variance ~ (9/5 - 1) v^2 / Ne
    se = ratio * math.sqrt(0.8 / Ne)
    assert abs(var1 / sig ** 2 - ratio) < 4 * se
    assert abs(mu1 - a) < 4 * sig * math.sqrt(ratio / Ne)


def test_ce_converges_to_brute_force_argmin(oracle):
    # 1-D quadratic from mu0 = a + 3 sigma0; the grid argmin is a
    a = -0.4137
    grid = np.linspace(-5, 5, 100001)
    a_grid = grid[np.argmin((grid - a) ** 2)]
    mu, sig = a + 3.0, 1.0
    for it in range(12):
        mu, var = _ce_step_1d(oracle, 9, it, a, mu, sig, 1024, 64)
        sig = math.sqrt(var)
    assert abs(mu - a_grid) < 1e-3


def test_plan_solve_push_improves_and_accounts(oracle):
    w = workloads.load("push")
    r = oracle.plan_solve(w, 0)
    st = r["stats"]
    pop = w["cem"]["pop"]
    assert np.all(st[:, 1:5].sum(1) == pop)
    assert np.all(np.diff(st[:, 7]) <= 0)                  # best-ever is monotone
    assert st[-1, 7] == r["best_cost"] and r["best_tier"] == 0
    assert r["best_cost"] < 0.5 * st[0, 0]                 # CE improves on iteration 0
    # the best row reproduces its cost when rolled out alone
    c, t, _, _ = oracle.rollout(w, 0, r["best_z"][None, :])
    assert abs(c[0] - r["best_cost"]) < 1e-12
