"""Pins of the oracle's sampler (Alg. 1 sampling step; Gaussian phi of Sec. IV-A).

Each check compares the oracle with something other than itself: published
Philox known answers, the FP64 libm, closed-form moments of N(0, 1), the
Kolmogorov-Smirnov distribution, and sample covariances.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox_raw(ctr, key)
        assert [int(x) for x in got] == want


def test_philox_counter_layout(oracle):
    # seed -> key (lo, hi); counter word 0 carries the stream tag in its top byte
    seed = 0x0123456789ABCDEF
    a = oracle.philox(seed, 1, 5, 7, 9, 11)
    b = oracle.philox_raw([(1 << 24) | 5, 7, 9, 11], [0x89ABCDEF, 0x01234567])
    assert np.array_equal(a, b)


def test_u01_exact_grid(oracle):
    x = np.array([0, 1 << 9, 0xFFFFFFFF, 0x80000000, 12345 << 9], np.uint32)
    u = oracle.u01(x)
    want = [(2 * (int(v) >> 9) + 1) / 2.0 ** 24 for v in x]
    assert [float(t) for t in u] == want
    assert u.min() > 0.0 and u.max() < 1.0


def test_u01_uniform_ks(oracle):
    w = np.stack([oracle.philox(7, 0, 0, i, 0, 0) for i in range(20000)]).ravel()
    u = oracle.u01(w).astype(np.float64)
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_logf_error_bound(oracle):
    # <= 2 ulp against the FP64 natural log over (0, 1) and a wide range
    u = oracle.u01(np.arange(0, 2 ** 32, 4099, dtype=np.uint64).astype(np.uint32))
    extra = np.array([1e-30, 1e-20, 3e-8, 0.5, 0.70710677, 0.7071068, 1.0 - 2 ** -24, 2.0, 1e10], np.float32)
    u = np.concatenate([u, extra])
    got = oracle.logf(u).astype(np.float64)
    ex = np.log(u.astype(np.float64))
    ulp = np.spacing(np.maximum(np.abs(ex), 1e-38).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ex) / ulp) <= 2.0


def test_sincos2pi_error_bound(oracle):
    u = oracle.u01(np.arange(0, 2 ** 32, 4099, dtype=np.uint64).astype(np.uint32))
    s, c = oracle.sincos2pi(u)
    ang = 2 * np.pi * u.astype(np.float64)
    assert np.max(np.abs(s - np.sin(ang))) <= 2.0 ** -23
    assert np.max(np.abs(c - np.cos(ang))) <= 2.0 ** -23
    # quadrant boundaries are exact
    s, c = oracle.sincos2pi(np.array([0.25, 0.5, 0.75], np.float32))
    assert list(s) == [1.0, 0.0, -1.0] and list(c) == [0.0, -1.0, 0.0]


def test_normals_moments_and_ks(oracle):
    eps = oracle.normals(3, 0, 0, 1 << 16, 16).astype(np.float64).ravel()  # 2^20 normals
    n = eps.size
    assert abs(eps.mean()) < 4 / math.sqrt(n)
    assert abs(eps.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    assert abs(stats.skew(eps)) < 4 * math.sqrt(6.0 / n)
    assert abs(stats.kurtosis(eps, fisher=False) - 3.0) < 4 * math.sqrt(24.0 / n)
    assert stats.kstest(eps, "norm").pvalue > 1e-3


def test_normals_independent_dims(oracle):
    eps = oracle.normals(5, 2, 1, 1 << 15, 8).astype(np.float64)
    C = np.corrcoef(eps.T)
    off = C[~np.eye(8, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / math.sqrt(eps.shape[0])


def test_sample_covariance(oracle):
    D = 4
    A = np.array([[2.0, 0.3, 0.0, 0.1], [0.3, 1.0, -0.2, 0.0], [0.0, -0.2, 0.5, 0.05], [0.1, 0.0, 0.05, 0.25]])
    L = np.linalg.cholesky(A)
    mu = np.array([1.0, -2.0, 0.5, 3.0])
    n = 1 << 17
    Z = oracle.sample(11, 4, 0, n, mu, L).astype(np.float64)
    assert np.all(np.abs(Z.mean(0) - mu) < 5 * np.sqrt(np.diag(A) / n))
    S = np.cov(Z.T, bias=True)
    se = np.sqrt((A ** 2 + np.outer(np.diag(A), np.diag(A))) / n)
    assert np.all(np.abs(S - A) < 5 * se)


def test_sample_diag_is_mu_plus_sigma_eps(oracle):
    # with a diagonal factor z_d = fl32(mu_d + sigma_d eps_d) exactly
    mu = np.array([0.0, 0.0, 0.5])
    sig = np.sqrt(np.array([0.5, 0.5, 0.5]))
    Z = oracle.sample(0, 3, 0, 64, mu, np.diag(sig))
    eps = oracle.normals(0, 3, 0, 64, 3)
    want = (mu[None, :] + sig[None, :] * eps.astype(np.float64)).astype(np.float32)
    assert np.array_equal(Z, want)


def test_samples_differ_across_counters(oracle):
    a = oracle.normals(0, 0, 0, 64, 3)
    b = oracle.normals(0, 1, 0, 64, 3)
    c = oracle.normals(0, 0, 1, 64, 3)
    d = oracle.normals(1, 0, 0, 64, 3)
    for o in (b, c, d):
        assert not np.any(a == o)
