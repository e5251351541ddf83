"""Pins of the oracle's domain randomisation (Sec. IV-C: plans made robust to
bounded uncertainty in friction or mass).

  - scenario draws: inside their ranges and uniform (Kolmogorov-Smirnov at the
    1 % level), fixed per (seed, instance), independent of the instance's own
    draws;
  - plumbing: a scenario whose range is a single value rolls out exactly as a
    scene that carries that friction / mass;
  - reduction: a row's outcome under R scenarios is the worst of the R
    single-scenario tiers, the mean (or the maximum) of their costs and
    scenario 0's pose, each scenario rolled out on its own as a plain scene.
"""
import copy
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads


def _dr(w, R, reduce="mean", mu=(0.3, 0.7), mass=(0.15, 0.35)):
    w = copy.deepcopy(w)
    w["scene"]["domain_randomization"] = {"scenarios": R, "reduce": reduce, "mu": list(mu), "mass": list(mass)}
    return w


def _plain(w, mu, mass):
    """The scene with one friction value for every object contact and the given mass."""
    w = copy.deepcopy(w)
    w["scene"].pop("domain_randomization", None)
    w["scene"]["object"]["mu"] = [mu, mu]
    w["scene"]["object"]["mass"] = mass
    return w


def test_scenario_draws(oracle):
    w = _dr(workloads.load("movepush"), 64)
    mu, mass = oracle.scenarios(w, 3, inst=1)
    assert np.all((mu >= 0.3) & (mu <= 0.7)) and np.all((mass >= 0.15) & (mass <= 0.35))
    us = np.concatenate([(oracle.scenarios(w, s, inst=1)[0] - 0.3) / 0.4 for s in range(40)])
    um = np.concatenate([(oracle.scenarios(w, s, inst=1)[1] - 0.15) / 0.2 for s in range(40)])
    for u in (us, um):
        v = np.sort(u)
        n = v.size
        ks = max(np.max(np.arange(1, n + 1) / n - v), np.max(v - np.arange(n) / n))
        assert ks < 1.63 / math.sqrt(n)
    assert abs(np.corrcoef(us, um)[0, 1]) < 4 / math.sqrt(us.size)
    mu2, _ = oracle.scenarios(w, 3, inst=1)
    assert np.array_equal(mu, mu2)
    assert not np.array_equal(mu, oracle.scenarios(w, 3, inst=2)[0])
    # the instance's own draw (word 2 of block 0) is not a scenario's
    assert oracle.draw_instance(w, 3, inst=1)[2] not in set(mu)


def _rows(oracle, w, seed, n):
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(cem["cov0_diag"]))
    return oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)


def test_single_value_scenario_is_the_plain_scene(oracle):
    base = copy.deepcopy(workloads.load("movepush"))
    base["scene"]["horizon"] = 600
    Z = _rows(oracle, base, 2, 8)
    a = oracle.rollout(_dr(base, 2, mu=(0.45, 0.45), mass=(0.25, 0.25)), 2, Z)
    b = oracle.rollout(_plain(base, 0.45, 0.25), 2, Z)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("reduce", ["mean", "max"])
def test_reduction_over_scenarios(oracle, reduce):
    base = copy.deepcopy(workloads.load("movepush"))
    base["scene"]["horizon"] = 1500
    R, seed = 4, 5
    w = _dr(base, R, reduce)
    Z = _rows(oracle, base, seed, 12)
    cost, tier, pose, _, steps = oracle.rollout(w, seed, Z, with_steps=True)
    mu, mass = oracle.scenarios(w, seed)
    runs = [oracle.rollout(_plain(base, mu[r], mass[r]), seed, Z, with_steps=True) for r in range(R)]
    C = np.stack([r_[0] for r_ in runs])
    T = np.stack([r_[1] for r_ in runs])
    want = C.mean(0) if reduce == "mean" else C.max(0)
    assert np.allclose(cost, want, rtol=1e-12, atol=0)
    assert np.array_equal(tier, T.max(0))
    assert np.array_equal(pose, runs[0][2])
    assert np.array_equal(steps, np.stack([r_[4] for r_ in runs]).sum(0))
    # the scenarios matter on these rows
    assert np.any(C.min(0) != C.max(0)) or np.any(T.min(0) != T.max(0))

