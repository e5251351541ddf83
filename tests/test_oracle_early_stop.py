"""Pins of the oracle's early stop of robot rollouts (scene settle_steps > 0).

The stop does not alter the dynamics before it, so a full-horizon run of the
same rows fixes what an early-stopped one must report:
  - the cost is identical (it stops growing once the last action has ended,
    and the stop waits for that; a stop while an action still runs, such as
    the object resting on its shelf during the first move, would cut it short);
  - the pose returned is the full run's pose at the stop step;
  - the object's speed is below the rest threshold on each of the last
    settle_steps steps before the stop;
  - a run without the option simulates T steps.
"""
import copy

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

SETTLE = 100


def _rows(oracle, w, seed, n):
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(cem["cov0_diag"]))
    return oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)


@pytest.mark.parametrize("name,n", [("movepush", 24), ("pickplace", 12)])
def test_early_stop_against_the_full_horizon_run(oracle, name, n):
    w = workloads.load(name)
    H = w["scene"]["horizon"]
    Z = _rows(oracle, w, 1, n)
    c0, t0, p0, tr, s0 = oracle.rollout(w, 1, Z, trace_steps=H, with_steps=True)
    assert np.all(s0 == H)
    we = copy.deepcopy(w)
    we["scene"]["settle_steps"] = SETTLE
    c1, t1, p1, _, s1 = oracle.rollout(we, 1, Z, with_steps=True)
    assert np.array_equal(c1, c0)
    assert np.all((s1 >= SETTLE) & (s1 <= H))
    stopped = np.where(s1 < H)[0]
    assert stopped.size >= n // 2 if name == "movepush" else stopped.size >= 1
    rest = w["scene"]["rest_speed"]
    for i in stopped:
        k = s1[i]
        assert np.array_equal(p1[i], tr[i, k - 1, :7])
        speed = np.linalg.norm(tr[i, k - SETTLE:k, 7:10], axis=1)
        assert np.all(speed < rest), (i, k)
    # psi_g read at the stop agrees with the full horizon on these rows
    assert np.mean(t1 == t0) >= 0.9


# ---- stop on a failed action (scene fail_stop = 1) ----
# Once an action has timed out without success the plan can no longer be
# feasible (Problem 2 needs every action to succeed), and Alg. 1 evaluates only
# the costs of successful plans.  The full-horizon run's action log fixes what
# the stopped run must report: unchanged outcome for plans whose every action
# that ended succeeded; otherwise tier 2, the steps up to the first failure,
# and the cost of those steps.

def _first_failure(log, n_act):
    for a in range(n_act):
        if log["ends"][a] >= 0 and not (log["ok"] >> a) & 1:
            return int(log["ends"][a])
    return None


@pytest.mark.parametrize("name,n", [("pickplace", 24), ("movepush", 16)])
def test_fail_stop_against_the_full_horizon_log(oracle, name, n):
    w = workloads.load(name)
    H, dt = w["scene"]["horizon"], w["scene"]["dt"]
    n_act = 4 if name == "pickplace" else 2
    Z = _rows(oracle, w, 4, n)
    c0, t0, p0, tr, s0 = oracle.rollout(w, 4, Z, trace_steps=H, with_steps=True)
    wf = copy.deepcopy(w)
    wf["scene"]["fail_stop"] = 1
    c1, t1, p1, _, s1 = oracle.rollout(wf, 4, Z, with_steps=True)
    stopped = 0
    for i in range(n):
        tf = _first_failure(oracle.robot_log(w, 4, Z[i]), n_act)
        if tf is None:
            # nothing failed: the same rollout, to the bit
            assert (c1[i], t1[i], s1[i]) == (c0[i], t0[i], s0[i]) and np.array_equal(p1[i], p0[i])
        else:
            stopped += 1
            assert t0[i] >= 2 and t1[i] == 2
            assert s1[i] == tf and abs(c1[i] - dt * tf) < 1e-12
            assert np.array_equal(p1[i], tr[i, tf - 1, :7] if tf > 0 else p1[i])
    assert stopped >= 2 and stopped < n


@pytest.mark.parametrize("name,pop,ne,iters", [("pickplace", 96, 8, 3), ("movepush", 64, 8, 2)])
def test_fail_stop_leaves_the_ce_run_unchanged(oracle, name, pop, ne, iters):
    # the update reads only tier 0 and tier 1 samples, which the stop never touches
    w = workloads.load(name)
    w["cem"].update(pop=pop, n_elite=ne)
    wf = copy.deepcopy(w)
    wf["scene"]["fail_stop"] = 1
    for seed in (0, 1):
        a = oracle.plan_solve(w, seed, iters=iters)
        b = oracle.plan_solve(wf, seed, iters=iters)
        assert np.array_equal(a["mu"], b["mu"]) and np.array_equal(a["S"], b["S"])
        sa, sb = a["stats"], b["stats"]
        assert np.array_equal(sa[:, [1, 2, 5, 6]], sb[:, [1, 2, 5, 6]])        # tiers 0, 1; n_e; mode
        assert np.array_equal(sa[:, 3] + sa[:, 4], sb[:, 3] + sb[:, 4])       # tiers 2 + 3
        if a["best_tier"] <= 1:
            assert (a["best_cost"], a["best_tier"]) == (b["best_cost"], b["best_tier"])
            assert np.array_equal(a["best_z"], b["best_z"])
