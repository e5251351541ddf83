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
