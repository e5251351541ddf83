"""Early stop of robot rollouts (scene settle_steps > 0) and the per-context
count of simulated control steps, on the GPU through the C ABI.

Bit-exact: without the option every rollout counts T steps (push,
pick-and-place, move-and-push, a ragged population).  Against the GPU's own
full-horizon run of the same rows: identical cost wherever both are finite (the
stop waits for the last action to end), psi_g agrees on nearly every row, and
fewer steps are simulated.  Against the FP64 oracle with the same option:
tier and cost on certified rows as for the full horizon, and the total of
simulated steps within 5 %.  With domain-randomisation scenarios the costs
still equal the full-horizon ones, and batched instances that stop early give
the bits and step counts of their single runs.  The cost-and-goal test also
runs at the lanes per plan the benchmarks use (8 for move-push, 16 for
pick-and-place).
"""
import copy

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SETTLE = 100


@pytest.fixture(scope="module")
def Context():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd.binding import Context
    return Context


def _rows(oracle, w, seed, n):
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(cem["cov0_diag"]))
    return oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)


def _early(w):
    we = copy.deepcopy(w)
    we["scene"]["settle_steps"] = SETTLE
    return we


def _gpu(Context, w, Z, seed, lanes=1):
    """cost, tier and the control steps the rollouts simulated."""
    n = Z.shape[0]
    with Context(w, seed=seed, pop=max(n, 64), n_elite=1, lanes=lanes) as c:
        assert c.env_steps() == 0
        Zd = torch.from_numpy(np.ascontiguousarray(Z)).to("cuda:0")
        cost = torch.empty(n, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        c.rollout_batch(Zd, cost, tier)
        torch.cuda.synchronize()
        return cost.cpu().numpy().astype(np.float64), tier.cpu().numpy(), c.env_steps()


@pytest.mark.parametrize("name", ["push", "pickplace", "movepush"])
def test_full_horizon_counts_T_steps_per_rollout(oracle, Context, name):
    w = copy.deepcopy(workloads.load(name))
    w["scene"]["horizon"] = min(w["scene"]["horizon"], 400)
    n = 100                                      # one full wave and a ragged one
    Z = _rows(oracle, w, 3, n)
    _, _, steps = _gpu(Context, w, Z, 3)
    assert steps == n * w["scene"]["horizon"]
    with Context(w, seed=3, pop=n, n_elite=8) as c:
        c.plan_solve(2)
        assert c.env_steps() == 2 * n * w["scene"]["horizon"]


@pytest.mark.parametrize("name,lanes", [("movepush", 1), ("pickplace", 1), ("movepush", 8), ("pickplace", 16)])
def test_early_stop_keeps_cost_and_goal(oracle, Context, name, lanes):
    w = workloads.load(name)
    H = w["scene"]["horizon"]
    n = 256
    Z = _rows(oracle, w, 1, n)
    cf, tf, sf = _gpu(Context, w, Z, 1, lanes)
    ce, te, se = _gpu(Context, _early(w), Z, 1, lanes)
    assert sf == n * H
    both = np.isfinite(cf) & np.isfinite(ce)
    assert both.mean() >= 0.99
    assert np.array_equal(cf[both], ce[both])
    assert np.mean(tf == te) >= 0.98
    assert n * SETTLE <= se < sf
    if name == "movepush":
        assert se < 0.5 * sf                     # most plans end well before T


def _certified(oracle, w, seed, Z):
    """Oracle outcome, steps, and the rows whose cost and tier a one-ulp nudge
    of every parameter either way does not change."""
    c0, t0, _, _, s0 = oracle.rollout(w, seed, Z, with_steps=True)
    up = np.nextafter(Z, np.float32(np.inf)).astype(np.float32)
    dn = np.nextafter(Z, np.float32(-np.inf)).astype(np.float32)
    c1, t1, _, _ = oracle.rollout(w, seed, up)
    c2, t2, _, _ = oracle.rollout(w, seed, dn)
    ok = (t0 == t1) & (t0 == t2) & (np.abs(c1 - c0) < 1e-9) & (np.abs(c2 - c0) < 1e-9)
    return ok, c0, t0, s0


def test_early_stop_parity_with_the_oracle(oracle, Context):
    w = _early(workloads.load("movepush"))
    seed = 1
    Z = _rows(oracle, w, seed, 128)
    ok, cr, tr, sr = _certified(oracle, w, seed, Z)
    assert ok.sum() >= 48
    cg, tg, sg = _gpu(Context, w, Z, seed)
    assert np.mean(tg[ok] == tr[ok]) >= 0.95
    same = ok & (tg == tr) & (tr < 3)
    assert np.max(np.abs(cg[same] - cr[same])) <= 2 * w["scene"]["dt"] + 1e-6
    assert abs(sg - int(sr.sum())) <= 0.05 * sr.sum()


def test_early_stop_with_scenarios_and_in_a_batch(oracle, Context):
    # early stop composes with domain randomisation (each scenario stops on its
    # own; the cost is still the full-horizon one) and with batching (a batched
    # instance that stops early gives the bits of its single run)
    from paper_2512_11571_amd import binding
    w = copy.deepcopy(workloads.load("movepush"))
    w["scene"]["horizon"] = 1500
    w["scene"]["domain_randomization"] = {"scenarios": 4, "mu": [0.3, 0.7], "mass": [0.2, 0.4]}
    Z = _rows(oracle, w, 2, 96)
    cf, tf, sf = _gpu(Context, w, Z, 2)
    ce, te, se = _gpu(Context, _early(w), Z, 2)
    both = np.isfinite(cf) & np.isfinite(ce)
    assert both.mean() >= 0.99 and np.array_equal(cf[both], ce[both])
    assert np.mean(tf == te) >= 0.95
    assert se < sf
    we = _early(w)
    we["cem"].update(pop=128, n_elite=8)
    pp = copy.deepcopy(workloads.load("pickplace"))
    pp["scene"]["horizon"] = 600
    pp["cem"].update(pop=100, n_elite=8)
    insts = [{"workload": we, "seed": 0, "instance": 0, "iters": 2},
             {"workload": _early(pp), "seed": 1, "instance": 1, "iters": 2}]
    with binding.Batch(insts) as bt:
        res = bt.solve(2)
        counted = [bt.instance(k).env_steps() for k in range(2)]
    for inst, r, n in zip(insts, res, counted):
        with Context(inst["workload"], seed=inst["seed"], instance=inst["instance"]) as c:
            s = c.plan_solve(inst["iters"])
            assert c.env_steps() == n
        assert r["best_cost"] == s["best_cost"] and np.array_equal(r["mu"], s["mu"])
