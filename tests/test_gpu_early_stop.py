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
from parity_util import certify, tier_mismatches

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
    """Oracle outcome, the certified rows (cost and tier), the rows whose tier is
    certified, and the steps each rollout simulated."""
    r = certify(oracle, w, seed, Z)
    return r["ok"], r["cost"], r["tier"], r["okt"], r["steps"]


def test_early_stop_parity_with_the_oracle(oracle, Context):
    w = _early(workloads.load("movepush"))
    seed = 1
    Z = _rows(oracle, w, seed, 128)
    ok, cr, tr, dec, sr = _certified(oracle, w, seed, Z)
    assert ok.sum() >= 48
    cg, tg, sg = _gpu(Context, w, Z, seed)
    assert not tier_mismatches("movepush early stop", dec, tg, tr, cg, cr)
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


# ---- stop on a failed action (scene fail_stop = 1) ----

def _failstop(w):
    wf = copy.deepcopy(w)
    wf["scene"]["fail_stop"] = 1
    return wf


def _gpu_full(Context, w, Z, seed, lanes=1):
    n = Z.shape[0]
    with Context(w, seed=seed, pop=max(n, 64), n_elite=1, lanes=lanes) as c:
        Zd = torch.from_numpy(np.ascontiguousarray(Z)).to("cuda:0")
        cost = torch.empty(n, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        pose = torch.empty((n, 7), dtype=torch.float32, device="cuda:0")
        c.rollout_batch(Zd, cost, tier, pose)
        torch.cuda.synchronize()
        return cost.cpu().numpy().astype(np.float64), tier.cpu().numpy(), pose.cpu().numpy(), c.env_steps()


@pytest.mark.parametrize("name,lanes", [("pickplace", 1), ("pickplace", 16), ("movepush", 1), ("movepush", 8)])
def test_fail_stop_against_the_gpus_full_run(oracle, Context, name, lanes):
    # plans whose actions all succeed are untouched, to the bit; the others
    # report tier 2 and stop early, at a cost no larger than the full run's
    w = workloads.load(name)
    n = 256
    Z = _rows(oracle, w, 5, n)
    cf, tf, pf, sf = _gpu_full(Context, w, Z, 5, lanes)
    cs, ts, ps, ss = _gpu_full(Context, _failstop(w), Z, 5, lanes)
    keep = tf <= 1
    assert np.array_equal(cs[keep], cf[keep]) and np.array_equal(ts[keep], tf[keep])
    assert np.array_equal(ps[keep], pf[keep])
    stopped = ~keep & (ts == 2)
    assert np.all(ts[~keep] >= 2)
    assert np.all(cs[stopped] <= cf[stopped] + 1e-6)
    assert ss < sf and stopped.sum() > 0
    print("%s, %d lanes: %d of %d plans stopped early, %.1f %% of the full run's steps"
          % (name, lanes, stopped.sum(), n, 100.0 * ss / sf))


def test_fail_stop_parity_with_the_oracle(oracle, Context):
    w = _failstop(workloads.load("pickplace"))
    seed = 6
    Z = _rows(oracle, w, seed, 128)
    ok, cr, tr, dec, sr = _certified(oracle, w, seed, Z)
    assert ok.sum() >= 48
    cg, tg, sg = _gpu(Context, w, Z, seed)
    assert not tier_mismatches("pickplace fail stop", dec, tg, tr, cg, cr)
    same = ok & (tg == tr) & (tr < 3)
    assert np.max(np.abs(cg[same] - cr[same])) <= 2 * w["scene"]["dt"] + 1e-6
    assert abs(sg - int(sr.sum())) <= 0.05 * sr.sum()


def test_fail_stop_leaves_the_ce_run_unchanged(Context):
    # the update reads tier 0 and tier 1 samples only, which the stop does not touch
    w = copy.deepcopy(workloads.load("pickplace"))
    w["cem"].update(pop=256, n_elite=16)
    for seed in (0, 1):
        with Context(w, seed=seed) as c:
            a = c.plan_solve(3)
            na = c.env_steps()
        with Context(_failstop(w), seed=seed) as c:
            b = c.plan_solve(3)
            nb = c.env_steps()
        assert np.array_equal(a["mu"], b["mu"]) and np.array_equal(a["cov"], b["cov"])
        assert np.array_equal(a["stats"][:, [1, 2, 5, 6]], b["stats"][:, [1, 2, 5, 6]])
        if a["best_tier"] <= 1:
            assert a["best_cost"] == b["best_cost"] and np.array_equal(a["best_z"], b["best_z"])
        assert nb < na


def test_pooled_batch_with_stops_equals_single_runs(oracle, Context):
    # in a batch, lanes whose rollout stopped take the instance's next plan; the
    # outcomes and step counts are those of the instances run alone
    from paper_2512_11571_amd import binding
    insts = []
    for k, name in enumerate(("pickplace", "movepush", "pickplace")):
        w = _failstop(_early(workloads.load(name)))
        w["scene"]["horizon"] = 900 + 300 * k
        w["cem"].update(pop=200 + 64 * k, n_elite=8)
        insts.append({"workload": w, "seed": k, "instance": k, "iters": 2})
    with binding.Batch(insts) as bt:
        res = bt.solve(2)
        counted = [bt.instance(k).env_steps() for k in range(3)]
        last = [bt.instance(k).outcomes() for k in range(3)]
    for inst, r, n, (cb, tb, pb) in zip(insts, res, counted, last):
        with Context(inst["workload"], seed=inst["seed"], instance=inst["instance"]) as c:
            s = c.plan_solve(inst["iters"])
            assert c.env_steps() == n
            cs, ts, ps = c.outcomes()
        assert r["best_cost"] == s["best_cost"] and np.array_equal(r["mu"], s["mu"])
        assert np.array_equal(cb, cs) and np.array_equal(tb, ts) and np.array_equal(pb, ps)
        full = inst["iters"] * inst["workload"]["cem"]["pop"] * inst["workload"]["scene"]["horizon"]
        assert n < full
