"""Domain randomisation on the GPU (Sec. IV-C), through the C ABI.

Draws: each scenario's friction and mass equal the oracle's FP64 draw rounded
to FP32.  Composition, exact on the GPU itself: a row's outcome under R
scenarios is the worst tier, the mean (butterfly order) or maximum cost and
scenario 0's pose of R plain rollouts that carry the scenarios' friction and
mass, and the step count covers all pop x R rollouts.  Against the oracle:
tier and cost on certified rows (cost within two control steps).  Batched
instances with scenarios give the bits of their single runs.  Statistical:
over 32 seeds of plan_solve, at least half the seeds' best costs within 1e-2
relative of the oracle's, and the medians within 1e-2 or two standard errors
of the median (parity_util.median_agreement).  The
composition, oracle and population tests also run with 2 to 16 lanes per
environment (the scenario butterfly then pairs lanes G, 2G, ... apart).
"""
import copy
import json
import os

import numpy as np
import pytest

from paper_2512_11571_amd import workloads
from parity_util import certify, median_agreement, tier_mismatches

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plan_solve_oracle.json")

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    return binding


def _dr(w, R, reduce="mean", mu=(0.3, 0.7), mass=(0.2, 0.4), H=None):
    w = copy.deepcopy(w)
    w["scene"]["domain_randomization"] = {"scenarios": R, "reduce": reduce, "mu": list(mu), "mass": list(mass)}
    if H:
        w["scene"]["horizon"] = H
    return w


def _plain(w, mu, mass):
    w = copy.deepcopy(w)
    w["scene"].pop("domain_randomization", None)
    w["scene"]["object"]["mu"] = [float(mu), float(mu)]
    w["scene"]["object"]["mass"] = float(mass)
    return w


def _rows(oracle, w, seed, n):
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(cem["cov0_diag"]))
    return oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)


def _run(B, w, Z, seed, lanes=1):
    n = Z.shape[0]
    with B.Context(w, seed=seed, pop=max(n, 64), n_elite=1, lanes=lanes) as c:
        Zd = torch.from_numpy(np.ascontiguousarray(Z)).to("cuda:0")
        cost = torch.empty(n, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        pose = torch.empty((n, 7), dtype=torch.float32, device="cuda:0")
        c.rollout_batch(Zd, cost, tier, pose)
        torch.cuda.synchronize()
        return cost.cpu().numpy(), tier.cpu().numpy(), pose.cpu().numpy(), c.env_steps(), c.get_scenarios()


def test_scenario_draws_match_the_oracle(oracle, B):
    w = _dr(workloads.load("movepush"), 64)
    for seed, inst in ((0, 0), (3, 1)):
        with B.Context(w, seed=seed, instance=inst) as c:
            mu, mass = c.get_scenarios()
        rmu, rmass = oracle.scenarios(w, seed, inst)
        # the same uniforms; the range ends differ by the FP32 rounding of the scene
        assert np.max(np.abs(mu - rmu)) < 1e-6 and np.max(np.abs(mass - rmass)) < 1e-6


@pytest.mark.parametrize("name,R,reduce,lanes", [("movepush", 4, "mean", 1), ("pickplace", 8, "max", 1),
                                                 ("movepush", 4, "mean", 4), ("pickplace", 8, "max", 2),
                                                 ("movepush", 8, "mean", 8)])
def test_rows_compose_their_scenarios(oracle, B, name, R, reduce, lanes):
    base = workloads.load(name)
    w = _dr(base, R, reduce, H=600)
    n = 100                                           # ragged: 100 x R environments
    Z = _rows(oracle, base, 1, n)
    cost, tier, pose, steps, (mu, mass) = _run(B, w, Z, 1, lanes)
    runs = [_run(B, _plain(w, mu[r], mass[r]), Z, 1, lanes) for r in range(R)]
    assert steps == sum(r_[3] for r_ in runs) and 0.99 * n * R * 600 <= steps <= n * R * 600
    C = np.stack([r_[0] for r_ in runs])
    T = np.stack([r_[1] for r_ in runs])
    if reduce == "mean":
        while C.shape[0] > 1:                         # the kernel's butterfly: pairs at distance 1, 2, 4, ...
            C = np.stack([C[k] + C[k + 1] for k in range(0, C.shape[0], 2)])
        want = (C[0] * np.float32(1.0 / R)).astype(np.float32)
    else:
        want = C.max(0)
    fin = np.isfinite(want)
    assert np.array_equal(cost[fin], want[fin]) and np.all(~np.isfinite(cost[~fin]))
    assert np.array_equal(tier, T.max(0))
    assert np.array_equal(pose, runs[0][2])


@pytest.mark.parametrize("lanes", [1, 4])
def test_parity_with_the_oracle(oracle, B, lanes):
    w = _dr(workloads.load("movepush"), 4)
    seed = 2
    Z = _rows(oracle, w, seed, 64)
    r = certify(oracle, w, seed, Z)            # certified: nudges of 1 to 256 ulps either way change nothing
    ok, c0, t0 = r["ok"], r["cost"], r["tier"]
    assert ok.sum() >= 24
    cg, tg, _, _, _ = _run(B, w, Z, seed, lanes)
    # scenario 0's final state stands for the row's in the goal certification
    okt = r["okt"]
    assert not tier_mismatches("movepush 4 scenarios, %d lanes" % lanes, okt, tg, t0, cg, c0)
    same = ok & (tg == t0) & (t0 < 3)
    assert np.max(np.abs(cg[same] - c0[same])) <= 2 * w["scene"]["dt"] + 1e-6


def test_batched_with_scenarios_equals_single_runs(B):
    a = _dr(workloads.load("pickplace"), 8, H=300)
    b = _dr(workloads.load("movepush"), 2, "max", H=400)
    for w, pop in ((a, 100), (b, 130)):
        w["cem"].update(pop=pop, n_elite=8)
    insts = [{"workload": a, "seed": 0, "instance": 0, "iters": 2},
             {"workload": workloads.load("push"), "seed": 1, "instance": 1, "iters": 3},
             {"workload": b, "seed": 2, "instance": 2, "iters": 2}]
    with B.Batch(insts) as bt:
        res = bt.solve(3)
        counted = [bt.instance(k).env_steps() for k in range(3)]
    for inst, r, n in zip(insts, res, counted):
        w = inst["workload"]
        R = w["scene"].get("domain_randomization", {}).get("scenarios", 1)
        assert n >= 0.99 * inst["iters"] * w["cem"]["pop"] * R * w["scene"]["horizon"]
        with B.Context(w, seed=inst["seed"], instance=inst["instance"]) as c:
            s = c.plan_solve(inst["iters"])
            assert c.env_steps() == n
        assert r["best_cost"] == s["best_cost"] and r["best_tier"] == s["best_tier"]
        assert np.array_equal(r["best_z"], s["best_z"]) and np.array_equal(r["mu"], s["mu"])


def test_plan_solve_median_matches_oracle(B):
    # the oracle's runs are tests/golden/plan_solve_oracle.json ("dr_small"), written by
    # tests/golden/make_plan_solve_goldens.py
    gold = json.load(open(GOLDEN))["dr_small"]["runs"]
    w = _dr(workloads.load("pickplace"), 4)
    w["cem"].update(pop=64, n_elite=8)
    iters = 2
    g, r = [], []
    for seed in range(32):
        with B.Context(w, seed=seed) as c:
            g.append(c.plan_solve(iters)["best_cost"])
        assert gold[str(seed)]["iters"] == iters
        r.append(gold[str(seed)]["best_cost"])
    median_agreement("DR pick-and-place (4 scenarios, pop 64, 2 iterations)", g, r)


@pytest.mark.parametrize("name,R,lanes", [("pickplace", 1, 1), ("movepush", 64, 1), ("pickplace", 1, 4), ("movepush", 16, 4),
                                          ("movepush", 8, 8), ("pickplace", 4, 16)])
def test_rows_do_not_depend_on_the_population(oracle, B, name, R, lanes):
    # a row's outcome is the same whether it runs alone (pop 1 or 3; with 64
    # scenarios one row fills a wave) or among 100 rows
    base = workloads.load(name)
    w = _dr(base, R, H=300) if R > 1 else dict(base, scene=dict(base["scene"], horizon=300))
    Z = _rows(oracle, base, 3, 100)
    full = _run(B, w, Z, 3, lanes)
    for n in (1, 3):
        part = _run(B, w, Z[:n], 3, lanes)
        for a, b in zip(part[:3], full[:3]):
            assert np.array_equal(a, b[:n])
        assert 0.99 * n * R * 300 <= part[3] <= n * R * 300
