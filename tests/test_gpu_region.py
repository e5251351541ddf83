"""The initial distribution as a region and the n_env schedule on the GPU,
through the C ABI.

Bit-exact: iteration-0 rows of a region (rings and boxes) against the oracle,
at the paper setting's full size (3000) and a ragged population; iteration 1
returns to the Gaussian rows.  Exact counts: plan_solve under a schedule
simulates sum_j n_env(j) x T control steps and its per-iteration tier counts
add up to n_env(j).  Statistical: the median best cost of plan_solve with a
region and a schedule over 32 seeds against the oracle's, within 1e-2
relative.  Batches reject a schedule.
"""
import copy
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    return binding


def _push_region():
    w = copy.deepcopy(workloads.load("push"))
    w["cem"].update(pop=256, n_elite=8, iters=5, pop_schedule={"final": 64, "iters": 3},
                    init_region={"lo": [-math.pi, -0.3, 0.1], "hi": [math.pi, 0.3, 1.5], "rings": []})
    return w


@pytest.mark.parametrize("pop", [3000, 1000, 77])
def test_region_rows_bit_exact(oracle, B, pop):
    w = copy.deepcopy(workloads.load("pickplace_paper"))
    w["cem"].pop("pop_schedule")             # sampling only: any population size
    seed = 4
    with B.Context(w, seed=seed, pop=pop, n_elite=min(50, pop)) as c:
        Z = torch.empty((pop, 16), dtype=torch.float32, device="cuda:0")
        c.cem_sample(0, Z)
        torch.cuda.synchronize()
        Z0 = Z.cpu().numpy()
        c.cem_sample(1, Z)
        torch.cuda.synchronize()
        Z1 = Z.cpu().numpy()
    assert np.array_equal(Z0, oracle.sample_region(w, seed, 0, pop))
    L, _ = oracle.factor_cov(np.diag(w["cem"]["cov0_diag"]))
    assert np.array_equal(Z1, oracle.sample(seed, 1, 0, pop, np.asarray(w["cem"]["mu0"], np.float64), L))


def test_schedule_counts(oracle, B):
    w = copy.deepcopy(workloads.load("pickplace_paper"))
    w["scene"]["horizon"] = 150
    w["cem"].update(pop=300, n_elite=20, pop_schedule={"final": 100, "iters": 3})
    iters = 5
    with B.Context(w, seed=1) as c:
        n = [c.pop_at(j) for j in range(iters)]
        assert n == [oracle.n_env_at(w, j) for j in range(iters)] == [300, 234, 167, 100, 100]
        res = c.plan_solve(iters)
        assert c.env_steps() == sum(n) * 150
    assert np.array_equal(res["stats"][:, 1:5].sum(1), n)
    assert res["iters_done"] == iters


def test_region_and_schedule_median_matches_oracle(oracle, B):
    w = _push_region()
    iters = w["cem"]["iters"]
    g, r = [], []
    for seed in range(32):
        with B.Context(w, seed=seed) as c:
            res = c.plan_solve(iters)
        assert np.array_equal(res["stats"][:, 1:5].sum(1), [oracle.n_env_at(w, j) for j in range(iters)])
        g.append(res["best_cost"])
        r.append(oracle.plan_solve(w, seed)["best_cost"])
    assert abs(np.median(g) - np.median(r)) <= 1e-2 * np.median(r)


def test_batch_rejects_a_schedule(B):
    w = _push_region()
    with pytest.raises(B.CemError):
        B.Batch([{"workload": w, "seed": 0, "instance": 0, "iters": 2}])


@pytest.mark.parametrize("lanes", [1, 4])
def test_diverged_rows_against_the_oracle(oracle, B, lanes):
    # the paper setting's iteration-0 region rows (3000): every row the GPU
    # reports as diverged (tier 3) is one the oracle also cannot complete
    # (tier 2: an action fails, or tier 3: it diverges too), so no plan that
    # could enter the update is lost to FP32 arithmetic alone
    w = copy.deepcopy(workloads.load("pickplace_paper"))
    w["cem"].pop("pop_schedule")
    seed, pop = 0, 3000
    with B.Context(w, seed=seed, pop=pop, n_elite=50, lanes=lanes) as c:
        Z = torch.empty((pop, 16), dtype=torch.float32, device="cuda:0")
        cost = torch.empty(pop, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(pop, dtype=torch.uint8, device="cuda:0")
        c.cem_sample(0, Z)
        c.rollout_batch(Z, cost, tier)
        torch.cuda.synchronize()
        Zh, th = Z.cpu().numpy(), tier.cpu().numpy()
    bad = np.nonzero(th == 3)[0]
    print("pickplace_paper iteration 0, %d lanes: %d of %d rows diverged on the GPU: %s"
          % (lanes, bad.size, pop, bad.tolist()))
    if bad.size:
        cr, tr, _, _ = oracle.rollout(w, seed, Zh[bad])
        print("  oracle tiers of those rows:", tr.tolist())
        assert np.all(tr >= 2), list(zip(bad.tolist(), tr.tolist()))
    assert bad.size <= 0.01 * pop
