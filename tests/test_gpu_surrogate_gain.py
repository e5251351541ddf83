"""What the trained surrogate gains over the method without it (pick-and-place).

A network trained on rollouts the simulator records (plain-CE runs on training
seeds) screens a 16x oversampled population; only the kept candidates are
simulated.  Against plain CE with the same number of simulated rollouts per
iteration, on held-out seeds:
  - the share of simulated plans that are feasible (tier 0) in the first
    iteration is higher: the surrogate picks better candidates;
  - the median best plan cost after the same number of iterations is lower.
Full simulation decides every cost that enters the refit in both runs.
"""
import copy

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


def test_trained_surrogate_beats_plain_ce_at_equal_simulations(B):
    spec = copy.deepcopy(workloads.load("surrogate")["surrogate"])
    spec["dataset"].update(n_instances=12, pop=1024, n_elite=64, iters=4)
    insts = workloads.surrogate_dataset_instances(spec)
    cap = sum(i["workload"]["cem"]["pop"] * i["iters"] for i in insts)
    X = torch.empty((cap, 16), dtype=torch.float32, device="cuda:0")
    Y = torch.empty((cap, 8), dtype=torch.float32, device="cuda:0")
    with B.Batch(insts) as bt:
        n = bt.record(spec["dataset"]["iters"], X, Y)
    assert n == cap

    base = workloads.load("pickplace")
    n_sim, screen_pop, n_elite, iters = 1024, 16384, 64, 3
    with B.Mlp(seed=1, max_rows=screen_pop) as m:
        m.fit_norm(X, Y, n)
        losses = m.train(X, Y, n, 1024, 12, 1e-3, seed=1)
        assert losses[-1] < losses[0]
        share = {False: [], True: []}
        best = {False: [], True: []}
        for seed in (0, 1, 2, 3):                      # disjoint from the training seeds (1000+)
            # first iteration: simulate n_sim plans drawn plainly vs n_sim kept by the screen
            w = dict(base, cem=dict(base["cem"], pop=n_sim, n_elite=n_elite))
            with B.Context(w, seed=seed) as c:
                Z = torch.empty((n_sim, 16), dtype=torch.float32, device="cuda:0")
                cost = torch.empty(n_sim, dtype=torch.float32, device="cuda:0")
                tier = torch.empty(n_sim, dtype=torch.uint8, device="cuda:0")
                c.cem_sample(0, Z)
                c.rollout_batch(Z, cost, tier)
                torch.cuda.synchronize()
                share[False].append(float((tier.cpu().numpy() == 0).mean()))
                best[False].append(c.plan_solve(iters)["best_cost"])
            ws = dict(base, cem=dict(base["cem"], pop=screen_pop, n_elite=n_elite))
            with B.Context(ws, seed=seed) as c:
                Zs = torch.empty((n_sim, 16), dtype=torch.float32, device="cuda:0")
                m.screen(c, 0, n_sim, Zs)
                with B.Context(w, seed=seed) as cs:
                    cost = torch.empty(n_sim, dtype=torch.float32, device="cuda:0")
                    tier = torch.empty(n_sim, dtype=torch.uint8, device="cuda:0")
                    cs.rollout_batch(Zs, cost, tier)
                    torch.cuda.synchronize()
                    share[True].append(float((tier.cpu().numpy() == 0).mean()))
                best[True].append(m.plan_solve_screened(c, iters, n_sim)["best_cost"])
    print("feasible share", share, "best", best)
    assert np.mean(share[True]) >= np.mean(share[False]) + 0.1
    assert np.median(best[True]) < np.median(best[False])
