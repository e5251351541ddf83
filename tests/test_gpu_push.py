"""GPU parity of the push plan through the C ABI against the CPU oracle.

Bit-exact: Cholesky factor of theta, Philox samples, elite index sets and the
refit theta given identical inputs, run-to-run results, eager vs graph-replayed
iterations.  Tolerance: FP32 rollout states within 1e-3 m / rad of the FP64
oracle over the first 100 control steps and costs within 1e-3 on cases the
oracle certifies as non-chaotic (a one-ulp nudge of every parameter moves the
oracle's own trajectory by under 1e-4).  Statistical: the median best cost of
plan_solve over seeds 0-9 within 1e-2 relative.
"""
import numpy as np
import pytest

from paper_2512_11571_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def push():
    return workloads.load("push")


@pytest.fixture(scope="module")
def Context():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd.binding import Context
    return Context


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _cov0(w):
    return np.diag(np.asarray(w["cem"]["cov0_diag"], np.float64))


def test_factor_and_instance_draw(oracle, push, Context):
    for seed in (0, 3, 2 ** 40 + 17):
        with Context(push, seed=seed, instance=2) as c:
            Lr, rc = oracle.factor_cov(_cov0(push))
            assert rc == 0 and np.array_equal(c.get_factor(), Lr)
            g = c.get_instance()
            gr = oracle.draw_instance(push, seed, inst=2)
            # same uniforms; the ABI carries the draw ranges in FP32, the oracle in FP64
            assert np.max(np.abs(g - gr)) < 1e-6


@pytest.mark.parametrize("pop", [1, 64, 1000, 65536])
def test_sample_bit_exact(oracle, push, Context, pop):
    seed, inst = 12345, 3
    with Context(push, seed=seed, instance=inst, pop=pop, n_elite=1) as c:
        L = c.get_factor()
        mu = np.asarray(push["cem"]["mu0"], np.float64)
        Z = torch.empty((pop, 3), dtype=torch.float32, device="cuda:0")
        for it in (0, 1, 7):
            c.cem_sample(it, Z)
            torch.cuda.synchronize()
            Zr = oracle.sample(seed, it, inst, pop, mu, L)
            assert np.array_equal(Z.cpu().numpy().view(np.uint32), Zr.view(np.uint32))


def test_full_covariance_factor_and_sample_bit_exact(oracle, push, Context):
    w = dict(push, cem=dict(push["cem"], cov_mode="full"))
    A = np.array([[0.5, 0.1, -0.05], [0.1, 0.3, 0.02], [-0.05, 0.02, 0.2]])
    mu = np.array([0.1, -0.2, 0.7])
    with Context(w, seed=9, pop=4096) as c:
        c.set_theta(mu, A)
        Lr, _ = oracle.factor_cov(A)
        L = c.get_factor()
        assert np.array_equal(L, Lr)
        Z = torch.empty((4096, 3), dtype=torch.float32, device="cuda:0")
        c.cem_sample(5, Z)
        torch.cuda.synchronize()
        Zr = oracle.sample(9, 5, 0, 4096, mu, Lr)
        assert np.array_equal(Z.cpu().numpy(), Zr)


def _certified(oracle, w, seed, Zs, steps):
    """Rows whose oracle trajectory moves < 1e-4 when every parameter is nudged by one ulp."""
    _, _, _, t0 = oracle.rollout(w, seed, Zs, trace_steps=steps)
    nud = np.nextafter(Zs, np.float32(np.inf)).astype(np.float32)
    _, _, _, t1 = oracle.rollout(w, seed, nud, trace_steps=steps)
    dev = np.max(np.abs(t0[:, :, :7] - t1[:, :, :7]), axis=(1, 2))
    return dev < 1e-4, t0


def test_rollout_trace_parity_100_steps(oracle, push, Context):
    seed = 1
    rng = np.random.default_rng(0)
    g = oracle.draw_instance(push, seed)
    base = np.arctan2(g[1], g[0])
    Zs = np.stack([base + rng.uniform(-0.4, 0.4, 96), rng.uniform(-0.1, 0.1, 96),
                   rng.uniform(0.2, 1.5, 96)], 1).astype(np.float32)
    ok, tr_ref = _certified(oracle, push, seed, Zs, 100)
    assert ok.sum() >= 48
    Zc = Zs[ok]
    with Context(push, seed=seed) as c:
        Zd = _dev(Zc)
        tr = torch.empty((Zc.shape[0], 100, 13), dtype=torch.float32, device="cuda:0")
        c.rollout_trace(Zd, 100, tr)
        torch.cuda.synchronize()
        tr = tr.cpu().numpy().astype(np.float64)
    ref = tr_ref[ok]
    assert np.max(np.abs(tr[:, :, 0:3] - ref[:, :, 0:3])) < 1e-3          # position, m
    # orientation error angle ~ 2 |q - q_ref| for nearby unit quaternions
    assert np.max(2 * np.linalg.norm(tr[:, :, 3:7] - ref[:, :, 3:7], axis=2)) < 1e-3
    assert np.max(np.abs(tr[:, :, 7:13] - ref[:, :, 7:13])) < 2e-2        # velocities


@pytest.mark.parametrize("pop", [1, 100, 1000])
def test_rollout_costs_match_oracle(oracle, push, Context, pop):
    seed = 2
    H = push["scene"]["horizon"]
    with Context(push, seed=seed, pop=max(pop, 8), n_elite=8) as c:
        Z = torch.empty((pop, 3), dtype=torch.float32, device="cuda:0")
        c.cem_sample(0, Z)
        cost = torch.empty(pop, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(pop, dtype=torch.uint8, device="cuda:0")
        pose = torch.empty((pop, 7), dtype=torch.float32, device="cuda:0")
        c.rollout_batch(Z, cost, tier, pose)
        torch.cuda.synchronize()
        Zh = Z.cpu().numpy()
    cr, tr_, pr, _ = oracle.rollout(push, seed, Zh)
    ok, _ = _certified(oracle, push, seed, Zh, H)
    nud_c, _, _, _ = oracle.rollout(push, seed, np.nextafter(Zh, np.float32(np.inf)).astype(np.float32))
    stable = ok & (np.abs(nud_c - cr) < 1e-4)
    assert np.array_equal(tier.cpu().numpy(), tr_)
    assert stable.sum() >= max(1, int(0.5 * pop))
    c_gpu = cost.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(c_gpu[stable] - cr[stable])) < 1e-3
    assert np.max(np.abs(pose.cpu().numpy()[stable, :3] - pr[stable, :3])) < 1e-3


def test_rollout_pop_zero_is_a_no_op(push, Context):
    with Context(push) as c:
        Z = torch.empty((0, 3), dtype=torch.float32, device="cuda:0")
        cost = torch.empty(0, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(0, dtype=torch.uint8, device="cuda:0")
        c.rollout_batch(Z, cost, tier)


def _refit_case(oracle, push, Context, cost, tier, n_elite, cov_mode="diag", seed=4):
    pop = cost.size
    w = dict(push, cem=dict(push["cem"], cov_mode=cov_mode))
    with Context(w, seed=seed, pop=pop, n_elite=n_elite) as c:
        Z = torch.empty((pop, 3), dtype=torch.float32, device="cuda:0")
        c.cem_sample(0, Z)
        elite = torch.full((n_elite,), -7, dtype=torch.int32, device="cuda:0")
        info = torch.zeros(6, dtype=torch.int32, device="cuda:0")
        c.cem_refit(Z, _dev(cost.astype(np.float32)), _dev(tier.astype(np.uint8)), elite, info)
        torch.cuda.synchronize()
        mu_g, S_g = c.get_theta()
        L_g = c.get_factor()
        Zh = Z.cpu().numpy()
        elite = elite.cpu().numpy()
        info = info.cpu().numpy()
    idx, mode, counts = oracle.select(cost, tier, n_elite)
    cov0 = _cov0(w)
    mu_r, S_r, L_r, _ = oracle.refit(Zh, idx, mode, 0 if cov_mode == "diag" else 1, cov0,
                                     np.asarray(w["cem"]["mu0"], np.float64), cov0)
    ne = len(idx)
    assert list(elite[:ne]) == list(idx) and np.all(elite[ne:] == -1)
    assert info[0] == ne and info[1] == mode and list(info[2:]) == list(counts)
    assert np.array_equal(mu_g, mu_r) and np.array_equal(S_g, S_r) and np.array_equal(L_g, L_r)
    return mode


@pytest.mark.parametrize("cov_mode", ["diag", "full"])
def test_refit_bit_exact_given_oracle_costs(oracle, push, Context, cov_mode):
    seed = 4
    with Context(push, seed=seed) as c:
        Z = torch.empty((64, 3), dtype=torch.float32, device="cuda:0")
        c.cem_sample(0, Z)
        torch.cuda.synchronize()
        Zh = Z.cpu().numpy()
    cr, tr_, _, _ = oracle.rollout(push, seed, Zh)
    assert _refit_case(oracle, push, Context, cr.astype(np.float32), tr_, 8, cov_mode) == 0


def test_refit_edge_cases(oracle, push, Context):
    rng = np.random.default_rng(3)
    nan = np.float32("nan")
    # ties everywhere (index order decides), a ragged population
    c = np.full(1000, 0.25, np.float32)
    assert _refit_case(oracle, push, Context, c, np.zeros(1000, np.uint8), 64) == 0
    # NaN costs rank as diverged; fewer feasible than N_e
    c = rng.uniform(0, 1, 300).astype(np.float32)
    t = np.full(300, 2, np.uint8)
    t[:20] = 0
    c[3] = nan
    assert _refit_case(oracle, push, Context, c, t, 64) == 1
    # exactly one feasible -> that sample with artificial noise
    t = np.full(300, 2, np.uint8)
    t[17] = 0
    assert _refit_case(oracle, push, Context, c, t, 64) == 2
    # none feasible, some with all actions succeeded -> tier 1 elites
    t = rng.integers(1, 4, 300).astype(np.uint8)
    assert _refit_case(oracle, push, Context, c, t, 32) == 3
    # nothing usable -> theta unchanged
    t = np.full(300, 3, np.uint8)
    assert _refit_case(oracle, push, Context, c, t, 32) == 4
    # a single sample, N_e = 1; and the largest population
    assert _refit_case(oracle, push, Context, np.array([0.5], np.float32), np.zeros(1, np.uint8), 1) == 0
    big = rng.uniform(0, 10, 65536).astype(np.float32)
    big[rng.integers(0, 65536, 1000)] = 1.0   # heavy ties
    assert _refit_case(oracle, push, Context, big, rng.integers(0, 2, 65536).astype(np.uint8), 256,
                       "full") == 0


def test_plan_solve_equals_eager_iterations_and_is_deterministic(push, Context):
    iters = push["cem"]["iters"]
    seed = 6
    with Context(push, seed=seed) as c:
        r1 = c.plan_solve(iters)
        mu1, S1 = c.get_theta()
    with Context(push, seed=seed) as c:
        r2 = c.plan_solve(2)
        r2b = c.plan_solve(iters - 2)          # replays continue the counter
        mu2, S2 = c.get_theta()
    with Context(push, seed=seed) as c:       # the same iterations issued eagerly
        Z = torch.empty((64, 3), dtype=torch.float32, device="cuda:0")
        cost = torch.empty(64, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(64, dtype=torch.uint8, device="cuda:0")
        for j in range(iters):
            c.cem_sample(j, Z)
            c.rollout_batch(Z, cost, tier)
            c.cem_refit(Z, cost, tier)
            torch.cuda.synchronize()
        mu3, S3 = c.get_theta()
    assert np.array_equal(mu1, mu2) and np.array_equal(S1, S2)
    assert np.array_equal(mu1, mu3) and np.array_equal(S1, S3)
    assert r1["best_cost"] == r2b["best_cost"] and np.array_equal(r1["best_z"], r2b["best_z"])
    assert np.array_equal(r1["stats"][2:], r2b["stats"])


def test_plan_solve_median_matches_oracle(oracle, push, Context):
    iters = push["cem"]["iters"]
    g, r = [], []
    for seed in push["cem"]["seeds"]:
        with Context(push, seed=seed) as c:
            res = c.plan_solve(iters)
        st = res["stats"]
        assert np.all(st[:, 1:5].sum(1) == push["cem"]["pop"])
        assert np.all(np.diff(st[:, 7]) <= 0)
        g.append(res["best_cost"])
        r.append(oracle.plan_solve(push, seed)["best_cost"])
    mg, mr = np.median(g), np.median(r)
    assert abs(mg - mr) <= 1e-2 * mr
