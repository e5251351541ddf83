"""The BF16-MFMA surrogate network against the oracle: bit-exact He
initialisation, forward against the oracle's BF16-emulated forward (up to
16,384 rows), the whole-network inference kernel against the layer-by-layer
GEMMs bit for bit, loss and gradients against the oracle's FP64 backward, Adam
against the oracle's Adam,
training progress, the screening top-k against a host sort of the same keys,
and the recorded dataset against the simulator's own outputs."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda:0")


def test_init_bit_exact(oracle, B):
    with B.Mlp(seed=11, max_rows=1024) as m:
        P = m.get_params()
    Pr = oracle.mlp_init(11)
    assert np.array_equal(P.astype(np.float64), Pr)


@pytest.mark.parametrize("n", [1, 77, 1000, 16384])
def test_forward_matches_bf16_oracle(oracle, B, n):
    rng = np.random.default_rng(n)
    with B.Mlp(seed=3, max_rows=16384) as m:
        P = m.get_params()
        P = P + rng.normal(size=P.size).astype(np.float32) * 0.01   # nonzero biases
        m.set_params(P)
        x = rng.normal(size=(n, 16)).astype(np.float32)
        Y = torch.empty((n, 8), dtype=torch.float32, device="cuda:0")
        m.forward(_dev(x), Y)
        torch.cuda.synchronize()
        y = Y.cpu().numpy().astype(np.float64)
    yr = oracle.mlp_forward(P.astype(np.float64), x, bf16=True)
    y64 = oracle.mlp_forward(P.astype(np.float64), x)
    scale = np.max(np.abs(y64))
    # same BF16 operands; FP32 vs FP64 accumulation order and BF16 rounding of
    # hidden activations are the only differences
    assert np.max(np.abs(y - yr)) <= 2e-2 * scale
    assert np.max(np.abs(y - y64)) <= 5e-2 * scale


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 8192])
def test_fused_forward_equals_the_layer_by_layer_forward(B, n):
    # the whole-network kernel (64 rows per workgroup, activations in LDS)
    # against the layer-by-layer tiled GEMMs of the allocation-free entry, bit
    # for bit: the same BF16 operands, the same MFMA per 32-step of the
    # contraction in the same order, the same epilogue expressions; n spans
    # one row, ragged and whole workgroups and the fixed array's limit
    rng = np.random.default_rng(100 + n)
    with B.Mlp(seed=5, max_rows=8192) as m:
        m.set_params(m.get_params() + rng.normal(size=m.n_params).astype(np.float32) * 0.01)
        m.set_norm(np.concatenate([rng.normal(size=16), rng.uniform(0.5, 2.0, 16),
                                   rng.normal(size=8), rng.uniform(0.5, 2.0, 8)]).astype(np.float32))
        x = _dev(rng.normal(size=(n, 16)) * 2.0)
        y_f = torch.full((n, 8), float("nan"), dtype=torch.float32, device="cuda:0")
        y_l = torch.full((n, 8), float("nan"), dtype=torch.float32, device="cuda:0")
        m.forward(x, y_f)
        m.forward_static(x, y_l)
        torch.cuda.synchronize()
        a, b = y_f.cpu().numpy(), y_l.cpu().numpy()
    assert np.all(np.isfinite(a))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (n, np.max(np.abs(a - b)))


@pytest.mark.parametrize("n", [200, 4096])
def test_loss_and_gradient_match_the_oracle_elementwise(oracle, B, n):
    # n = 4096: the training batch.  Every gradient element against the
    # oracle's backward with the same BF16 operands (FP32 against FP64
    # accumulation and the order of the sums the only differences), and against
    # the plain FP64 backward at the 1e-2 bound of the BF16 arithmetic:
    #   |g - g_ref| <= rtol |g_ref| + atol max_layer |g_ref|
    rng = np.random.default_rng(5)
    with B.Mlp(seed=4, max_rows=4096) as m:
        P = m.get_params() + rng.normal(size=m.n_params).astype(np.float32) * 0.01
        m.set_params(P)
        x = rng.normal(size=(n, 16)).astype(np.float32)
        t = rng.normal(size=(n, 8)).astype(np.float32)
        G = torch.empty(m.n_params, dtype=torch.float32, device="cuda:0")
        L = torch.empty(1, dtype=torch.float32, device="cuda:0")
        m.loss_grad(_dev(x), _dev(t), G, L)
        torch.cuda.synchronize()
        g, loss = G.cpu().numpy().astype(np.float64), float(L.cpu()[0])
    P64 = P.astype(np.float64)
    le, ge = oracle.mlp_loss_grad(P64, x, t, bf16=True)
    lr, gr = oracle.mlp_loss_grad(P64, x, t)
    assert abs(loss - le) <= 1e-4 * le and abs(loss - lr) <= 2e-2 * lr
    worst = {}
    for l, (ws, shape, bs) in enumerate(oracle.mlp_slices()):
        for name, sl in (("W%d" % (l + 1), ws), ("b%d" % (l + 1), bs)):
            a, e, r = g[sl], ge[sl], gr[sl]
            me, mr = np.max(np.abs(e)), np.max(np.abs(r))
            # same arithmetic: rtol 1e-2, atol 1e-3 of the layer's largest element
            ex = np.abs(a - e) - (1e-2 * np.abs(e) + 1e-3 * me)
            # against FP64: the O-8 bound, 1e-2 relative plus 1e-2 of the largest element
            fx = np.abs(a - r) - (1e-2 * np.abs(r) + 1e-2 * mr)
            worst[name] = (float(np.max(np.abs(a - e)) / me), float(np.max(np.abs(a - r)) / mr))
            assert np.all(ex <= 0), (name, int(np.argmax(ex)), float(np.max(ex)))
            assert np.all(fx <= 0), (name, int(np.argmax(fx)), float(np.max(fx)))
    print("n %d: largest |g - g_bf16| / max and |g - g_fp64| / max per tensor:" % n,
          {k: "%.1e / %.1e" % v for k, v in worst.items()})


def test_adam_step_matches_oracle(oracle, B):
    rng = np.random.default_rng(6)
    n = 128
    with B.Mlp(seed=5, max_rows=1024) as m:
        P0 = m.get_params()
        x = _dev(rng.normal(size=(n, 16)))
        t = _dev(rng.normal(size=(n, 8)))
        G = torch.empty(m.n_params, dtype=torch.float32, device="cuda:0")
        m.loss_grad(x, t, G)
        m.train_step(x, t, 1e-3)
        torch.cuda.synchronize()
        P1 = m.get_params().astype(np.float64)
        g = G.cpu().numpy().astype(np.float64)
    P = P0.astype(np.float64)
    mm, vv = np.zeros_like(P), np.zeros_like(P)
    oracle.adam_step(P, g, mm, vv, 1, lr=1e-3)
    assert np.max(np.abs(P1 - P)) <= 2e-6


def test_training_reduces_loss(oracle, B):
    rng = np.random.default_rng(7)
    N = 8192
    A = rng.normal(size=(16, 8)) * 0.3
    x = rng.normal(size=(N, 16)).astype(np.float32)
    y = np.sin(x @ A).astype(np.float32)
    with B.Mlp(seed=1, max_rows=4096) as m:
        X, Y = _dev(x), _dev(y)
        m.fit_norm(X, Y)
        losses = m.train(X, Y, N, 1024, 6, 3e-3, seed=2)
    assert losses[-1] < 0.2 * losses[0]


def test_screen_topk_is_the_k_smallest_keys(oracle, B):
    pp = workloads.load("pickplace")
    rng = np.random.default_rng(8)
    pop, k = 5000, 700
    with B.Context(pp, seed=3, pop=pop, n_elite=64) as c, B.Mlp(seed=2, max_rows=pop) as m:
        norm = np.concatenate([np.asarray(pp["cem"]["mu0"]), np.sqrt(pp["cem"]["cov0_diag"]),
                               [5.0, 2.0, 0.0, 0.4, 0.5, 0, 0, 0], [2.0, 1.0, 0.5, 0.1, 0.5, 0.5, 0.5, 0.5]])
        m.set_norm(norm.astype(np.float32))
        P = m.get_params() + rng.normal(size=m.n_params).astype(np.float32) * 0.05
        m.set_params(P)
        Zs = torch.empty((k, 16), dtype=torch.float32, device="cuda:0")
        Ps = torch.empty((k, 8), dtype=torch.float32, device="cuda:0")
        m.screen(c, 0, k, Zs, Ps)
        Zall = torch.empty((pop, 16), dtype=torch.float32, device="cuda:0")
        c.cem_sample(0, Zall)
        Yall = torch.empty((pop, 8), dtype=torch.float32, device="cuda:0")
        m.forward(Zall, Yall)
        torch.cuda.synchronize()
        Zs, Ps, Zall, Yall = Zs.cpu().numpy(), Ps.cpu().numpy(), Zall.cpu().numpy(), Yall.cpu().numpy()
    t2 = pp["scene"]["static_boxes"][pp["scene"]["goal_static"]]
    top = t2["center"][2] + t2["half"][2]
    he = pp["scene"]["object"]["half"][2]
    goal = ((np.abs(Yall[:, 1] - t2["center"][0]) <= t2["half"][0]) & (np.abs(Yall[:, 2] - t2["center"][1]) <= t2["half"][1])
            & (Yall[:, 3] >= top - he) & (Yall[:, 3] <= top + 3 * he))
    order = np.lexsort((np.arange(pop), Yall[:, 0], (~goal).astype(int)))
    want = np.sort(order[:k])
    assert np.array_equal(Zs, Zall[want])
    assert np.array_equal(Ps, Yall[want])


def test_recorded_dataset_is_the_simulated_outcome(oracle, B):
    spec = dict(workloads.load("batch")["batch"])
    spec.update(n_instances=3, kinds=["pickplace"], horizon=[150, 150], pop=[64, 64], iters={"pickplace": 2}, seed=1)
    insts = workloads.batch_instances(spec)
    cap = 3 * 64 * 2
    X = torch.empty((cap, 16), dtype=torch.float32, device="cuda:0")
    Y = torch.empty((cap, 8), dtype=torch.float32, device="cuda:0")
    with B.Batch(insts) as bt:
        n = bt.record(2, X, Y)
    assert n == cap
    X, Y = X.cpu().numpy(), Y.cpu().numpy()
    # first iteration rows of instance 0 are its iteration-0 samples; their outcome is the rollout's
    w = insts[0]["workload"]
    L, _ = oracle.factor_cov(np.diag(w["cem"]["cov0_diag"]))
    Z0 = oracle.sample(insts[0]["seed"], 0, insts[0]["instance"], 64, np.asarray(w["cem"]["mu0"]), L)
    assert np.array_equal(X[:64], Z0)
    with B.Context(w, seed=insts[0]["seed"], instance=insts[0]["instance"]) as c:
        cost = torch.empty(64, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(64, dtype=torch.uint8, device="cuda:0")
        pose = torch.empty((64, 7), dtype=torch.float32, device="cuda:0")
        c.rollout_batch(_dev(Z0), cost, tier, pose)
        torch.cuda.synchronize()
        cost, pose = cost.cpu().numpy(), pose.cpu().numpy()
    assert np.array_equal(Y[:64, 0], cost)
    s = np.where(pose[:, 3:4] < 0, -1.0, 1.0).astype(np.float32)
    assert np.array_equal(Y[:64, 1:4], pose[:, :3]) and np.array_equal(Y[:64, 4:8], s * pose[:, 3:7])
    assert np.all(np.isfinite(Y))


def _screening_setup(B, pp, m, rng):
    norm = np.concatenate([np.asarray(pp["cem"]["mu0"]), np.sqrt(pp["cem"]["cov0_diag"]),
                           [5.0, 2.0, 0.0, 0.4, 0.5, 0, 0, 0], [2.0, 1.0, 0.5, 0.1, 0.5, 0.5, 0.5, 0.5]])
    m.set_norm(norm.astype(np.float32))
    m.set_params(m.get_params() + rng.normal(size=m.n_params).astype(np.float32) * 0.05)


def _short_pickplace(pop, n_elite):
    pp = workloads.load("pickplace")
    return dict(pp, scene=dict(pp["scene"], horizon=400), cem=dict(pp["cem"], pop=pop, n_elite=n_elite))


@pytest.mark.parametrize("lanes", [1, 4])
def test_plan_solve_screened_equals_eager_steps(B, lanes):
    # the captured screened iteration = screen, simulate the kept candidates,
    # refit (also with the rollout at 4 lanes per plan, as the A/B runs it)
    w = _short_pickplace(2048, 32)
    n_sim, iters = 256, 2
    with B.Mlp(seed=3, max_rows=2048) as m:
        _screening_setup(B, w, m, np.random.default_rng(9))
        with B.Context(w, seed=4, lanes=lanes) as c:
            r = m.plan_solve_screened(c, iters, n_sim)
            mu_g, S_g = c.get_theta()
        with B.Context(w, seed=4, lanes=lanes) as c2:
            Zs = torch.empty((n_sim, 16), dtype=torch.float32, device="cuda:0")
            Ps = torch.empty((n_sim, 8), dtype=torch.float32, device="cuda:0")
            cost = torch.empty(n_sim, dtype=torch.float32, device="cuda:0")
            tier = torch.empty(n_sim, dtype=torch.uint8, device="cuda:0")
            for it in range(iters):
                m.screen(c2, it, n_sim, Zs, Ps)
                c2.rollout_batch(Zs, cost, tier, None)
                c2.cem_refit(Zs, cost, tier, None, None)
            torch.cuda.synchronize()
            mu_e, S_e = c2.get_theta()
    assert np.array_equal(mu_g, mu_e) and np.array_equal(S_g, S_e)
    assert r["iters_done"] == iters and np.isfinite(r["best_cost"])
    assert np.all(np.isfinite(r["surrogate_err"]))


def test_screened_solves_on_successive_contexts(B):
    # contexts created and freed one after another (a freed context's host
    # address is reused by the next): each solve uses its own context's buffers
    w = _short_pickplace(2048, 32)
    n_sim = 256
    outs = []
    with B.Mlp(seed=3, max_rows=2048) as m:
        _screening_setup(B, w, m, np.random.default_rng(9))
        P, nrm = m.get_params(), m.get_norm()
        for seed in (5, 6, 5):
            with B.Context(w, seed=seed) as c:
                outs.append(m.plan_solve_screened(c, 1, n_sim))
    with B.Mlp(seed=3, max_rows=2048) as m2:
        m2.set_params(P)
        m2.set_norm(nrm)
        with B.Context(w, seed=6) as c:
            fresh = m2.plan_solve_screened(c, 1, n_sim)
    same = lambda a, b: a["best_cost"] == b["best_cost"] and np.array_equal(a["best_z"], b["best_z"]) and \
        np.array_equal(a["mu"], b["mu"])
    assert same(outs[0], outs[2]) and same(outs[1], fresh)
