"""The batched persistent launch against the oracle, at the configured batch's
shape: 64 independent instances (push, and pick-and-place on a ramp whose pose
is jittered per instance), horizons up to 4000 steps, populations up to 4096,
one persistent rollout launch per CE iteration; and the mixed batch, whose
instances run three different action sequences in one launch.

- Iteration 0 of sampled instances (the longest-horizon pick-and-place, the
  other pick-and-place instances with H >= 2000, and push instances): the
  sampled rows are the oracle's bit for bit; on 48 random rows of each, the
  rows the oracle certifies (cost and tier unchanged by 1- to 256-ulp nudges of
  every parameter) have the oracle's tier, and their costs agree within two
  control steps (robot plans) or 1e-3 (push).
- The whole batch's iteration 0: every row the batched launch reports as
  diverged (tier 3) is one the oracle cannot complete either (tier 2 or 3).
- The full CE runs of the 32 push instances (each its own problem, 5
  iterations): the median over instances of the best cost is within 1e-2
  relative of the oracle's (tests/golden/plan_solve_oracle.json, written by
  tests/golden/make_plan_solve_goldens.py from the oracle alone).
"""
import json
import os

import numpy as np
import pytest

from paper_2512_11571_amd import workloads
from parity_util import certify, tier_mismatches

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plan_solve_oracle.json")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    return binding


def _certified(oracle, w, seed, inst, Z):
    r = certify(oracle, w, seed, Z, inst=inst)
    return r["okt"], r["cost"], r["tier"]


def _iteration0(oracle, binding, insts, picks, tag):
    """One batched step; then each picked instance's iteration-0 outcomes against the oracle."""
    with binding.Batch(insts) as B:
        rows = {}
        for k in picks:                                 # the rows the step will draw (theta still at theta_0)
            c = B.instance(k)
            Zd = torch.empty((insts[k]["workload"]["cem"]["pop"], c.D), dtype=torch.float32, device="cuda:0")
            c.cem_sample(0, Zd)
            rows[k] = Zd
        B.step()
        torch.cuda.synchronize()
        got = {}
        for k in picks:
            c = B.instance(k)
            got[k] = (rows[k].cpu().numpy(),) + c.outcomes(insts[k]["workload"]["cem"]["pop"])
    checked = 0
    for k in picks:
        inst = insts[k]
        w = inst["workload"]
        Zh, cg, tg, _ = got[k]
        cem = w["cem"]
        L, _ = oracle.factor_cov(np.diag(np.asarray(cem["cov0_diag"], np.float64)))
        Zr = oracle.sample(inst["seed"], 0, inst["instance"], cem["pop"], np.asarray(cem["mu0"], np.float64), L)
        assert np.array_equal(Zh, Zr), k
        idx = np.random.default_rng(k).choice(cem["pop"], 48, replace=False)
        ok, cr, tr = _certified(oracle, w, inst["seed"], inst["instance"], Zh[idx])
        kind = w["scene"]["kind"]
        assert ok.sum() >= 12, (k, ok.sum())
        assert not tier_mismatches("%s instance %d (%s, H %d, pop %d)" % (tag, k, kind, w["scene"]["horizon"],
                                                                       cem["pop"]),
                                   ok, tg[idx], tr, cg[idx].astype(np.float64), cr, idx)
        same = ok & (tg[idx] == tr) & (tr < 3)
        tol = 2 * w["scene"]["dt"] + 1e-6 if kind != "push" else 1e-3
        assert np.max(np.abs(cg[idx][same] - cr[same])) <= tol, k
        checked += int(ok.sum())
    return checked


def test_batch_iteration0_against_oracle(oracle, binding):
    insts = workloads.batch_instances()
    assert len(insts) == 64
    H = np.array([i["workload"]["scene"]["horizon"] for i in insts])
    kinds = [i["workload"]["scene"]["kind"] for i in insts]
    pp = [k for k in range(64) if kinds[k] == "pickplace"]
    longest = max(pp, key=lambda k: H[k])
    long_pp = [k for k in pp if H[k] >= 2000 and k != longest][:2]
    push = [k for k in range(64) if kinds[k] == "push"][:3]
    picks = [longest] + long_pp + push
    assert H[longest] >= 3500
    # the jittered ramp really moved
    ramps = [b["center"][:2] for b in insts[longest]["workload"]["scene"]["static_boxes"] if b.get("ramp")]
    base = [b["center"][:2] for b in workloads.load("pickplace")["scene"]["static_boxes"] if b.get("ramp")]
    assert ramps != base
    assert _iteration0(oracle, binding, insts, picks, "batch") >= 100


def test_mixed_batch_iteration0_against_oracle(oracle, binding):
    spec = dict(workloads.load("batch_mixed")["batch"])
    insts = workloads.batch_instances(spec)
    kinds = [i["workload"]["scene"]["kind"] for i in insts]
    picks = [kinds.index("push"), kinds.index("pickplace"), kinds.index("movepush")]
    assert _iteration0(oracle, binding, insts, picks, "mixed batch") >= 40


def test_batch_diverged_rows_against_the_oracle(oracle, binding):
    # the configured batch's iteration 0 (141,184 plans of 64 instances, the
    # pools in their launch order): every row the batched launch reports as
    # diverged (tier 3) is one the FP64 oracle cannot complete either (tier 2:
    # an action fails, or tier 3: it diverges too), so no plan that could enter
    # an update is lost to FP32 arithmetic alone
    insts = workloads.batch_instances()
    with binding.Batch(insts) as B:
        B.step()
        torch.cuda.synchronize()
        tiers = [B.instance(k).outcomes(i["workload"]["cem"]["pop"])[1] for k, i in enumerate(insts)]
    n_bad = 0
    for k, (inst, th) in enumerate(zip(insts, tiers)):
        bad = np.nonzero(th == 3)[0]
        if bad.size == 0:
            continue
        n_bad += bad.size
        w, cem = inst["workload"], inst["workload"]["cem"]
        L, _ = oracle.factor_cov(np.diag(np.asarray(cem["cov0_diag"], np.float64)))
        Z = oracle.sample(inst["seed"], 0, inst["instance"], cem["pop"], np.asarray(cem["mu0"], np.float64), L)
        _, tr, _, _ = oracle.rollout(w, inst["seed"], Z[bad], inst=inst["instance"])
        print("batch instance %d (%s, H %d, pop %d): GPU tier-3 rows %s, oracle tiers %s"
              % (k, w["scene"]["kind"], w["scene"]["horizon"], cem["pop"], bad.tolist(), tr.tolist()))
        assert np.all(tr >= 2), (k, list(zip(bad.tolist(), tr.tolist())))
    print("batch iteration 0: %d of %d rows diverged on the GPU" % (n_bad, sum(t.size for t in tiers)))
    assert n_bad <= 1e-3 * sum(t.size for t in tiers)


def test_batch_push_instances_median_best_cost(binding):
    if not os.path.exists(GOLDEN):
        pytest.fail("missing %s (tests/golden/make_plan_solve_goldens.py)" % GOLDEN)
    gold = json.load(open(GOLDEN))["batch_push"]["runs"]
    insts = workloads.batch_instances()
    with binding.Batch(insts) as B:
        res = B.solve(max(i["iters"] for i in insts))
    g, r = [], []
    for inst, out in zip(insts, res):
        if inst["workload"]["scene"]["kind"] != "push":
            continue
        ref = gold[str(inst["instance"])]
        assert out["iters_done"] == ref["iters"]
        g.append(out["best_cost"])
        r.append(ref["best_cost"])
    assert len(g) == 32
    g, r = np.array(g), np.array(r)
    rel = np.abs(g - r) / r
    print("push instances: median best cost GPU %.6f oracle %.6f; per-instance relative gaps: median %.2e, max %.2e"
          % (np.median(g), np.median(r), np.median(rel), rel.max()))
    assert abs(np.median(g) - np.median(r)) <= 1e-2 * np.median(r)
