"""Batched instances in one persistent launch: every instance's CE run is
bit-identical to running it alone, iteration caps hold, and the autotuner's
choice changes only speed."""
import copy

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    return binding


def _small_batch():
    spec = dict(workloads.load("batch")["batch"])
    spec.update(n_instances=6, horizon=[100, 300], pop=[64, 200], iters={"push": 3, "pickplace": 2}, seed=7)
    return workloads.batch_instances(spec)


def _same(a, b):
    return (a["best_cost"] == b["best_cost"] and a["best_tier"] == b["best_tier"]
            and np.array_equal(a["best_z"], b["best_z"]) and np.array_equal(a["mu"], b["mu"])
            and np.array_equal(a["cov"], b["cov"]))


def test_batched_equals_single_instance_runs(binding):
    insts = _small_batch()
    with binding.Batch(insts) as B:
        res = B.solve(max(i["iters"] for i in insts))
    for inst, r in zip(insts, res):
        assert r["iters_done"] == inst["iters"]
        with binding.Context(inst["workload"], seed=inst["seed"], instance=inst["instance"]) as c:
            s = c.plan_solve(inst["iters"])
        assert _same(r, s), inst["instance"]


def test_autotune_changes_only_speed(binding):
    insts = _small_batch()
    with binding.Batch(insts) as B:
        cfg = B.autotune()
        assert cfg["envs_per_item"] in (32, 64) and cfg["grid"] > 0 and cfg["rollout_us"] > 0
        # the tuner's trial passes are not the CE run's: no counted steps, no iteration advanced
        assert [B.instance(k).env_steps() for k in range(len(insts))] == [0] * len(insts)
        tuned = B.solve(3)
    with binding.Batch(copy.deepcopy(insts)) as B:
        plain = B.solve(3)
    for a, b in zip(tuned, plain):
        assert _same(a, b)


def test_extra_steps_past_the_caps_change_nothing(binding):
    insts = _small_batch()
    with binding.Batch(insts) as B:
        r1 = B.solve(3)
        r2 = B.solve(2)           # every instance is already at its cap
    for a, b in zip(r1, r2):
        assert _same(a, b)


def test_mixed_plans_batched_equal_single_runs(binding):
    # push, pick-and-place and move-and-push instances (three action sequences) in one launch
    spec = dict(workloads.load("batch_mixed")["batch"])
    spec.update(n_instances=6, horizon=[100, 300], pop=[64, 200], iters={"push": 3, "pickplace": 2, "movepush": 2},
                seed=3)
    insts = workloads.batch_instances(spec)
    assert {i["workload"]["scene"]["kind"] for i in insts} == {"push", "pickplace", "movepush"}
    with binding.Batch(insts) as B:
        res = B.solve(3)
        # each instance's context counts the control steps its own rollouts ran
        counted = [B.instance(k).env_steps() for k in range(len(insts))]
    for inst, r, n in zip(insts, res, counted):
        assert r["iters_done"] == inst["iters"]
        w = inst["workload"]
        full = inst["iters"] * w["cem"]["pop"] * w["scene"]["horizon"]
        assert n == full, (inst["instance"], n, full)
        with binding.Context(w, seed=inst["seed"], instance=inst["instance"]) as c:
            s = c.plan_solve(inst["iters"])
            assert c.env_steps() == full
        assert _same(r, s), inst["instance"]
