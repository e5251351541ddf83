"""The two rollout instances for robot scenes: the one compiled for the robot
model (used whenever a scene's robot is the model, so by every other robot
test) and the generic one (any robot; cem_set_robot_specialization(0) forces
it).

- The generic instance against the oracle on the pick-and-place plan: joint
  angles and object position over the first 100 control steps on rows the
  oracle certifies as non-chaotic (1e-3), and full-horizon tier and cost on
  certified rows, at one and at sixteen lanes per environment.
- The two instances against each other on those rows: the same dynamics up
  to rounding, so over 100 steps they stay within half the distance either
  may keep from the oracle.
- A robot that is not the model (one link 10 % heavier, one centre of mass
  off its axis) takes the generic instance and matches the oracle run on the
  same robot.
"""
import copy

import numpy as np
import pytest

from paper_2512_11571_amd import workloads
from parity_util import certify, tier_mismatches

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    return binding


@pytest.fixture
def generic(B):
    B.set_robot_specialization(False)
    try:
        yield
    finally:
        B.set_robot_specialization(True)


def _rows(oracle, w, seed, n):
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(cem["cov0_diag"]))
    return oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)


def _run(B, w, Z, trace_steps=0, lanes=1):
    n = Z.shape[0]
    with B.Context(w, pop=max(n, 64), n_elite=1, lanes=lanes) as c:
        Zd = torch.from_numpy(np.ascontiguousarray(Z)).to("cuda:0")
        if trace_steps:
            tr = torch.empty((n, trace_steps, 35), dtype=torch.float32, device="cuda:0")
            c.rollout_trace(Zd, trace_steps, tr)
            torch.cuda.synchronize()
            return tr.cpu().numpy().astype(np.float64)
        cost = torch.empty(n, dtype=torch.float32, device="cuda:0")
        tier = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        c.rollout_batch(Zd, cost, tier)
        torch.cuda.synchronize()
        return cost.cpu().numpy().astype(np.float64), tier.cpu().numpy()


_MEMO = {}


def _stable_trace_rows(oracle, w, Z):
    key = Z.tobytes()
    if key not in _MEMO:
        t0 = oracle.rollout(w, 0, Z, trace_steps=100)[3]
        t1 = oracle.rollout(w, 0, np.nextafter(Z, np.float32(np.inf)).astype(np.float32), trace_steps=100)[3]
        ok = np.max(np.abs(t0 - t1)[:, :, list(range(7)) + list(range(13, 24))], axis=(1, 2)) < 1e-4
        _MEMO[key] = (t0, ok)
    return _MEMO[key]


def _check_trace(tg, ref):
    assert np.max(np.abs(tg[:, :, 13:24] - ref[:, :, 13:24])) < 1e-3     # joint angles / base position
    assert np.max(np.abs(tg[:, :, 0:3] - ref[:, :, 0:3])) < 1e-3         # object position
    assert np.max(np.abs(tg[:, :, 24:35] - ref[:, :, 24:35])) < 2e-2     # joint velocities


@pytest.mark.parametrize("lanes", [1, 16])
def test_generic_instance_trace_and_outcomes_against_the_oracle(oracle, B, generic, lanes):
    w = workloads.load("pickplace")
    Z = _rows(oracle, w, 0, 64)
    t0, ok = _stable_trace_rows(oracle, w, Z)
    assert ok.sum() >= 32
    _check_trace(_run(B, w, Z[ok], trace_steps=100, lanes=lanes), t0[ok])
    Z = _rows(oracle, w, 1, 128)
    r = certify(oracle, w, 1, Z)
    cg, tg = _run(B, w, Z, lanes=lanes)
    assert not tier_mismatches("generic instance, pickplace seed 1, %d lanes" % lanes, r["okt"], tg, r["tier"], cg,
                               r["cost"])
    same = r["ok"] & (tg == r["tier"]) & (r["tier"] < 3)
    assert same.sum() >= 48
    assert np.max(np.abs(cg[same] - r["cost"][same])) <= 2 * w["scene"]["dt"] + 1e-6


def test_specialised_and_generic_instances_agree(oracle, B):
    w = workloads.load("pickplace")
    Z = _rows(oracle, w, 0, 64)
    t0, ok = _stable_trace_rows(oracle, w, Z)
    ts = _run(B, w, Z[ok], trace_steps=100)
    B.set_robot_specialization(False)
    try:
        tgen = _run(B, w, Z[ok], trace_steps=100)
    finally:
        B.set_robot_specialization(True)
    d_inst = np.max(np.abs(ts[:, :, 13:24] - tgen[:, :, 13:24]))
    d_orac = max(np.max(np.abs(ts[:, :, 13:24] - t0[ok][:, :, 13:24])),
                 np.max(np.abs(tgen[:, :, 13:24] - t0[ok][:, :, 13:24])))
    print("joint angles over 100 steps: specialised vs generic %.2e; either vs the oracle %.2e" % (d_inst, d_orac))
    assert d_inst < 5e-4                                                  # half the bar against the oracle
    assert np.max(np.abs(ts[:, :, 0:3] - tgen[:, :, 0:3])) < 5e-4


def test_a_robot_other_than_the_model_matches_the_oracle(oracle, B):
    w = copy.deepcopy(workloads.load("pickplace"))
    joints = w["scene"]["robot"]["joints"]
    joints[5]["mass"] = joints[5]["mass"] * 1.1
    joints[4]["com"] = [0.004, 0.0, joints[4]["com"][2]]
    Z = _rows(oracle, w, 3, 96)
    r = certify(oracle, w, 3, Z)
    cg, tg = _run(B, w, Z)
    assert not tier_mismatches("modified robot, pickplace seed 3", r["okt"], tg, r["tier"], cg, r["cost"])
    same = r["ok"] & (tg == r["tier"]) & (r["tier"] < 3)
    assert same.sum() >= 32
    assert np.max(np.abs(cg[same] - r["cost"][same])) <= 2 * w["scene"]["dt"] + 1e-6
