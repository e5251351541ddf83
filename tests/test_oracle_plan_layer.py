"""Pins of the oracle's plan layer: the controllers, the action sequencing,
the success predicates and the cost count of the robot plans.

Each expected value comes from the definitions, not from the oracle:
- the joint PD law and its torque clamp: a finger (a prismatic joint whose
  mirror twin cancels its reaction on the palm) follows the exact discrete
  recurrence of a PD-driven point mass under semi-implicit Euler;
- the sequencing of Problem 1 (an action ends when it succeeds or times out
  and the next one controls from the following step, t_{0,i+1} = T_i + 1) and
  Problem 2's cost (one per control step while the active action is
  unsuccessful, scaled by dt): scripted plans whose actions all time out
  cost the sum of the timeouts, a move that already holds at the start ends
  at once, and a move ends at the first step whose entering state satisfies
  Eq. 4, read off the state trace;
- the grasp predicates (Eq. 5 and its text) on hand-set finger and object
  poses, decided by interval geometry;
- the smoothstep reference of a move: it starts at the start pose, ends at
  the target at the duration the speed limits give, and has zero speed at
  both ends and 1.5 times the mean speed at its middle.
"""
import copy
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads


@pytest.fixture(scope="module")
def pp():
    return workloads.load("pickplace")


@pytest.fixture(scope="module")
def mp():
    return workloads.load("movepush")


def _steps_to(timeout, dt):
    """The first control-step count n with n * dt >= timeout (the elapsed time of an action in FP64)."""
    n = 0
    while float(n) * dt < timeout:
        n += 1
    return n


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


def test_finger_pd_and_clamp_follow_the_exact_recurrence(oracle, pp):
    # No gravity, no base torques (the base PD gains set to zero), the object
    # far away: only the fingers move, from closed to the open command, and
    # their reactions on the palm cancel, so each finger is a point mass m on
    # its slide:  tau = clamp(inom (wc^2 (r - q) - 2 zeta wc qd), +-inom a_max),
    # qd += h tau / m,  q += h qd  (h = dt / substeps).
    w = copy.deepcopy(pp)
    sc = w["scene"]
    sc["gravity"] = 0.0
    for j in (0, 1, 2):
        sc["robot"]["joints"][j]["inom"] = 0.0
    sc["robot"]["q0"][9] = sc["robot"]["q0"][10] = 0.0
    sc["object"]["pos0"] = [10.0, 10.0, 0.025]
    ct = sc["controller"]
    z = np.array(w["cem"]["mu0"], np.float32)
    z[0:4] = [1.0, -30.0, math.pi, 1.5]          # a move that cannot end within the logged steps
    T = 200
    log = oracle.robot_log(w, 0, z, steps=T, trace_steps=T)
    assert np.all(log["act"] == 0)
    fin = sc["robot"]["joints"][9]
    m, inom = fin["mass"], fin["inom"]
    wc, zeta, amax = ct["omega_c"], ct["zeta"], ct["accel_max"]
    r = ct["finger_open"]
    h = sc["dt"] / sc["substeps"]
    q, qd = 0.0, 0.0
    clamped = 0
    want = []
    for t in range(T):
        for _ in range(sc["substeps"]):
            u = inom * (wc * wc * (r - q) - 2.0 * zeta * wc * qd)
            lim = inom * amax
            tau = max(-lim, min(lim, u))
            clamped += abs(u) > lim
            qd = qd + h * tau / m
            q = q + h * qd
        want.append((q, qd))
    want = np.array(want)
    tr = log["trace"]
    for f in (9, 10):
        assert np.allclose(tr[:, 13 + f], want[:, 0], rtol=0, atol=1e-12)
        assert np.allclose(tr[:, 24 + f], want[:, 1], rtol=0, atol=1e-10)
    assert clamped > 0 and abs(want[-1, 0] - r) < 1e-6          # both regimes, then settled on the command
    # nothing else moved
    q0 = np.array(sc["robot"]["q0"])
    assert np.max(np.abs(tr[:, 13:13 + 9] - q0[:9])) < 1e-12
    assert np.max(np.abs(tr[:, 24:24 + 9])) < 1e-12


def _far_pickplace(pp, horizon=3000):
    w = copy.deepcopy(pp)
    w["scene"]["horizon"] = horizon
    return w


def test_all_timeouts_cost_the_sum_of_the_timeouts_pickplace(oracle, pp):
    w = _far_pickplace(pp)
    sc, ct = w["scene"], w["scene"]["controller"]
    # every action out of reach: two moves 20+ m away, a grasp of an object
    # the robot never comes near, a place 10 m up
    z = np.array([1.0, -20.0, math.pi, 1.5, 0.0, 1.0, 0.0, 0.0,
                  1.0, -40.0, math.pi, 1.5, 1.0, -30.0, 10.0, 0.0], np.float32)
    dt = sc["dt"]
    n = [_steps_to(ct["timeout_move"], dt), _steps_to(ct["timeout_pick"], dt),
         _steps_to(ct["timeout_move"], dt), _steps_to(ct["timeout_place"], dt)]
    ends = np.cumsum(n)
    log = oracle.robot_log(w, 0, z)
    assert list(log["ends"]) == list(ends)
    assert log["ok"] == 0 and log["tier"] == 2
    assert abs(log["cost"] - dt * ends[-1]) < 1e-12
    # t_{0,i+1} = T_i + 1: action i controls exactly the steps [ends[i-1], ends[i])
    want = np.searchsorted(ends, np.arange(sc["horizon"]), side="right")
    assert np.array_equal(log["act"], want)


def test_all_timeouts_cost_the_sum_of_the_timeouts_movepush(oracle, mp):
    w = copy.deepcopy(mp)
    sc, ct = w["scene"], w["scene"]["controller"]
    z = np.array([-0.8, -30.0, math.pi / 2, 1.5, -0.8, -5.0, 10.0, 0.0, 0.3, 0.4, 0.1, 0.0], np.float32)
    dt = sc["dt"]
    ends = np.cumsum([_steps_to(ct["timeout_move"], dt), _steps_to(ct["timeout_push"], dt)])
    log = oracle.robot_log(w, 0, z)
    assert list(log["ends"][:2]) == list(ends) and list(log["ends"][2:]) == [-1, -1]
    assert log["ok"] == 0 and log["tier"] == 2
    assert abs(log["cost"] - dt * ends[-1]) < 1e-12
    assert np.array_equal(log["act"], np.searchsorted(ends, np.arange(sc["horizon"]), side="right"))


def test_a_move_already_at_its_target_ends_before_its_first_step(oracle, pp):
    # Eq. 4 holds on the initial state: the move ends at t = 0 having
    # controlled no step, at no cost; the grasp starts at once
    w = _far_pickplace(pp)
    sc, ct = w["scene"], w["scene"]["controller"]
    q0 = sc["robot"]["q0"]
    z = np.array([q0[0], q0[1], q0[2], 1.0, 0.0, 1.0, 0.0, 0.0,
                  1.0, -40.0, math.pi, 1.5, 1.0, -30.0, 10.0, 0.0], np.float32)
    # the grasp target is the object on table 1, 0.9 m away: out of reach from the start pose
    dt = sc["dt"]
    ends = np.cumsum([0, _steps_to(ct["timeout_pick"], dt), _steps_to(ct["timeout_move"], dt),
                      _steps_to(ct["timeout_place"], dt)])
    log = oracle.robot_log(w, 0, z)
    assert list(log["ends"]) == list(ends)
    assert log["ok"] == 1                      # the move succeeded, nothing else
    assert abs(log["cost"] - dt * ends[-1]) < 1e-12


def test_a_move_ends_at_the_first_step_whose_state_satisfies_eq4(oracle, pp):
    w = _far_pickplace(pp)
    sc, ct = w["scene"], w["scene"]["controller"]
    tgt = (1.0, -1.0, math.pi)
    z = np.array([tgt[0], tgt[1], tgt[2], 1.0, 0.0, 1.0, 0.0, 0.0,
                  1.0, -40.0, math.pi, 1.5, 1.0, -30.0, 10.0, 0.0], np.float32)
    T = sc["horizon"]
    log = oracle.robot_log(w, 0, z, trace_steps=T)
    tr = log["trace"]
    q0 = np.array(sc["robot"]["q0"])
    zt = z.astype(np.float64)

    def eq4(q):        # base within tolerance of the target position and heading
        return (math.hypot(q[0] - zt[0], q[1] - zt[1]) <= ct["base_tol"]
                and abs(_wrap(q[2] - zt[2])) <= ct["yaw_tol"])

    # the state entering step t is the initial state for t = 0, else the state after step t - 1
    entering = [q0] + [tr[t - 1, 13:24] for t in range(1, T)]
    t_s = next(t for t in range(T) if eq4(entering[t]))
    assert t_s > 100
    dt = sc["dt"]
    ends = t_s + np.cumsum([0, _steps_to(ct["timeout_pick"], dt), _steps_to(ct["timeout_move"], dt),
                            _steps_to(ct["timeout_place"], dt)])
    assert list(log["ends"]) == list(ends)
    assert log["ok"] == 1
    assert abs(log["cost"] - dt * ends[-1]) < 1e-12


def test_cost_counts_the_steps_of_unfinished_actions(oracle, pp):
    # on sampled plans: cost = dt * #{t : an action is active at t}, and each
    # action controls the steps between the previous end and its own
    L, _ = oracle.factor_cov(np.diag(np.asarray(pp["cem"]["cov0_diag"], np.float64)))
    Z = oracle.sample(3, 0, 0, 12, np.asarray(pp["cem"]["mu0"], np.float64), L)
    dt, H = pp["scene"]["dt"], pp["scene"]["horizon"]
    tiers = set()
    for z in Z:
        log = oracle.robot_log(pp, 3, z)
        act = log["act"]
        active = int(np.sum(act < 4))
        assert abs(log["cost"] - dt * active) < 1e-9
        e = [x for x in log["ends"] if x >= 0]
        assert e == sorted(e)
        assert np.array_equal(act, np.searchsorted(np.array(e), np.arange(H), side="right"))
        tiers.add(log["tier"])
    assert len(tiers) >= 2


def _rot_to_quat(R):
    w = math.sqrt(max(0.0, 1.0 + R[0, 0] + R[1, 1] + R[2, 2])) / 2.0
    x = math.copysign(math.sqrt(max(0.0, 1.0 + R[0, 0] - R[1, 1] - R[2, 2])) / 2.0, R[2, 1] - R[1, 2])
    y = math.copysign(math.sqrt(max(0.0, 1.0 - R[0, 0] + R[1, 1] - R[2, 2])) / 2.0, R[0, 2] - R[2, 0])
    zz = math.copysign(math.sqrt(max(0.0, 1.0 - R[0, 0] - R[1, 1] + R[2, 2])) / 2.0, R[1, 0] - R[0, 1])
    return np.array([w, x, y, zz])


@pytest.mark.parametrize("qf,y_off,want", [
    # fingers at +-0.02 on a 0.05 m cube centred between them: both overlap it by 5 mm
    (0.02, 0.0, (True, True, True, True)),
    # fingers open wider than the cube: no contact
    (0.04, 0.0, (False, False, True, False)),
    # the cube shifted 30 mm toward the left finger: it touches that finger only, centre outside
    (0.02, 0.03, (True, False, False, False)),
    # shifted 19 mm: centre still inside, the right finger free
    (0.02, 0.019, (True, False, True, False)),
    # fingers nearly closed (inner faces +-5 mm), cube 10 mm off centre: both touch, centre outside
    (0.005, 0.01, (True, True, False, False)),
    (0.005, -0.01, (True, True, False, False)),
])
def test_grasp_predicates_on_hand_set_poses(oracle, pp, qf, y_off, want):
    sc = pp["scene"]
    tree = oracle.make_tree(sc["robot"]["joints"])
    q = np.array(sc["robot"]["q0"], np.float64)
    q[9] = q[10] = qf
    R, p = oracle.tree_fk(tree, q)
    e = sc["robot"]["ee_body"]
    # the fingers' boxes span palm z in [0.06, 0.09] and palm x in +-0.015; the
    # cube (half 0.025) sits at palm z 0.075, aligned with the palm
    centre = p[e] + R[e] @ np.array([0.0, y_off, 0.075])
    got = oracle.grasp_check(pp, q, centre, _rot_to_quat(R[e]))
    assert got == want


def _smooth(x):
    c = min(1.0, max(0.0, x))
    return c * c * (3.0 - 2.0 * c)


@pytest.mark.parametrize("target", [(1.0, 0.0, math.pi, 1.0), (0.2, 0.4, 2.0, 0.7), (1.3, 1.2, -2.8, 3.0)])
def test_move_reference_is_a_smoothstep_of_the_limited_duration(oracle, pp, target):
    # a negative tolerance the base cannot meet keeps the move running to its timeout,
    # so the whole reference is logged; the duration is set by the distance
    # and the clamped speed, or by the turn and the yaw-rate limit
    w = copy.deepcopy(pp)
    sc, ct = w["scene"], w["scene"]["controller"]
    ct["base_tol"] = -1.0
    z = np.array(w["cem"]["mu0"], np.float32)
    z[0:4] = target
    T = 820
    log = oracle.robot_log(w, 0, z, steps=T)
    e0 = int(log["ends"][0])
    assert e0 == _steps_to(ct["timeout_move"], sc["dt"])
    ref = log["qref"]
    q0 = np.array(sc["robot"]["q0"])
    frm = q0[:3]
    zt = z.astype(np.float64)
    to = np.array([zt[0], zt[1], q0[2] + _wrap(zt[2] - q0[2])])
    v = min(ct["base_vmax"], max(ct["base_vmin"], zt[3]))
    dur = max(math.hypot(*(to[:2] - frm[:2])) / v, abs(to[2] - frm[2]) / ct["base_wmax"], sc["dt"])
    dt = sc["dt"]
    tau = np.arange(e0) * dt
    want = frm[None, :] + np.array([_smooth(x) for x in tau / dur])[:, None] * (to - frm)[None, :]
    assert np.allclose(ref[:e0, :3], want, rtol=0, atol=1e-12)
    # the arm holds its start pose during a move, the fingers their open command
    assert np.all(ref[:e0, 3:9] == q0[3:9]) and np.all(ref[:e0, 9:] == ct["finger_open"])
    # shape: at rest at both ends (the first and last step move the reference by
    # 3 (dt / T)^2 of the distance, to first order), peak speed 1.5x the mean at mid-duration
    k = int(math.ceil(dur / dt))
    assert k + 2 < e0
    d = np.linalg.norm(np.diff(ref[:k + 2, :2], axis=0), axis=1) / dt
    mean = math.hypot(*(to[:2] - frm[:2])) / dur
    end = 3.0 * dt / dur * mean
    assert d[0] <= 1.05 * end and d[k - 1] <= 1.05 * end and d[k] == 0.0
    assert abs(d.max() - 1.5 * mean) < 0.01 * mean
    assert abs(np.argmax(d) - k / 2) <= 2
