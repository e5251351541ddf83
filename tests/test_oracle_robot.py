"""Pins of the oracle's articulated dynamics, IK and the pick-and-place plan.

ABA (forward dynamics) against the joint-space equation M(q) qdd = tau - bias
built from a different algorithm (RNEA and its unit-acceleration columns),
closed-form pendulum dynamics and mass matrices, energy drift of a passive
chain, IK against forward kinematics of known configurations, the incline
law on the scene's tilted ramp, and the scripted plan at its initial mean.
"""
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

G = 9.81


@pytest.fixture(scope="module")
def pp():
    return workloads.load("pickplace")


@pytest.fixture(scope="module")
def robot_tree(oracle, pp):
    return oracle.make_tree(pp["scene"]["robot"]["joints"])


def test_aba_matches_mass_matrix_solve(oracle, robot_tree):
    rng = np.random.default_rng(0)
    n = robot_tree.n
    for _ in range(20):
        q = rng.uniform(-2, 2, n)
        qd = rng.normal(size=n)
        tau = rng.normal(size=n) * 5
        fext = rng.normal(size=(n, 6))
        qdd = oracle.tree_aba(robot_tree, q, qd, tau, fext)
        M = oracle.tree_crba(robot_tree, q)
        bias = oracle.tree_rnea(robot_tree, q, qd, np.zeros(n), fext)
        want = np.linalg.solve(M, tau - bias)
        assert np.allclose(qdd, want, rtol=1e-9, atol=1e-9 * np.max(np.abs(want)))
        assert np.allclose(M, M.T, atol=1e-12)
        assert np.all(np.linalg.eigvalsh(M) > 0)


def _link(type_, axis, parent, origin, mass, com, half):
    return dict(type=type_, axis=axis, parent=parent, origin=origin, mass=mass, com=com, half=half)


def test_single_pendulum_closed_form(oracle):
    # revolute about +y, a thin box of mass m whose COM is at distance l below
    # the axis at q = 0 swinging in the x-z plane: I th'' = -m g l sin(th)
    m, l, hz = 2.0, 0.7, 0.05
    t = oracle.make_tree([_link(0, 1, -1, [0, 0, 0], m, [0, 0, -l], [0.01, 0.01, hz])])
    Ic = m * (0.01 ** 2 + hz ** 2) / 3
    I = Ic + m * l * l
    for th in (0.3, 1.2, -2.5):
        qdd = oracle.tree_aba(t, [th], [0.7], [0.0])
        assert abs(qdd[0] - (-m * G * l * math.sin(th) / I)) < 1e-12


def test_double_pendulum_mass_matrix_closed_form(oracle):
    m1, m2, l1, c1, c2 = 1.5, 0.8, 0.6, 0.3, 0.25
    h1, h2 = (0.02, 0.02, 0.3), (0.02, 0.02, 0.25)
    t = oracle.make_tree([_link(0, 1, -1, [0, 0, 0], m1, [0, 0, c1], list(h1)),
                          _link(0, 1, 0, [0, 0, l1], m2, [0, 0, c2], list(h2))])
    I1 = m1 * (h1[0] ** 2 + h1[2] ** 2) / 3
    I2 = m2 * (h2[0] ** 2 + h2[2] ** 2) / 3
    for q2 in (0.0, 0.9, -2.0):
        M = oracle.tree_crba(t, [0.4, q2])
        cq = math.cos(q2)
        M11 = I1 + I2 + m1 * c1 * c1 + m2 * (l1 * l1 + c2 * c2 + 2 * l1 * c2 * cq)
        M12 = I2 + m2 * (c2 * c2 + l1 * c2 * cq)
        M22 = I2 + m2 * c2 * c2
        assert np.allclose(M, [[M11, M12], [M12, M22]], rtol=1e-12, atol=1e-14)


def _energy(oracle, tree, q, qd):
    M = oracle.tree_crba(tree, q)
    R, p = oracle.tree_fk(tree, q)
    pe = 0.0
    for j in range(tree.n):
        com = R[j] @ np.array(tree.com[j][:]) + p[j]
        pe += tree.mass[j] * G * com[2]
    return 0.5 * qd @ M @ qd + pe


def test_passive_arm_energy_drift_first_order(oracle, pp):
    # the six arm links alone on a fixed base, swinging under gravity
    J = pp["scene"]["robot"]["joints"][3:9]
    arm = []
    for i, j in enumerate(J):
        d = dict(j)
        d["parent"] = i - 1
        arm.append(d)
    t = oracle.make_tree(arm)
    q0 = np.array([0.3, 0.8, -0.6, 0.4, 1.0, 0.2])
    qd0 = np.zeros(6)
    E0 = _energy(oracle, t, q0, qd0)
    drift = []
    for h in (2e-4, 1e-4):
        n = int(round(0.5 / h))
        q, qd = oracle.tree_sim(t, q0, qd0, G, h, n)
        drift.append(abs(_energy(oracle, t, q[-1], qd[-1]) - E0))
    assert drift[0] < 0.05 * abs(E0) + 0.05
    assert 0.3 < drift[1] / drift[0] < 0.7


def test_ik_reaches_forward_kinematics_targets(oracle, pp):
    rng = np.random.default_rng(1)
    q0 = np.array(pp["scene"]["robot"]["q0"])
    tree = oracle.make_tree(pp["scene"]["robot"]["joints"])
    ee = pp["scene"]["robot"]["ee_body"]
    off = np.array(pp["scene"]["robot"]["ee_offset"])
    for _ in range(10):
        qt = q0.copy()
        qt[3:9] += rng.uniform(-0.5, 0.5, 6)
        R, p = oracle.tree_fk(tree, qt)
        pt, Rt = p[ee] + R[ee] @ off, R[ee]
        qs = qt.copy()
        qs[3:9] += rng.uniform(-0.15, 0.15, 6)
        qo, pe, Re = oracle.ik(pp, qs, pt, Rt)
        assert np.linalg.norm(pe - pt) < 1e-6
        assert np.linalg.norm(Re - Rt) < 1e-6
        assert np.all(qo[:3] == qs[:3]) and np.all(qo[9:] == qs[9:])


def test_object_slides_down_the_ramp_at_coulomb_acceleration(oracle, pp):
    # the scene's 15 degree ramp, friction 0.2 < tan 15: a = g (sin - mu cos)
    sc = pp["scene"]
    ramp = [b for b in sc["static_boxes"] if b.get("ramp")][0]
    th = ramp["pitch"]
    c = np.array(ramp["center"])
    # a point on the ramp top, 0.15 m down-slope from its upper edge
    up = np.array([math.cos(th), 0.0, -math.sin(th)])       # down-slope direction
    nrm = np.array([math.sin(th), 0.0, math.cos(th)])      # outward normal of the top face
    top_hi = c + ramp["half"][2] * nrm - ramp["half"][0] * up
    he = sc["object"]["half"][2]
    m = sc["object"]["mass"]
    pen = m * G * math.cos(th) / (4 * sc["k_contact"])
    p0 = top_hi + 0.15 * up + (he - pen) * nrm
    q0 = [math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]      # object aligned with the slope
    h = sc["dt"] / sc["substeps"]
    tr = oracle.object_sim(pp, p0, q0, [0, 0, 0], 1000)
    v = tr[:, 7:10] @ up
    # late window: v >> eps_v, so the regularised friction is within 0.2% of Coulomb's
    a = (v[999] - v[600]) / (399 * h)
    a_want = G * (math.sin(th) - sc["mu_ramp"] * math.cos(th))
    assert abs(a - a_want) < 0.01 * a_want
    assert np.all(np.abs(tr[:, 1]) < 1e-9)                  # stays in its plane


def test_pick_place_plan_at_initial_mean_is_feasible(oracle, pp):
    mu = np.array(pp["cem"]["mu0"], np.float32)[None, :]
    cost, tier, pose, tr = oracle.rollout(pp, 0, mu, trace_steps=pp["scene"]["horizon"])
    assert tier[0] == 0
    t2 = pp["scene"]["static_boxes"][pp["scene"]["goal_static"]]
    assert abs(pose[0, 0] - t2["center"][0]) <= t2["half"][0]
    # picked: the object leaves the table top while the plan runs
    assert tr[0, :, 2].max() > 0.5
    assert 0 < cost[0] < pp["scene"]["horizon"] * pp["scene"]["dt"]
