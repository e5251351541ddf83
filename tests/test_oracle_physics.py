"""Pins of the oracle's dynamics f (Problem 1, Eq. 1b) against closed forms.

The paper runs its rollouts in a GPU physics engine; the oracle writes the
dynamics out (free bodies, penalty contact with regularised Coulomb friction,
semi-implicit Euler).  These tests tie it to results that do not come from the
oracle: exact discrete recurrences, textbook rigid-body and friction results,
and brute-force geometry.
"""
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads

G = 9.81
ID = [1.0, 0.0, 0.0, 0.0]


def test_free_fall_exact_discrete(oracle):
    h, n = 1e-3, 500
    tr = oracle.box_sim([0.1] * 3, 1.0, [0, 0, 5.0], ID, [0, 0, 0], [0, 0, 0], [0, 0, -G],
                        1e4, 100, 0.5, 0.01, h, False, n)
    k = np.arange(1, n + 1)
    # semi-implicit Euler: v_n = -g n h, z_n = z0 - g h^2 n (n + 1) / 2
    assert np.allclose(tr[:, 9], -G * k * h, rtol=0, atol=1e-12)
    assert np.allclose(tr[:, 2], 5.0 - G * h * h * k * (k + 1) / 2, rtol=0, atol=1e-12)
    assert np.all(tr[:, [0, 1, 7, 8, 10, 11, 12]] == 0.0)


def test_resting_spring_damper_exact_recurrence(oracle):
    # A box pressed 0.5 mm into the plane, flat: four identical corner
    # contacts act as one spring 4k and damper 4c on the COM height:
    #   v+ = v + h ((4k (he - z) - 4c v) / m - g),  z+ = z + h v+
    he, m, k, c, h, n = 0.1, 1.0, 1e4, 100.0, 1.25e-3, 400
    z0 = he - 5e-4
    tr = oracle.box_sim([he] * 3, m, [0, 0, z0], ID, [0, 0, 0], [0, 0, 0], [0, 0, -G],
                        k, c, 0.5, 0.01, h, True, n)
    z, v = z0, 0.0
    want = []
    for _ in range(n):
        v = v + h * ((4 * k * (he - z) - 4 * c * v) / m - G)
        z = z + h * v
        want.append(z)
    assert np.max(np.abs(tr[:, 2] - np.array(want))) < 1e-14
    # settles at the resting penetration m g / (4 k) = 0.245 mm
    assert abs((he - tr[-1, 2]) - m * G / (4 * k)) < 1e-7


def test_torque_free_axisymmetric_top_precession(oracle):
    # Body-frame angular velocity of an axisymmetric body (I1 = I2 != I3)
    # precesses about the symmetry axis at Omega = (I3 - I1) / I1 * w3.
    hx, hz = 0.1, 0.05       # box: I1 = I2 = m (hx^2 + hz^2)/3, I3 = 2 m hx^2 / 3
    m = 1.0
    I1 = m * (hx * hx + hz * hz) / 3
    I3 = m * (2 * hx * hx) / 3
    w0 = np.array([0.3, 0.0, 5.0])
    T = 1.0
    errs = []
    for h in (1e-4, 5e-5):
        n = int(round(T / h))
        tr = oracle.box_sim([hx, hx, hz], m, [0, 0, 0], ID, [0, 0, 0], w0, [0, 0, 0],
                            0, 0, 0, 0.01, h, False, n)
        q = tr[-1, 3:7]
        w = tr[-1, 10:13]
        R = _quat_mat(q)
        wb = R.T @ w
        Omega = (I3 - I1) / I1 * w0[2]
        ang = math.atan2(wb[1], wb[0])
        want = Omega * T  # Euler's equations: d/dt (w1 + i w2) = i Omega (w1 + i w2)
        errs.append(abs(math.remainder(ang - want, 2 * math.pi)))
    assert errs[0] < 2e-2
    assert errs[1] < 0.65 * errs[0]     # first order in h


def test_angular_momentum_drift_first_order(oracle):
    he = [0.15, 0.1, 0.05]
    m = 2.0
    I = np.array([m * (he[1] ** 2 + he[2] ** 2), m * (he[0] ** 2 + he[2] ** 2), m * (he[0] ** 2 + he[1] ** 2)]) / 3
    w0 = np.array([1.0, 2.0, 0.5])
    drift = []
    for h in (2e-4, 1e-4):
        n = int(round(0.5 / h))
        tr = oracle.box_sim(he, m, [0, 0, 0], ID, [0, 0, 0], w0, [0, 0, 0], 0, 0, 0, 0.01, h, False, n)
        R = _quat_mat(tr[-1, 3:7])
        L_end = R @ (I * (R.T @ tr[-1, 10:13]))
        L0 = I * w0
        drift.append(np.linalg.norm(L_end - L0) / np.linalg.norm(L0))
    assert drift[0] < 1e-2
    assert 0.35 < drift[1] / drift[0] < 0.65


def _incline(oracle, theta_deg, mu, T, h=1e-3, eps_v=0.01):
    th = math.radians(theta_deg)
    g = [G * math.sin(th), 0.0, -G * math.cos(th)]   # plane tilted: slope along +x
    he, m, k = 0.1, 1.0, 1e4
    z0 = he - m * G * math.cos(th) / (4 * k)
    n = int(round(T / h))
    return oracle.box_sim([he] * 3, m, [0, 0, z0], ID, [0, 0, 0], [0, 0, 0], g, k, 100.0, mu, eps_v, h, True, n), h


def test_incline_sticks_with_regularised_creep(oracle):
    # tan(10 deg) < 0.5: stick; regularised friction creeps at
    # v_ss = eps_v r / sqrt(1 - r^2), r = tan(theta) / mu   (3.77 mm/s)
    tr, h = _incline(oracle, 10.0, 0.5, 2.0)
    r = math.tan(math.radians(10.0)) / 0.5
    v_ss = 0.01 * r / math.sqrt(1 - r * r)
    v_late = tr[-200:, 7].mean()
    assert abs(v_late - v_ss) < 0.03 * v_ss
    assert tr[-1, 0] < v_ss * 2.0 + 1e-3   # displacement bounded by creep plus transient


def test_incline_slides_at_coulomb_acceleration(oracle):
    # tan(30 deg) > 0.5: a -> g (sin theta - mu cos theta) = 0.657 m/s^2
    tr, h = _incline(oracle, 30.0, 0.5, 2.0)
    th = math.radians(30.0)
    a_want = G * (math.sin(th) - 0.5 * math.cos(th))
    i0, i1 = 1000, 1999
    a = (tr[i1, 7] - tr[i0, 7]) / ((i1 - i0) * h)
    assert abs(a - a_want) < 0.01 * a_want


def test_sphere_box_hand_cases(oracle):
    he = [0.1, 0.1, 0.1]
    # sphere of radius 0.1 centred 0.05 in front of the +x face: depth 0.05, n = -x
    ct = oracle.sphere_box([0.15, 0, 0], 0.1, [0, 0, 0], ID, he)
    assert np.allclose(ct[:3], [0.1, 0, 0]) and np.allclose(ct[3:6], [-1, 0, 0]) and abs(ct[6] - 0.05) < 1e-15
    # separated
    assert oracle.sphere_box([0.31, 0, 0], 0.1, [0, 0, 0], ID, he) is None
    # near an edge: closest point is the edge point (0.1, 0.1, 0)
    c = np.array([0.15, 0.15, 0.0])
    ct = oracle.sphere_box(c, 0.1, [0, 0, 0], ID, he)
    dist = math.hypot(0.05, 0.05)
    assert abs(ct[6] - (0.1 - dist)) < 1e-15 and np.allclose(ct[3:6], [-math.sqrt(0.5), -math.sqrt(0.5), 0])
    # rotated box (45 deg about z), sphere on the world x axis hits a vertical edge
    q = [math.cos(math.pi / 8), 0, 0, math.sin(math.pi / 8)]
    ct = oracle.sphere_box([0.2, 0, 0.0], 0.1, [0, 0, 0], q, he)
    assert abs(ct[6] - (0.1 - (0.2 - 0.1 * math.sqrt(2)))) < 1e-12
    assert np.allclose(ct[3:6], [-1, 0, 0], atol=1e-12)
    # centre inside the box: nearest face +y at distance 0.02
    ct = oracle.sphere_box([0.0, 0.08, 0.0], 0.05, [0, 0, 0], ID, he)
    assert np.allclose(ct[3:6], [0, -1, 0]) and abs(ct[6] - 0.07) < 1e-15


def test_box_box_depth_matches_brute_force_sdf(oracle):
    rng = np.random.default_rng(0)
    heB = np.array([0.3, 0.2, 0.15])
    # densely sampled surface of B (in its own frame) for a brute-force distance
    g = np.linspace(-1, 1, 161)
    pts = []
    for ax in range(3):
        o = [a for a in range(3) if a != ax]
        U, V = np.meshgrid(g, g)
        for s in (-1, 1):
            P = np.zeros((U.size, 3))
            P[:, ax] = s * heB[ax]
            P[:, o[0]] = U.ravel() * heB[o[0]]
            P[:, o[1]] = V.ravel() * heB[o[1]]
            pts.append(P)
    surf = np.concatenate(pts)
    n_checked = 0
    for _ in range(40):
        qB = rng.normal(size=4); qB /= np.linalg.norm(qB)
        qA = rng.normal(size=4); qA /= np.linalg.norm(qA)
        pB = rng.normal(size=3) * 0.1
        pA = pB + rng.normal(size=3) * 0.2
        heA = rng.uniform(0.05, 0.2, size=3)
        cts = oracle.box_box(pA, qA, heA, pB, qB, heB)
        RB = _quat_mat(qB)
        for row in cts:
            x, n, d = row[:3], row[3:6], row[6]
            assert abs(np.linalg.norm(n) - 1) < 1e-12 and d > 0
            xb = RB.T @ (x - pB)
            dmin = np.min(np.linalg.norm(surf - xb[None, :], axis=1))
            assert abs(dmin - d) < 2.5e-3      # grid spacing 2/160 of the half extents
            # moving the vertex out along n by d puts it on B's surface
            xo = RB.T @ (x + d * n - pB)
            assert np.max(np.abs(xo) - heB) < 1e-12 and np.min(np.abs(np.abs(xo) - heB)) < 1e-12
            n_checked += 1
    assert n_checked > 20


def _quat_mat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# ---- the push plan --------------------------------------------------------

@pytest.fixture(scope="module")
def push():
    return workloads.load("push")


def test_push_cost_when_nothing_moves(oracle, push):
    # zero speed: the box rests, cost = |goal - start| + w dt H exactly
    g = oracle.draw_instance(push, 4)
    cost, tier, pose, _ = oracle.rollout(push, 4, np.array([[0.3, 0.0, 0.0], [0.0, 0.0, -1.0]], np.float32))
    d = math.hypot(g[0], g[1])
    sc = push["scene"]
    want = d + sc["goal"]["time_weight"] * sc["dt"] * sc["horizon"]
    assert np.all(tier == 0)
    assert np.allclose(cost, want, rtol=0, atol=1e-9)


def test_push_goal_draw_ranges(oracle, push):
    rho, phi = [], []
    for s in range(400):
        g = oracle.draw_instance(push, s)
        rho.append(math.hypot(g[0], g[1]))
        phi.append(math.atan2(g[1], g[0]))
    go = push["scene"]["goal"]
    assert go["rho"][0] <= min(rho) and max(rho) <= go["rho"][1]
    assert go["phi"][0] <= min(phi) and max(phi) <= go["phi"][1]
    assert np.std(rho) > 0.1 and np.std(phi) > 0.4


def test_push_symmetric_push_stays_on_axis(oracle, push):
    _, _, pose, tr = oracle.rollout(push, 0, np.array([[0.0, 0.0, 1.0]], np.float32), trace_steps=200)
    assert np.max(np.abs(tr[0, :, 1])) < 1e-9             # y
    assert np.max(np.abs(tr[0, :, [4, 6]])) < 1e-9        # roll and yaw quaternion parts


def test_push_steady_speed_penetration_and_slide(oracle, push):
    # pushed at 1 m/s: the box moves with the pusher, the pusher contact carries
    # the friction mu m g (penetration mu m g / k = 0.49 mm), and after the
    # pusher stops the box slides v^2 / (2 mu g) = 0.102 m (+ O(eps_v)).
    _, _, _, tr = oracle.rollout(push, 0, np.array([[0.0, 0.0, 1.0]], np.float32), trace_steps=200)
    x, v = tr[0, :, 0], tr[0, :, 7]
    assert abs(v[60:99].mean() - 1.0) < 2e-3
    # pusher centre at x = -0.35 + t, radius 0.1; box face at x - 0.1
    t = (np.arange(200) + 1) * 0.01
    gap = (x[60:99] - 0.1) - (-0.35 + t[60:99] + 0.1)
    assert abs(-gap.mean() - 0.5 * 9.81 / 1e4) < 5e-5
    slide = x[-1] - x[99]
    assert abs(slide - 1.0 / (2 * 0.5 * 9.81)) < 0.01
