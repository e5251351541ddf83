"""Pins of the oracle's initial distribution phi(theta^0) as a region (Sec.
III-B: iteration 0 uniform inside each parameter's region) and of the n_env
schedule (Sec. IV-A, "Algorithm setting": 3000 falling linearly to 300 by
iteration 10, constant afterwards).

  - every row lies in its region: box dimensions within [lo, hi], ring pairs
    within their radii;
  - the law: the box coordinates, the ring's squared radius (the area
    fraction) and its angle are uniform (Kolmogorov-Smirnov at the 1 % level);
  - the uniforms are the Philox words behind iteration 0's normals: on a unit
    box they are recovered from the Box-Muller normals by inverting the
    transform, u_a = exp(-(n0^2 + n1^2) / 2), u_b = atan2(n1, n0) / (2 pi);
    a ring's point follows from those uniforms by the area law and the angle
    2 pi u measured counter-clockwise from +x;
  - rows do not depend on the population size;
  - the schedule's values at the paper's numbers.
"""
import copy
import math

import numpy as np
import pytest

from paper_2512_11571_amd import workloads


@pytest.fixture(scope="module")
def pp():
    return workloads.load("pickplace_paper")


def _ks(u):
    u = np.sort(np.asarray(u, np.float64))
    n = u.size
    return max(np.max(np.arange(1, n + 1) / n - u), np.max(u - np.arange(n) / n))


def test_rows_lie_in_their_regions_with_the_uniform_law(oracle, pp):
    reg = pp["cem"]["init_region"]
    n = 4000
    Z = oracle.sample_region(pp, 5, 0, n).astype(np.float64)
    ring_dims = set()
    for g in reg["rings"]:
        d = g["dim"]
        ring_dims |= {d, d + 1}
        cx, cy = g["center"]
        r0, r1 = g["radius"]
        x, y = Z[:, d] - cx, Z[:, d + 1] - cy
        rad = np.hypot(x, y)
        assert np.all(rad >= r0 * (1 - 1e-6)) and np.all(rad <= r1 * (1 + 1e-6))
        area = (rad ** 2 - r0 ** 2) / (r1 ** 2 - r0 ** 2)
        ang = np.mod(np.arctan2(y, x), 2 * np.pi) / (2 * np.pi)
        assert _ks(np.clip(area, 0, 1)) < 1.63 / math.sqrt(n)
        assert _ks(ang) < 1.63 / math.sqrt(n)
    for d in range(Z.shape[1]):
        if d in ring_dims:
            continue
        lo, hi = reg["lo"][d], reg["hi"][d]
        lo32, hi32 = np.float32(lo), np.float32(hi)
        assert np.all(Z[:, d] >= lo32) and np.all(Z[:, d] <= hi32)
        assert _ks((Z[:, d] - lo) / (hi - lo)) < 1.63 / math.sqrt(n)


def test_uniforms_are_the_words_behind_the_iteration0_normals(oracle, pp):
    w = copy.deepcopy(pp)
    D = 16
    w["cem"]["init_region"] = {"lo": [0.0] * D, "hi": [1.0] * D, "rings": []}
    n = 64
    U = oracle.sample_region(w, 9, 2, n).astype(np.float64)
    N = oracle.sample(9, 0, 2, n, np.zeros(D), np.eye(D)).astype(np.float64)
    for h in range(0, D, 2):
        n0, n1 = N[:, h], N[:, h + 1]
        ua = np.exp(-(n0 * n0 + n1 * n1) / 2)
        ub = np.mod(np.arctan2(n1, n0), 2 * np.pi) / (2 * np.pi)
        assert np.max(np.abs(U[:, h] - ua)) < 1e-5
        # the angle's uniform is defined modulo 1
        dub = np.abs(U[:, h + 1] - ub)
        assert np.max(np.minimum(dub, 1 - dub)) < 1e-5
    # a ring on (4, 5) takes its radius from u_4 (by area) and its angle,
    # counter-clockwise from +x, from u_5
    w["cem"]["init_region"]["rings"] = [{"dim": 4, "center": [0.5, -2.0], "radius": [1.0, 2.0]}]
    R = oracle.sample_region(w, 9, 2, n).astype(np.float64)
    r = np.sqrt(1.0 + 3.0 * U[:, 4])
    assert np.max(np.abs(R[:, 4] - (0.5 + r * np.cos(2 * np.pi * U[:, 5])))) < 1e-5
    assert np.max(np.abs(R[:, 5] - (-2.0 + r * np.sin(2 * np.pi * U[:, 5])))) < 1e-5
    assert np.array_equal(np.delete(R, [4, 5], 1), np.delete(U, [4, 5], 1))


def test_rows_do_not_depend_on_the_population(oracle, pp):
    a = oracle.sample_region(pp, 3, 1, 1000)
    b = oracle.sample_region(pp, 3, 1, 77)
    assert np.array_equal(a[:77], b)
    c = oracle.sample_region(pp, 3, 2, 77)
    assert not np.array_equal(b, c)


def test_schedule_values(oracle, pp):
    n = [oracle.n_env_at(pp, j) for j in range(25)]
    assert n[0] == 3000 and n[10] == 300 and all(v == 300 for v in n[10:])
    assert n[5] == 1650 and n[1] == 2730
    assert all(a > b for a, b in zip(n[:10], n[1:11]))
    plain = workloads.load("pickplace")
    assert all(oracle.n_env_at(plain, j) == plain["cem"]["pop"] for j in range(12))
