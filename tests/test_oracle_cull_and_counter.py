"""Two parts of the oracle that are not physics: the face-axis broadphase of
the box-box tests, and the operation counter behind the FLOP figures.

- The broadphase skips a box pair when one of the six face normals separates
  the boxes.  Separated boxes have no vertex inside each other, so skipping
  them must change nothing: rollouts with the broadphase switched off are
  bit-identical, on sampled rows of every robot scene, in FP64.
- The counter (the oracle's templates run on a counting scalar) tallies + - *
  as 1, fma as 2, / and sqrt as 1, and skips operations fixed by structure
  (on exact 0 / +-1 operands).  Its tallies of single building blocks on
  generic operands equal hand counts of their definitions.
"""
import numpy as np
import pytest

from paper_2512_11571_amd import workloads


def _rows(oracle, w, n, seed):
    """n rows around the configured mean; with an iteration-0 region, half of them from the region."""
    cem = w["cem"]
    L, _ = oracle.factor_cov(np.diag(np.asarray(cem["cov0_diag"], np.float64)))
    Z = oracle.sample(seed, 0, 0, n, np.asarray(cem["mu0"], np.float64), L)
    if cem.get("init_region"):
        Z[: n // 2] = oracle.sample_region(w, seed, 0, n // 2)
    return Z


@pytest.mark.parametrize("name", ["pickplace", "movepush", "pickplace_box", "pickplace_paper"])
def test_face_cull_changes_no_rollout(oracle, name):
    w = workloads.load(name)
    Z = _rows(oracle, w, 96, 5)
    if name == "pickplace":
        Z = np.concatenate([Z, np.asarray([w["cem"]["mu0"]], np.float32)])   # a plan that grasps and places
    try:
        oracle.set_face_cull(True)
        on = oracle.rollout(w, 5, Z, trace_steps=200)
        oracle.set_face_cull(False)
        off = oracle.rollout(w, 5, Z, trace_steps=200)
    finally:
        oracle.set_face_cull(True)
    for a, b in zip(on, off):
        assert np.array_equal(a, b, equal_nan=True)
    # the rows exercise contacts: some plans succeed, some fail
    assert len(set(on[1].tolist())) >= 2


def test_counter_free_body_step(oracle):
    # integrate_free on generic operands (gravity (0, 0, -g): two structural zeros):
    #   R = rotation of q .................................. 27 mul, 12 add
    #   v += h (f / m + g): 1/m, 3 mul, +g (z only), h*, +  ... 1 div, 6 mul, 4 add
    #   w_body = R^T w ..................................... 9 mul, 6 add
    #   L = I w_body ....................................... 3 mul
    #   gyro = R L ......................................... 9 mul, 6 add
    #   rhs = tau - w x gyro ............................... 6 mul, 6 add
    #   R^T rhs, / I ....................................... 9 mul, 6 add, 3 div
    #   w += h R dw ........................................ 12 mul, 9 add
    #   p += h v ........................................... 3 mul, 3 add
    #   h/2; dq = (0, w) x q ............................... 1 mul; 12 mul, 8 add
    #   q + (h/2) dq ....................................... 4 mul, 4 add
    #   1 / sqrt(|q|^2), q * inv ........................... 8 mul, 3 add, 1 sqrt, 1 div
    c = oracle.count_block(0)
    assert (c["add"], c["mul"], c["fma"], c["div"], c["sqrt"], c["trans"]) == (67, 109, 0, 5, 1, 0)
    assert c["flops"] == 182


def test_counter_penalty_force(oracle):
    # normal (0.6, 0, 0.8): its zero y component makes the y products structural
    #   v_rel = vA - vB ..................... 3 add
    #   v_n = n . v_rel ..................... 2 mul, 1 add
    #   f_n = max(0, k d - c v_n) ........... 2 mul, 1 add
    #   v_t = v_rel - v_n n ................. 2 mul, 2 add
    #   sqrt(|v_t|^2 + eps^2) ............... 4 mul, 3 add, 1 sqrt
    #   s = -(mu f_n) / denom ............... 1 mul, 1 div
    #   f_n n + s v_t ....................... 5 mul, 2 add
    c = oracle.count_block(1)
    assert (c["add"], c["mul"], c["fma"], c["div"], c["sqrt"], c["trans"]) == (12, 16, 0, 1, 1, 0)


def test_counter_small_blocks(oracle):
    c = oracle.count_block(2)            # cross product: 6 mul, 3 add
    assert (c["add"], c["mul"], c["flops"]) == (3, 6, 9)
    c = oracle.count_block(3)            # rotation of a quaternion: 3 x (3 mul, 2 add) + 6 x (3 mul, 1 add)
    assert (c["add"], c["mul"], c["flops"]) == (12, 27, 39)
