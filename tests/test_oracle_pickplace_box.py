"""Pins of the oracle's box-obstacle pick-and-place scene (Sec. IV-A setup 2:
the obstacle without its slanted side).

The plan that releases the cube over the obstacle (the initial mean of the
ramp workload) lets the cube slide down the ramp onto Table 2 (psi_g holds),
but leaves it resting on the box's top face: every action succeeds, psi_g
fails, and the cube rests at the top face's height plus its half size minus
the penalty springs' static compression m g / (4 k) (four corners share the
weight).  A plan that goes around the obstacle on its +y side and releases the
cube over Table 2 reaches psi_g in both scenes.
"""
import numpy as np

from paper_2512_11571_amd import workloads

AROUND = [0.06, 0.93, -2.03, 0.9, 0.11, 0.88, -0.04, 0.03, 2.99, 0.8, -2.18, 1.5, 2.59, 0.19, 0.52, 3.4]


def test_box_obstacle_blocks_the_ramp_mode(oracle):
    ramp, box = workloads.load("pickplace_paper"), workloads.load("pickplace_box")
    Z = np.array([workloads.load("pickplace")["cem"]["mu0"], AROUND], np.float32)
    cr, tr, pr, _ = oracle.rollout(ramp, 0, Z)
    cb, tb, pb, _ = oracle.rollout(box, 0, Z)
    sc = box["scene"]
    ob = sc["object"]
    sink = ob["mass"] * sc["gravity"] / (4 * sc["k_contact"])
    # the ramp plan: on Table 2 with the ramp, on the box top without it
    t2 = ramp["scene"]["static_boxes"][1]
    assert tr[0] == 0
    assert abs(pr[0, 2] - (t2["center"][2] + t2["half"][2] + ob["half"][2] - sink)) < 1e-6
    obst = sc["static_boxes"][2]
    assert tb[0] == 1
    assert abs(pb[0, 2] - (obst["center"][2] + obst["half"][2] + ob["half"][2] - sink)) < 1e-6
    assert abs(pb[0, 0] - obst["center"][0]) <= obst["half"][0]
    # the actions are the same and succeed alike: the cost counts their steps
    assert cb[0] == cr[0]
    # around the obstacle: feasible in both scenes
    assert tr[1] == 0 and tb[1] == 0
