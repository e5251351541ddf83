"""Writes the mobile-manipulator workloads (pickplace.json, movepush.json, and
the paper-setting variants pickplace_paper.json, pickplace_box.json, and the
domain-randomised movepush_dr.json).

All use the same synthetic 11-joint robot: a holonomic base (x and y
prismatic joints on massless bodies, then yaw), a six-joint arm and two
prismatic fingers on the palm.  Geometry is stated in metres, masses in kg.
A "measurement" block already in a file (the FLOP count written by the oracle's
counter) is kept.

    python paper_2512_11571_amd/configs/make_robot_configs.py
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))

JOINTS = [
    dict(name="base_x", inom=24.0, type=1, axis=0, parent=-1, origin=[0, 0, 0], mass=0.0, com=[0, 0, 0],
         half=[0, 0, 0], collide=0),
    dict(name="base_y", inom=24.0, type=1, axis=1, parent=0, origin=[0, 0, 0], mass=0.0, com=[0, 0, 0],
         half=[0, 0, 0], collide=0),
    dict(name="base_yaw", inom=1.6, type=0, axis=2, parent=1, origin=[0, 0, 0], mass=20.0, com=[0, 0, 0.2],
         half=[0.3, 0.25, 0.15], collide=1),
    dict(name="shoulder_yaw", inom=0.2, type=0, axis=2, parent=2, origin=[0.2, 0, 0.35], mass=1.0,
         com=[0, 0, 0.05], half=[0.05, 0.05, 0.05], collide=0),
    dict(name="shoulder_pitch", inom=0.35, type=0, axis=1, parent=3, origin=[0, 0, 0.1], mass=1.0,
         com=[0, 0, 0.175], half=[0.04, 0.04, 0.175], collide=0),
    dict(name="elbow", inom=0.25, type=0, axis=1, parent=4, origin=[0, 0, 0.35], mass=0.8, com=[0, 0, 0.175],
         half=[0.035, 0.035, 0.175], collide=0),
    dict(name="wrist_roll", inom=0.005, type=0, axis=2, parent=5, origin=[0, 0, 0.35], mass=0.4,
         com=[0, 0, 0.05], half=[0.03, 0.03, 0.05], collide=0),
    dict(name="wrist_pitch", inom=0.0045, type=0, axis=1, parent=6, origin=[0, 0, 0.1], mass=0.3,
         com=[0, 0, 0.025], half=[0.03, 0.03, 0.025], collide=0),
    dict(name="ee_roll", inom=0.001, type=0, axis=2, parent=7, origin=[0, 0, 0.05], mass=0.2, com=[0, 0, 0.02],
         half=[0.03, 0.05, 0.02], collide=0),
    dict(name="finger_l", inom=0.1, type=1, axis=1, parent=8, origin=[0, 0, 0.04], mass=0.1,
         com=[0, 0.01, 0.035], half=[0.015, 0.01, 0.015], collide=2),
    dict(name="finger_r", inom=0.1, type=1, axis=4, parent=8, origin=[0, 0, 0.04], mass=0.1,
         com=[0, -0.01, 0.035], half=[0.015, 0.01, 0.015], collide=2),
]
TUCK = [0.0, -0.3, 2.2, 0.0, 1.2, 0.0]   # arm joints at the start
CONTROLLER = {"omega_c": 60.0, "zeta": 1.0, "ik_iters": 30, "ik_lambda": 0.05,
              "base_vmin": 0.1, "base_vmax": 1.5, "base_wmax": 1.0, "base_tol": 0.05, "yaw_tol": 0.1, "ee_tol": 0.02,
              "t_approach": 1.0, "t_descend": 0.75, "t_close": 0.5, "t_lift": 0.75, "t_transfer": 1.0,
              "t_release": 0.5, "timeout_move": 4.0, "timeout_pick": 3.5, "timeout_place": 2.0,
              "joint_speed_max": 2.0, "accel_max": 100.0, "pregrasp": 0.2, "finger_open": 0.04,
              "finger_closed": 0.015}


def pickplace():
    t15 = math.radians(15.0)
    # ramp plate: top surface from (2.0, 0.48) down to (2.6, 0.4) = table 2's top
    # edge, 1.0 m wide (y in [-0.5, 0.5]), 0.8 m thick, pitched 15 degrees about y
    thick = 0.8
    ltop = 0.6 / math.cos(t15)
    top_c = (2.3, 0.0, 0.4 + 0.3 * math.tan(t15))
    cx = top_c[0] - math.sin(t15) * thick / 2
    cz = top_c[2] - math.cos(t15) * thick / 2
    return {
        "name": "pickplace",
        "description": "Plain CEM, mobile manipulator move-pick-move-place over a 15 degree ramp obstacle: holonomic "
                       "base (3 DOF), 6-DOF arm by ABA with joint PD, two-box parallel gripper, 0.05 m 0.2 kg box "
                       "object; 4 actions x 4 params = 16 params; pop 1024, 64 elites, 10 iterations; dt 0.005 s, "
                       "2000 steps",
        "scene": {
            "kind": "pickplace", "dt": 0.005, "substeps": 5, "horizon": 2000,
            "gravity": 9.81, "k_contact": 10000.0, "c_contact": 10.0, "eps_v": 0.02,
            "mu_ground": 0.5, "mu_tool": 0.8, "mu_static": 0.5, "mu_ramp": 0.2,
            "object": {"half": [0.025, 0.025, 0.025], "mass": 0.2, "pos0": [0.25, 0.0, 0.425], "yaw0": 0.0},
            "static_boxes": [
                {"name": "table1", "center": [0.0, 0.0, 0.2], "half": [0.4, 0.4, 0.2]},
                {"name": "table2", "center": [3.0, 0.0, 0.2], "half": [0.4, 0.4, 0.2]},
                {"name": "ramp", "center": [cx, 0.0, cz], "half": [ltop / 2, 0.5, thick / 2], "pitch": t15,
                 "ramp": True},
            ],
            "goal_static": 1, "rest_speed": 0.05,
            "robot": {"joints": JOINTS, "q0": [1.0, 1.0, math.pi] + TUCK + [0.04, 0.04],
                      "ee_body": 8, "ee_offset": [0.0, 0.0, 0.075]},
            "controller": dict(CONTROLLER),
            "goal": {"tol": 0.0, "time_weight": 1.0},
        },
        "cem": {"pop": 1024, "n_elite": 64, "iters": 10, "cov_mode": "diag",
                "mu0": [0.85, 0.0, math.pi, 1.0, 0.0, 1.0, 0.0, 0.0, 1.35, 0.0, 0.0, 1.0, 2.1, 0.0, 0.6, math.pi],
                "cov0_diag": [0.09, 0.09, 0.25, 0.09, 0.0225, 0.0225, 0.0225, 0.0225, 0.09, 0.09, 0.25, 0.09,
                              0.01, 0.01, 0.0025, 0.25],
                "seeds": list(range(10))},
    }


# Sec. IV-A, "Algorithm setting": iteration 0 uniform inside the parameter
# regions, then independent normals; n_env 3000 falling linearly to 300 by
# iteration 10; N_e = 50; a budget of 20 iterations.  The regions follow
# Sec. IV-A's list, with the rings sized to this robot's reach (an arm of
# about 1 m from a shoulder 0.2 m ahead of the base centre): Table_1 and
# Table_2 rings, the grasp quaternion in a box of side 0.3 around the
# top-down grasp (0, 1, 0, 0), the release point in a 0.2 x 0.4 x 0.6 m box
# straddling Table 2's near edge and the obstacle, the release yaw within
# +-0.15 rad of pi; headings anywhere, base speeds in [0.5, 1.5] m/s.
PP_RING_1 = {"dim": 0, "center": [0.0, 0.0], "radius": [0.7, 1.1]}
PP_RING_2 = {"dim": 8, "center": [3.0, 0.0], "radius": [0.7, 1.2]}


def paper_setting(w, name, description):
    pi = math.pi
    w = json.loads(json.dumps(w))
    w["name"] = name
    w["description"] = description
    lo = [0.0, 0.0, -pi, 0.5, -0.15, 0.85, -0.15, -0.15, 0.0, 0.0, -pi, 0.5, 2.5, -0.2, 0.45, pi - 0.15]
    hi = [0.0, 0.0, pi, 1.5, 0.15, 1.15, 0.15, 0.15, 0.0, 0.0, pi, 1.5, 2.7, 0.2, 1.05, pi + 0.15]
    w["cem"].update({"pop": 3000, "n_elite": 50, "iters": 20,
                     "pop_schedule": {"final": 300, "iters": 10},
                     "init_region": {"lo": lo, "hi": hi, "rings": [PP_RING_1, PP_RING_2]}})
    return w


def pickplace_paper():
    return paper_setting(pickplace(), "pickplace_paper",
                         "Pick-and-place over the ramp obstacle with the paper's algorithm setting: iteration 0 "
                         "uniform in the parameter regions (rings around the tables, grasp and release boxes), "
                         "n_env 3000 -> 300 linearly by iteration 10, 50 elites, 20 iterations")


def pickplace_box():
    w = paper_setting(pickplace(), "pickplace_box",
                      "Pick-and-place with the box obstacle (Sec. IV-A setup 2: the obstacle without its slanted "
                      "side, a rectangular prism on the ramp's footprint and up to its top edge) and the paper's "
                      "algorithm setting")
    boxes = w["scene"]["static_boxes"]
    boxes[2] = {"name": "box", "center": [2.3, 0.0, 0.24], "half": [0.3, 0.5, 0.24]}
    return w


def movepush():
    # shelf 0.6 x 0.6 x 0.5 m at the origin; a 0.1 m, 0.3 kg block near its +x
    # edge; an open container (floor + 4 walls 0.3 m high, 0.4 x 0.4 m inside,
    # 0.02 m thick) against the shelf's +x face
    wall_h, t, inner = 0.3, 0.02, 0.4
    floor_top = t
    cx = 0.3 + t + inner / 2          # container centre x (inner x in [0.32, 0.72])
    zc = floor_top + wall_h / 2
    boxes = [
        {"name": "shelf", "center": [0.0, 0.0, 0.25], "half": [0.3, 0.3, 0.25]},
        {"name": "floor", "center": [cx, 0.0, t / 2], "half": [inner / 2 + t, inner / 2 + t, t / 2]},
        {"name": "wall_near", "center": [0.3 + t / 2, 0.0, zc], "half": [t / 2, inner / 2 + t, wall_h / 2]},
        {"name": "wall_far", "center": [0.3 + 1.5 * t + inner, 0.0, zc], "half": [t / 2, inner / 2 + t, wall_h / 2]},
        {"name": "wall_left", "center": [cx, inner / 2 + t / 2, zc], "half": [inner / 2, t / 2, wall_h / 2]},
        {"name": "wall_right", "center": [cx, -inner / 2 - t / 2, zc], "half": [inner / 2, t / 2, wall_h / 2]},
    ]
    ctl = dict(CONTROLLER)
    ctl.update({"push_vmin": 0.05, "push_vmax": 1.0, "push_dmax": 0.6, "timeout_push": 4.0})
    return {
        "name": "movepush",
        "description": "Plain CEM, mobile manipulator move-and-push: the robot moves beside a shelf and pushes a "
                       "0.1 m, 0.3 kg block (friction U[0.3, 0.7] per instance) off it into an open container "
                       "(5 static boxes); 2 actions, 4 + 8 = 12 params; pop 8192, 256 elites, 15 iterations; "
                       "dt 0.005 s, 3000 steps",
        "scene": {
            "kind": "movepush", "dt": 0.005, "substeps": 5, "horizon": 3000,
            "gravity": 9.81, "k_contact": 10000.0, "c_contact": 10.0, "eps_v": 0.02,
            "mu_ground": 0.5, "mu_tool": 0.8, "mu_static": 0.5, "mu_ramp": 0.5,
            "object": {"half": [0.05, 0.05, 0.05], "mass": 0.3, "pos0": [0.2, 0.0, 0.55], "yaw0": 0.0,
                       "mu": [0.3, 0.7]},
            "static_boxes": boxes,
            "goal_static": -1,
            "goal_box": {"center": [cx, 0.0, zc], "half": [inner / 2, inner / 2, wall_h / 2]},
            "rest_speed": 0.05,
            "robot": {"joints": JOINTS, "q0": [-0.8, -1.2, math.pi / 2] + TUCK + [0.04, 0.04],
                      "ee_body": 8, "ee_offset": [0.0, 0.0, 0.075]},
            "controller": ctl,
            "goal": {"tol": 0.0, "time_weight": 1.0},
        },
        "cem": {"pop": 8192, "n_elite": 256, "iters": 15, "cov_mode": "diag",
                # move: x, y, psi, v; push: start x, y, z, heading, distance, speed, approach height, gripper yaw
                "mu0": [0.05, -0.68, math.pi / 2, 1.0, 0.125, 0.0, 0.55, 0.0, 0.3, 0.4, 0.1, 0.0],
                "cov0_diag": [0.04, 0.01, 0.04, 0.09, 0.0025, 0.01, 0.0004, 0.04, 0.01, 0.04, 0.0025, 0.1],
                "seeds": list(range(10))},
    }


def movepush_dr():
    # Sec. IV-C: plans made robust to bounded uncertainty in friction or mass;
    # every candidate is scored by its mean cost over 8 scenarios whose block
    # friction and mass are drawn per instance
    w = movepush()
    w["name"] = "movepush_dr"
    w["description"] = ("Move-and-push with domain randomisation: each parameter row rolled out under 8 scenarios "
                        "(block friction U[0.3, 0.7], mass U[0.2, 0.4] kg), cost the mean, tier the worst; "
                        "pop 8192 (65,536 rollouts per iteration), 256 elites, 15 iterations")
    w["scene"]["domain_randomization"] = {"scenarios": 8, "reduce": "mean", "mu": [0.3, 0.7], "mass": [0.2, 0.4]}
    return w


def write(w):
    path = os.path.join(HERE, w["name"] + ".json")
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if "measurement" in old:
            w["measurement"] = old["measurement"]
    with open(path, "w") as f:
        json.dump(w, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    write(pickplace())
    write(movepush())
    write(pickplace_paper())
    write(pickplace_box())
    write(movepush_dr())
