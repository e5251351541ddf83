"""The robot model compiled into the specialised rollout instance
(paper_2512_11571_amd/csrc/robot_model.hpp) is the robot every robot
configuration carries: the committed header equals what its generator writes
from the configuration, and the configurations share one robot."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_11571_amd", "csrc")
CONFIGS = os.path.join(ROOT, "paper_2512_11571_amd", "configs")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_robot_model", os.path.join(CSRC, "gen_robot_model.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_header_is_the_generated_one():
    g = _gen()
    joints = json.load(open(g.CONFIG))["scene"]["robot"]["joints"]
    assert open(os.path.join(CSRC, "robot_model.hpp")).read() == g.render(joints)


def test_robot_configurations_share_the_model():
    ref = json.load(open(os.path.join(CONFIGS, "pickplace.json")))["scene"]["robot"]["joints"]
    n = 0
    for name in sorted(os.listdir(CONFIGS)):
        if not name.endswith(".json"):
            continue
        sc = json.load(open(os.path.join(CONFIGS, name))).get("scene", {})
        if "robot" in sc:
            assert sc["robot"]["joints"] == ref, name
            n += 1
    assert n >= 4


def test_hex_literals_are_the_fp32_roundings():
    import numpy as np
    g = _gen()
    for v in (0.35, 0.2, -0.01, 20.0, 0.0):
        lit = g.f32(v)
        assert lit.endswith("f")
        assert np.float32(float.fromhex(lit[:-1])) == np.float32(v)
