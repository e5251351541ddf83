"""Workload descriptions: the synthetic scenes and CEM settings, read from JSON.

This module only reads files and draws nothing: it holds no arithmetic of the
method.  It is the one input source shared by the GPU library's binding and by
the test harness that drives the CPU oracle.
"""
import json
import os

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def names():
    return sorted(f[:-5] for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))


def load(name):
    """Return the workload dict for `name` (a file stem under configs/)."""
    with open(os.path.join(CONFIG_DIR, name + ".json")) as f:
        return json.load(f)


def batch_instances(spec=None, seed=None):
    """The batched workload's task instances, drawn from a seeded generator.

    Returns a list of dicts {"workload", "seed", "instance", "iters"}: the kinds
    alternate; each instance gets its own horizon and population (rounded up to
    the population multiple), N_e = pop / elite_divisor, and pick-place
    instances an obstacle (ramp) pose jittered in x, y and yaw.  Push goals are
    drawn per instance from the instance id by the method itself.
    """
    import copy

    import numpy as np

    spec = spec or load("batch")["batch"]
    rng = np.random.default_rng(spec["seed"] if seed is None else seed)
    base = {k: load(k) for k in spec["kinds"]}
    out = []
    for b in range(spec["n_instances"]):
        kind = spec["kinds"][b % len(spec["kinds"])]
        w = copy.deepcopy(base[kind])
        H = int(rng.integers(spec["horizon"][0], spec["horizon"][1] + 1))
        m = spec["pop_multiple"]
        pop = int(rng.integers(spec["pop"][0], spec["pop"][1] + 1))
        pop = -(-pop // m) * m
        w["scene"]["horizon"] = H
        w["cem"]["pop"] = pop
        w["cem"]["n_elite"] = max(1, min(256, pop // spec["elite_divisor"]))
        jx, jy, jyaw = rng.uniform(-1, 1, 3)
        for box in w["scene"].get("static_boxes", []):
            if box.get("ramp"):
                box["center"] = [box["center"][0] + spec["jitter_xy"] * jx, box["center"][1] + spec["jitter_xy"] * jy,
                                 box["center"][2]]
                box["yaw"] = box.get("yaw", 0.0) + np.radians(spec["jitter_yaw_deg"]) * jyaw
        out.append({"workload": w, "seed": int(spec["seed"] if seed is None else seed), "instance": b,
                    "iters": int(spec["iters"][kind])})
    return out


def surrogate_dataset_instances(spec=None):
    """Task instances whose plain-CE runs make the surrogate's training data:
    the base workload with the dataset's population and elites, one seed per
    instance from seed_base on (disjoint from the evaluation seeds)."""
    import copy

    spec = spec or load("surrogate")["surrogate"]
    d = spec["dataset"]
    base = load(spec["workload"])
    out = []
    for b in range(d["n_instances"]):
        w = copy.deepcopy(base)
        w["cem"]["pop"] = d["pop"]
        w["cem"]["n_elite"] = d["n_elite"]
        out.append({"workload": w, "seed": int(d["seed_base"] + b), "instance": b, "iters": int(d["iters"])})
    return out
