"""Counts the algorithmic FP operations per environment step of each workload.

Runs the oracle's rollout instantiated with its counting scalar type over the
iteration-0 population of seed 0 (up to 64 rows), and stores the mean
operations per control step (with its substeps) in the workload file under
"measurement".  +, -, * count 1, fma 2, / and sqrt 1; transcendental calls are
listed separately and not included.  Calls only the oracle.

    python oracle/count_flops.py push [pickplace ...]
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path[0] = os.path.dirname(HERE)  # the repo root, not this folder
from oracle import oracle as O  # noqa: E402

CONFIGS = os.path.join(os.path.dirname(HERE), "paper_2512_11571_amd", "configs")


def count(name, rows=64):
    path = os.path.join(CONFIGS, name + ".json")
    with open(path) as f:
        w = json.load(f)
    cem = w["cem"]
    mu0 = np.asarray(cem["mu0"], np.float64)
    L, _ = O.factor_cov(np.diag(np.asarray(cem["cov0_diag"], np.float64)))
    n = min(rows, cem["pop"])
    Z = O.sample_region(w, 0, 0, n) if cem.get("init_region") else O.sample(0, 0, 0, n, mu0, L)
    H = w["scene"]["horizon"]
    tallies = [O.count_ops(w, 0, Z[i]) for i in range(n)]
    per_step = {k: float(np.mean([t[k] for t in tallies])) / H for k in tallies[0]}
    w["measurement"] = {
        "flops_per_env_step": per_step["flops"],
        "ops_per_env_step": {k: v for k, v in per_step.items() if k != "flops"},
        "counted_over": "%d iteration-0 rows of seed 0, full horizon, by oracle/count_flops.py" % n,
    }
    with open(path, "w") as f:
        json.dump(w, f, indent=2)
        f.write("\n")
    return per_step["flops"]


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        print(nm, count(nm))
