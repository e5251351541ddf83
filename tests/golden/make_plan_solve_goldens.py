"""Writes plan_solve_oracle.json beside this script: the FP64 oracle's Alg. 1
runs that the GPU's plan_solve medians are compared with.

- pickplace: the configured problem (pop 1024, N_e 64, 10 iterations), seeds 0-31;
- movepush: a subset of the configured problem (pop 1024, N_e 64, 5 iterations,
  of the configured 8192 / 256 / 15), seeds 0-31;
- batch_push: the push instances of the batched workload (jittered goals,
  their own horizon, population and N_e), each for its iteration budget, as
  the batch runs them (seed of the batch recipe, instance id as the Philox
  instance);
- box_small: the box-obstacle scene in the paper's setting (iteration-0
  region, n_env schedule) at pop 256 -> 64 by iteration 2, N_e 16, 3
  iterations, seeds 0-31;
- dr_small: pick-and-place with 4 domain-randomisation scenarios (block
  friction and mass), pop 64, N_e 8, 2 iterations, seeds 0-31.

Only the oracle and the seeded workload descriptions are used.  Results are
saved after every run, so an interrupted run keeps what it finished and a new
run resumes.

    python tests/golden/make_plan_solve_goldens.py [--threads N] [--only NAME]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2512_11571_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "plan_solve_oracle.json")
SEEDS = list(range(32))


def problems():
    """name -> (workload, list of (key, seed, instance, iters))."""
    out = {}
    pp = workloads.load("pickplace")
    pp["cem"].update(pop=1024, n_elite=64)
    out["pickplace"] = (pp, [(str(s), s, 0, 10) for s in SEEDS])
    mp = workloads.load("movepush")
    mp["cem"].update(pop=1024, n_elite=64)
    out["movepush"] = (mp, [(str(s), s, 0, 5) for s in SEEDS])
    box = workloads.load("pickplace_box")
    box["cem"].update(pop=256, n_elite=16, pop_schedule={"final": 64, "iters": 2})
    out["box_small"] = (box, [(str(s), s, 0, 3) for s in SEEDS])
    dr = workloads.load("pickplace")
    dr["scene"]["domain_randomization"] = {"scenarios": 4, "reduce": "mean", "mu": [0.3, 0.7], "mass": [0.2, 0.4]}
    dr["cem"].update(pop=64, n_elite=8)
    out["dr_small"] = (dr, [(str(s), s, 0, 2) for s in SEEDS])
    for inst in workloads.batch_instances():
        if inst["workload"]["scene"]["kind"] == "push":
            out.setdefault("batch_push", ([], []))
            out["batch_push"][0].append(inst["workload"])
            out["batch_push"][1].append((str(inst["instance"]), inst["seed"], inst["instance"], inst["iters"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name, (w, runs) in problems().items():
        if a.only and name != a.only:
            continue
        block = res.setdefault(name, {"runs": {}})
        for k, (key, seed, inst, iters) in enumerate(runs):
            if key in block["runs"]:
                continue
            wk = w[k] if isinstance(w, list) else w
            t0 = time.perf_counter()
            r = O.plan_solve(wk, seed, inst=inst, iters=iters, threads=a.threads)
            block["runs"][key] = {"seed": seed, "instance": inst, "iters": iters, "pop": wk["cem"]["pop"],
                                  "n_elite": wk["cem"]["n_elite"], "horizon": wk["scene"]["horizon"],
                                  "best_cost": r["best_cost"], "best_tier": r["best_tier"],
                                  "best_per_iteration": [float(v) for v in r["stats"][:, 7]]}
            tmp = OUT + ".tmp"
            with open(tmp, "w") as f:
                json.dump(res, f, indent=1, sort_keys=True)
            os.replace(tmp, OUT)
            print("%s %s: best %.6f tier %d (%.0f s)" % (name, key, r["best_cost"], r["best_tier"],
                                                       time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
