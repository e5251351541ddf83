"""Throughput of the CE hot path on one MI355X.

One step = one CE iteration of the whole hot path on one batch of synthetic
input: Philox sampling of the population, the rollout of every sampled plan
over the full horizon, elite selection and the FP64 refit.  Prints one JSON
line with env-steps/s (one env-step = one control step dt of one environment,
with all its physics substeps), CE iterations/s, the roofline of the rollout
kernel and the CPU oracle's throughput on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--settle-steps N] [--lanes auto|1|2|4|8|16]

Workloads: batch (the default: 64 push and pick-and-place instances with
uneven horizons and populations, one persistent launch per CE iteration, the
largest configuration that fits one GPU), batch_mixed (push, pick-and-place
and move-push instances), pickplace (1024 plans x 2000 steps), push,
movepush, pickplace_paper and pickplace_box (iteration-0 regions, n_env
schedule), movepush_dr (8 friction/mass scenarios per plan), surrogate
(screened against plain CE to the same cost) and mlp (the surrogate network's
forward over 65,536 rows and its training step, against the BF16 MFMA peak).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: FP32 vector (packed) 157.3 TFLOP/s, HBM3E 8 TB/s.
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0   # dense BF16 MFMA
MLP_FLOP_PER_ROW = 2 * (16 * 256 + 256 * 256 + 256 * 256 + 256 * 8)   # one forward pass, multiply-adds x 2
DEFAULT_WORKLOAD = "batch"

# HBM traffic per rollout launch measured with rocprofv3 (FETCH_SIZE + WRITE_SIZE,
# scaled by the copy-kernel calibration), keyed by workload; valid only while
# the rollout sources hash to the recorded value.
MEASURED_TRAFFIC = {
    # one batched rollout launch (64 instances, 141,184 plans, 357.7 M env-steps): FETCH_SIZE 5852.1875 KiB x 2.0
    # (items of 32 envs) + WRITE_SIZE 7208.25 KiB x 1.0 (items of 64 envs; a 256 MiB copy reads as 131083.5 /
    # 262144 KiB); algorithmic 10,243,712 B (Z in, cost, tier and pose out); the plans' launch order scatters the
    # rows' reads and the outcomes' writes
    "batch": {"bytes_per_launch": int((5852.1875 * 2.0 + 7208.25 * 1.0) * 1024), "src_hash": "a0f6363f63c6f0f4"},
    # rollout of 1024 pick-and-place plans over 2000 steps, 16 lanes per plan: FETCH_SIZE
    # 553.5 KiB x 2.0 + WRITE_SIZE 24.0 KiB x 1.0
    "pickplace": {"bytes_per_launch": int((553.5 * 2.0 + 24.0 * 1.0) * 1024), "lanes": 16,
                  "src_hash": "a0f6363f63c6f0f4"},
}

_KERNEL_FILES = ["rollout.hip", "push_env.hpp", "robot_env.hpp", "robot_dyn.hpp", "robot_spec.hpp", "robot_model.hpp",
                 "rigid.hpp", "devmath.hpp", "internal.hpp"]
ROLLOUT_SOURCES = {"push": _KERNEL_FILES, "pickplace": _KERNEL_FILES, "movepush": _KERNEL_FILES,
                   "batch": _KERNEL_FILES}


def _src_hash(workload):
    h = hashlib.sha256()
    for f in ROLLOUT_SOURCES.get(workload, []):
        with open(os.path.join(ROOT, "paper_2512_11571_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Host threads of the CPU baseline: every core the host shows, up to the 16
# that one GPU's share of the GPU machine's host allows.
CPU_SHARE = 16


def cpu_threads():
    return max(1, min(CPU_SHARE, os.cpu_count() or 1))


def cpu_baseline(w, seed, budget_s):
    """The oracle (FP64, all host threads up to the one-GPU share) on a bounded sample of the same workload."""
    import numpy as np
    from oracle import oracle as O
    cem = w["cem"]
    threads = cpu_threads()
    H = w["scene"]["horizon"]
    mu0 = np.asarray(cem["mu0"], np.float64)
    L, _ = O.factor_cov(np.diag(np.asarray(cem["cov0_diag"], np.float64)))
    n = min(cem["pop"], 4 * threads)
    Z = O.sample(seed, 0, 0, n, mu0, L)
    done, reps = 0, 0
    t0 = time.perf_counter()
    settle = w["scene"].get("settle_steps", 0)
    while True:
        steps = O.rollout(w, seed, Z, threads=threads, with_steps=True)[4]
        done += int(steps.sum())
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    span = ("full horizon %d steps" % H) if not settle else ("horizon %d, early stop after %d settled steps" % (H, settle))
    return {"value": done / dt, "unit": "env-steps/s", "cores": threads, "host_nproc": os.cpu_count(),
            "kind": "oracle",
            "sample": "%d x %d rollouts of %d iteration-0 samples (%s), %.1f s" % (reps, n, n, span, dt),
            "env_steps": done, "seconds": dt}


def _valu_ceiling():
    """The device's measured unpacked FP32 FMA rate (TFLOP/s): the ceiling of the rollout's arithmetic."""
    from paper_2512_11571_amd.binding import valu_fma_rate
    return valu_fma_rate() / 1e12


def auto_lanes(scene, pop, scenarios, simds=None):
    """Lanes per environment for a single robot instance: the most (16, 8, 4,
    2 or 1) whose waves still fit one per SIMD (64 lanes a wave, 4 SIMDs a CU;
    the device's unless `simds` is given).  Where the object has at most four
    world tests, 8 or 16 lanes split corners rather than tests, which pays
    less: then only while the waves fit one per CU (measured: pick-and-place
    at 1024 plans 314 ms at 16 lanes, 318 at 8, 326 at 4; at 3000 plans 317 at
    8 against 305 at 4)."""
    if scene["kind"] == "push":
        return 1
    if simds is None:
        import torch
        simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    halves = len(scene.get("static_boxes", [])) + 1 <= 4
    for G in (16, 8, 4, 2):
        limit = simds // 4 if (G >= 8 and halves) else simds
        if scenarios * G <= 64 and -(-pop * scenarios * G // 64) <= limit:
            return G
    return 1


def bench_batch(a):
    """The batched workload: all instances, one CE iteration of every instance per step (graph replay).

    A timed step is one CE iteration of every instance.  Where the driver asks
    for more steps than an instance's nominal iteration budget (5 push, 10
    pick-and-place), the timed batch raises every budget to the step count, so
    that each timed step still iterates all 64 instances."""
    import torch
    from paper_2512_11571_amd import workloads
    from paper_2512_11571_amd.binding import Batch

    spec = workloads.load(a.workload)["batch"]
    kinds = list(spec["kinds"])
    insts = workloads.batch_instances(spec)
    for i in insts:                   # early stops on the robot instances
        if i["workload"]["scene"]["kind"] != "push":
            i["workload"]["scene"]["settle_steps"] = a.settle_steps
            i["workload"]["scene"]["fail_stop"] = int(a.fail_stop)
    K = a.steps if a.steps is not None else 3
    nominal = {k: int(spec["iters"][k]) for k in kinds}
    timed = [dict(i, iters=max(i["iters"], K)) for i in insts]
    torch.cuda.set_device(0)
    with Batch([dict(i, iters=max(i["iters"], a.warmup)) for i in insts]) as B:   # warm-up on a batch of its own
        for _ in range(a.warmup):
            B.step()
        torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    with Batch(timed) as B:
        tune = B.autotune()           # untimed; leaves the CE state and step counters as they were
        torch.cuda.synchronize()
        per0 = [B.instance(k).env_steps() for k in range(len(insts))]
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        t0 = time.perf_counter()
        for j in range(K):            # one CE iteration of every instance per replay
            evs[j][0].record(stream)
            B.step(stream)
            evs[j][1].record(stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        step_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
        per = [B.instance(k).env_steps() - per0[k] for k in range(len(insts))]
    counted = sum(per)
    env_steps_iter = sum(i["workload"]["cem"]["pop"] * i["workload"]["scene"]["horizon"] for i in insts)
    dims = {"push": 3, "pickplace": 16, "movepush": 12}
    # HBM bytes the method must move per launch: each plan's parameter row in, its cost, tier and pose out
    alg_bytes = sum(i["workload"]["cem"]["pop"] * (4 * dims[i["workload"]["scene"]["kind"]] + 4 + 1 + 28)
                    for i in insts)
    assert counted <= env_steps_iter * K, (counted, env_steps_iter * K)   # fewer only where rollouts stopped early
    fps = {k: workloads.load(k).get("measurement", {}).get("flops_per_env_step") for k in kinds}
    # algorithmic FLOPs of the steps the rollouts actually simulated, per scene kind
    flops = sum(n * (fps[i["workload"]["scene"]["kind"]] or 0.0) for n, i in zip(per, insts))
    # the replayed step is sampling + the rollout launch + refit; the rollout is > 99.8 % of it,
    # so the step's event time bounds the rollout kernel's duration from above
    roll_s = sum(step_ms) / len(step_ms) / 1e3
    achieved = flops / K / roll_s / 1e12 if roll_s > 0 else None
    ceiling = _valu_ceiling()
    tr = MEASURED_TRAFFIC.get(a.workload)
    traffic = (tr["bytes_per_launch"] if tr and tr.get("src_hash") == _src_hash(a.workload)
               and not a.settle_steps and not a.fail_stop else None)
    out = {
        "metric": "env-steps/s (CE iterations/s alongside)",
        "value": counted / elapsed,
        "unit": "env-steps/s", "n_gpus": 1, "steps": K, "warmup": a.warmup,
        "ms_per_step": elapsed / K * 1e3, "cem_iters_per_s": K / elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (FP64 refit and Cholesky)", "data": "synthetic (seeded instances, scenes and Philox samples)",
        "config": {"workload": a.workload, "instances": len(insts), "kinds": kinds,
                   "env_steps_per_iter": env_steps_iter, "nominal_iters": nominal,
                   "timed_iters_per_instance": K, "autotune": tune, "settle_steps": a.settle_steps,
                   "fail_stop": int(a.fail_stop)},
        "env_steps_simulated": counted, "env_steps_full_horizon": env_steps_iter * K,
        "step_event_ms": roll_s * 1e3,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS if achieved else None, "traffic": traffic,
                     "algorithmic_bytes": alg_bytes,
                     "flops_per_env_step": fps, "unpacked_fma_measured": ceiling,
                     "frac_of_measured": achieved / ceiling if achieved and ceiling else None},
    }
    if not a.no_cpu_baseline:
        per_kind = []
        for k in kinds:
            w = next(i["workload"] for i in insts if i["workload"]["scene"]["kind"] == k)
            per_kind.append(cpu_baseline(w, a.seed, a.cpu_seconds / len(kinds)))
        tot_t = sum(p["seconds"] for p in per_kind)
        steps = sum(p["env_steps"] for p in per_kind)
        out["cpu_baseline"] = {"value": steps / tot_t, "unit": "env-steps/s", "cores": per_kind[0]["cores"],
                               "host_nproc": os.cpu_count(), "kind": "oracle",
                               "sample": "; ".join(p["sample"] for p in per_kind)}
    print(json.dumps(out))


def _first_reach(curve, target):
    """First iteration count k (1-based) whose value is within the target band, else None."""
    for k, v in enumerate(curve, 1):
        if v <= target:
            return k
    return None


def mlp_kernel_times(m, X, Y, rows, batch, reps=20):
    """The surrogate's kernels alone: the mean of `reps` forward passes over `rows` rows of X and of `reps`
    training steps (forward, backward, Adam) on the first `batch` rows, timed with HIP events."""
    import torch
    stream = torch.cuda.current_stream()
    Yp = torch.empty((rows, 8), dtype=torch.float32, device=X.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    m.forward(X[:rows], Yp, stream)
    e0.record(stream)
    for _ in range(reps):
        m.forward(X[:rows], Yp, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / reps / 1e3
    m.train_step(X[:batch], Y[:batch], 0.0, None, stream)
    e0.record(stream)
    for _ in range(reps):
        m.train_step(X[:batch], Y[:batch], 0.0, None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    step_s = e0.elapsed_time(e1) / reps / 1e3
    return {"forward_rows": rows, "forward_ms": fwd_s * 1e3,
            "forward_tflops": rows * MLP_FLOP_PER_ROW / fwd_s / 1e12,
            "forward_frac_of_bf16_peak": rows * MLP_FLOP_PER_ROW / fwd_s / 1e12 / PEAK_BF16_TFLOPS,
            "train_step_rows": batch, "train_step_ms": step_s * 1e3,
            "train_step_tflops": 3 * batch * MLP_FLOP_PER_ROW / step_s / 1e12}


def bench_mlp(a):
    """The surrogate network's kernels on synthetic rows: the screening forward over the screening population
    (65,536 rows) and one training step at the training batch, on a freshly initialised network."""
    import torch
    from paper_2512_11571_amd import workloads
    from paper_2512_11571_amd.binding import Mlp

    spec = workloads.load("surrogate")["surrogate"]
    rows, batch = spec["eval"]["screen_pop"], spec["train"]["batch"]
    torch.cuda.set_device(0)
    g = torch.Generator(device="cpu").manual_seed(a.seed)
    X = torch.randn((rows, 16), generator=g).to("cuda:0")
    Y = torch.randn((rows, 8), generator=g).to("cuda:0")
    with Mlp(seed=a.seed, max_rows=rows) as m:
        m.fit_norm(X, Y, rows)
        for _ in range(max(1, a.warmup)):
            mlp_kernel_times(m, X, Y, rows, batch, reps=2)
        t = mlp_kernel_times(m, X, Y, rows, batch, reps=a.steps or 20)
    ach = t["forward_tflops"]
    print(json.dumps({
        "metric": "surrogate forward TFLOP/s (training step alongside)", "value": ach, "unit": "TFLOP/s",
        "n_gpus": 1, "steps": a.steps or 20, "warmup": a.warmup, "ms_per_step": t["forward_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 operands, f32 accumulation",
        "data": "synthetic (seeded normal rows, freshly initialised network)",
        "config": {"workload": "mlp", "forward_rows": rows, "train_batch": batch, "layers": [16, 256, 256, 256, 8]},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_BF16_TFLOPS, "traffic": None},
        "mlp": t}))


def bench_surrogate(a):
    """Surrogate screening against plain CE on the pick-and-place plan: wall time
    to reach plain CE's final plan cost.  Dataset recording and training are
    timed and reported on their own (amortised over every later solve)."""
    import numpy as np
    import torch
    from paper_2512_11571_amd import workloads
    from paper_2512_11571_amd.binding import Batch, Context, Mlp

    spec = workloads.load("surrogate")["surrogate"]
    base = workloads.load(spec["workload"])
    ev, tr = spec["eval"], spec["train"]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    log = lambda *x: print(*x, file=sys.stderr, flush=True)

    insts = workloads.surrogate_dataset_instances(spec)
    cap = sum(i["workload"]["cem"]["pop"] * i["iters"] for i in insts)
    X = torch.empty((cap, 16), dtype=torch.float32, device=dev)
    Y = torch.empty((cap, 8), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    with Batch(insts) as bt:
        n = bt.record(spec["dataset"]["iters"], X, Y)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    env_steps_data = sum(i["workload"]["cem"]["pop"] * i["iters"] * i["workload"]["scene"]["horizon"] for i in insts)
    log("dataset: %d rows in %.1f s" % (n, t_data))

    # both arms simulate n_sim plans per iteration, with the same lanes per environment
    lanes = auto_lanes(base["scene"], ev["n_sim"], 1) if a.lanes == "auto" else int(a.lanes)

    def solve(seed, screened, m):
        cem = dict(base["cem"], n_elite=ev["n_elite"], pop=ev["screen_pop"] if screened else ev["n_sim"])
        w = dict(base, cem=cem)
        with Context(w, seed=seed, lanes=lanes) as c:
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = m.plan_solve_screened(c, ev["iters"], ev["n_sim"]) if screened else c.plan_solve(ev["iters"])
            return r, time.perf_counter() - t

    with Mlp(seed=tr["seed"], max_rows=ev["screen_pop"]) as m:
        t0 = time.perf_counter()
        m.fit_norm(X, Y, n)
        losses = m.train(X, Y, n, tr["batch"], tr["epochs"], tr["lr"], seed=tr["seed"])
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        log("training: %d epochs in %.1f s, loss %.4f -> %.4f" % (tr["epochs"], t_train, losses[0], losses[-1]))
        # the network's kernels alone: the screening forward over one population, one training step
        mlp = mlp_kernel_times(m, X, Y, ev["screen_pop"], tr["batch"])
        log("mlp:", mlp)
        del X, Y
        solve(ev["seeds"][0], False, m)          # warm-up of both paths (graph capture, code load)
        solve(ev["seeds"][0], True, m)
        curves = {False: [], True: []}
        times = {False: [], True: []}
        err = []
        for seed in ev["seeds"]:
            for screened in (False, True):
                r, t = solve(seed, screened, m)
                curves[screened].append(r["stats"][:, 7])
                times[screened].append(t)
                if screened:
                    err.append(r["surrogate_err"])
            log("seed %d: plain %.3f, screened %.3f" % (seed, curves[False][-1][-1], curves[True][-1][-1]))

    med = {k: np.median(np.stack(v), axis=0) for k, v in curves.items()}
    target = float(med[False][-1])
    band = target * (1.0 + ev["target_tol"])
    t_iter = {k: float(np.mean(v)) / ev["iters"] for k, v in times.items()}
    k_plain, k_scr = _first_reach(med[False], band), _first_reach(med[True], band)
    t_plain = k_plain * t_iter[False]
    t_scr = k_scr * t_iter[True] if k_scr else None
    # per seed: the wall time each arm needs to bring that seed's best cost into the band, and their ratio;
    # the median ratio with a bootstrap interval over seeds (resampled with a seeded generator)
    per_seed = []
    for c0, c1, s0, s1 in zip(curves[False], curves[True], times[False], times[True]):
        k0, k1 = _first_reach(c0, band), _first_reach(c1, band)
        t0 = k0 * s0 / ev["iters"] if k0 else float("inf")
        t1 = k1 * s1 / ev["iters"] if k1 else float("inf")
        per_seed.append((t0, t1))
    ratios = np.array([t1 / t0 for t0, t1 in per_seed if np.isfinite(t0)])
    rng = np.random.default_rng(0)
    boot = [float(np.median(rng.choice(ratios, ratios.size))) for _ in range(int(ev.get("bootstrap", 2000)))]
    lo, hi = (float(np.percentile(boot, 2.5)), float(np.percentile(boot, 97.5))) if ratios.size else (None, None)
    # inclusive: the one-off dataset and training charged to the screened arm, over every evaluated seed
    fin = [(t0, t1) for t0, t1 in per_seed if np.isfinite(t0) and np.isfinite(t1)]
    incl = (t_data + t_train + sum(t1 for _, t1 in fin)) / sum(t0 for t0, _ in fin) if fin else None
    out = {
        "metric": "wall time to plain CE's final plan cost, screened / plain (median over seeds of per-seed ratios)",
        "value": float(np.median(ratios)) if ratios.size else None,
        "unit": "x", "n_gpus": 1, "steps": ev["iters"], "warmup": 1,
        "ms_per_step": t_iter[True] * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 rollouts, bf16 MFMA surrogate (f32 accumulate)",
        "data": "synthetic (seeded pick-and-place instances and Philox samples)",
        "config": {"workload": "surrogate (pick-and-place)", "n_sim": ev["n_sim"], "screen_pop": ev["screen_pop"],
                   "n_elite": ev["n_elite"], "iters": ev["iters"], "seeds": len(ev["seeds"]), "lanes_per_env": lanes,
                   "dataset_rows": n, "dataset_env_steps": env_steps_data},
        "target_cost": target, "target_band": band,
        "per_seed_ratio": {"median": float(np.median(ratios)) if ratios.size else None,
                           "bootstrap_95": [lo, hi], "seeds_counted": int(ratios.size),
                           "screened_never_reached": int(sum(1 for t0, t1 in per_seed if np.isfinite(t0)
                                                              and not np.isfinite(t1)))},
        "median_curve_ratio": (t_scr / t_plain) if t_scr else None,
        "inclusive_ratio_with_dataset_and_training": incl,
        "median_best_cost_per_iter": {"plain": [float(x) for x in med[False]],
                                      "screened": [float(x) for x in med[True]]},
        "iters_to_target": {"plain": k_plain, "screened": k_scr},
        "seconds_per_iter": {"plain": t_iter[False], "screened": t_iter[True]},
        "seconds_to_target": {"plain": t_plain, "screened": t_scr},
        "surrogate_cost_error_mean_per_iter": [float(x) for x in np.mean(np.stack(err), axis=0)],
        "dataset_seconds": t_data, "train_seconds": t_train, "mlp": mlp,
        "train_loss_first_last": [float(losses[0]), float(losses[-1])],
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--settle-steps", type=int, default=0,
                    help="robot workloads: stop a rollout once its plan has ended and the object has rested this "
                         "many control steps (0: every rollout runs the full horizon); throughput then counts the "
                         "steps actually simulated")
    ap.add_argument("--fail-stop", action="store_true",
                    help="robot workloads: stop a rollout when an action fails (its plan can no longer be "
                         "feasible); throughput then counts the steps actually simulated")
    ap.add_argument("--lanes", default="auto",
                    help="lanes per environment of a single robot instance (1, 2, 4, 8, 16; auto: the most whose "
                         "waves fit one per SIMD)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (the known-size "
                         "reference for the HBM byte counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would run its own "
              "share of the population independently); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if a.copy_calibration:
        import torch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "launches": 3}))
        return
    if a.workload in ("batch", "batch_mixed"):
        bench_batch(a)
        return
    if a.workload == "surrogate":
        bench_surrogate(a)
        return
    if a.workload == "mlp":
        bench_mlp(a)
        return

    import torch
    from paper_2512_11571_amd import workloads
    from paper_2512_11571_amd.binding import Context

    w = workloads.load(a.workload)
    if a.settle_steps or a.fail_stop:
        if w["scene"]["kind"] == "push":
            print("--settle-steps and --fail-stop apply to the robot workloads only", file=sys.stderr)
            sys.exit(2)
        w["scene"]["settle_steps"] = a.settle_steps
        w["scene"]["fail_stop"] = int(a.fail_stop)
    cem, sc = w["cem"], w["scene"]
    pop, H, D = cem["pop"], sc["horizon"], {"push": 3, "pickplace": 16, "movepush": 12}[sc["kind"]]
    sched = cem.get("pop_schedule")
    K = a.steps if a.steps is not None else cem["iters"]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    Z = torch.empty((pop, D), dtype=torch.float32, device=dev)
    cost = torch.empty(pop, dtype=torch.float32, device=dev)
    tier = torch.empty(pop, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    R = max(1, sc.get("domain_randomization", {}).get("scenarios", 1))
    lanes = auto_lanes(sc, pop, R) if a.lanes == "auto" else int(a.lanes)
    with Context(w, seed=a.seed, lanes=lanes) as c:
        def step(j, evs=None):
            n = c.pop_at(j)                    # n_env(j): pop unless the workload has a schedule
            c.cem_sample(j, Z, stream)
            if evs is not None:
                evs[0].record(stream)
            c.rollout_batch(Z[:n], cost[:n], tier[:n], None, stream)
            if evs is not None:
                evs[1].record(stream)
            c.cem_refit(Z[:n], cost[:n], tier[:n], None, None, stream)

        for j in range(a.warmup):
            step(j)
        torch.cuda.synchronize()
        c.reset()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        counted0 = c.env_steps()
        pops = [c.pop_at(j) for j in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(K):
            step(j, evs[j])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        env_steps = c.env_steps() - counted0   # the control steps the rollouts simulated
        roll_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
        mu, S = c.get_theta()

    full = sum(pops) * H * R
    assert env_steps <= full, (env_steps, full)   # fewer only where rollouts stopped early or diverged
    value = env_steps / elapsed
    roll_avg_s = sum(roll_ms) / len(roll_ms) / 1e3
    meas = w.get("measurement", {})
    fps = meas.get("flops_per_env_step")
    achieved = (fps * env_steps / K / roll_avg_s / 1e12) if fps else None
    ceiling = _valu_ceiling()
    tr = MEASURED_TRAFFIC.get(a.workload)
    traffic = (tr["bytes_per_launch"] if tr and tr.get("src_hash") == _src_hash(a.workload)
               and tr.get("lanes", 1) == lanes and not sc.get("settle_steps", 0) and not sc.get("fail_stop", 0)
               else None)
    out = {
        "metric": "env-steps/s (CE iterations/s alongside)",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": a.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "cem_iters_per_s": K / elapsed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 refit and Cholesky)",
        "data": "synthetic (seeded scene and Philox samples)",
        "config": {"workload": a.workload, "pop": pop, "horizon": H, "substeps": sc["substeps"], "dim": D,
                   "n_elite": cem["n_elite"], "dt": sc["dt"], "seed": a.seed,
                   "settle_steps": sc.get("settle_steps", 0), "fail_stop": sc.get("fail_stop", 0),
                   "pop_schedule": sched,
                   "init_region": bool(cem.get("init_region")), "dr_scenarios": R, "lanes_per_env": lanes},
        "env_steps_simulated": env_steps,
        "env_steps_full_horizon": full,
        "rollout_kernel_ms": roll_avg_s * 1e3,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP32_TFLOPS) if achieved else None, "traffic": traffic,
                     "flops_per_env_step": fps,
                     "unpacked_fma_measured": ceiling,
                     "frac_of_measured": (achieved / ceiling) if achieved and ceiling else None},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.seed, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
