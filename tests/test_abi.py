"""The C-ABI library loads and exports every entry point include/cemtamp.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cemtamp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|size_t|cem_ctx)\s*\*?\s*([a-z_0-9]+)\s*\(", src,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_the_method_calls():
    names = _declared()
    for n in ("cem_init", "cem_sample", "rollout_batch", "cem_refit", "plan_solve", "cem_free", "cem_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2512_11571_amd import binding
    L = binding.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(binding.EXPORTS) == set(_declared())


def test_struct_layouts_match():
    from paper_2512_11571_amd import binding
    L = binding.lib()
    assert L.cem_sizeof(0) == ctypes.sizeof(binding.CemScene)
    assert L.cem_sizeof(1) == ctypes.sizeof(binding.CemProblem)
    assert L.cem_sizeof(2) == ctypes.sizeof(binding.CemResult)
    assert L.cem_sizeof(3) == ctypes.sizeof(binding.CemInitRegion)
    assert L.cem_sizeof(7) == 0


def test_strerror_without_gpu():
    from paper_2512_11571_amd import binding
    L = binding.lib()
    assert L.cem_strerror(0) == b"ok"
    assert L.cem_strerror(5).startswith(b"covariance")
    assert L.cem_last_error(None) == b"null context"


def test_init_rejects_bad_arguments_before_touching_the_device():
    from paper_2512_11571_amd import binding, workloads
    w = workloads.load("push")
    with pytest.raises(binding.CemError) as e:
        binding.Context(w, pop=0)
    assert e.value.code == 1
    with pytest.raises(binding.CemError) as e:
        binding.Context(w, n_elite=65)
    assert e.value.code == 1
    bad = dict(w, scene=dict(w["scene"], substeps=0))
    with pytest.raises(binding.CemError) as e:
        binding.Context(bad)
    assert e.value.code == 2


def test_batch_workload_recipe():
    from paper_2512_11571_amd import workloads
    spec = workloads.load("batch")["batch"]
    a = workloads.batch_instances()
    b = workloads.batch_instances()
    assert len(a) == spec["n_instances"] == 64
    for i, (x, y) in enumerate(zip(a, b)):
        w = x["workload"]
        assert w == y["workload"]
        assert w["scene"]["kind"] == spec["kinds"][i % 2]
        assert spec["horizon"][0] <= w["scene"]["horizon"] <= spec["horizon"][1]
        assert w["cem"]["pop"] % 64 == 0 and spec["pop"][0] <= w["cem"]["pop"] <= spec["pop"][1] + 63
        assert w["cem"]["n_elite"] == w["cem"]["pop"] // 16
        assert x["iters"] == spec["iters"][w["scene"]["kind"]]
    pops = [x["workload"]["cem"]["pop"] * x["workload"]["scene"]["horizon"] for x in a]
    assert 1e8 < sum(pops) < 6e8


def _rejects(binding, w, code, **kw):
    with pytest.raises(binding.CemError) as e:
        binding.Context(w, **kw)
    assert e.value.code == code


def test_options_are_validated_before_touching_the_device():
    import copy
    from paper_2512_11571_amd import binding, workloads
    pp = workloads.load("pickplace_paper")
    # iteration-0 region: box bounds, ring dimensions, overlap, radii
    for change in (lambda r: r["lo"].__setitem__(2, 4.0),
                   lambda r: r["lo"].__setitem__(3, float("nan")),
                   lambda r: r["rings"][0].__setitem__("dim", 15),
                   lambda r: r["rings"][1].__setitem__("dim", 1),
                   lambda r: r["rings"][0].__setitem__("radius", [1.2, 1.1]),
                   lambda r: r["rings"][0].__setitem__("radius", [-0.1, 1.1])):
        w = copy.deepcopy(pp)
        change(w["cem"]["init_region"])
        _rejects(binding, w, 1)
    # n_env schedule: final below N_e, no ramp
    w = copy.deepcopy(pp)
    w["cem"]["pop_schedule"] = {"final": 10, "iters": 10}
    _rejects(binding, w, 1)
    w["cem"]["pop_schedule"] = {"final": 300, "iters": 0}
    _rejects(binding, w, 1)
    with pytest.raises(ValueError):
        binding.Context(pp, pop=200)             # final 300 exceeds the population
    # early stop window, domain-randomisation scenarios, reduction and ranges
    mp = workloads.load("movepush")
    for scene in ({"settle_steps": -1}, {"settle_steps": 3001},
                  {"domain_randomization": {"scenarios": 3, "mu": [0.3, 0.7]}},
                  {"domain_randomization": {"scenarios": 128, "mu": [0.3, 0.7]}},
                  {"domain_randomization": {"scenarios": 4, "reduce": "max", "mu": [0.7, 0.3]}},
                  {"domain_randomization": {"scenarios": 4, "mass": [0.0, 0.4]}}):
        w = copy.deepcopy(mp)
        w["scene"].update(scene)
        _rejects(binding, w, 2)
    w = copy.deepcopy(workloads.load("push"))
    w["scene"]["domain_randomization"] = {"scenarios": 4, "mu": [0.3, 0.7]}
    _rejects(binding, w, 2)                      # robot scenes only


def test_lanes_per_env_is_validated_before_touching_the_device():
    import copy
    from paper_2512_11571_amd import binding, workloads
    pp = workloads.load("pickplace")
    for lanes in (-1, 3, 32, 64):
        _rejects(binding, pp, 1, lanes=lanes)
    _rejects(binding, workloads.load("push"), 1, lanes=2)    # robot scenes only
    w = copy.deepcopy(workloads.load("movepush"))
    w["scene"]["domain_randomization"] = {"scenarios": 32, "mu": [0.3, 0.7]}
    _rejects(binding, w, 1, lanes=4)                        # lanes x scenarios <= 64
    insts = [{"workload": copy.deepcopy(pp), "seed": 0, "instance": 0, "iters": 1}]
    insts[0]["workload"]["cem"]["lanes_per_env"] = 2
    with pytest.raises(binding.CemError) as e:
        binding.Batch(insts)                                 # batches run one lane per environment
    assert e.value.code == 1


def test_bench_lane_choice():
    # the most lanes whose waves still fit one per SIMD (1024 SIMDs on MI355X)
    import bench
    from paper_2512_11571_amd import workloads
    pick = lambda name, pop=None, R=1: bench.auto_lanes(workloads.load(name)["scene"],
                                                        pop or workloads.load(name)["cem"]["pop"], R, simds=1024)
    assert pick("pickplace") == 16                # 1024 plans: 256 waves, within one per CU
    assert pick("pickplace_paper") == 4           # 3000 plans: 375 waves at 8 lanes is over one per CU
    assert pick("pickplace", 4096) == 4           # the surrogate comparison's 4096 plans
    assert pick("movepush") == 8                  # 8192 plans: 1024 waves (seven object-world tests)
    assert pick("movepush", 8192, 8) == 1         # 65,536 rollouts already fill the chip
    assert pick("movepush", 16384) == 4
    assert pick("pickplace", 1024, 16) == 4       # 16 scenarios x 4 lanes fill a wave per plan
    assert pick("push") == 1
    assert pick("pickplace", 65536) == 1


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: --gpus N > 1 exits with a message before touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
