"""Python binding of the CPU oracle (liboracle.so, built by oracle/build.sh).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow FP64 implementation of
the method written from the paper; the only callers are tests/, the smoke
check and the CPU-baseline leg of the benchmark.  It shares no code with the
GPU library and imports nothing from it.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CEM_ORACLE_LIB selects another build of the same sources (the sanitizer build)
LIB_PATH = os.environ.get("CEM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

SCENE_KIND = {"push": 1, "pickplace": 2, "movepush": 3}
MAX_STATIC = 8

_d = ctypes.c_double
_i = ctypes.c_int32


class RefScene(ctypes.Structure):
    _fields_ = [
        ("kind", _i), ("substeps", _i), ("horizon", _i),
        ("dt", _d), ("gravity", _d), ("k_contact", _d), ("c_contact", _d), ("eps_v", _d),
        ("mu_ground", _d), ("mu_tool", _d), ("mu_static", _d), ("mu_ramp", _d),
        ("obj_half", _d * 3), ("obj_mass", _d), ("obj_pos0", _d * 3), ("obj_yaw0", _d),
        ("n_static", _i),
        ("st_center", (_d * 3) * MAX_STATIC), ("st_half", (_d * 3) * MAX_STATIC),
        ("st_yaw", _d * MAX_STATIC), ("st_pitch", _d * MAX_STATIC), ("st_ramp", _i * MAX_STATIC),
        ("pusher_radius", _d), ("pusher_standoff", _d), ("pusher_height", _d), ("pusher_vmax", _d),
        ("pusher_steps", _i),
        ("goal_rho_lo", _d), ("goal_rho_hi", _d), ("goal_phi_lo", _d), ("goal_phi_hi", _d),
        ("goal_tol", _d), ("time_weight", _d),
        ("n_joints", _i), ("j_type", _i * 12), ("j_axis", _i * 12), ("j_parent", _i * 12), ("b_collide", _i * 12),
        ("j_origin", (_d * 3) * 12), ("b_mass", _d * 12), ("b_com", (_d * 3) * 12), ("b_half", (_d * 3) * 12),
        ("j_inom", _d * 12), ("q0", _d * 12),
        ("ee_body", _i), ("ee_offset", _d * 3),
        ("ik_iters", _i), ("omega_c", _d), ("zeta", _d), ("ik_lambda", _d),
        ("base_vmin", _d), ("base_vmax", _d), ("base_wmax", _d), ("base_tol", _d), ("yaw_tol", _d), ("ee_tol", _d),
        ("t_approach", _d), ("t_descend", _d), ("t_close", _d), ("t_lift", _d), ("t_transfer", _d),
        ("t_release", _d), ("timeout_move", _d), ("timeout_pick", _d), ("timeout_place", _d),
        ("pregrasp", _d), ("finger_open", _d), ("finger_closed", _d), ("rest_speed", _d),
        ("goal_static", _i), ("joint_speed_max", _d), ("accel_max", _d),
        ("push_vmin", _d), ("push_vmax", _d), ("push_dmax", _d), ("timeout_push", _d),
        ("obj_mu_lo", _d), ("obj_mu_hi", _d), ("goal_box_center", _d * 3), ("goal_box_half", _d * 3),
        ("settle_steps", _i), ("fail_stop", _i), ("dr_scenarios", _i), ("dr_reduce", _i),
        ("dr_mu_lo", _d), ("dr_mu_hi", _d), ("dr_mass_lo", _d), ("dr_mass_hi", _d),
    ]


class Tree(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("type", ctypes.c_int * 12), ("axis", ctypes.c_int * 12),
                ("parent", ctypes.c_int * 12), ("origin", (_d * 3) * 12), ("mass", _d * 12),
                ("com", (_d * 3) * 12), ("half", (_d * 3) * 12)]


def make_tree(joints):
    """Kinematic tree from a list of joint dicts (type 0 revolute / 1 prismatic, axis 0..5 = +x..-z)."""
    t = Tree()
    t.n = len(joints)
    for j, jd in enumerate(joints):
        t.type[j], t.axis[j], t.parent[j] = jd["type"], jd["axis"], jd["parent"]
        t.mass[j] = jd["mass"]
        for k in range(3):
            t.origin[j][k] = jd["origin"][k]
            t.com[j][k] = jd["com"][k]
            t.half[j][k] = jd["half"][k]
    return t


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("oracle not built: run oracle/build.sh")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        u64, u32 = ctypes.c_uint64, ctypes.c_uint32
        L.ref_scene_size.restype = ctypes.c_int
        L.ref_philox.argtypes = [u64, u32, u32, u32, u32, u32, vp]
        L.ref_philox_raw.argtypes = [vp, vp, vp]
        L.ref_u01.argtypes = [vp, ctypes.c_int, vp]
        L.ref_logf_vec.argtypes = [vp, ctypes.c_int, vp]
        L.ref_sincos2pi_vec.argtypes = [vp, ctypes.c_int, vp, vp]
        L.ref_normals.argtypes = [u64, u32, u32, ctypes.c_int, ctypes.c_int, vp]
        L.ref_sample.argtypes = [u64, u32, u32, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.ref_draw_instance.argtypes = [P(RefScene), u64, u32, vp]
        L.ref_rollout.argtypes = [P(RefScene), u64, u32, ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int,
                                  ctypes.c_int, vp, vp, vp]
        L.ref_count_ops.argtypes = [P(RefScene), u64, u32, vp, vp]
        L.ref_select.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp]
        L.ref_cholesky.argtypes = [ctypes.c_int, vp, vp]
        L.ref_factor_cov.argtypes = [ctypes.c_int, vp, vp]
        L.ref_refit.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int32, vp, vp, vp, vp]
        L.ref_plan_solve.argtypes = [P(RefScene), u64, u32, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                     vp, vp, ctypes.c_int, vp, vp]
        L.ref_sample_region.argtypes = [u64, u32, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp]
        L.ref_n_env_at.argtypes = [ctypes.c_int] * 4
        L.ref_scenarios.argtypes = [P(RefScene), u64, u32, ctypes.c_int, vp, vp]
        L.ref_tree_aba.argtypes = [P(Tree), vp, vp, vp, vp, ctypes.c_double, vp]
        L.ref_tree_rnea.argtypes = [P(Tree), vp, vp, vp, vp, ctypes.c_double, vp]
        L.ref_tree_crba.argtypes = [P(Tree), vp, vp]
        L.ref_tree_fk.argtypes = [P(Tree), vp, vp, vp]
        L.ref_ik.argtypes = [P(RefScene), vp, vp, vp, vp, vp, vp]
        L.ref_tree_sim.argtypes = [P(Tree), vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp]
        L.ref_mlp_n_params.restype = ctypes.c_long
        L.ref_mlp_init.argtypes = [u64, vp]
        L.ref_mlp_forward.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int]
        L.ref_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.ref_mlp_loss_grad.restype = ctypes.c_double
        L.ref_mlp_loss_grad_bf16.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.ref_mlp_loss_grad_bf16.restype = ctypes.c_double
        L.ref_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.ref_object_sim.argtypes = [P(RefScene), vp, vp, vp, ctypes.c_int, vp]
        L.ref_set_face_cull.argtypes = [ctypes.c_int]
        L.ref_set_face_cull.restype = None
        L.ref_robot_log.argtypes = [P(RefScene), u64, u32, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, ctypes.c_int]
        L.ref_grasp_check.argtypes = [P(RefScene), vp, vp, vp, vp]
        L.ref_grasp_check.restype = None
        L.ref_count_block.argtypes = [ctypes.c_int, vp]
        L.ref_count_block.restype = None
        L.ref_gelu_vec.argtypes = [vp, ctypes.c_int, vp, vp]
        L.ref_gelu_vec.restype = None
        L.ref_to_bf16_vec.argtypes = [vp, ctypes.c_int, vp]
        L.ref_to_bf16_vec.restype = None
        if L.ref_tree_size() != ctypes.sizeof(Tree):
            raise RuntimeError("oracle Tree layout mismatch")
        L.ref_box_sim.argtypes = [vp, ctypes.c_int, vp]
        L.ref_sphere_box.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
        L.ref_box_box.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        if L.ref_scene_size() != ctypes.sizeof(RefScene):
            raise RuntimeError("oracle RefScene layout mismatch")
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads():
    """Host threads for the parallel oracle loops: the machine's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def param_dim(workload):
    return {"push": 3, "pickplace": 16, "movepush": 12}[workload["scene"]["kind"]]


def make_scene(workload):
    """Fill the oracle's scene record from a workload dict."""
    sc = workload["scene"]
    s = RefScene()
    s.kind = SCENE_KIND[sc["kind"]]
    s.substeps, s.horizon = sc["substeps"], sc["horizon"]
    s.dt, s.gravity = sc["dt"], sc["gravity"]
    s.k_contact, s.c_contact, s.eps_v = sc["k_contact"], sc["c_contact"], sc["eps_v"]
    s.mu_ground, s.mu_tool, s.mu_static, s.mu_ramp = sc["mu_ground"], sc["mu_tool"], sc["mu_static"], sc["mu_ramp"]
    ob = sc["object"]
    for i in range(3):
        s.obj_half[i] = ob["half"][i]
        s.obj_pos0[i] = ob["pos0"][i]
    s.obj_mass, s.obj_yaw0 = ob["mass"], ob["yaw0"]
    boxes = sc.get("static_boxes", [])
    assert len(boxes) <= MAX_STATIC
    s.n_static = len(boxes)
    for j, b in enumerate(boxes):
        for i in range(3):
            s.st_center[j][i] = b["center"][i]
            s.st_half[j][i] = b["half"][i]
        s.st_yaw[j], s.st_pitch[j] = b.get("yaw", 0.0), b.get("pitch", 0.0)
        s.st_ramp[j] = 1 if b.get("ramp", False) else 0
    pu = sc.get("pusher")
    if pu:
        s.pusher_radius, s.pusher_standoff, s.pusher_height = pu["radius"], pu["standoff"], pu["height"]
        s.pusher_vmax, s.pusher_steps = pu["vmax"], pu["steps"]
    go = sc.get("goal")
    if go:
        s.goal_rho_lo, s.goal_rho_hi = go.get("rho", (0.0, 0.0))
        s.goal_phi_lo, s.goal_phi_hi = go.get("phi", (0.0, 0.0))
        s.goal_tol, s.time_weight = go["tol"], go["time_weight"]
    rb = sc.get("robot")
    if rb:
        J = rb["joints"]
        s.n_joints = len(J)
        for j, jd in enumerate(J):
            s.j_type[j], s.j_axis[j], s.j_parent[j], s.b_collide[j] = jd["type"], jd["axis"], jd["parent"], jd["collide"]
            s.b_mass[j], s.j_inom[j], s.q0[j] = jd["mass"], jd["inom"], rb["q0"][j]
            for k in range(3):
                s.j_origin[j][k] = jd["origin"][k]
                s.b_com[j][k] = jd["com"][k]
                s.b_half[j][k] = jd["half"][k]
        s.ee_body = rb["ee_body"]
        for k in range(3):
            s.ee_offset[k] = rb["ee_offset"][k]
        ct = sc["controller"]
        s.ik_iters = ct["ik_iters"]
        for f in ("omega_c", "zeta", "ik_lambda", "base_vmin", "base_vmax", "base_wmax", "base_tol", "yaw_tol",
                  "ee_tol", "t_approach", "t_descend", "t_close", "t_lift", "t_transfer", "t_release",
                  "timeout_move", "timeout_pick", "timeout_place", "pregrasp", "finger_open", "finger_closed",
                  "joint_speed_max", "accel_max"):
            setattr(s, f, ct[f])
        for f in ("push_vmin", "push_vmax", "push_dmax", "timeout_push"):
            setattr(s, f, ct.get(f, 0.0))
        s.rest_speed = sc["rest_speed"]
        s.goal_static = sc["goal_static"]
        gb = sc.get("goal_box")
        if gb:
            for k in range(3):
                s.goal_box_center[k] = gb["center"][k]
                s.goal_box_half[k] = gb["half"][k]
    s.obj_mu_lo, s.obj_mu_hi = ob.get("mu", (0.0, 0.0))
    s.settle_steps = sc.get("settle_steps", 0)
    s.fail_stop = int(sc.get("fail_stop", 0))
    dr = sc.get("domain_randomization")
    if dr:
        s.dr_scenarios = int(dr["scenarios"])
        s.dr_reduce = {"mean": 0, "max": 1}[dr.get("reduce", "mean")]
        s.dr_mu_lo, s.dr_mu_hi = dr.get("mu", (0.0, 0.0))
        s.dr_mass_lo, s.dr_mass_hi = dr.get("mass", (0.0, 0.0))
    return s


def philox(seed, tag, block, sample, it, inst):
    out = np.zeros(4, np.uint32)
    lib().ref_philox(seed, tag, block, sample, it, inst, _ptr(out))
    return out


def philox_raw(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().ref_philox_raw(_ptr(c), _ptr(k), _ptr(out))
    return out


def u01(x):
    x = np.ascontiguousarray(x, np.uint32)
    out = np.zeros(x.shape, np.float32)
    lib().ref_u01(_ptr(x), x.size, _ptr(out))
    return out


def logf(u):
    u = np.ascontiguousarray(u, np.float32)
    out = np.zeros(u.shape, np.float32)
    lib().ref_logf_vec(_ptr(u), u.size, _ptr(out))
    return out


def sincos2pi(u):
    u = np.ascontiguousarray(u, np.float32)
    s = np.zeros(u.shape, np.float32)
    c = np.zeros(u.shape, np.float32)
    lib().ref_sincos2pi_vec(_ptr(u), u.size, _ptr(s), _ptr(c))
    return s, c


def normals(seed, it, inst, pop, D):
    out = np.zeros((pop, D), np.float32)
    lib().ref_normals(seed, it, inst, pop, D, _ptr(out))
    return out


def sample(seed, it, inst, pop, mu, L):
    mu = np.ascontiguousarray(mu, np.float64)
    L = np.ascontiguousarray(L, np.float64)
    D = mu.size
    out = np.zeros((pop, D), np.float32)
    lib().ref_sample(seed, it, inst, pop, D, _ptr(mu), _ptr(L), _ptr(out))
    return out


def _region_arrays(reg, D):
    """FP32 arrays of an init_region dict: lo, hi (D), ring dims, rings (n x (cx, cy, r0, r1))."""
    lo = np.ascontiguousarray(reg["lo"][:D], np.float32)
    hi = np.ascontiguousarray(reg["hi"][:D], np.float32)
    rings = reg.get("rings", [])
    dims = np.ascontiguousarray([g["dim"] for g in rings] or [0], np.int32)
    ring = np.ascontiguousarray([list(g["center"]) + list(g["radius"]) for g in rings] or [[0, 0, 0, 0]],
                                np.float32)
    return lo, hi, len(rings), dims, ring


def sample_region(workload, seed, inst, pop):
    """Iteration-0 rows from the workload's init_region (Sec. III-B initial distribution)."""
    D = param_dim(workload)
    lo, hi, n, dims, ring = _region_arrays(workload["cem"]["init_region"], D)
    out = np.zeros((pop, D), np.float32)
    lib().ref_sample_region(seed, inst, pop, D, _ptr(lo), _ptr(hi), n, _ptr(dims), _ptr(ring), _ptr(out))
    return out


def n_env_at(workload, j):
    """n_env(j) of the workload's schedule (its pop when it has none)."""
    cem = workload["cem"]
    sch = cem.get("pop_schedule") or {"final": 0, "iters": 1}
    return int(lib().ref_n_env_at(cem["pop"], sch["final"], sch["iters"], j))


def scenarios(workload, seed, inst=0, n=64):
    """Domain-randomisation scenarios: (friction[n], mass[n]), 0 where the scene draws none."""
    s = make_scene(workload)
    mu = np.zeros(n, np.float64)
    mass = np.zeros(n, np.float64)
    lib().ref_scenarios(ctypes.byref(s), seed, inst, n, _ptr(mu), _ptr(mass))
    return mu, mass


def draw_instance(workload, seed, inst=0):
    """Per-instance scene draws: (goal x, goal y, object friction or 0)."""
    s = make_scene(workload)
    g = np.zeros(3, np.float64)
    lib().ref_draw_instance(ctypes.byref(s), seed, inst, _ptr(g))
    return g


def rollout(workload, seed, Z, inst=0, trace_steps=0, threads=None, with_steps=False, with_rest=False):
    """FP64 rollouts of the rows of Z: returns cost (f64), tier (u8), pose (pop x 7), trace or None
    (and, with_steps, the control steps each rollout simulated; with_rest, the object's final speed and
    the consecutive final control steps it spent below the rest speed)."""
    s = make_scene(workload)
    Z = np.ascontiguousarray(Z, np.float32)
    pop = Z.shape[0]
    cost = np.zeros(pop, np.float64)
    tier = np.zeros(pop, np.uint8)
    pose = np.zeros((pop, 7), np.float64)
    tw = 13 if workload["scene"]["kind"] == "push" else 35
    trace = np.zeros((pop, trace_steps, tw), np.float64) if trace_steps else None
    threads = threads or default_threads()
    steps = np.zeros(pop, np.int32)
    speed = np.zeros(pop, np.float64)
    rest = np.zeros(pop, np.int32)
    rc = lib().ref_rollout(ctypes.byref(s), seed, inst, pop, _ptr(Z), _ptr(cost), _ptr(tier), _ptr(pose),
                           _ptr(trace) if trace is not None else None, trace_steps, threads, _ptr(steps),
                           _ptr(speed), _ptr(rest))
    if rc != 0:
        raise RuntimeError("oracle rollout failed (%d)" % rc)
    out = (cost, tier, pose, trace)
    if with_steps:
        out = out + (steps,)
    if with_rest:
        out = out + (speed, rest)
    return out


def count_ops(workload, seed, z, inst=0):
    """Operation tally of one rollout: dict(add, mul, fma, div, sqrt, trans, flops)."""
    s = make_scene(workload)
    z = np.ascontiguousarray(z, np.float32)
    out = np.zeros(6, np.uint64)
    lib().ref_count_ops(ctypes.byref(s), seed, inst, _ptr(z), _ptr(out))
    d = dict(zip(["add", "mul", "fma", "div", "sqrt", "trans"], [int(v) for v in out]))
    d["flops"] = d["add"] + d["mul"] + 2 * d["fma"] + d["div"] + d["sqrt"]
    return d


def select(cost, tier, n_elite):
    cost = np.ascontiguousarray(cost, np.float32)
    tier = np.ascontiguousarray(tier, np.uint8)
    idx = np.zeros(max(n_elite, 1), np.int32)
    mode = np.zeros(1, np.int32)
    counts = np.zeros(4, np.int32)
    ne = lib().ref_select(cost.size, _ptr(cost), _ptr(tier), n_elite, _ptr(idx), _ptr(mode), _ptr(counts))
    return idx[:ne].copy(), int(mode[0]), counts


def cholesky(A):
    A = np.ascontiguousarray(A, np.float64)
    L = np.zeros_like(A)
    rc = lib().ref_cholesky(A.shape[0], _ptr(A), _ptr(L))
    return L, rc


def factor_cov(S):
    S = np.ascontiguousarray(S, np.float64)
    L = np.zeros_like(S)
    rc = lib().ref_factor_cov(S.shape[0], _ptr(S), _ptr(L))
    return L, rc


def refit(Z, elite, mode, cov_mode, cov0, mu, S):
    Z = np.ascontiguousarray(Z, np.float32)
    D = Z.shape[1]
    elite = np.ascontiguousarray(elite, np.int32)
    cov0 = np.ascontiguousarray(cov0, np.float64)
    mu = np.array(mu, np.float64)
    S = np.array(S, np.float64)
    L = np.zeros((D, D), np.float64)
    rc = lib().ref_refit(D, cov_mode, _ptr(Z), _ptr(elite), elite.size, mode, _ptr(cov0), _ptr(mu), _ptr(S),
                         _ptr(L))
    return mu, S, L, rc


def plan_solve(workload, seed, inst=0, threads=None, iters=None, pop=None):
    cem = workload["cem"]
    D = param_dim(workload)
    pop = pop or cem["pop"]
    iters = iters if iters is not None else cem["iters"]
    cov_mode = 0 if cem["cov_mode"] == "diag" else 1
    mu0 = np.asarray(cem["mu0"], np.float64)
    cov0 = np.diag(np.asarray(cem["cov0_diag"], np.float64))
    s = make_scene(workload)
    best_z = np.zeros(D, np.float32)
    best_cost = np.zeros(1, np.float64)
    best_tier = np.zeros(1, np.int32)
    mu = np.zeros(D, np.float64)
    S = np.zeros((D, D), np.float64)
    stats = np.zeros((iters, 8), np.float64)
    threads = threads or default_threads()
    sch = cem.get("pop_schedule") or {"final": 0, "iters": 1}
    if sch["final"] > pop:
        raise ValueError("pop_schedule final exceeds pop")
    reg = cem.get("init_region")
    lo = hi = dims = ring = None
    n_rings = 0
    if reg:
        lo, hi, n_rings, dims, ring = _region_arrays(reg, D)
    lib().ref_plan_solve(ctypes.byref(s), seed, inst, pop, cem["n_elite"], iters, cov_mode, _ptr(mu0), _ptr(cov0),
                         threads, _ptr(best_z), _ptr(best_cost), _ptr(best_tier), _ptr(mu), _ptr(S), _ptr(stats),
                         sch["final"], sch["iters"], _ptr(lo) if reg else None, _ptr(hi) if reg else None, n_rings,
                         _ptr(dims) if reg else None, _ptr(ring) if reg else None)
    return dict(best_z=best_z, best_cost=float(best_cost[0]), best_tier=int(best_tier[0]), mu=mu, S=S, stats=stats)


def box_sim(he, m, p0, q0, v0, w0, gvec, k, c, mu, eps_v, h, plane, nsteps):
    """Single free box (optionally on the plane z = 0): nsteps x 13 trace of p q v w."""
    prm = np.array(list(he) + [m] + list(p0) + list(q0) + list(v0) + list(w0) + list(gvec)
                   + [k, c, mu, eps_v, h, 1.0 if plane else 0.0, 0.0], np.float64)
    out = np.zeros((nsteps, 13), np.float64)
    lib().ref_box_sim(_ptr(prm), nsteps, _ptr(out))
    return out


def sphere_box(c, r, p, q, he):
    a = [np.ascontiguousarray(v, np.float64) for v in (c, p, q, he)]
    out = np.zeros(7, np.float64)
    n = lib().ref_sphere_box(_ptr(a[0]), ctypes.c_double(r), _ptr(a[1]), _ptr(a[2]), _ptr(a[3]), _ptr(out))
    return out if n else None


def box_box(pA, qA, heA, pB, qB, heB):
    """Contacts of A's vertices inside B: rows x[3] n[3] d (n from B into A)."""
    a = [np.ascontiguousarray(v, np.float64) for v in (pA, qA, heA, pB, qB, heB)]
    out = np.zeros((8, 7), np.float64)
    n = lib().ref_box_box(*[_ptr(v) for v in a], _ptr(out))
    return out[:n].copy()


def _f64(a, n=None):
    return np.ascontiguousarray(a if a is not None else np.zeros(n), np.float64)


def tree_aba(tree, q, qd, tau, fext=None, g=9.81):
    n = tree.n
    fx = _f64(fext, (n, 6)) if fext is not None else np.zeros((n, 6))
    out = np.zeros(n)
    lib().ref_tree_aba(ctypes.byref(tree), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(tau)), _ptr(fx), g, _ptr(out))
    return out


def tree_rnea(tree, q, qd, qdd, fext=None, g=9.81):
    n = tree.n
    fx = _f64(fext, (n, 6)) if fext is not None else np.zeros((n, 6))
    out = np.zeros(n)
    lib().ref_tree_rnea(ctypes.byref(tree), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(qdd)), _ptr(fx), g, _ptr(out))
    return out


def tree_crba(tree, q):
    M = np.zeros((tree.n, tree.n))
    lib().ref_tree_crba(ctypes.byref(tree), _ptr(_f64(q)), _ptr(M))
    return M


def tree_fk(tree, q):
    R = np.zeros((tree.n, 3, 3))
    p = np.zeros((tree.n, 3))
    lib().ref_tree_fk(ctypes.byref(tree), _ptr(_f64(q)), _ptr(R), _ptr(p))
    return R, p


MLP_DIMS = (16, 256, 256, 256, 8)


def mlp_n_params():
    return int(lib().ref_mlp_n_params())


def mlp_init(seed):
    P = np.zeros(mlp_n_params())
    lib().ref_mlp_init(seed, _ptr(P))
    return P


def mlp_forward(P, x, bf16=False):
    x = _f64(x)
    n = x.shape[0]
    y = np.zeros((n, MLP_DIMS[-1]))
    lib().ref_mlp_forward(_ptr(_f64(P)), _ptr(x), n, _ptr(y), 1 if bf16 else 0)
    return y


def mlp_loss_grad(P, x, t, want_grad=True, bf16=False):
    """MSE loss and its gradient; bf16: with BF16 operands in every product (forward and backward)."""
    x, t = _f64(x), _f64(t)
    g = np.zeros(mlp_n_params()) if want_grad else None
    f = lib().ref_mlp_loss_grad_bf16 if bf16 else lib().ref_mlp_loss_grad
    loss = f(_ptr(_f64(P)), _ptr(x), _ptr(t), x.shape[0], _ptr(g) if want_grad else None)
    return loss, g


def adam_step(P, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays P, m, v (t = step number from 1)."""
    lib().ref_adam_step(_ptr(P), _ptr(_f64(g)), _ptr(m), _ptr(v), P.size, lr, b1, b2, eps, t)


def mlp_slices():
    """(W, b) slices of the flat parameter vector per layer; W as (out, in)."""
    out, o = [], 0
    for l in range(4):
        ni, no = MLP_DIMS[l], MLP_DIMS[l + 1]
        out.append((slice(o, o + ni * no), (no, ni), slice(o + ni * no, o + ni * no + no)))
        o += ni * no + no
    return out


def tree_sim(tree, q0, qd0, g, h, n):
    out = np.zeros((n, 2 * tree.n))
    lib().ref_tree_sim(ctypes.byref(tree), _ptr(_f64(q0)), _ptr(_f64(qd0)), g, h, n, _ptr(out))
    return out[:, :tree.n], out[:, tree.n:]


def object_sim(workload, p0, q0, v0, n):
    s = make_scene(workload)
    out = np.zeros((n, 13))
    lib().ref_object_sim(ctypes.byref(s), _ptr(_f64(p0)), _ptr(_f64(q0)), _ptr(_f64(v0)), n, _ptr(out))
    return out


def ik(workload, q, pt, Rt):
    s = make_scene(workload)
    qo = np.zeros(len(q))
    pe = np.zeros(3)
    Re = np.zeros(9)
    lib().ref_ik(ctypes.byref(s), _ptr(_f64(q)), _ptr(_f64(pt)), _ptr(_f64(np.asarray(Rt).ravel())), _ptr(qo),
                 _ptr(pe), _ptr(Re))
    return qo, pe, Re.reshape(3, 3)


def set_face_cull(on):
    """Face-axis broadphase of the box-box tests on (default) or off."""
    lib().ref_set_face_cull(1 if on else 0)


def robot_log(workload, seed, z, steps=None, trace_steps=0, inst=0):
    """One robot rollout with its action-sequencing record:
    dict(act[steps], qref[steps][11], ends[4], ok bits, cost, tier, trace)."""
    s = make_scene(workload)
    steps = steps if steps is not None else workload["scene"]["horizon"]
    z = np.ascontiguousarray(z, np.float32)
    act = np.zeros(max(steps, 1), np.int32)
    qref = np.zeros((max(steps, 1), 11), np.float64)
    ends = np.zeros(4, np.int32)
    ok = np.zeros(1, np.int32)
    out = np.zeros(2, np.float64)
    trace = np.zeros((trace_steps, 35), np.float64) if trace_steps else None
    rc = lib().ref_robot_log(ctypes.byref(s), seed, inst, _ptr(z), steps, _ptr(act), _ptr(qref), _ptr(ends),
                             _ptr(ok), _ptr(out), _ptr(trace) if trace is not None else None, trace_steps)
    if rc != 0:
        raise RuntimeError("robot_log needs a robot scene")
    return dict(act=act[:steps], qref=qref[:steps], ends=ends, ok=int(ok[0]), cost=float(out[0]), tier=int(out[1]),
                trace=trace)


def grasp_check(workload, q, obj_p, obj_q):
    """(left touches, right touches, centre between the fingers, all three) at a hand-set state."""
    s = make_scene(workload)
    out = np.zeros(4, np.int32)
    lib().ref_grasp_check(ctypes.byref(s), _ptr(_f64(q)), _ptr(_f64(obj_p)), _ptr(_f64(obj_q)), _ptr(out))
    return tuple(bool(v) for v in out)


def count_block(which):
    """Operation tally of one building block (0 free-body step, 1 penalty force, 2 cross, 3 quaternion matrix)."""
    out = np.zeros(6, np.uint64)
    lib().ref_count_block(int(which), _ptr(out))
    d = dict(zip(["add", "mul", "fma", "div", "sqrt", "trans"], [int(v) for v in out]))
    d["flops"] = d["add"] + d["mul"] + 2 * d["fma"] + d["div"] + d["sqrt"]
    return d


def gelu(x):
    """The network's GELU (tanh form) and its derivative at the points x."""
    x = _f64(np.atleast_1d(x))
    y, dy = np.zeros_like(x), np.zeros_like(x)
    lib().ref_gelu_vec(_ptr(x), x.size, _ptr(y), _ptr(dy))
    return y, dy


def to_bf16(x):
    """The oracle's bfloat16 rounding (through FP32, ties to even), as float64 values."""
    x = _f64(np.atleast_1d(x))
    y = np.zeros_like(x)
    lib().ref_to_bf16_vec(_ptr(x), x.size, _ptr(y))
    return y
