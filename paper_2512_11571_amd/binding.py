"""Thin ctypes binding of libcemtamp.so (include/cemtamp.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module turns
workload dicts into the C structs, torch device tensors into pointers and the
current torch stream into a hipStream_t.  There is no fallback: if the
library is not built or no GPU is present, calls raise.
"""
import ctypes
import math
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcemtamp.so")

CEM_OK = 0
ERRORS = {1: "CEM_E_ARG", 2: "CEM_E_SCENE", 3: "CEM_E_ALLOC", 4: "CEM_E_HIP", 5: "CEM_E_NUMERIC", 6: "CEM_E_STATE"}
SCENE_KIND = {"push": 1, "pickplace": 2, "movepush": 3}
DIM = {"push": 3, "pickplace": 16, "movepush": 12}
MAX_STATIC = 8
MAX_D = 16
MAX_ANNULI = 4
MAX_DR = 64
MAX_JOINTS = 12
STATS_COLS = 8
TRACE_FREE = 13
TRACE_ROBOT = 35
CONTROLLER_FIELDS = ("omega_c", "zeta", "ik_lambda", "base_vmin", "base_vmax", "base_wmax", "base_tol", "yaw_tol",
                     "ee_tol", "t_approach", "t_descend", "t_close", "t_lift", "t_transfer", "t_release",
                     "timeout_move", "timeout_pick", "timeout_place", "pregrasp", "finger_open", "finger_closed",
                     "joint_speed_max", "accel_max")

_f = ctypes.c_float
_i = ctypes.c_int32


class CemScene(ctypes.Structure):
    _fields_ = [
        ("kind", _i), ("substeps", _i), ("horizon", _i),
        ("dt", _f), ("gravity", _f), ("k_contact", _f), ("c_contact", _f), ("eps_v", _f),
        ("mu_ground", _f), ("mu_tool", _f), ("mu_static", _f), ("mu_ramp", _f),
        ("obj_half", _f * 3), ("obj_mass", _f), ("obj_pos0", _f * 3), ("obj_yaw0", _f),
        ("n_static", _i),
        ("st_center", (_f * 3) * MAX_STATIC), ("st_half", (_f * 3) * MAX_STATIC),
        ("st_yaw", _f * MAX_STATIC), ("st_pitch", _f * MAX_STATIC), ("st_ramp", _i * MAX_STATIC),
        ("pusher_radius", _f), ("pusher_standoff", _f), ("pusher_height", _f), ("pusher_vmax", _f),
        ("pusher_steps", _i),
        ("goal_rho_lo", _f), ("goal_rho_hi", _f), ("goal_phi_lo", _f), ("goal_phi_hi", _f),
        ("goal_tol", _f), ("time_weight", _f),
        ("n_joints", _i), ("j_type", _i * MAX_JOINTS), ("j_axis", _i * MAX_JOINTS), ("j_parent", _i * MAX_JOINTS),
        ("j_origin", (_f * 3) * MAX_JOINTS), ("b_mass", _f * MAX_JOINTS), ("b_com", (_f * 3) * MAX_JOINTS),
        ("b_half", (_f * 3) * MAX_JOINTS), ("j_inom", _f * MAX_JOINTS), ("q0", _f * MAX_JOINTS),
        ("ee_body", _i), ("ee_offset", _f * 3),
        ("ik_iters", _i), ("omega_c", _f), ("zeta", _f), ("ik_lambda", _f),
        ("base_vmin", _f), ("base_vmax", _f), ("base_wmax", _f), ("base_tol", _f), ("yaw_tol", _f), ("ee_tol", _f),
        ("t_approach", _f), ("t_descend", _f), ("t_close", _f), ("t_lift", _f), ("t_transfer", _f),
        ("t_release", _f), ("timeout_move", _f), ("timeout_pick", _f), ("timeout_place", _f),
        ("pregrasp", _f), ("finger_open", _f), ("finger_closed", _f), ("rest_speed", _f),
        ("goal_static", _i), ("joint_speed_max", _f), ("accel_max", _f),
        ("push_vmin", _f), ("push_vmax", _f), ("push_dmax", _f), ("timeout_push", _f),
        ("obj_mu_lo", _f), ("obj_mu_hi", _f), ("goal_box_center", _f * 3), ("goal_box_half", _f * 3),
        ("settle_steps", _i), ("fail_stop", _i), ("dr_scenarios", _i), ("dr_reduce", _i),
        ("dr_mu_lo", _f), ("dr_mu_hi", _f), ("dr_mass_lo", _f), ("dr_mass_hi", _f),
    ]


class CemInitRegion(ctypes.Structure):
    _fields_ = [
        ("lo", _f * MAX_D), ("hi", _f * MAX_D), ("n_annuli", _i), ("ann_dim", _i * MAX_ANNULI),
        ("ann_center", (_f * 2) * MAX_ANNULI), ("ann_radius", (_f * 2) * MAX_ANNULI),
    ]


class CemProblem(ctypes.Structure):
    _fields_ = [
        ("scene", ctypes.POINTER(CemScene)),
        ("pop", _i), ("n_elite", _i), ("cov_mode", _i), ("lanes_per_env", _i),
        ("mu0", ctypes.POINTER(ctypes.c_double)), ("cov0", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32),
        ("pop_final", _i), ("pop_ramp_iters", _i),
        ("init_region", ctypes.POINTER(CemInitRegion)),
    ]


class CemResult(ctypes.Structure):
    _fields_ = [
        ("best_z", _f * MAX_D), ("best_cost", _f), ("best_tier", _i), ("iters_done", _i), ("dim", _i),
        ("mu", ctypes.c_double * MAX_D), ("cov", ctypes.c_double * (MAX_D * MAX_D)),
    ]


EXPORTS = ["cem_init", "cem_free", "cem_dim", "cem_sizeof", "cem_strerror", "cem_last_error", "cem_sample", "rollout_batch",
           "rollout_trace", "cem_refit", "plan_solve", "cem_get_theta", "cem_set_theta", "cem_get_factor",
           "cem_get_instance", "cem_get_scenarios", "cem_env_steps", "cem_get_outcomes", "cem_pop_at", "cem_reset",
           "cem_valu_fma_rate", "cem_batch_init", "cem_batch_free", "cem_batch_size",
           "cem_batch_last_error", "cem_batch_instance", "cem_batch_autotune", "cem_batch_step", "cem_batch_solve",
           "cem_batch_record", "cem_mlp_init", "cem_mlp_free", "cem_mlp_n_params", "cem_mlp_last_error",
           "cem_mlp_get_params", "cem_mlp_set_params", "cem_mlp_get_norm", "cem_mlp_set_norm", "cem_mlp_fit_norm",
           "cem_mlp_forward", "cem_mlp_forward_static", "cem_mlp_loss_grad", "cem_mlp_train_step", "cem_mlp_train", "cem_screen",
           "plan_solve_screened", "cem_set_robot_specialization"]

_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcemtamp.so is not built: run `python -m paper_2512_11571_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        L.cem_init.argtypes = [P(CemProblem), P(vp)]
        L.cem_free.argtypes = [vp]
        L.cem_free.restype = None
        L.cem_dim.argtypes = [vp]
        L.cem_strerror.argtypes = [ctypes.c_int]
        L.cem_strerror.restype = ctypes.c_char_p
        L.cem_last_error.argtypes = [vp]
        L.cem_last_error.restype = ctypes.c_char_p
        L.cem_sample.argtypes = [vp, _i, vp, vp]
        L.rollout_batch.argtypes = [vp, vp, _i, vp, vp, vp, vp]
        L.rollout_trace.argtypes = [vp, vp, _i, _i, vp, vp]
        L.cem_refit.argtypes = [vp, vp, vp, vp, _i, vp, vp, vp]
        L.plan_solve.argtypes = [vp, _i, P(CemResult), vp, vp]
        L.cem_get_theta.argtypes = [vp, vp, vp]
        L.cem_set_theta.argtypes = [vp, vp, vp]
        L.cem_get_factor.argtypes = [vp, vp]
        L.cem_get_instance.argtypes = [vp, vp]
        L.cem_env_steps.argtypes = [vp, P(ctypes.c_uint64)]
        L.cem_get_outcomes.argtypes = [vp, _i, vp, vp, vp]
        L.cem_pop_at.argtypes = [vp, _i]
        L.cem_get_scenarios.argtypes = [vp, vp, vp]
        L.cem_valu_fma_rate.argtypes = [P(ctypes.c_double), vp]
        L.cem_set_robot_specialization.argtypes = [ctypes.c_int32]
        L.cem_set_robot_specialization.restype = None
        L.cem_reset.argtypes = [vp]
        L.cem_sizeof.argtypes = [ctypes.c_int]
        L.cem_batch_init.argtypes = [vp, vp, _i, P(vp)]
        L.cem_batch_free.argtypes = [vp]
        L.cem_batch_free.restype = None
        L.cem_batch_size.argtypes = [vp]
        L.cem_batch_last_error.argtypes = [vp]
        L.cem_batch_last_error.restype = ctypes.c_char_p
        L.cem_batch_instance.argtypes = [vp, _i]
        L.cem_batch_instance.restype = vp
        L.cem_batch_autotune.argtypes = [vp, vp]
        L.cem_batch_step.argtypes = [vp, vp]
        L.cem_batch_solve.argtypes = [vp, _i, vp, vp]
        i64 = ctypes.c_int64
        L.cem_batch_record.argtypes = [vp, _i, vp, vp, i64, vp, vp]
        L.cem_mlp_init.argtypes = [ctypes.c_uint64, _i, P(vp)]
        L.cem_mlp_free.argtypes = [vp]
        L.cem_mlp_free.restype = None
        L.cem_mlp_last_error.argtypes = [vp]
        L.cem_mlp_last_error.restype = ctypes.c_char_p
        L.cem_mlp_get_params.argtypes = [vp, vp]
        L.cem_mlp_set_params.argtypes = [vp, vp]
        L.cem_mlp_get_norm.argtypes = [vp, vp]
        L.cem_mlp_set_norm.argtypes = [vp, vp]
        L.cem_mlp_fit_norm.argtypes = [vp, vp, vp, i64, vp]
        L.cem_mlp_forward.argtypes = [vp, vp, _i, vp, vp]
        L.cem_mlp_forward_static.argtypes = [vp, vp, _i, vp, vp]
        L.cem_mlp_loss_grad.argtypes = [vp, vp, vp, _i, vp, vp, vp]
        L.cem_mlp_train_step.argtypes = [vp, vp, vp, _i, ctypes.c_float, vp, vp]
        L.cem_mlp_train.argtypes = [vp, vp, vp, i64, _i, _i, ctypes.c_float, ctypes.c_uint64, vp]
        L.cem_screen.argtypes = [vp, vp, _i, _i, vp, vp, vp]
        L.plan_solve_screened.argtypes = [vp, vp, _i, _i, P(CemResult), vp, vp, vp]
        for which, st in enumerate((CemScene, CemProblem, CemResult, CemInitRegion)):
            if L.cem_sizeof(which) != ctypes.sizeof(st):
                raise RuntimeError("ABI struct layout mismatch for %s" % st.__name__)
        _lib = L
    return _lib


def valu_fma_rate(stream=None):
    """Measured FP32 vector FMA rate of the current device, FLOP/s (a measurement aid)."""
    r = ctypes.c_double(0.0)
    rc = lib().cem_valu_fma_rate(ctypes.byref(r), _stream(stream) if stream is not None else None)
    if rc != CEM_OK:
        raise CemError(rc, lib().cem_strerror(rc).decode())
    return r.value


def set_robot_specialization(enable):
    """cem_set_robot_specialization: False makes launches prepared afterwards take the
    generic rollout instance instead of the one compiled for the robot model."""
    lib().cem_set_robot_specialization(1 if enable else 0)


class CemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


def make_scene(workload):
    """cem_scene from a workload dict."""
    sc = workload["scene"]
    s = CemScene()
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
    if len(boxes) > MAX_STATIC:
        raise ValueError("at most %d static boxes" % MAX_STATIC)
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
        if len(J) > MAX_JOINTS:
            raise ValueError("at most %d joints" % MAX_JOINTS)
        s.n_joints = len(J)
        for j, jd in enumerate(J):
            s.j_type[j], s.j_axis[j], s.j_parent[j] = jd["type"], jd["axis"], jd["parent"]
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
        for f in CONTROLLER_FIELDS:
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
    s.settle_steps = int(sc.get("settle_steps", 0))
    s.fail_stop = int(sc.get("fail_stop", 0))
    dr = sc.get("domain_randomization")
    if dr:
        s.dr_scenarios = int(dr["scenarios"])
        s.dr_reduce = {"mean": 0, "max": 1}[dr.get("reduce", "mean")]
        s.dr_mu_lo, s.dr_mu_hi = dr.get("mu", (0.0, 0.0))
        s.dr_mass_lo, s.dr_mass_hi = dr.get("mass", (0.0, 0.0))
    return s


def _dptr(t):
    """Device pointer of a CUDA/HIP torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_problem(workload, seed=0, instance=0, pop=None, n_elite=None, mu0=None, cov0=None, lanes=None):
    """(cem_problem, keep-alive list) for a workload dict.  `lanes` (else the
    workload's cem.lanes_per_env, else 1) is the lanes per environment."""
    cem = workload["cem"]
    scene = make_scene(workload)
    mu0 = np.ascontiguousarray(mu0 if mu0 is not None else cem["mu0"], np.float64)
    if cov0 is None:
        cov0 = np.diag(np.asarray(cem["cov0_diag"], np.float64))
    cov0 = np.ascontiguousarray(cov0, np.float64)
    p = CemProblem()
    p.scene = ctypes.pointer(scene)
    p.pop = int(pop if pop is not None else cem["pop"])
    p.n_elite = int(n_elite if n_elite is not None else cem["n_elite"])
    p.cov_mode = 0 if cem["cov_mode"] == "diag" else 1
    p.mu0 = mu0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.cov0 = cov0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.seed, p.instance = int(seed), int(instance)
    p.lanes_per_env = int(lanes if lanes is not None else cem.get("lanes_per_env", 0))
    keep = [scene, mu0, cov0]
    sch = cem.get("pop_schedule")
    if sch:
        if sch["final"] > p.pop:
            raise ValueError("pop_schedule final %d exceeds pop %d" % (sch["final"], p.pop))
        p.pop_final, p.pop_ramp_iters = int(sch["final"]), int(sch["iters"])
    reg = cem.get("init_region")
    if reg:
        r = make_region(reg)
        p.init_region = ctypes.pointer(r)
        keep.append(r)
    return p, keep


def make_region(reg):
    """cem_init_region from {"lo": [D], "hi": [D], "rings": [{"dim", "center", "radius"}]}."""
    r = CemInitRegion()
    for d, (a, b) in enumerate(zip(reg["lo"], reg["hi"])):
        r.lo[d], r.hi[d] = a, b
    rings = reg.get("rings", [])
    if len(rings) > MAX_ANNULI:
        raise ValueError("at most %d rings" % MAX_ANNULI)
    r.n_annuli = len(rings)
    for k, g in enumerate(rings):
        r.ann_dim[k] = g["dim"]
        r.ann_center[k][0], r.ann_center[k][1] = g["center"]
        r.ann_radius[k][0], r.ann_radius[k][1] = g["radius"]
    return r



def _result_dict(res, D):
    return dict(best_z=np.array(res.best_z[:D], np.float32), best_cost=float(res.best_cost),
                best_tier=int(res.best_tier), iters_done=int(res.iters_done),
                mu=np.array(res.mu[:D]), cov=np.array(res.cov[:D * D]).reshape(D, D))


class Context:
    """One CE problem on the current device (wraps cem_ctx*)."""

    def __init__(self, workload, seed=0, instance=0, pop=None, n_elite=None, mu0=None, cov0=None, handle=None,
                 lanes=None):
        self.workload = workload
        self.kind = workload["scene"]["kind"]
        self.D = DIM[self.kind]
        if handle is not None:          # borrowed from a batch, which owns it
            self.h, self._owned = handle, False
            self.pop, self.n_elite = workload["cem"]["pop"], workload["cem"]["n_elite"]
            return
        p, self._keep = make_problem(workload, seed, instance, pop, n_elite, mu0, cov0, lanes)
        self.pop, self.n_elite = p.pop, p.n_elite
        h = ctypes.c_void_p()
        rc = lib().cem_init(ctypes.byref(p), ctypes.byref(h))
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_strerror(rc).decode())
        self.h, self._owned = h, True

    def _check(self, rc):
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owned", False):
                lib().cem_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- the C ABI calls -------------------------------------------------
    def cem_sample(self, it, Z, stream=None):
        self._check(lib().cem_sample(self.h, int(it), _dptr(Z), _stream(stream)))

    def rollout_batch(self, Z, cost, tier, pose=None, stream=None):
        self._check(lib().rollout_batch(self.h, _dptr(Z), Z.shape[0], _dptr(cost), _dptr(tier), _dptr(pose),
                                        _stream(stream)))

    def rollout_trace(self, Z, n_steps, trace, stream=None):
        self._check(lib().rollout_trace(self.h, _dptr(Z), Z.shape[0], int(n_steps), _dptr(trace), _stream(stream)))

    def cem_refit(self, Z, cost, tier, elite_idx=None, sel_info=None, stream=None):
        self._check(lib().cem_refit(self.h, _dptr(Z), _dptr(cost), _dptr(tier), Z.shape[0], _dptr(elite_idx),
                                    _dptr(sel_info), _stream(stream)))

    def plan_solve(self, iters, stream=None):
        res = CemResult()
        stats = np.zeros((max(iters, 1), STATS_COLS), np.float32)
        s = _stream(stream) if stream is not None else None
        self._check(lib().plan_solve(self.h, int(iters), ctypes.byref(res), _np_ptr(stats), s))
        out = _result_dict(res, self.D)
        out["stats"] = stats[:iters]
        return out

    def get_theta(self):
        mu = np.zeros(self.D)
        cov = np.zeros((self.D, self.D))
        self._check(lib().cem_get_theta(self.h, _np_ptr(mu), _np_ptr(cov)))
        return mu, cov

    def set_theta(self, mu, cov):
        mu = np.ascontiguousarray(mu, np.float64)
        cov = np.ascontiguousarray(cov, np.float64)
        self._check(lib().cem_set_theta(self.h, _np_ptr(mu), _np_ptr(cov)))

    def get_factor(self):
        L = np.zeros((self.D, self.D))
        self._check(lib().cem_get_factor(self.h, _np_ptr(L)))
        return L

    def get_instance(self):
        """Per-instance scene draws: (goal x, goal y, object friction or 0)."""
        g = np.zeros(3)
        self._check(lib().cem_get_instance(self.h, _np_ptr(g)))
        return g

    def get_scenarios(self):
        """Domain-randomisation scenarios: (friction[64], mass[64]) as drawn (0 where none)."""
        mu = np.zeros(MAX_DR, np.float32)
        mass = np.zeros(MAX_DR, np.float32)
        self._check(lib().cem_get_scenarios(self.h, _np_ptr(mu), _np_ptr(mass)))
        return mu, mass

    def pop_at(self, it):
        """n_env(it) of the problem's schedule (its pop when it has none)."""
        return int(lib().cem_pop_at(self.h, int(it)))

    def env_steps(self):
        """Control steps simulated by this context's rollouts so far (summed over environments)."""
        n = ctypes.c_uint64(0)
        self._check(lib().cem_env_steps(self.h, ctypes.byref(n)))
        return int(n.value)

    def outcomes(self, n=None):
        """(cost, tier, pose) of rows 0..n-1 of the context's own outcome buffers (the last iteration's)."""
        n = self.pop if n is None else int(n)
        cost = np.zeros(n, np.float32)
        tier = np.zeros(n, np.uint8)
        pose = np.zeros((n, 7), np.float32)
        self._check(lib().cem_get_outcomes(self.h, n, _np_ptr(cost), _np_ptr(tier), _np_ptr(pose)))
        return cost, tier, pose

    def reset(self):
        self._check(lib().cem_reset(self.h))


class Batch:
    """Many independent CE problems iterated together (wraps cem_batch*).

    instances: list of dicts {"workload", "seed", "instance", "iters"}."""

    def __init__(self, instances):
        self.instances = instances
        n = len(instances)
        probs = (CemProblem * n)()
        self._keep = []
        for i, inst in enumerate(instances):
            p, keep = make_problem(inst["workload"], inst["seed"], inst["instance"])
            probs[i] = p
            self._keep.append(keep)
        self._probs = probs
        iters = np.ascontiguousarray([inst["iters"] for inst in instances], np.int32)
        h = ctypes.c_void_p()
        rc = lib().cem_batch_init(probs, _np_ptr(iters), n, ctypes.byref(h))
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_strerror(rc).decode())
        self.h = h

    def _check(self, rc):
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().cem_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def instance(self, i):
        """Borrowed Context view of instance i (theta, factor, instance draws)."""
        return Context(self.instances[i]["workload"], handle=lib().cem_batch_instance(self.h, i))

    def autotune(self):
        cfg = np.zeros(3, np.int32)
        self._check(lib().cem_batch_autotune(self.h, _np_ptr(cfg)))
        return dict(grid=int(cfg[0]), envs_per_item=int(cfg[1]), rollout_us=int(cfg[2]))

    def step(self, stream=None):
        self._check(lib().cem_batch_step(self.h, _stream(stream) if stream is not None else None))

    def solve(self, iters, stream=None):
        n = len(self.instances)
        res = (CemResult * n)()
        self._check(lib().cem_batch_solve(self.h, int(iters), res, _stream(stream) if stream is not None else None))
        return [_result_dict(res[i], DIM[self.instances[i]["workload"]["scene"]["kind"]]) for i in range(n)]

    def record(self, iters, X, Y):
        """Run iters iterations, appending (parameters, outcome) rows to device tensors X, Y; returns rows."""
        n = ctypes.c_int64()
        self._check(lib().cem_batch_record(self.h, int(iters), _dptr(X), _dptr(Y), X.shape[0], ctypes.byref(n),
                                           None))
        return int(n.value)


class Mlp:
    """The screening surrogate (wraps cem_mlp*)."""

    def __init__(self, seed=0, max_rows=65536):
        h = ctypes.c_void_p()
        rc = lib().cem_mlp_init(int(seed), int(max_rows), ctypes.byref(h))
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_strerror(rc).decode())
        self.h = h
        self.n_params = lib().cem_mlp_n_params()

    def _check(self, rc):
        if rc != CEM_OK:
            raise CemError(rc, lib().cem_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().cem_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get_params(self):
        P = np.zeros(self.n_params, np.float32)
        self._check(lib().cem_mlp_get_params(self.h, _np_ptr(P)))
        return P

    def set_params(self, P):
        P = np.ascontiguousarray(P, np.float32)
        self._check(lib().cem_mlp_set_params(self.h, _np_ptr(P)))

    def get_norm(self):
        v = np.zeros(48, np.float32)
        self._check(lib().cem_mlp_get_norm(self.h, _np_ptr(v)))
        return v

    def set_norm(self, v):
        v = np.ascontiguousarray(v, np.float32)
        self._check(lib().cem_mlp_set_norm(self.h, _np_ptr(v)))

    def fit_norm(self, X, Y, n=None):
        self._check(lib().cem_mlp_fit_norm(self.h, _dptr(X), _dptr(Y), int(n if n is not None else X.shape[0]),
                                           _stream(None)))

    def forward(self, X, Y, stream=None):
        self._check(lib().cem_mlp_forward(self.h, _dptr(X), X.shape[0], _dptr(Y), _stream(stream)))

    def forward_static(self, X, Y, stream=None):
        """The allocation-free forward (work buffers in the library's fixed device array)."""
        self._check(lib().cem_mlp_forward_static(self.h, _dptr(X), X.shape[0], _dptr(Y), _stream(stream)))

    def loss_grad(self, X, Y, grad=None, loss=None, stream=None):
        self._check(lib().cem_mlp_loss_grad(self.h, _dptr(X), _dptr(Y), X.shape[0], _dptr(grad), _dptr(loss),
                                            _stream(stream)))

    def train_step(self, X, Y, lr, loss=None, stream=None):
        self._check(lib().cem_mlp_train_step(self.h, _dptr(X), _dptr(Y), X.shape[0], float(lr), _dptr(loss),
                                             _stream(stream)))

    def train(self, X, Y, n, batch, epochs, lr, seed=0):
        losses = np.zeros(max(epochs, 1), np.float32)
        self._check(lib().cem_mlp_train(self.h, _dptr(X), _dptr(Y), int(n), int(batch), int(epochs), float(lr),
                                        int(seed), _np_ptr(losses)))
        return losses[:epochs]

    def screen(self, ctx, it, n_sim, Zsim, pred=None, stream=None):
        self._check(lib().cem_screen(ctx.h, self.h, int(it), int(n_sim), _dptr(Zsim), _dptr(pred), _stream(stream)))

    def plan_solve_screened(self, ctx, iters, n_sim):
        res = CemResult()
        stats = np.zeros((max(iters, 1), STATS_COLS), np.float32)
        err = np.zeros(max(iters, 1), np.float32)
        self._check(lib().plan_solve_screened(ctx.h, self.h, int(iters), int(n_sim), ctypes.byref(res),
                                              _np_ptr(stats), _np_ptr(err), None))
        out = _result_dict(res, ctx.D)
        out["stats"] = stats[:iters]
        out["surrogate_err"] = err[:iters]
        return out
