// Oracle: the mobile-manipulator plans.  TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Pick-and-place (Sec. IV-A, plan pi_p&p without the final move to Exit):
//   move_to(x, y, psi, v) -> grasp(q in SO(3)) -> move_to(x, y, psi, v) -> place(x, y, z, psi)
// Each action is a controller run from the step after the previous one ends
// (Problem 1: t_{0,i+1} = T_i + 1) until it succeeds or times out.  Per-step
// cost 1 while the active action is unsuccessful (Eqs. 4-6 and text), scaled
// by dt; success: base within tolerance of the target (move, Eq. 4), end
// effector at the grasp / place pose within tolerance, and for grasping the
// gripper enclosing the object (Eqs. 5-6 and text).  The goal psi_g holds when
// the object rests on the top face of the goal table at T.
//
// Move-and-push (Sec. IV-A, plan pi_m&p):
//   move_to(x, y, psi, v) -> push(start point, heading, distance, speed,
//   approach height, gripper yaw)
// The push controller reaches a start pose above and then at the start point
// with closed fingers, moves the end effector along the push line, then opens
// the gripper; it succeeds when the end effector is at the end of the line
// after the release.  psi_g: the pushed block rests with its centre inside
// the container's inner volume at T.  Every contact of the block uses the
// block's friction coefficient, drawn per instance.
//
// Controllers (the paper's geometric fabrics and A* are replaced, see the
// design notes): straight-line base reference at a commanded speed tracked by
// joint PD; arm joint targets from damped-least-squares IK solved at action
// start, tracked by joint PD along linear joint-space interpolation; gripper
// fingers by PD.  Dynamics: ABA for the 11-joint robot with contact forces on
// the base and finger links as external spatial forces; the object is a free
// box; contacts as in ref_rigid.hpp.
#pragma once
#include "ref_rigid.hpp"
#include "ref_scene.hpp"
#include "ref_spatial.hpp"
#include "ref_push.hpp"

namespace ref {

constexpr int TRACE_ROBOT = 13 + 11 + 11;  // object p q v w, robot q, robot qd
constexpr int NJ = 11;
constexpr int ARM0 = 3, NARM = 6, FL = 9, FR = 10, BASE_BODY = 2;

inline Tree tree_of(const RefScene &s) {
  Tree t;
  t.n = s.n_joints;
  for (int j = 0; j < t.n; ++j) {
    t.type[j] = s.j_type[j];
    t.axis[j] = s.j_axis[j];
    t.parent[j] = s.j_parent[j];
    for (int k = 0; k < 3; ++k) {
      t.origin[j][k] = s.j_origin[j][k];
      t.com[j][k] = s.b_com[j][k];
      t.half[j][k] = s.b_half[j][k];
    }
    t.mass[j] = s.b_mass[j];
  }
  return t;
}

template <class T> inline T wrap_pi(T a) {
  const double pi = 3.14159265358979323846;
  double v = r_val(a);
  // bring to [-pi, pi) by whole turns
  double k = std::floor((v + pi) / (2.0 * pi));
  return a - T(k * 2.0 * pi);
}

// End-effector pose: R (EE -> world) and the EE point.
template <class T>
inline void ee_pose(const RefScene &s, const Tree &tr, const T *q, M3<T> *R, V3<T> *p) {
  M3<T> Rw[MAXJ];
  V3<T> pw[MAXJ];
  forward_kinematics(tr, q, Rw, pw);
  const int e = s.ee_body;
  *R = Rw[e];
  *p = pw[e] + mul(Rw[e], V3<T>(T(s.ee_offset[0]), T(s.ee_offset[1]), T(s.ee_offset[2])));
}

// Solve the n x n SPD system A x = b by Cholesky (in place on copies).
template <class T> inline void spd_solve(int n, const T *A, const T *b, T *x) {
  T L[36];
  for (int i = 0; i < n * n; ++i) L[i] = T(0.0);
  for (int j = 0; j < n; ++j) {
    T d = A[j * n + j];
    for (int k = 0; k < j; ++k) d = d - L[j * n + k] * L[j * n + k];
    const T ljj = r_sqrt(d);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      T t = A[i * n + j];
      for (int k = 0; k < j; ++k) t = t - L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / ljj;
    }
  }
  T y[6];
  for (int i = 0; i < n; ++i) {
    T t = b[i];
    for (int k = 0; k < i; ++k) t = t - L[i * n + k] * y[k];
    y[i] = t / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T t = y[i];
    for (int k = i + 1; k < n; ++k) t = t - L[k * n + i] * x[k];
    x[i] = t / L[i * n + i];
  }
}

// Damped least squares on the six arm joints: `iters` steps of
// dq = J^T (J J^T + lambda^2 I)^-1 e, e = (position error, orientation error
// 1/2 sum_k r_k x r*_k), J the geometric Jacobian at the EE point.
template <class T>
inline void ik_dls(const RefScene &s, const Tree &tr, T *q, const V3<T> &pt, const M3<T> &Rt) {
  const T lam2 = T(s.ik_lambda * s.ik_lambda);
  for (int it = 0; it < s.ik_iters; ++it) {
    M3<T> Rw[MAXJ];
    V3<T> pw[MAXJ];
    forward_kinematics(tr, q, Rw, pw);
    const int e = s.ee_body;
    const V3<T> pe = pw[e] + mul(Rw[e], V3<T>(T(s.ee_offset[0]), T(s.ee_offset[1]), T(s.ee_offset[2])));
    T err[6];
    const V3<T> ep = pt - pe;
    V3<T> eo;
    for (int k = 0; k < 3; ++k) {
      const V3<T> rc(Rw[e].m[0][k], Rw[e].m[1][k], Rw[e].m[2][k]);
      const V3<T> rt(Rt.m[0][k], Rt.m[1][k], Rt.m[2][k]);
      eo = eo + cross(rc, rt);
    }
    err[0] = ep.x; err[1] = ep.y; err[2] = ep.z;
    err[3] = T(0.5) * eo.x; err[4] = T(0.5) * eo.y; err[5] = T(0.5) * eo.z;
    T J[6][NARM];
    for (int c = 0; c < NARM; ++c) {
      const int j = ARM0 + c;
      const V3<T> z = mul(Rw[j], axis_vec<T>(tr.axis[j]));
      const V3<T> jv = cross(z, pe - pw[j]);
      J[0][c] = jv.x; J[1][c] = jv.y; J[2][c] = jv.z;
      J[3][c] = z.x; J[4][c] = z.y; J[5][c] = z.z;
    }
    T A[36];
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) {
        T acc = r == c ? lam2 : T(0.0);
        for (int k = 0; k < NARM; ++k) acc = acc + J[r][k] * J[c][k];
        A[r * 6 + c] = acc;
      }
    T y[6];
    spd_solve(6, A, err, y);
    for (int c = 0; c < NARM; ++c) {
      T d = T(0.0);
      for (int r = 0; r < 6; ++r) d = d + J[r][c] * y[r];
      q[ARM0 + c] = q[ARM0 + c] + d;
    }
  }
}

template <class T> inline M3<T> quat_mat_normalized(T w, T x, T y, T z) {
  T n2 = w * w + x * x + y * y + z * z;
  Q4<T> q;
  if (!(n2 > T(1e-12))) { q.w = T(1.0); q.x = T(0.0); q.y = T(0.0); q.z = T(0.0); }
  else {
    const T inv = T(1.0) / r_sqrt(n2);
    q.w = w * inv; q.x = x * inv; q.y = y * inv; q.z = z * inv;
  }
  return quat_to_mat(q);
}

// Static box pose: rotation Rz(yaw) Ry(pitch).
template <class T> inline M3<T> static_rot(const RefScene &s, int k) {
  const M3<T> Rz = axis_rot(2, r_cos(T(s.st_yaw[k])), r_sin(T(s.st_yaw[k])));
  const M3<T> Ry = axis_rot(1, r_cos(T(s.st_pitch[k])), r_sin(T(s.st_pitch[k])));
  return matmul(Rz, Ry);
}

enum Act { MOVE = 0, PICK = 1, PLACE = 2, PUSH = 3 };

// Smooth 0 -> 1 blend of the references: x^2 (3 - 2x) on [0, 1], clamped.
template <class T> inline T smooth(T x) {
  const T c = r_max(T(0.0), r_min(T(1.0), x));
  return c * c * (T(3.0) - T(2.0) * c);
}

// Collision box of link j from its frame pose (Rw, pw): centre and half extents.
template <class T>
inline void link_box(const RefScene &s, int j, const M3<T> &Rw, const V3<T> &pw, V3<T> *c, V3<T> *h) {
  *c = pw + mul(Rw, V3<T>(T(s.b_com[j][0]), T(s.b_com[j][1]), T(s.b_com[j][2])));
  *h = V3<T>(T(s.b_half[j][0]), T(s.b_half[j][1]), T(s.b_half[j][2]));
}

// The contacts between a finger box (fc, Rf, fh) and the object box (op, oR,
// ohe), both ways: finger vertices inside the object (a[0..*na)) and object
// vertices inside the finger (b[0..*nb)).  The finger touches the object when
// there is at least one.
template <class T>
inline void finger_object_contacts(const V3<T> &fc, const M3<T> &Rf, const V3<T> &fh, const V3<T> &op, const M3<T> &oR,
                                   const V3<T> &ohe, Contact<T> a[8], int *na, Contact<T> b[8], int *nb) {
  const bool nearf = !face_separated(fc, Rf, fh, op, oR, ohe);
  *na = nearf ? box_verts_in_box(fc, Rf, fh, op, oR, ohe, a) : 0;
  *nb = nearf ? box_verts_in_box(op, oR, ohe, fc, Rf, fh, b) : 0;
}

// The gripper encloses the object (Eq. 5 and its text): the object's centre
// lies between the fingers' inner faces.  The fingers slide along the palm's
// y axis, the left one's inner face at palm y = q_L, the right one's at -q_R.
template <class T>
inline bool object_between_fingers(const M3<T> &R_palm, const V3<T> &p_palm, const T *q, const V3<T> &obj_p) {
  const V3<T> ob_palm = mulT(R_palm, obj_p - p_palm);
  return ob_palm.y < q[FL] && ob_palm.y > -q[FR];
}

// Per-step record of a robot rollout's action sequencing: act[t] the action
// that controls step t (n_act once every action has ended) and, optionally,
// the joint references of that step, for the first `steps` control steps;
// ends[a] the step at which action a stopped controlling (T_a + 1 =
// t_{0,a+1}, -1 if it never ended); ok the success bits of the actions.
struct RobotLog {
  int32_t *act = nullptr;
  double *qref = nullptr;  // nullable: the joint references of each logged step, steps x 11
  int steps = 0;
  int32_t ends[4] = {-1, -1, -1, -1};
  int32_t ok = 0;
};

template <class T>
RolloutOut robot_rollout(const RefScene &s, const Instance &inst, const float *z, double *trace, int trace_steps,
                         RobotLog *log = nullptr) {
  const Tree tr = tree_of(s);
  Mat6<T> Ibody[MAXJ];  // body inertias: constants of the tree, built once
  for (int j = 0; j < tr.n; ++j) Ibody[j] = body_inertia<T>(tr, j);
  const T h = T(s.dt) / T((double)s.substeps);
  const T dt = T(s.dt);
  const T g = T(s.gravity);
  const T k = T(s.k_contact), damp = T(s.c_contact), eps_v = T(s.eps_v);
  const T wc = T(s.omega_c), zeta = T(s.zeta);
  const V3<T> ohe(T(s.obj_half[0]), T(s.obj_half[1]), T(s.obj_half[2]));
  const T om = T(inst.obj_mass > 0.0 ? inst.obj_mass : s.obj_mass);
  const V3<T> oIb(om * (ohe.y * ohe.y + ohe.z * ohe.z) / T(3.0), om * (ohe.x * ohe.x + ohe.z * ohe.z) / T(3.0),
                  om * (ohe.x * ohe.x + ohe.y * ohe.y) / T(3.0));
  const V3<T> gv(T(0.0), T(0.0), -g);

  // static geometry
  M3<T> SR[MAX_STATIC];
  V3<T> SP[MAX_STATIC], SH[MAX_STATIC];
  for (int b = 0; b < s.n_static; ++b) {
    SR[b] = static_rot<T>(s, b);
    SP[b] = V3<T>(T(s.st_center[b][0]), T(s.st_center[b][1]), T(s.st_center[b][2]));
    SH[b] = V3<T>(T(s.st_half[b][0]), T(s.st_half[b][1]), T(s.st_half[b][2]));
  }

  // friction of the object's contacts: the instance's draw, else the per-class values
  const bool mu_drawn = inst.obj_mu > 0.0;
  const double mu_obj_ground = mu_drawn ? inst.obj_mu : s.mu_ground;
  const double mu_obj_tool = mu_drawn ? inst.obj_mu : s.mu_tool;

  // plan: pick-and-place = move, pick, move, place with four parameters each;
  // move-push = move (4 parameters), push (8 parameters)
  const bool pnp = s.kind == SCENE_PICKPLACE;
  const int acts[4] = {MOVE, pnp ? PICK : PUSH, MOVE, PLACE};
  const int n_act = pnp ? 4 : 2;
  const int n_par = pnp ? 16 : 12;
  T zp[16];
  for (int i = 0; i < 16; ++i) zp[i] = T(i < n_par ? (double)z[i] : 0.0);

  T q[NJ], qd[NJ];
  for (int j = 0; j < NJ; ++j) { q[j] = T(s.q0[j]); qd[j] = T(0.0); }
  Body<T> ob;
  ob.p = V3<T>(T(s.obj_pos0[0]), T(s.obj_pos0[1]), T(s.obj_pos0[2]) - om * g / (T(4.0) * k));
  ob.q.w = r_cos(T(0.5 * s.obj_yaw0)); ob.q.x = T(0.0); ob.q.y = T(0.0); ob.q.z = r_sin(T(0.5 * s.obj_yaw0));

  int act = 0, t_start = 0;
  bool ok[4] = {false, false, false, false};
  T qref[NJ];
  for (int j = 0; j < NJ; ++j) qref[j] = q[j];
  T qstart[NJ], qa[NJ], qb[NJ], qc[NJ];  // interpolation anchors
  V3<T> ptarget;                 // EE target used in the success test
  T base_from[3], base_to[3], t_move = T(1.0);
  T Ta = T(s.t_approach), Td = T(s.t_descend), Tl = T(s.t_lift), Tp = T(s.t_transfer), Tq = dt;
  const T Tc = T(s.t_close), Tr = T(s.t_release), qd_max = T(s.joint_speed_max);
  // phase duration: the nominal one, stretched so no arm joint reference moves faster than qd_max
  auto span = [&](const T *from, const T *to, T nominal) {
    T m = T(0.0);
    for (int j = ARM0; j < ARM0 + NARM; ++j) m = r_max(m, r_abs(to[j] - from[j]));
    return r_max(nominal, m / qd_max);
  };
  T finger_cmd = T(s.finger_open);
  bool touch[2] = {false, false};
  long unsuccessful = 0;

  auto start_action = [&](int a, int t) {
    t_start = t;
    for (int j = 0; j < NJ; ++j) qstart[j] = q[j];
    const T *pz = zp + 4 * a;
    if (acts[a] == MOVE) {
      base_from[0] = q[0]; base_from[1] = q[1]; base_from[2] = q[2];
      base_to[0] = pz[0]; base_to[1] = pz[1];
      const T dpsi = wrap_pi(pz[2] - q[2]);
      base_to[2] = q[2] + dpsi;
      const T v = r_max(T(s.base_vmin), r_min(T(s.base_vmax), pz[3]));
      const T dx = base_to[0] - q[0], dy = base_to[1] - q[1];
      const T L = r_sqrt(dx * dx + dy * dy);
      t_move = r_max(r_max(L / v, r_abs(dpsi) / T(s.base_wmax)), dt);
    } else if (acts[a] == PICK) {
      const M3<T> Rg = quat_mat_normalized(pz[0], pz[1], pz[2], pz[3]);
      const V3<T> zax(Rg.m[0][2], Rg.m[1][2], Rg.m[2][2]);
      const V3<T> pg = ob.p;
      const V3<T> ppre = pg - T(s.pregrasp) * zax;
      for (int j = 0; j < NJ; ++j) qa[j] = q[j];
      ik_dls(s, tr, qa, ppre, Rg);          // pre-grasp (also the lift target)
      for (int j = 0; j < NJ; ++j) qb[j] = qa[j];
      ik_dls(s, tr, qb, pg, Rg);            // grasp
      ptarget = ppre;
      Ta = span(qstart, qa, T(s.t_approach));
      Td = span(qa, qb, T(s.t_descend));
      Tl = span(qb, qa, T(s.t_lift));
    } else if (acts[a] == PUSH) {
      // push: EE start point ps, heading phi, distance d, speed v, approach
      // height dz, gripper yaw gamma; top-down gripper with closed fingers.
      // Joint targets by IK: above the start (qa), at the start (qb), at the
      // end ps + d (cos phi, sin phi, 0) (qc); the push phase lasts d / v.
      const T cg = r_cos(pz[7]), sg = r_sin(pz[7]);
      M3<T> Rt;
      Rt.m[0][0] = cg; Rt.m[0][1] = sg; Rt.m[0][2] = T(0.0);
      Rt.m[1][0] = sg; Rt.m[1][1] = -cg; Rt.m[1][2] = T(0.0);
      Rt.m[2][0] = T(0.0); Rt.m[2][1] = T(0.0); Rt.m[2][2] = T(-1.0);
      const V3<T> ps(pz[0], pz[1], pz[2]);
      const T dist = r_max(T(0.0), r_min(T(s.push_dmax), pz[4]));
      const T vp = r_max(T(s.push_vmin), r_min(T(s.push_vmax), pz[5]));
      const T dz = r_max(T(0.0), pz[6]);
      const V3<T> pe = ps + dist * V3<T>(r_cos(pz[3]), r_sin(pz[3]), T(0.0));
      for (int j = 0; j < NJ; ++j) qa[j] = q[j];
      ik_dls(s, tr, qa, ps + V3<T>(T(0.0), T(0.0), dz), Rt);
      for (int j = 0; j < NJ; ++j) qb[j] = qa[j];
      ik_dls(s, tr, qb, ps, Rt);
      for (int j = 0; j < NJ; ++j) qc[j] = qb[j];
      ik_dls(s, tr, qc, pe, Rt);
      ptarget = pe;
      Ta = span(qstart, qa, T(s.t_approach));
      Td = span(qa, qb, T(s.t_descend));
      Tq = r_max(span(qb, qc, dist / vp), dt);
    } else {
      const T cy = r_cos(pz[3]), sy = r_sin(pz[3]);
      // top-down: EE z axis along -z, yaw psi about z: Rz(psi) Rx(pi)
      M3<T> Rt;
      Rt.m[0][0] = cy; Rt.m[0][1] = sy; Rt.m[0][2] = T(0.0);
      Rt.m[1][0] = sy; Rt.m[1][1] = -cy; Rt.m[1][2] = T(0.0);
      Rt.m[2][0] = T(0.0); Rt.m[2][1] = T(0.0); Rt.m[2][2] = T(-1.0);
      ptarget = V3<T>(pz[0], pz[1], pz[2]);
      for (int j = 0; j < NJ; ++j) qa[j] = q[j];
      ik_dls(s, tr, qa, ptarget, Rt);
      Tp = span(qstart, qa, T(s.t_transfer));
    }
  };

  auto success = [&](int a, T tau) -> bool {
    const T *pz = zp + 4 * a;
    if (acts[a] == MOVE) {
      const T dx = q[0] - pz[0], dy = q[1] - pz[1];
      return r_sqrt(dx * dx + dy * dy) <= T(s.base_tol) && r_abs(wrap_pi(q[2] - pz[2])) <= T(s.yaw_tol);
    }
    M3<T> Re;
    V3<T> pe;
    ee_pose(s, tr, q, &Re, &pe);
    const T err = norm(pe - ptarget);
    if (acts[a] == PICK) {
      const T tend = Ta + Td + Tc + Tl;
      if (tau < tend) return false;
      // gripper encloses the object: both fingers touching it and the object
      // centre between their inner faces (palm frame y)
      M3<T> Rw[MAXJ];
      V3<T> pw[MAXJ];
      forward_kinematics(tr, q, Rw, pw);
      const bool between = object_between_fingers(Rw[s.ee_body], pw[s.ee_body], q, ob.p);
      return touch[0] && touch[1] && between && err <= T(s.ee_tol);
    }
    const T tend = acts[a] == PUSH ? Ta + Td + Tq + Tr : Tp + Tr;
    return tau >= tend && err <= T(s.ee_tol);
  };

  auto timeout_of = [&](int a) -> double {
    return acts[a] == MOVE ? s.timeout_move
           : acts[a] == PICK ? s.timeout_pick
           : acts[a] == PUSH ? s.timeout_push
                             : s.timeout_place;
  };

  start_action(0, 0);
  bool diverged = false;
  int steps = s.horizon;
  int calm = 0;  // consecutive control steps with every action ended and the object at rest
  int rest_run = 0;  // consecutive control steps with the object at rest (observed only)
  for (int t = 0; t < s.horizon; ++t) {
    // action sequencing
    if (act < n_act) {
      const T tau = T((double)(t - t_start)) * dt;
      const bool succ = success(act, tau);
      const bool tout = r_val(tau) >= timeout_of(act);
      if (succ || tout) {
        ok[act] = succ;
        if (log) {
          log->ends[act] = t;
          if (succ) log->ok |= 1 << act;
        }
        ++act;
        if (!succ && s.fail_stop) {
          // the plan cannot become feasible any more: stop before step t
          steps = t;
          break;
        }
        if (act < n_act) start_action(act, t);
      }
    }
    if (log && t < log->steps) log->act[t] = act;
    if (act < n_act) ++unsuccessful;
    // references for this control step
    if (act < n_act) {
      const T tau = T((double)(t - t_start)) * dt;
      if (acts[act] == MOVE) {
        const T sft = smooth(tau / t_move);
        for (int c = 0; c < 3; ++c) qref[c] = base_from[c] + sft * (base_to[c] - base_from[c]);
        for (int j = ARM0; j < ARM0 + NARM; ++j) qref[j] = qstart[j];
      } else if (acts[act] == PICK) {
        for (int c = 0; c < 3; ++c) qref[c] = qstart[c];
        for (int j = ARM0; j < ARM0 + NARM; ++j) {
          T r;
          if (tau < Ta) r = qstart[j] + smooth(tau / Ta) * (qa[j] - qstart[j]);
          else if (tau < Ta + Td) r = qa[j] + smooth((tau - Ta) / Td) * (qb[j] - qa[j]);
          else if (tau < Ta + Td + Tc) r = qb[j];
          else if (tau < Ta + Td + Tc + Tl) r = qb[j] + smooth((tau - Ta - Td - Tc) / Tl) * (qa[j] - qb[j]);
          else r = qa[j];
          qref[j] = r;
        }
        finger_cmd = tau < Ta + Td ? T(s.finger_open) : T(s.finger_closed);
      } else if (acts[act] == PUSH) {
        for (int c = 0; c < 3; ++c) qref[c] = qstart[c];
        for (int j = ARM0; j < ARM0 + NARM; ++j) {
          T r;
          if (tau < Ta) r = qstart[j] + smooth(tau / Ta) * (qa[j] - qstart[j]);
          else if (tau < Ta + Td) r = qa[j] + smooth((tau - Ta) / Td) * (qb[j] - qa[j]);
          else if (tau < Ta + Td + Tq) r = qb[j] + smooth((tau - Ta - Td) / Tq) * (qc[j] - qb[j]);
          else r = qc[j];
          qref[j] = r;
        }
        finger_cmd = tau < Ta + Td + Tq ? T(s.finger_closed) : T(s.finger_open);
      } else {
        for (int c = 0; c < 3; ++c) qref[c] = qstart[c];
        for (int j = ARM0; j < ARM0 + NARM; ++j)
          qref[j] = tau < Tp ? qstart[j] + smooth(tau / Tp) * (qa[j] - qstart[j]) : qa[j];
        finger_cmd = tau < Tp ? T(s.finger_closed) : T(s.finger_open);
      }
    }
    qref[FL] = finger_cmd;
    qref[FR] = finger_cmd;
    if (log && log->qref && t < log->steps)
      for (int j = 0; j < NJ; ++j) log->qref[(long)t * NJ + j] = r_val(qref[j]);

    for (int si = 0; si < s.substeps; ++si) {
      // kinematics and velocities of all links
      M3<T> Rw[MAXJ];
      V3<T> pw[MAXJ];
      forward_kinematics(tr, q, Rw, pw);
      T vb[MAXJ][6];
      body_velocities(tr, q, qd, vb);
      auto link_vel = [&](int j, const V3<T> &x) {
        const V3<T> xb = mulT(Rw[j], x - pw[j]);
        const V3<T> w(vb[j][0], vb[j][1], vb[j][2]), v(vb[j][3], vb[j][4], vb[j][5]);
        return mul(Rw[j], v + cross(w, xb));
      };
      T fext[MAXJ][6];
      for (int j = 0; j < NJ; ++j)
        for (int c = 0; c < 6; ++c) fext[j][c] = T(0.0);
      auto link_force = [&](int j, const V3<T> &x, const V3<T> &F) {
        const V3<T> Fb = mulT(Rw[j], F), xb = mulT(Rw[j], x - pw[j]);
        const V3<T> n = cross(xb, Fb);
        fext[j][0] = fext[j][0] + n.x; fext[j][1] = fext[j][1] + n.y; fext[j][2] = fext[j][2] + n.z;
        fext[j][3] = fext[j][3] + Fb.x; fext[j][4] = fext[j][4] + Fb.y; fext[j][5] = fext[j][5] + Fb.z;
      };
      const M3<T> oR = quat_to_mat(ob.q);
      Wrench<T> W;
      auto obj_vel = [&](const V3<T> &x) { return ob.v + cross(ob.w, x - ob.p); };
      Contact<T> cs[8];
      // object on the ground
      int nc = box_plane(ob.p, oR, ohe, cs);
      for (int i = 0; i < nc; ++i)
        add_force(W, ob.p, cs[i].x, penalty_force(cs[i], obj_vel(cs[i].x), V3<T>(), k, damp, T(mu_obj_ground), eps_v));
      // object against static boxes, both ways
      for (int b = 0; b < s.n_static; ++b) {
        const T mu = T(mu_drawn ? inst.obj_mu : (s.st_ramp[b] ? s.mu_ramp : s.mu_static));
        if (face_separated(ob.p, oR, ohe, SP[b], SR[b], SH[b])) continue;
        nc = box_verts_in_box(ob.p, oR, ohe, SP[b], SR[b], SH[b], cs);
        for (int i = 0; i < nc; ++i)
          add_force(W, ob.p, cs[i].x, penalty_force(cs[i], obj_vel(cs[i].x), V3<T>(), k, damp, mu, eps_v));
        nc = box_verts_in_box(SP[b], SR[b], SH[b], ob.p, oR, ohe, cs);
        for (int i = 0; i < nc; ++i)
          add_force(W, ob.p, cs[i].x, -penalty_force(cs[i], V3<T>(), obj_vel(cs[i].x), k, damp, mu, eps_v));
      }
      // fingers against the object, both ways
      const bool last = si == s.substeps - 1;
      for (int f = 0; f < 2; ++f) {
        const int j = f == 0 ? FL : FR;
        V3<T> fc, fh;
        link_box(s, j, Rw[j], pw[j], &fc, &fh);
        Contact<T> cb[8];
        int nb = 0;
        finger_object_contacts(fc, Rw[j], fh, ob.p, oR, ohe, cs, &nc, cb, &nb);
        for (int i = 0; i < nc; ++i) {
          const V3<T> F = penalty_force(cs[i], link_vel(j, cs[i].x), obj_vel(cs[i].x), k, damp, T(mu_obj_tool), eps_v);
          link_force(j, cs[i].x, F);
          add_force(W, ob.p, cs[i].x, -F);
        }
        for (int i = 0; i < nb; ++i) {
          const V3<T> F = penalty_force(cb[i], obj_vel(cb[i].x), link_vel(j, cb[i].x), k, damp, T(mu_obj_tool), eps_v);
          add_force(W, ob.p, cb[i].x, F);
          link_force(j, cb[i].x, -F);
        }
        if (last) touch[f] = nc + nb > 0;
      }
      // base against static boxes, both ways
      {
        const int j = BASE_BODY;
        const V3<T> bc = pw[j] + mul(Rw[j], V3<T>(T(s.b_com[j][0]), T(s.b_com[j][1]), T(s.b_com[j][2])));
        const V3<T> bh(T(s.b_half[j][0]), T(s.b_half[j][1]), T(s.b_half[j][2]));
        for (int b = 0; b < s.n_static; ++b) {
          if (face_separated(bc, Rw[j], bh, SP[b], SR[b], SH[b])) continue;
          nc = box_verts_in_box(bc, Rw[j], bh, SP[b], SR[b], SH[b], cs);
          for (int i = 0; i < nc; ++i)
            link_force(j, cs[i].x, penalty_force(cs[i], link_vel(j, cs[i].x), V3<T>(), k, damp, T(s.mu_static), eps_v));
          nc = box_verts_in_box(SP[b], SR[b], SH[b], bc, Rw[j], bh, cs);
          for (int i = 0; i < nc; ++i)
            link_force(j, cs[i].x, -penalty_force(cs[i], V3<T>(), link_vel(j, cs[i].x), k, damp, T(s.mu_static), eps_v));
        }
      }
      // joint PD: tau = I_nom (wc^2 (q_ref - q) - 2 zeta wc qd), limited to +-I_nom a_max
      T tau[NJ];
      for (int j = 0; j < NJ; ++j) {
        const T lim = T(s.j_inom[j] * s.accel_max);
        const T u = T(s.j_inom[j]) * (wc * wc * (qref[j] - q[j]) - T(2.0) * zeta * wc * qd[j]);
        tau[j] = r_max(-lim, r_min(lim, u));
      }
      T qdd[NJ];
      aba<T>(tr, q, qd, tau, fext, g, qdd, nullptr, Ibody);
      for (int j = 0; j < NJ; ++j) {
        qd[j] = qd[j] + h * qdd[j];
        q[j] = q[j] + h * qd[j];
      }
      integrate_free(ob, W, om, oIb, gv, h);
    }
    if (trace && t < trace_steps) {
      double *o = trace + (long)t * TRACE_ROBOT;
      o[0] = r_val(ob.p.x); o[1] = r_val(ob.p.y); o[2] = r_val(ob.p.z);
      o[3] = r_val(ob.q.w); o[4] = r_val(ob.q.x); o[5] = r_val(ob.q.y); o[6] = r_val(ob.q.z);
      o[7] = r_val(ob.v.x); o[8] = r_val(ob.v.y); o[9] = r_val(ob.v.z);
      o[10] = r_val(ob.w.x); o[11] = r_val(ob.w.y); o[12] = r_val(ob.w.z);
      for (int j = 0; j < NJ; ++j) { o[13 + j] = r_val(q[j]); o[24 + j] = r_val(qd[j]); }
    }
    if (!r_finite(ob.p.x) || !r_finite(q[0])) { diverged = true; steps = t + 1; break; }
    rest_run = std::sqrt(r_val(dot(ob.v, ob.v))) < s.rest_speed ? rest_run + 1 : 0;
    if (s.settle_steps > 0) {
      // early stop: the plan has ended and the object has stayed at rest; the
      // cost no longer changes and psi_g is read at this step
      const bool at_rest = std::sqrt(r_val(dot(ob.v, ob.v))) < s.rest_speed;
      calm = (act >= n_act && at_rest) ? calm + 1 : 0;
      if (calm >= s.settle_steps) { steps = t + 1; break; }
    }
  }
  // goal psi_g at T, the object at rest and either on the goal table's top
  // face (pick-and-place) or with its centre inside the goal box (move-push:
  // the container's inner volume)
  bool goal = false;
  const double px = r_val(ob.p.x), py = r_val(ob.p.y), pz = r_val(ob.p.z);
  const bool rest = std::sqrt(r_val(dot(ob.v, ob.v))) < s.rest_speed;
  if (s.goal_static >= 0 && s.goal_static < s.n_static) {
    const int b = s.goal_static;
    const double top = s.st_center[b][2] + s.st_half[b][2];
    goal = std::fabs(px - s.st_center[b][0]) <= s.st_half[b][0] && std::fabs(py - s.st_center[b][1]) <= s.st_half[b][1] &&
           pz >= top && pz <= top + 2.0 * s.obj_half[2] && rest;
  } else if (s.goal_static < 0) {
    const double *c = s.goal_box_center, *hb = s.goal_box_half;
    goal = std::fabs(px - c[0]) <= hb[0] && std::fabs(py - c[1]) <= hb[1] && std::fabs(pz - c[2]) <= hb[2] && rest;
  }
  RolloutOut out;
  out.steps = steps;
  out.speed = std::sqrt(r_val(dot(ob.v, ob.v)));
  out.rest_steps = rest_run;
  const T cost = T(s.time_weight) * dt * T((double)unsuccessful);
  out.cost = r_val(cost);
  out.pose[0] = r_val(ob.p.x); out.pose[1] = r_val(ob.p.y); out.pose[2] = r_val(ob.p.z);
  out.pose[3] = r_val(ob.q.w); out.pose[4] = r_val(ob.q.x); out.pose[5] = r_val(ob.q.y); out.pose[6] = r_val(ob.q.z);
  bool fin = !diverged;
  for (int i = 0; i < 7; ++i) fin = fin && std::isfinite(out.pose[i]);
  for (int j = 0; j < NJ; ++j) fin = fin && std::isfinite(r_val(q[j])) && std::fabs(r_val(q[j])) < 1e3;
  fin = fin && std::fabs(out.pose[0]) < 1e3 && std::fabs(out.pose[1]) < 1e3 && std::fabs(out.pose[2]) < 1e3;
  bool all_ok = true;
  for (int a = 0; a < n_act; ++a) all_ok = all_ok && ok[a];
  out.tier = !fin ? 3 : (all_ok ? (goal ? 0 : 1) : 2);
  if (!fin) out.cost = INFINITY;
  return out;
}

}  // namespace ref
