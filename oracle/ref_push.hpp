// Oracle: the single-action push plan (a kinematic, velocity-controlled sphere
// pushes one box across the ground plane towards a goal).
// TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Cost (Problem 2): the per-step action cost J = 1 while the action is not
// successful (Sec. IV-A, Eq. 4 and the text after it), scaled to seconds by dt
// and weighted, plus the final cost J_end = distance of the box to the goal at
// T.  "Successful" here means the box is within goal_tol of the goal.
#pragma once
#include "ref_rigid.hpp"
#include "ref_scene.hpp"

namespace ref {

struct RolloutOut {
  double cost;
  int32_t tier;      // 0 ok, 3 diverged (the push plan has no other predicate)
  double pose[7];    // final object pose p (3), q (4)
  int32_t steps;     // control steps simulated
  // observations for the parity tests, no part of the outcome: the object's
  // final speed and the number of consecutive final control steps it spent
  // slower than the scene's rest speed (robot scenes)
  double speed = 0.0;
  int32_t rest_steps = 0;
};

// Free-body state trace layout per control step: p(3) q(4) v(3) w(3).
constexpr int TRACE_FREE = 13;

template <class T>
RolloutOut push_rollout(const RefScene &s, const Instance &inst, const float *z, double *trace, int trace_steps) {
  const T h = T(s.dt) / T((double)s.substeps);
  const T g = T(s.gravity);
  const T k = T(s.k_contact), damp = T(s.c_contact), eps_v = T(s.eps_v);
  const V3<T> he(T(s.obj_half[0]), T(s.obj_half[1]), T(s.obj_half[2]));
  const T m = T(s.obj_mass);
  // solid box: I = m/3 (b^2 + c^2) with half extents a, b, c
  const V3<T> Ib = V3<T>(m * (he.y * he.y + he.z * he.z) / T(3.0), m * (he.x * he.x + he.z * he.z) / T(3.0),
                         m * (he.x * he.x + he.y * he.y) / T(3.0));

  // Controller parameters: approach angle theta, lateral offset o, speed s.
  const T theta = T((double)z[0]);
  const T off = T((double)z[1]);
  const T sp = r_max(T(0.0), r_min(T(s.pusher_vmax), T((double)z[2])));
  const T ct = r_cos(theta), st = r_sin(theta);
  const V3<T> u(ct, st, T(0.0));
  const V3<T> uperp(-st, ct, T(0.0));
  const V3<T> c0(T(s.obj_pos0[0]), T(s.obj_pos0[1]), T(0.0));
  V3<T> p0 = c0 - T(s.pusher_standoff) * u + off * uperp;
  p0.z = T(s.pusher_height);
  const T r = T(s.pusher_radius);
  const long push_sub = (long)s.pusher_steps * (long)s.substeps;

  Body<T> b;
  // resting height minus the penetration m g / (4 k) of four bottom corners
  b.p = V3<T>(T(s.obj_pos0[0]), T(s.obj_pos0[1]), T(s.obj_pos0[2]) - m * g / (T(4.0) * k));
  const T cy = r_cos(T(0.5 * s.obj_yaw0)), sy = r_sin(T(0.5 * s.obj_yaw0));
  b.q.w = cy; b.q.x = T(0.0); b.q.y = T(0.0); b.q.z = sy;

  const T gx = T(inst.goal[0]), gy = T(inst.goal[1]);
  const T tol = T(s.goal_tol);
  long unsuccessful = 0;
  long sub = 0;
  for (int t = 0; t < s.horizon; ++t) {
    for (int si = 0; si < s.substeps; ++si, ++sub) {
      const long active = sub < push_sub ? sub : push_sub;
      const T tau = T((double)active) * h;
      const V3<T> pc = p0 + (sp * tau) * u;
      const V3<T> vc = (sub < push_sub) ? sp * u : V3<T>();
      const M3<T> R = quat_to_mat(b.q);
      Wrench<T> W;
      Contact<T> cs[8];
      const int nc = box_plane(b.p, R, he, cs);
      for (int ci = 0; ci < nc; ++ci) {
        const V3<T> vA = b.v + cross(b.w, cs[ci].x - b.p);
        const V3<T> F = penalty_force(cs[ci], vA, V3<T>(), k, damp, T(s.mu_ground), eps_v);
        add_force(W, b.p, cs[ci].x, F);
      }
      Contact<T> sc;
      if (sphere_box(pc, r, b.p, R, he, &sc)) {
        const V3<T> vA = b.v + cross(b.w, sc.x - b.p);
        const V3<T> F = penalty_force(sc, vA, vc, k, damp, T(s.mu_tool), eps_v);
        add_force(W, b.p, sc.x, F);
      }
      integrate_free(b, W, m, Ib, V3<T>(T(0.0), T(0.0), -g), h);
    }
    const T dx = b.p.x - gx, dy = b.p.y - gy;
    const T dist = r_sqrt(dx * dx + dy * dy);
    if (dist > tol) ++unsuccessful;
    if (trace && t < trace_steps) {
      double *o = trace + (long)t * TRACE_FREE;
      o[0] = r_val(b.p.x); o[1] = r_val(b.p.y); o[2] = r_val(b.p.z);
      o[3] = r_val(b.q.w); o[4] = r_val(b.q.x); o[5] = r_val(b.q.y); o[6] = r_val(b.q.z);
      o[7] = r_val(b.v.x); o[8] = r_val(b.v.y); o[9] = r_val(b.v.z);
      o[10] = r_val(b.w.x); o[11] = r_val(b.w.y); o[12] = r_val(b.w.z);
    }
  }
  const T dx = b.p.x - gx, dy = b.p.y - gy;
  const T dist = r_sqrt(dx * dx + dy * dy);
  const T cost = dist + T(s.time_weight) * T(s.dt) * T((double)unsuccessful);
  RolloutOut out;
  out.steps = s.horizon;
  out.cost = r_val(cost);
  out.pose[0] = r_val(b.p.x); out.pose[1] = r_val(b.p.y); out.pose[2] = r_val(b.p.z);
  out.pose[3] = r_val(b.q.w); out.pose[4] = r_val(b.q.x); out.pose[5] = r_val(b.q.y); out.pose[6] = r_val(b.q.z);
  bool fin = r_finite(cost);
  for (int i = 0; i < 7; ++i) fin = fin && std::isfinite(out.pose[i]);
  fin = fin && std::fabs(out.pose[0]) < 1e3 && std::fabs(out.pose[1]) < 1e3 && std::fabs(out.pose[2]) < 1e3;
  out.tier = fin ? 0 : 3;
  if (!fin) out.cost = INFINITY;
  return out;
}

}  // namespace ref
