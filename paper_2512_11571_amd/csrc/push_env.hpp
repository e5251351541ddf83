// One environment of the single-action push plan (device function).
//
// Evaluation step of CE optimisation (Alg. 1) for the single-action push plan:
// a kinematic, velocity-controlled sphere pushes one box over the ground plane.
//
// Controller parameters z = (theta, o, s): approach direction u = (cos theta,
// sin theta), start 'standoff' behind the box centre with lateral offset o
// along u_perp, speed clamp(s, 0, vmax) for pusher_steps control steps.
// Plan cost (Problem 2): distance of the box to the goal at T plus
// time_weight * dt per control step in which the box is not within goal_tol
// of the goal (the per-step cost 1 of an unfinished action, Sec. IV-A).
//
// One environment per lane; the whole state (13 floats) stays in VGPRs for the
// H x n_sub substeps; HBM is touched only for z in and (cost, tier, pose) out.
#pragma once
#include "internal.hpp"
#include "rigid.hpp"

namespace cem {
namespace {

// Rolls out row i of Z (theta, o, s) and writes its cost, tier, pose and (TRACE) trace.
template <bool TRACE>
__device__ __forceinline__ void push_env(CScene &sc, CDevState *st,
                                         const float *__restrict__ Z, long i, float *__restrict__ cost_out,
                                         uint8_t *__restrict__ tier_out, float *__restrict__ pose_out,
                                         float *__restrict__ trace, int trace_steps) {
  const float h = sc.dt / (float)sc.substeps;
  const V3f gv = v3(0.0f, 0.0f, -sc.gravity);
  const float k = sc.k_contact, damp = sc.c_contact, eps2 = sc.eps_v * sc.eps_v;
  const V3f he = v3(sc.obj_half[0], sc.obj_half[1], sc.obj_half[2]);
  const float m = sc.obj_mass, inv_m = 1.0f / m;
  const V3f Ib = v3(m * (he.y * he.y + he.z * he.z) / 3.0f, m * (he.x * he.x + he.z * he.z) / 3.0f,
                    m * (he.x * he.x + he.y * he.y) / 3.0f);
  const V3f inv_Ib = v3(1.0f / Ib.x, 1.0f / Ib.y, 1.0f / Ib.z);

  const float th = Z[(long)i * 3 + 0], off = Z[(long)i * 3 + 1];
  const float sp = fmaxf(0.0f, fminf(sc.pusher_vmax, Z[(long)i * 3 + 2]));
  float sth, cth;
  sincosf(th, &sth, &cth);
  const V3f u = v3(cth, sth, 0.0f), up = v3(-sth, cth, 0.0f);
  V3f p0 = v3(sc.obj_pos0[0], sc.obj_pos0[1], 0.0f) - sc.pusher_standoff * u + off * up;
  p0.z = sc.pusher_height;
  const int push_sub = sc.pusher_steps * sc.substeps;

  FreeBody b;
  b.p = v3(sc.obj_pos0[0], sc.obj_pos0[1], sc.obj_pos0[2] - m * sc.gravity / (4.0f * k));
  float sy, cy;
  sincosf(0.5f * sc.obj_yaw0, &sy, &cy);
  b.q = Q4f{cy, 0.0f, 0.0f, sy};
  b.v = v3(0.0f, 0.0f, 0.0f);
  b.w = v3(0.0f, 0.0f, 0.0f);

  const float gx = (float)st->goal[0], gy = (float)st->goal[1];
  const float tol2 = sc.goal_tol * sc.goal_tol;
  int unsuccessful = 0;
  int sub = 0;
  for (int t = 0; t < sc.horizon; ++t) {
    for (int s = 0; s < sc.substeps; ++s, ++sub) {
      const bool pushing = sub < push_sub;
      const float tau = (float)(pushing ? sub : push_sub) * h;
      const V3f pc = p0 + (sp * tau) * u;
      const V3f vc = pushing ? sp * u : v3(0.0f, 0.0f, 0.0f);
      const M3f R = rot_of(b.q);
      Wrench W{v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)};
      box_ground(b, R, he, k, damp, sc.mu_ground, eps2, W);
      sphere_on_box(b, R, he, pc, sc.pusher_radius, vc, k, damp, sc.mu_tool, eps2, W);
      integrate(b, W, inv_m, Ib, inv_Ib, gv, h, R);
    }
    const float dx = b.p.x - gx, dy = b.p.y - gy;
    unsuccessful += (dx * dx + dy * dy > tol2) ? 1 : 0;
    if (TRACE && t < trace_steps) {
      float *o = trace + ((long)i * trace_steps + t) * CEM_TRACE_FREE;
      o[0] = b.p.x; o[1] = b.p.y; o[2] = b.p.z;
      o[3] = b.q.w; o[4] = b.q.x; o[5] = b.q.y; o[6] = b.q.z;
      o[7] = b.v.x; o[8] = b.v.y; o[9] = b.v.z;
      o[10] = b.w.x; o[11] = b.w.y; o[12] = b.w.z;
    }
  }
  const float dx = b.p.x - gx, dy = b.p.y - gy;
  float c = sqrtf(dx * dx + dy * dy) + sc.time_weight * sc.dt * (float)unsuccessful;
  const float pose[7] = {b.p.x, b.p.y, b.p.z, b.q.w, b.q.x, b.q.y, b.q.z};
  bool fin = isfinite(c);
  for (int j = 0; j < 7; ++j) fin = fin && isfinite(pose[j]);
  fin = fin && fabsf(b.p.x) < 1e3f && fabsf(b.p.y) < 1e3f && fabsf(b.p.z) < 1e3f;
  if (!fin) c = __int_as_float(0x7F800000);
  if (cost_out) cost_out[i] = c;
  if (tier_out) tier_out[i] = fin ? 0 : 3;
  if (pose_out)
    for (int j = 0; j < 7; ++j) pose_out[(long)i * 7 + j] = pose[j];
}

}  // namespace
}  // namespace cem
