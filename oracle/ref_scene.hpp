// Oracle: scene description and the seeded per-instance draws.
// TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
#pragma once
#include <cstdint>

#include "ref_random.hpp"

namespace ref {

constexpr int SCENE_PUSH = 1;
constexpr int SCENE_PICKPLACE = 2;
constexpr int SCENE_MOVEPUSH = 3;
constexpr int MAX_STATIC = 8;

// Everything a rollout needs, in FP64.  Filled by the oracle's Python binding
// from the same workload description the GPU library receives.
struct RefScene {
  int32_t kind;
  int32_t substeps, horizon;
  double dt, gravity, k_contact, c_contact, eps_v;
  // friction coefficients: ground, pusher/finger, static boxes, ramp
  double mu_ground, mu_tool, mu_static, mu_ramp;
  // the one free object: a box
  double obj_half[3], obj_mass, obj_pos0[3], obj_yaw0;
  // static boxes: centre, half extents, yaw (about z) then pitch (about y), friction class
  int32_t n_static;
  double st_center[MAX_STATIC][3], st_half[MAX_STATIC][3], st_yaw[MAX_STATIC], st_pitch[MAX_STATIC];
  int32_t st_ramp[MAX_STATIC];
  // kinematic pusher sphere (push scene)
  double pusher_radius, pusher_standoff, pusher_height, pusher_vmax;
  int32_t pusher_steps;
  // goal: drawn per instance on the scene stream; tolerance and time weight of the cost
  double goal_rho_lo, goal_rho_hi, goal_phi_lo, goal_phi_hi, goal_tol, time_weight;
  // articulated robot (pick-place, move-push): joints 0-2 base x, y, yaw;
  // 3-8 arm; 9, 10 fingers.  Tree layout as in ref_spatial.hpp.
  int32_t n_joints;
  int32_t j_type[12], j_axis[12], j_parent[12], b_collide[12];
  double j_origin[12][3], b_mass[12], b_com[12][3], b_half[12][3], j_inom[12], q0[12];
  int32_t ee_body;
  double ee_offset[3];
  // controller constants
  int32_t ik_iters;
  double omega_c, zeta, ik_lambda;
  double base_vmin, base_vmax, base_wmax, base_tol, yaw_tol, ee_tol;
  double t_approach, t_descend, t_close, t_lift, t_transfer, t_release;
  double timeout_move, timeout_pick, timeout_place;
  double pregrasp, finger_open, finger_closed, rest_speed;
  int32_t goal_static;   // static box whose top face is the goal region
  double joint_speed_max, accel_max;  // arm reference speed limit; torque limit I_nom * accel_max
  // move-push: push speed clamp, longest push, the push action's timeout
  double push_vmin, push_vmax, push_dmax, timeout_push;
  // friction of every contact of the object, drawn per instance when obj_mu_hi > 0
  double obj_mu_lo, obj_mu_hi;
  // goal region used when goal_static < 0: the object's centre inside this box, at rest
  double goal_box_center[3], goal_box_half[3];
  // early stop of a robot rollout (0 = off): once every action has ended, stop
  // after this many consecutive control steps with the object at rest
  int32_t settle_steps;
  // stop a robot rollout when an action fails (0 = off): the plan can then no
  // longer become feasible (every action must succeed, Problem 2), and Alg. 1
  // evaluates only the costs of successful plans; the stopped plan reports
  // tier 2 and the cost of the steps it ran
  int32_t fail_stop;
  // domain randomisation (Sec. IV-C): R scenarios per parameter row (<= 1 off),
  // each with its own object friction / mass draw; the row's tier is the worst
  // and its cost the mean (dr_reduce 0) or maximum (1) over scenarios
  int32_t dr_scenarios, dr_reduce;
  double dr_mu_lo, dr_mu_hi, dr_mass_lo, dr_mass_hi;
};

// Per-instance draws (scene stream 1, sample 0, iteration 0, instance b), one
// Philox block, words 0-2:
//   goal = object start + rho (cos phi, sin phi), rho ~ U[rho_lo, rho_hi],
//   phi ~ U[phi_lo, phi_hi]  (words 0, 1);
//   the object's friction coefficient obj_mu ~ U[obj_mu_lo, obj_mu_hi] if
//   obj_mu_hi > 0, else 0 = "use the per-class coefficients"  (word 2).
struct Instance {
  double goal[2];
  double obj_mu;
  double obj_mass = 0.0;  // 0: the scene's
};

inline Instance draw_instance(const RefScene &s, uint64_t seed, uint32_t b) {
  Word4 x = philox_draw(seed, STREAM_SCENE, 0, 0, 0, b);
  const double u0 = (double)u01(x.w[0]);
  const double u1 = (double)u01(x.w[1]);
  const double rho = s.goal_rho_lo + (s.goal_rho_hi - s.goal_rho_lo) * u0;
  const double phi = s.goal_phi_lo + (s.goal_phi_hi - s.goal_phi_lo) * u1;
  Instance in;
  in.goal[0] = s.obj_pos0[0] + rho * std::cos(phi);
  in.goal[1] = s.obj_pos0[1] + rho * std::sin(phi);
  in.obj_mu = s.obj_mu_hi > 0.0 ? s.obj_mu_lo + (s.obj_mu_hi - s.obj_mu_lo) * (double)u01(x.w[2]) : 0.0;
  return in;
}

// Domain-randomisation scenario r of instance b (scene stream 1, block 1,
// sample r, iteration 0, instance b): the object's friction ~ U[dr_mu_lo,
// dr_mu_hi] from word 0 when dr_mu_hi > 0 (else the instance's draw stands)
// and its mass ~ U[dr_mass_lo, dr_mass_hi] from word 1 when dr_mass_hi > 0
// (else the scene's mass).
inline Instance scenario_of(const RefScene &s, const Instance &base, uint64_t seed, uint32_t b, int r) {
  Instance in = base;
  Word4 x = philox_draw(seed, STREAM_SCENE, 1, (uint32_t)r, 0, b);
  if (s.dr_mu_hi > 0.0) in.obj_mu = s.dr_mu_lo + (s.dr_mu_hi - s.dr_mu_lo) * (double)u01(x.w[0]);
  if (s.dr_mass_hi > 0.0) in.obj_mass = s.dr_mass_lo + (s.dr_mass_hi - s.dr_mass_lo) * (double)u01(x.w[1]);
  return in;
}

}  // namespace ref
