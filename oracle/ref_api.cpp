// Oracle C entry points (ref_*), host pointers only.
// TEST INFRASTRUCTURE ONLY: the only callers are tests/, the smoke check and
// the CPU-baseline leg of the benchmark.  Nothing here is shared with, or
// called by, the GPU library.
//
// Built with g++ -O2 -ffp-contract=off so that no multiply-add is fused behind
// the code's back: every rounding step is the one written.
#include <atomic>
#include <cstdint>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "ref_cem.hpp"
#include "ref_mlp.hpp"
#include "ref_push.hpp"
#include "ref_random.hpp"
#include "ref_robot.hpp"
#include "ref_spatial.hpp"
#include "ref_scene.hpp"

namespace ref {
thread_local Tally g_tally;
}

using namespace ref;

namespace {

RolloutOut rollout_one(const RefScene &s, const Instance &in, const float *z, double *trace, int trace_steps) {
  if (s.kind == SCENE_PUSH) return push_rollout<double>(s, in, z, trace, trace_steps);
  return robot_rollout<double>(s, in, z, trace, trace_steps);
}

int param_dim(const RefScene &s) {
  if (s.kind == SCENE_PUSH) return 3;
  if (s.kind == SCENE_PICKPLACE) return 16;
  return 12;
}

void parallel_for(int n, int threads, const std::function<void(int)> &fn) {
  if (threads <= 1 || n <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&]() {
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= n) break;
        fn(i);
      }
    });
  for (auto &t : ts) t.join();
}

}  // namespace

extern "C" {

int ref_scene_size(void) { return (int)sizeof(RefScene); }

void ref_philox(uint64_t seed, uint32_t tag, uint32_t block, uint32_t sample, uint32_t iter, uint32_t inst,
                uint32_t out[4]) {
  Word4 x = philox_draw(seed, tag, block, sample, iter, inst);
  for (int i = 0; i < 4; ++i) out[i] = x.w[i];
}

void ref_philox_raw(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  Word4 c;
  for (int i = 0; i < 4; ++i) c.w[i] = ctr[i];
  Word4 x = philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = x.w[i];
}

void ref_u01(const uint32_t *x, int n, float *out) {
  for (int i = 0; i < n; ++i) out[i] = u01(x[i]);
}
void ref_logf_vec(const float *u, int n, float *out) {
  for (int i = 0; i < n; ++i) out[i] = ref_logf(u[i]);
}
void ref_sincos2pi_vec(const float *u, int n, float *s, float *c) {
  for (int i = 0; i < n; ++i) ref_sincos2pi(u[i], &s[i], &c[i]);
}

// eps[i][d] for samples 0..pop-1 of iteration iter, instance inst.
void ref_normals(uint64_t seed, uint32_t iter, uint32_t inst, int pop, int D, float *eps) {
  for (int i = 0; i < pop; ++i)
    for (int d = 0; d < D; ++d) eps[(long)i * D + d] = cem_normal(seed, d, (uint32_t)i, iter, inst);
}

// Z (pop x D, FP32) = mu + L eps for iteration iter, instance inst.
void ref_sample(uint64_t seed, uint32_t iter, uint32_t inst, int pop, int D, const double *mu, const double *L,
                float *Z) {
  for (int i = 0; i < pop; ++i) cem_sample_row(seed, (uint32_t)i, iter, inst, D, mu, L, Z + (long)i * D, nullptr);
}

// Iteration-0 rows (pop x D) drawn from a region.
void ref_sample_region(uint64_t seed, uint32_t inst, int pop, int D, const float *lo, const float *hi, int n_rings,
                       const int *ring_dim, const float *ring, float *Z) {
  const RefRegion R{lo, hi, n_rings, ring_dim, ring};
  for (int i = 0; i < pop; ++i) region_sample_row(seed, (uint32_t)i, inst, D, R, Z + (long)i * D);
}

int ref_n_env_at(int pop, int pop_final, int ramp, int j) { return n_env_at(pop, pop_final, ramp, j); }

// out = (goal x, goal y, object friction) of instance inst.
void ref_draw_instance(const RefScene *s, uint64_t seed, uint32_t inst, double out[3]) {
  Instance in = draw_instance(*s, seed, inst);
  out[0] = in.goal[0];
  out[1] = in.goal[1];
  out[2] = in.obj_mu;
}

// Roll out pop parameter rows; trace (optional) gets trace_steps states per env.
int ref_rollout(const RefScene *s, uint64_t seed, uint32_t inst, int pop, const float *Z, double *cost,
                uint8_t *tier, double *pose, double *trace, int trace_steps, int threads, int32_t *steps,
                double *speed, int32_t *rest_steps) {
  const int D = param_dim(*s);
  const Instance in = draw_instance(*s, seed, inst);
  if (s->kind != SCENE_PUSH && s->kind != SCENE_PICKPLACE && s->kind != SCENE_MOVEPUSH) return 1;
  const int tw = s->kind == SCENE_PUSH ? TRACE_FREE : TRACE_ROBOT;
  const int R = (s->kind != SCENE_PUSH && s->dr_scenarios > 1) ? s->dr_scenarios : 1;
  if (R > 1) {
    // domain randomisation: every row under each of the R scenarios; the
    // worst tier, the mean or maximum cost, scenario 0's pose, the steps summed
    if (trace) return 1;
    std::vector<Instance> scen(R);
    for (int r = 0; r < R; ++r) scen[r] = scenario_of(*s, in, seed, inst, r);
    parallel_for(pop, threads, [&](int i) {
      double c_sum = 0.0, c_max = -INFINITY;
      int t_max = 0, n_steps = 0;
      for (int r = 0; r < R; ++r) {
        RolloutOut o = rollout_one(*s, scen[r], Z + (long)i * D, nullptr, 0);
        c_sum += o.cost;
        c_max = std::max(c_max, o.cost);
        t_max = std::max(t_max, o.tier);
        n_steps += o.steps;
        if (r == 0 && pose)
          for (int c = 0; c < 7; ++c) pose[(long)i * 7 + c] = o.pose[c];
        if (r == 0 && speed) speed[i] = o.speed;
        if (r == 0 && rest_steps) rest_steps[i] = o.rest_steps;
      }
      cost[i] = s->dr_reduce ? c_max : c_sum / R;
      tier[i] = (uint8_t)t_max;
      if (steps) steps[i] = n_steps;
    });
    return 0;
  }
  parallel_for(pop, threads, [&](int i) {
    RolloutOut o = rollout_one(*s, in, Z + (long)i * D, trace ? trace + (long)i * trace_steps * tw : nullptr,
                               trace_steps);
    cost[i] = o.cost;
    tier[i] = (uint8_t)o.tier;
    if (pose)
      for (int c = 0; c < 7; ++c) pose[(long)i * 7 + c] = o.pose[c];
    if (steps) steps[i] = o.steps;
    if (speed) speed[i] = o.speed;
    if (rest_steps) rest_steps[i] = o.rest_steps;
  });
  return 0;
}

// Domain-randomisation scenarios of instance inst: friction and mass per
// scenario (0 where the scene draws none).
void ref_scenarios(const RefScene *s, uint64_t seed, uint32_t inst, int n, double *mu, double *mass) {
  const Instance in = draw_instance(*s, seed, inst);
  for (int r = 0; r < n; ++r) {
    const Instance sc = scenario_of(*s, in, seed, inst, r);
    mu[r] = s->dr_mu_hi > 0.0 ? sc.obj_mu : 0.0;
    mass[r] = s->dr_mass_hi > 0.0 ? sc.obj_mass : 0.0;
  }
}

// Operation tally of one rollout of parameter row z: add, mul, fma, div, sqrt, trans.
void ref_count_ops(const RefScene *s, uint64_t seed, uint32_t inst, const float *z, uint64_t out[6]) {
  const Instance in = draw_instance(*s, seed, inst);
  g_tally = Tally();
  if (s->kind == SCENE_PUSH) push_rollout<Cnt>(*s, in, z, nullptr, 0);
  else robot_rollout<Cnt>(*s, in, z, nullptr, 0);
  out[0] = g_tally.add; out[1] = g_tally.mul; out[2] = g_tally.fma;
  out[3] = g_tally.div; out[4] = g_tally.sqrt; out[5] = g_tally.trans;
}

// A single free box, optionally resting on the plane z = 0 (8 corner contacts),
// under an arbitrary gravity vector: the closed-form pins of the integrator and
// of the contact model run through this.  prm layout:
// he[3] m p0[3] q0[4] v0[3] w0[3] gvec[3] k c mu eps_v h plane(0/1)  (27 doubles).
// trace: nsteps x 13 (p q v w after each step).
void ref_box_sim(const double *prm, int nsteps, double *trace) {
  const V3<double> he(prm[0], prm[1], prm[2]);
  const double m = prm[3];
  Body<double> b;
  b.p = V3<double>(prm[4], prm[5], prm[6]);
  b.q.w = prm[7]; b.q.x = prm[8]; b.q.y = prm[9]; b.q.z = prm[10];
  b.v = V3<double>(prm[11], prm[12], prm[13]);
  b.w = V3<double>(prm[14], prm[15], prm[16]);
  const V3<double> gv(prm[17], prm[18], prm[19]);
  const double k = prm[20], c = prm[21], mu = prm[22], eps_v = prm[23], h = prm[24];
  const bool plane = prm[25] != 0.0;
  const V3<double> Ib(m * (he.y * he.y + he.z * he.z) / 3.0, m * (he.x * he.x + he.z * he.z) / 3.0,
                      m * (he.x * he.x + he.y * he.y) / 3.0);
  for (int n = 0; n < nsteps; ++n) {
    Wrench<double> W;
    if (plane) {
      Contact<double> cs[8];
      const int nc = box_plane(b.p, quat_to_mat(b.q), he, cs);
      for (int i = 0; i < nc; ++i) {
        const V3<double> vA = b.v + cross(b.w, cs[i].x - b.p);
        add_force(W, b.p, cs[i].x, penalty_force(cs[i], vA, V3<double>(), k, c, mu, eps_v));
      }
    }
    integrate_free(b, W, m, Ib, gv, h);
    double *o = trace + (long)n * 13;
    o[0] = b.p.x; o[1] = b.p.y; o[2] = b.p.z;
    o[3] = b.q.w; o[4] = b.q.x; o[5] = b.q.y; o[6] = b.q.z;
    o[7] = b.v.x; o[8] = b.v.y; o[9] = b.v.z;
    o[10] = b.w.x; o[11] = b.w.y; o[12] = b.w.z;
  }
}

// Narrowphase probes.  Poses are (p[3], q[4]).  Each contact row: x[3] n[3] d.
int ref_sphere_box(const double c[3], double r, const double p[3], const double q[4], const double he[3],
                   double out[7]) {
  Q4<double> qq; qq.w = q[0]; qq.x = q[1]; qq.y = q[2]; qq.z = q[3];
  Contact<double> ct;
  const int n = sphere_box(V3<double>(c[0], c[1], c[2]), r, V3<double>(p[0], p[1], p[2]), quat_to_mat(qq),
                           V3<double>(he[0], he[1], he[2]), &ct);
  if (n) {
    out[0] = ct.x.x; out[1] = ct.x.y; out[2] = ct.x.z;
    out[3] = ct.n.x; out[4] = ct.n.y; out[5] = ct.n.z; out[6] = ct.d;
  }
  return n;
}

int ref_box_box(const double pA[3], const double qA[4], const double heA[3], const double pB[3], const double qB[4],
                const double heB[3], double out[8 * 7]) {
  Q4<double> a; a.w = qA[0]; a.x = qA[1]; a.y = qA[2]; a.z = qA[3];
  Q4<double> b; b.w = qB[0]; b.x = qB[1]; b.y = qB[2]; b.z = qB[3];
  Contact<double> cs[8];
  const int n = box_verts_in_box(V3<double>(pA[0], pA[1], pA[2]), quat_to_mat(a), V3<double>(heA[0], heA[1], heA[2]),
                                 V3<double>(pB[0], pB[1], pB[2]), quat_to_mat(b), V3<double>(heB[0], heB[1], heB[2]),
                                 cs);
  for (int i = 0; i < n; ++i) {
    double *o = out + i * 7;
    o[0] = cs[i].x.x; o[1] = cs[i].x.y; o[2] = cs[i].x.z;
    o[3] = cs[i].n.x; o[4] = cs[i].n.y; o[5] = cs[i].n.z; o[6] = cs[i].d;
  }
  return n;
}

// Kinematic-tree probes for the dynamics pins (Tree layout of ref_spatial.hpp).
int ref_tree_size(void) { return (int)sizeof(Tree); }
void ref_tree_aba(const Tree *t, const double *q, const double *qd, const double *tau, const double *fext, double g,
                  double *qdd) {
  aba(*t, q, qd, tau, (const double(*)[6])fext, g, qdd);
}
void ref_tree_rnea(const Tree *t, const double *q, const double *qd, const double *qdd, const double *fext, double g,
                   double *tau) {
  rnea(*t, q, qd, qdd, (const double(*)[6])fext, g, tau);
}
void ref_tree_crba(const Tree *t, const double *q, double *M) { crba(*t, q, M); }
// Passive tree (zero joint torque, gravity g): n semi-implicit Euler steps of
// length h; trace n x 2*n_joints (q, qd after each step).
void ref_tree_sim(const Tree *t, const double *q0, const double *qd0, double g, double h, int n, double *trace) {
  double q[MAXJ], qd[MAXJ], tau[MAXJ], qdd[MAXJ];
  for (int j = 0; j < t->n; ++j) { q[j] = q0[j]; qd[j] = qd0[j]; tau[j] = 0.0; }
  for (int s = 0; s < n; ++s) {
    aba(*t, q, qd, tau, (const double(*)[6]) nullptr, g, qdd);
    for (int j = 0; j < t->n; ++j) {
      qd[j] = qd[j] + h * qdd[j];
      q[j] = q[j] + h * qd[j];
      trace[(long)s * 2 * t->n + j] = q[j];
      trace[(long)s * 2 * t->n + t->n + j] = qd[j];
    }
  }
}
// The scene's free object alone (ground and static boxes, no robot) from pose
// p0 (3) q0 (4) and velocity v0 (3): n substeps of the scene's h; trace n x 13.
void ref_object_sim(const RefScene *s, const double *p0, const double *q0, const double *v0, int n, double *trace) {
  const double h = s->dt / (double)s->substeps;
  const V3<double> he(s->obj_half[0], s->obj_half[1], s->obj_half[2]);
  const double m = s->obj_mass;
  const V3<double> Ib(m * (he.y * he.y + he.z * he.z) / 3.0, m * (he.x * he.x + he.z * he.z) / 3.0,
                      m * (he.x * he.x + he.y * he.y) / 3.0);
  Body<double> b;
  b.p = V3<double>(p0[0], p0[1], p0[2]);
  b.q.w = q0[0]; b.q.x = q0[1]; b.q.y = q0[2]; b.q.z = q0[3];
  b.v = V3<double>(v0[0], v0[1], v0[2]);
  for (int st = 0; st < n; ++st) {
    const M3<double> R = quat_to_mat(b.q);
    Wrench<double> W;
    Contact<double> cs[8];
    auto vel = [&](const V3<double> &x) { return b.v + cross(b.w, x - b.p); };
    int nc = box_plane(b.p, R, he, cs);
    for (int i = 0; i < nc; ++i)
      add_force(W, b.p, cs[i].x, penalty_force(cs[i], vel(cs[i].x), V3<double>(), s->k_contact, s->c_contact, s->mu_ground, s->eps_v));
    for (int k = 0; k < s->n_static; ++k) {
      const M3<double> SR = static_rot<double>(*s, k);
      const V3<double> SP(s->st_center[k][0], s->st_center[k][1], s->st_center[k][2]);
      const V3<double> SH(s->st_half[k][0], s->st_half[k][1], s->st_half[k][2]);
      const double mu = s->st_ramp[k] ? s->mu_ramp : s->mu_static;
      nc = box_verts_in_box(b.p, R, he, SP, SR, SH, cs);
      for (int i = 0; i < nc; ++i)
        add_force(W, b.p, cs[i].x, penalty_force(cs[i], vel(cs[i].x), V3<double>(), s->k_contact, s->c_contact, mu, s->eps_v));
      nc = box_verts_in_box(SP, SR, SH, b.p, R, he, cs);
      for (int i = 0; i < nc; ++i)
        add_force(W, b.p, cs[i].x, -penalty_force(cs[i], V3<double>(), vel(cs[i].x), s->k_contact, s->c_contact, mu, s->eps_v));
    }
    integrate_free(b, W, m, Ib, V3<double>(0.0, 0.0, -s->gravity), h);
    double *o = trace + (long)st * 13;
    o[0] = b.p.x; o[1] = b.p.y; o[2] = b.p.z;
    o[3] = b.q.w; o[4] = b.q.x; o[5] = b.q.y; o[6] = b.q.z;
    o[7] = b.v.x; o[8] = b.v.y; o[9] = b.v.z;
    o[10] = b.w.x; o[11] = b.w.y; o[12] = b.w.z;
  }
}
void ref_tree_fk(const Tree *t, const double *q, double *R, double *p) {
  M3<double> Rw[MAXJ];
  V3<double> pw[MAXJ];
  forward_kinematics(*t, q, Rw, pw);
  for (int j = 0; j < t->n; ++j) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) R[j * 9 + a * 3 + b] = Rw[j].m[a][b];
    p[j * 3 + 0] = pw[j].x; p[j * 3 + 1] = pw[j].y; p[j * 3 + 2] = pw[j].z;
  }
}
// EE pose after damped-least-squares IK from q (robot scenes): q_out, EE p, R.
void ref_ik(const RefScene *s, const double *q, const double pt[3], const double Rt[9], double *q_out, double pe[3],
            double Re[9]) {
  const Tree tr = tree_of(*s);
  double qq[MAXJ];
  for (int j = 0; j < tr.n; ++j) qq[j] = q[j];
  M3<double> R;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R.m[a][b] = Rt[a * 3 + b];
  ik_dls(*s, tr, qq, V3<double>(pt[0], pt[1], pt[2]), R);
  M3<double> E;
  V3<double> p;
  ee_pose(*s, tr, qq, &E, &p);
  for (int j = 0; j < tr.n; ++j) q_out[j] = qq[j];
  pe[0] = p.x; pe[1] = p.y; pe[2] = p.z;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Re[a * 3 + b] = E.m[a][b];
}

// ---- pins of the plan layer ----

// Switches the face-axis broadphase of the box-box tests on (1, the default)
// or off (0: every pair runs its vertex tests).  Set only between calls.
void ref_set_face_cull(int on) { g_face_cull = on != 0; }

// One robot rollout of row z with its action-sequencing record: act[t] and
// (nullable) the joint references qref[t][11] for the first `steps` control
// steps, ends[4] (T_a + 1, or -1), the success bits, (cost, tier) and
// optionally the state trace.
int ref_robot_log(const RefScene *s, uint64_t seed, uint32_t inst, const float *z, int steps, int32_t *act,
                  double *qref, int32_t ends[4], int32_t *ok, double out[2], double *trace, int trace_steps) {
  if (s->kind != SCENE_PICKPLACE && s->kind != SCENE_MOVEPUSH) return 1;
  const Instance in = draw_instance(*s, seed, inst);
  RobotLog log;
  log.act = act;
  log.qref = qref;
  log.steps = steps;
  for (int t = 0; t < steps; ++t) act[t] = -1;
  const RolloutOut o = robot_rollout<double>(*s, in, z, trace, trace_steps, &log);
  for (int a = 0; a < 4; ++a) ends[a] = log.ends[a];
  *ok = log.ok;
  out[0] = o.cost;
  out[1] = (double)o.tier;
  return 0;
}

// The grasp predicates on a hand-set state: the robot at configuration q[11],
// the object box at (p, quaternion w x y z).  out = (left finger touches,
// right finger touches, object centre between the inner faces, all three).
void ref_grasp_check(const RefScene *s, const double *q, const double obj_p[3], const double obj_q[4],
                     int32_t out[4]) {
  const Tree tr = tree_of(*s);
  M3<double> Rw[MAXJ];
  V3<double> pw[MAXJ];
  forward_kinematics(tr, q, Rw, pw);
  const V3<double> op(obj_p[0], obj_p[1], obj_p[2]);
  Q4<double> oq;
  oq.w = obj_q[0]; oq.x = obj_q[1]; oq.y = obj_q[2]; oq.z = obj_q[3];
  const M3<double> oR = quat_to_mat(oq);
  const V3<double> ohe(s->obj_half[0], s->obj_half[1], s->obj_half[2]);
  for (int f = 0; f < 2; ++f) {
    const int j = f == 0 ? FL : FR;
    V3<double> fc, fh;
    link_box(*s, j, Rw[j], pw[j], &fc, &fh);
    Contact<double> a[8], b[8];
    int na = 0, nb = 0;
    finger_object_contacts(fc, Rw[j], fh, op, oR, ohe, a, &na, b, &nb);
    out[f] = na + nb > 0;
  }
  out[2] = object_between_fingers(Rw[s->ee_body], pw[s->ee_body], q, op);
  out[3] = out[0] && out[1] && out[2];
}

// Operation tallies of single building blocks on generic (non-structural)
// operands, for checking the counter against hand counts: which = 0 one
// free-body step (integrate_free), 1 one penalty contact force, 2 a 3-vector
// cross product, 3 a quaternion's rotation matrix.  out: add, mul, fma, div,
// sqrt, trans.
void ref_count_block(int which, uint64_t out[6]) {
  g_tally = Tally();
  const Cnt a(0.3), b(-0.7), c(1.1), d(0.45), e(2.5), f(-1.3);
  if (which == 0) {
    Body<Cnt> bd;
    bd.p = V3<Cnt>(a, b, c);
    bd.q.w = Cnt(0.9); bd.q.x = Cnt(0.1); bd.q.y = Cnt(-0.3); bd.q.z = Cnt(0.2);
    bd.v = V3<Cnt>(d, e, f);
    bd.w = V3<Cnt>(b, c, d);
    Wrench<Cnt> W;
    W.f = V3<Cnt>(e, a, b);
    W.tau = V3<Cnt>(c, f, a);
    const V3<Cnt> Ib(Cnt(0.2), Cnt(0.3), Cnt(0.4)), gv(Cnt(0.0), Cnt(0.0), Cnt(-9.81));
    g_tally = Tally();  // the set-up above performs no counted operation; start clean anyway
    integrate_free(bd, W, Cnt(2.0), Ib, gv, Cnt(0.001));
  } else if (which == 1) {
    Contact<Cnt> ct;
    ct.x = V3<Cnt>(a, b, c);
    ct.n = V3<Cnt>(Cnt(0.6), Cnt(0.0), Cnt(0.8));
    ct.d = Cnt(0.002);
    const V3<Cnt> vA(d, e, f), vB(b, c, a);
    g_tally = Tally();
    penalty_force(ct, vA, vB, Cnt(1e4), Cnt(100.0), Cnt(0.5), Cnt(0.01));
  } else if (which == 2) {
    const V3<Cnt> x(a, b, c), y(d, e, f);
    g_tally = Tally();
    cross(x, y);
  } else if (which == 3) {
    Q4<Cnt> q;
    q.w = Cnt(0.9); q.x = Cnt(0.1); q.y = Cnt(-0.3); q.z = Cnt(0.2);
    g_tally = Tally();
    quat_to_mat(q);
  }
  out[0] = g_tally.add; out[1] = g_tally.mul; out[2] = g_tally.fma;
  out[3] = g_tally.div; out[4] = g_tally.sqrt; out[5] = g_tally.trans;
}

// ---- surrogate network ----
long ref_mlp_n_params(void) { return mlp_n_params(); }

// Elementwise building blocks of the network, for pins at known values.
void ref_gelu_vec(const double *x, int n, double *y, double *dy) {
  for (int i = 0; i < n; ++i) {
    y[i] = gelu(x[i]);
    dy[i] = gelu_grad(x[i]);
  }
}
void ref_to_bf16_vec(const double *x, int n, double *y) {
  for (int i = 0; i < n; ++i) y[i] = to_bf16(x[i]);
}

// He-normal initialisation: W entry p of layer l ~ N(0, 2 / fan_in) from the
// normals of Philox stream 2 (block p / 4, sample 0, iteration 0, instance 0),
// rounded to FP32; biases 0.
void ref_mlp_init(uint64_t seed, double *P) {
  for (long i = 0; i < mlp_n_params(); ++i) P[i] = 0.0;
  for (int l = 0; l < MLP_L; ++l) {
    const long w0 = mlp_w_off(l), nw = (long)MLP_DIMS[l] * MLP_DIMS[l + 1];
    const double s = std::sqrt(2.0 / (double)MLP_DIMS[l]);
    for (long k = 0; k < nw; ++k) {
      const long p = w0 + k;
      Word4 x = philox_draw(seed, STREAM_MLP_INIT, (uint32_t)(p / 4), 0, 0, 0);
      float nrm[4];
      normals4(x, nrm);
      P[p] = (double)(float)((double)nrm[p % 4] * s);
    }
  }
}

void ref_mlp_forward(const double *P, const double *x, int n, double *y, int bf16) {
  mlp_forward(P, x, n, y, bf16 != 0, nullptr);
}

double ref_mlp_loss_grad(const double *P, const double *x, const double *t, int n, double *dP) {
  return mlp_loss_grad(P, x, t, n, dP);
}

// The same with BF16 operands in the forward and backward products (bf16 = 1).
double ref_mlp_loss_grad_bf16(const double *P, const double *x, const double *t, int n, double *dP) {
  return mlp_loss_grad(P, x, t, n, dP, true);
}

void ref_adam_step(double *P, const double *g, double *m, double *v, long n, double lr, double b1, double b2,
                   double eps, int t) {
  adam_step(P, g, m, v, n, lr, b1, b2, eps, t);
}

int ref_select(int pop, const float *cost, const uint8_t *tier, int n_elite, int32_t *elite_idx, int32_t *mode,
               int32_t tier_counts[4]) {
  return select_elites(pop, cost, tier, n_elite, elite_idx, mode, tier_counts);
}

int ref_cholesky(int D, const double *A, double *L) { return cholesky(D, A, L) ? 0 : 1; }
int ref_factor_cov(int D, const double *S, double *L) { return factor_cov(D, S, L); }

int ref_refit(int D, int cov_mode, const float *Z, const int32_t *elite, int ne, int32_t mode, const double *cov0,
              double *mu, double *S, double *L) {
  return refit(D, cov_mode, Z, elite, ne, mode, cov0, mu, S, L);
}

// Alg. 1 end to end: `iters` CE iterations of sample -> rollout -> select ->
// refit on one instance, iteration j with n_env(j) samples (pop_final 0: pop
// each), iteration 0 from the region when lo is given.  Outputs: best-ever
// row and its cost/tier, final theta (mu, S), and per-iteration stats rows of
// 8 doubles: [best cost this iteration, n_tier0, n_tier1, n_tier2, n_tier3,
// n_elite, mode, best-ever cost].
int ref_plan_solve(const RefScene *s, uint64_t seed, uint32_t inst, int pop, int n_elite, int iters, int cov_mode,
                   const double *mu0, const double *cov0, int threads, float *best_z, double *best_cost,
                   int32_t *best_tier, double *mu_out, double *S_out, double *stats, int pop_final, int ramp,
                   const float *lo, const float *hi, int n_rings, const int *ring_dim, const float *ring) {
  const int D = param_dim(*s);
  std::vector<double> mu(mu0, mu0 + D), S(cov0, cov0 + D * D), L(D * D);
  if (cov_mode == 0)
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        if (a != b) S[a * D + b] = 0.0;
  factor_cov(D, S.data(), L.data());
  std::vector<float> Z((long)pop * D), costf(pop);
  std::vector<double> cost(pop);
  std::vector<uint8_t> tier(pop);
  std::vector<int32_t> elite(n_elite);
  int32_t bt = 4;
  double bc = INFINITY;
  const int pop_max = pop;
  for (int j = 0; j < iters; ++j) {
    pop = n_env_at(pop_max, pop_final, ramp, j);
    if (j == 0 && lo)
      ref_sample_region(seed, inst, pop, D, lo, hi, n_rings, ring_dim, ring, Z.data());
    else
      ref_sample(seed, (uint32_t)j, inst, pop, D, mu.data(), L.data(), Z.data());
    ref_rollout(s, seed, inst, pop, Z.data(), cost.data(), tier.data(), nullptr, nullptr, 0, threads, nullptr, nullptr,
                nullptr);
    for (int i = 0; i < pop; ++i) costf[i] = (float)cost[i];
    int32_t mode, counts[4];
    const int ne = select_elites(pop, costf.data(), tier.data(), n_elite, elite.data(), &mode, counts);
    // best of this iteration = first key in sorted order
    int bi = -1;
    for (int i = 0; i < pop; ++i) {
      const int ti = std::isnan(cost[i]) ? 3 : tier[i];
      const double ci = std::isnan(cost[i]) ? INFINITY : cost[i];
      if (bi < 0) { bi = i; continue; }
      const int tb = std::isnan(cost[bi]) ? 3 : tier[bi];
      const double cb = std::isnan(cost[bi]) ? INFINITY : cost[bi];
      if (ti < tb || (ti == tb && ci < cb)) bi = i;
    }
    if (bi >= 0) {
      const int ti = std::isnan(cost[bi]) ? 3 : tier[bi];
      if (ti < bt || (ti == bt && cost[bi] < bc)) {
        bt = ti;
        bc = cost[bi];
        for (int d = 0; d < D; ++d) best_z[d] = Z[(long)bi * D + d];
      }
    }
    if (stats) {
      double *st = stats + (long)j * 8;
      st[0] = bi >= 0 ? cost[bi] : INFINITY;
      for (int t = 0; t < 4; ++t) st[1 + t] = counts[t];
      st[5] = ne;
      st[6] = mode;
      st[7] = bc;
    }
    refit(D, cov_mode, Z.data(), elite.data(), ne, mode, cov0, mu.data(), S.data(), L.data());
  }
  *best_cost = bc;
  *best_tier = bt;
  for (int d = 0; d < D; ++d) mu_out[d] = mu[d];
  for (int i = 0; i < D * D; ++i) S_out[i] = S[i];
  return 0;
}

}  // extern "C"
