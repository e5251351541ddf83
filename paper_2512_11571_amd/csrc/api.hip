// The C ABI (include/cemtamp.h): context management, argument validation,
// launches and the replayed CE iteration.  Host code only; every step of the
// method runs in the kernels of the other translation units.
#include <atomic>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace cem;

namespace {

int fail(cem_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(cem_ctx *c, hipError_t e, const char *what) {
  return fail(c, CEM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                           \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

int dim_of(int kind) {
  switch (kind) {
    case CEM_SCENE_PUSH: return 3;
    case CEM_SCENE_PICKPLACE: return 16;
    case CEM_SCENE_MOVEPUSH: return 12;
    default: return 0;
  }
}

bool pos(float x) { return std::isfinite(x) && x > 0.0f; }
bool nonneg(float x) { return std::isfinite(x) && x >= 0.0f; }

// The iteration-0 region of a D-parameter problem: finite box bounds with
// lo <= hi, rings on disjoint in-range pairs with 0 <= r0 <= r1.
const char *check_region(const cem_init_region &R, int D) {
  for (int d = 0; d < D; ++d)
    if (!std::isfinite(R.lo[d]) || !std::isfinite(R.hi[d]) || !(R.lo[d] <= R.hi[d])) return "region box bound";
  if (R.n_annuli < 0 || R.n_annuli > CEM_MAX_ANNULI) return "region ring count";
  unsigned used = 0;
  for (int k = 0; k < R.n_annuli; ++k) {
    const int d = R.ann_dim[k];
    if (d < 0 || d + 1 >= D) return "region ring dimension";
    if (used & (3u << d)) return "region rings overlap";
    used |= 3u << d;
    const float r0 = R.ann_radius[k][0], r1 = R.ann_radius[k][1];
    if (!std::isfinite(R.ann_center[k][0]) || !std::isfinite(R.ann_center[k][1]) || !std::isfinite(r1) ||
        !(r0 >= 0.0f) || !(r0 <= r1))
      return "region ring radii";
  }
  return nullptr;
}

int pop_at(const cem_ctx *c, int j) {
  if (c->pop_final <= 0) return c->pop;
  const long k = std::min(j, c->pop_ramp);
  return c->pop - (int)(((long)(c->pop - c->pop_final) * k) / c->pop_ramp);
}

const char *check_scene(const cem_scene &s) {
  if (dim_of(s.kind) == 0) return "unknown scene kind";
  if (s.substeps < 1 || s.substeps > 1000) return "substeps out of range [1, 1000]";
  if (s.horizon < 1 || s.horizon > 100000) return "horizon out of range [1, 100000]";
  if (s.settle_steps < 0 || s.settle_steps > s.horizon) return "settle_steps out of range [0, horizon]";
  if (s.fail_stop != 0 && s.fail_stop != 1) return "fail_stop must be 0 or 1";
  if (s.dr_scenarios < 0 || s.dr_scenarios > CEM_MAX_DR || (s.dr_scenarios & (s.dr_scenarios - 1)))
    return "dr_scenarios must be 0 or a power of two <= 64";
  if (s.dr_scenarios > 1 && s.kind == CEM_SCENE_PUSH) return "domain randomisation needs a robot scene";
  if (s.dr_reduce != 0 && s.dr_reduce != 1) return "dr_reduce must be 0 (mean) or 1 (max)";
  if (!nonneg(s.dr_mu_lo) || !nonneg(s.dr_mu_hi) || (s.dr_mu_hi > 0.0f && !(s.dr_mu_lo <= s.dr_mu_hi)))
    return "invalid dr friction range";
  if (!nonneg(s.dr_mass_lo) || !nonneg(s.dr_mass_hi) ||
      (s.dr_mass_hi > 0.0f && !(s.dr_mass_lo > 0.0f && s.dr_mass_lo <= s.dr_mass_hi)))
    return "invalid dr mass range";
  if (!pos(s.dt) || !nonneg(s.gravity) || !nonneg(s.k_contact) || !nonneg(s.c_contact) || !pos(s.eps_v))
    return "invalid physical constants";
  if (!nonneg(s.mu_ground) || !nonneg(s.mu_tool) || !nonneg(s.mu_static) || !nonneg(s.mu_ramp))
    return "invalid friction coefficient";
  if (!nonneg(s.obj_mu_lo) || !nonneg(s.obj_mu_hi) || (s.obj_mu_hi > 0.0f && !(s.obj_mu_lo <= s.obj_mu_hi)))
    return "invalid object friction range";
  if (!pos(s.obj_half[0]) || !pos(s.obj_half[1]) || !pos(s.obj_half[2]) || !pos(s.obj_mass))
    return "invalid object";
  if (s.n_static < 0 || s.n_static > CEM_MAX_STATIC) return "n_static out of range";
  if (s.kind == CEM_SCENE_PUSH) {
    if (!pos(s.pusher_radius) || !nonneg(s.pusher_vmax) || s.pusher_steps < 0) return "invalid pusher";
    if (!nonneg(s.goal_tol) || !nonneg(s.time_weight)) return "invalid goal tolerance or time weight";
    if (!(s.goal_rho_lo <= s.goal_rho_hi) || !(s.goal_phi_lo <= s.goal_phi_hi)) return "invalid goal ranges";
  }
  if (s.kind == CEM_SCENE_PICKPLACE || s.kind == CEM_SCENE_MOVEPUSH) {
    // the kernels unroll the fixed tree: base x, y, yaw; a serial arm 3..8; fingers 9, 10 on body 8
    if (s.n_joints != 11) return "robot must have 11 joints";
    for (int j = 0; j < 11; ++j) {
      const int want = j == 0 ? -1 : (j <= 8 ? j - 1 : 8);
      if (s.j_parent[j] != want) return "robot topology differs from base(3) + arm(6) + fingers(2)";
      if (s.j_type[j] != 0 && s.j_type[j] != 1) return "joint type must be 0 or 1";
      if (s.j_axis[j] < 0 || s.j_axis[j] > 5) return "joint axis must be 0..5";
      if (!nonneg(s.b_mass[j]) || !nonneg(s.j_inom[j]) || !std::isfinite(s.q0[j])) return "invalid body";
    }
    if (s.j_type[0] != 1 || s.j_type[1] != 1 || s.j_type[9] != 1 || s.j_type[10] != 1)
      return "base x, y and the fingers must be prismatic";
    if (s.ee_body != 8) return "end effector must be body 8";
    if (s.ik_iters < 0 || s.ik_iters > 1000 || !pos(s.ik_lambda) || !pos(s.omega_c) || !nonneg(s.zeta))
      return "invalid controller gains";
    if (!pos(s.base_vmin) || !(s.base_vmax >= s.base_vmin) || !pos(s.base_wmax) || !pos(s.joint_speed_max) ||
        !pos(s.accel_max))
      return "invalid speed limits";
    if (!pos(s.t_approach) || !pos(s.t_descend) || !nonneg(s.t_close) || !pos(s.t_lift) || !pos(s.t_transfer) ||
        !nonneg(s.t_release))
      return "invalid phase durations";
    if (s.kind == CEM_SCENE_PICKPLACE) {
      if (s.goal_static < 0 || s.goal_static >= s.n_static) return "goal_static must index a static box";
    } else {
      if (s.goal_static >= s.n_static) return "goal_static out of range";
      if (s.goal_static < 0 && !(pos(s.goal_box_half[0]) && pos(s.goal_box_half[1]) && pos(s.goal_box_half[2]) &&
                                 std::isfinite(s.goal_box_center[0]) && std::isfinite(s.goal_box_center[1]) &&
                                 std::isfinite(s.goal_box_center[2])))
        return "invalid goal box";
      if (!pos(s.push_vmin) || !(s.push_vmax >= s.push_vmin) || !nonneg(s.push_dmax) || !pos(s.timeout_push))
        return "invalid push limits";
    }
  }
  return nullptr;
}

InstDesc desc_of(cem_ctx *c, const float *Z, int pop, float *cost, uint8_t *tier, float *pose) {
  InstDesc d{};
  d.st = c->st;
  d.Z = Z;
  d.cost = cost;
  d.tier = tier;
  d.pose = pose;
  d.stats = c->stats;
  d.kind = c->scene.kind;
  d.pop = pop;
  d.D = c->D;
  d.iters = 1 << 30;
  d.scen = scenarios(c->scene);
  d.lanes = c->lanes;
  d.spec = robot_spec_for(c->scene) ? 1 : 0;
  // one lane per environment: the launch hands out the plans in an order it
  // sets (rollout.hip, order_plans); lane groups keep index order
  if (c->perm && c->lanes == 1 && pop <= c->pop) d.perm = c->perm;
  return d;
}

int launch_rollout(cem_ctx *c, const float *Z, int pop, float *cost, uint8_t *tier, float *pose, float *trace,
                   int trace_steps, hipStream_t s) {
  const hipError_t e = launch_rollout_single(desc_of(c, Z, pop, cost, tier, pose), trace, trace_steps, s);
  if (e != hipSuccess) return hip_fail(c, e, "rollout launch");
  return CEM_OK;
}

int factor_and_check(cem_ctx *c, hipStream_t s) {
  HIPCHK(c, launch_factor(c->st, s));
  int32_t status = 0;
  HIPCHK(c, hipMemcpyAsync(&status, &c->st->factor_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (status != 0) return fail(c, CEM_E_NUMERIC, "covariance is not positive definite: diagonal fallback in use");
  return CEM_OK;
}

int reset_best(cem_ctx *c, hipStream_t s) {
  const int32_t iter = 0, tier = 4;
  const float inf = INFINITY;
  HIPCHK(c, hipMemcpyAsync(&c->st->iter, &iter, sizeof iter, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(&c->st->best_tier, &tier, sizeof tier, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(&c->st->best_cost, &inf, sizeof inf, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return CEM_OK;
}

// theta upload: mu (D), covariance (D x D; off-diagonals dropped in diag mode).
int upload_theta(cem_ctx *c, const double *mu, const double *cov, bool also_cov0, hipStream_t s) {
  const int D = c->D;
  double hm[MAX_D], hs[MAX_D * MAX_D];
  for (int d = 0; d < D; ++d) {
    if (!std::isfinite(mu[d])) return fail(c, CEM_E_ARG, "mu has a non-finite entry");
    hm[d] = mu[d];
  }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      const double v = cov[a * D + b];
      if (!std::isfinite(v)) return fail(c, CEM_E_ARG, "covariance has a non-finite entry");
      if (v != cov[b * D + a]) return fail(c, CEM_E_ARG, "covariance is not symmetric");
      hs[a * D + b] = (c->cov_mode == 0 && a != b) ? 0.0 : v;
    }
  HIPCHK(c, hipMemcpyAsync(c->st->mu, hm, sizeof(double) * D, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->st->S, hs, sizeof(double) * D * D, hipMemcpyHostToDevice, s));
  if (also_cov0) HIPCHK(c, hipMemcpyAsync(c->st->cov0, hs, sizeof(double) * D * D, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return CEM_OK;
}

void release(cem_ctx *c) {
  if (!c) return;
  if (c->iter_graph) (void)hipGraphExecDestroy(c->iter_graph);
  if (c->own) (void)hipStreamDestroy(c->own);
  (void)hipFree(c->st);
  (void)hipFree(c->Z);
  (void)hipFree(c->cost);
  (void)hipFree(c->pose);
  (void)hipFree(c->tier);
  (void)hipFree(c->stats);
  (void)hipFree(c->perm);
}

}  // namespace

extern "C" {

const char *cem_strerror(int code) {
  switch (code) {
    case CEM_OK: return "ok";
    case CEM_E_ARG: return "invalid argument";
    case CEM_E_SCENE: return "invalid scene";
    case CEM_E_ALLOC: return "device allocation failed";
    case CEM_E_HIP: return "HIP runtime error";
    case CEM_E_NUMERIC: return "covariance not factorable (diagonal fallback used)";
    case CEM_E_STATE: return "invalid context state";
    default: return "unknown error";
  }
}

const char *cem_last_error(const cem_ctx *c) { return c ? c->err.c_str() : "null context"; }

int cem_dim(const cem_ctx *c) { return c ? c->D : 0; }

int cem_sizeof(int which) {
  switch (which) {
    case 0: return (int)sizeof(cem_scene);
    case 1: return (int)sizeof(cem_problem);
    case 2: return (int)sizeof(cem_result);
    case 3: return (int)sizeof(cem_init_region);
    default: return 0;
  }
}

int cem_init(const cem_problem *p, cem_ctx **out) {
  if (!out) return CEM_E_ARG;
  *out = nullptr;
  if (!p || !p->scene || !p->mu0 || !p->cov0) return CEM_E_ARG;
  const char *why = check_scene(*p->scene);
  if (why) return CEM_E_SCENE;
  const int D = dim_of(p->scene->kind);
  if (p->pop < 1 || p->pop > MAX_POP) return CEM_E_ARG;
  if (p->n_elite < 1 || p->n_elite > p->pop || p->n_elite > MAX_ELITE) return CEM_E_ARG;
  if (p->cov_mode != 0 && p->cov_mode != 1) return CEM_E_ARG;
  if (p->pop_final != 0 && (p->pop_final < p->n_elite || p->pop_final > p->pop || p->pop_ramp_iters < 1))
    return CEM_E_ARG;
  if (p->init_region && check_region(*p->init_region, D)) return CEM_E_ARG;
  const int lanes = p->lanes_per_env <= 1 ? 1 : p->lanes_per_env;
  if (p->lanes_per_env < 0 || (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16) ||
      (lanes > 1 && p->scene->kind == CEM_SCENE_PUSH) || lanes * scenarios(*p->scene) > 64)
    return CEM_E_ARG;

  cem_ctx *c = new (std::nothrow) cem_ctx();
  if (!c) return CEM_E_ALLOC;
  c->scene = *p->scene;
  c->D = D;
  c->pop = p->pop;
  c->n_elite = p->n_elite;
  c->cov_mode = p->cov_mode;
  c->pop_final = p->pop_final;
  c->pop_ramp = p->pop_final ? p->pop_ramp_iters : 0;
  c->lanes = lanes;
  c->seed = p->seed;
  c->inst = p->instance;
  static std::atomic<uint64_t> next_serial{1};
  c->serial = next_serial.fetch_add(1);
  int rc = CEM_OK;
  do {
    if (hipGetDevice(&c->device) != hipSuccess) { rc = fail(c, CEM_E_HIP, "hipGetDevice"); break; }
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
      rc = fail(c, CEM_E_HIP, "stream create");
      break;
    }
    const size_t P = (size_t)p->pop;
    if (hipMalloc(&c->st, sizeof(DevState)) != hipSuccess || hipMalloc(&c->Z, sizeof(float) * P * D) != hipSuccess ||
        hipMalloc(&c->cost, sizeof(float) * P) != hipSuccess || hipMalloc(&c->pose, sizeof(float) * P * 7) != hipSuccess ||
        hipMalloc(&c->tier, P) != hipSuccess ||
        hipMalloc(&c->stats, sizeof(float) * MAX_STATS_ITERS * CEM_STATS_COLS) != hipSuccess ||
        (c->scene.kind != CEM_SCENE_PUSH && hipMalloc(&c->perm, sizeof(int32_t) * P) != hipSuccess)) {
      rc = fail(c, CEM_E_ALLOC, "device allocation");
      break;
    }
    DevState h;
    std::memset(&h, 0, sizeof h);
    h.D = D;
    h.cov_mode = p->cov_mode;
    h.n_elite = p->n_elite;
    h.best_cost = INFINITY;
    h.best_tier = 4;
    h.seed = c->seed;
    h.inst_id = c->inst;
    h.pop = c->pop;
    h.scene = c->scene;
    if (p->init_region) {
      h.region = *p->init_region;
      h.region_on = 1;
    }
    if (hipMemcpyAsync(c->st, &h, sizeof h, hipMemcpyHostToDevice, c->own) != hipSuccess) {
      rc = fail(c, CEM_E_HIP, "state upload");
      break;
    }
    if ((rc = upload_theta(c, p->mu0, p->cov0, true, c->own)) != CEM_OK) break;
    if (launch_instance_draw(c->scene, c->seed, c->inst, c->st, c->own) != hipSuccess ||
        launch_scene_consts(c->st, c->own) != hipSuccess) {
      rc = fail(c, CEM_E_HIP, "instance set-up launch");
      break;
    }
    rc = factor_and_check(c, c->own);
    if (rc == CEM_E_NUMERIC) rc = fail(c, CEM_E_ARG, "cov0 is not positive definite");
  } while (0);
  if (rc != CEM_OK) {
    release(c);
    delete c;
    return rc;
  }
  *out = c;
  return CEM_OK;
}

void cem_free(cem_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->own);
  release(c);
  delete c;
}

int cem_sample(cem_ctx *c, int32_t iter, float *Z_dev, void *stream) {
  if (!c) return CEM_E_ARG;
  if (!Z_dev || iter < 0) return fail(c, CEM_E_ARG, "Z_dev is null or iter < 0");
  HIPCHK(c, launch_sample(c->seed, c->inst, iter, c->st, c->pop, c->D, Z_dev, (hipStream_t)stream));
  return CEM_OK;
}

int rollout_batch(cem_ctx *c, const float *Z_dev, int32_t pop, float *cost_dev, uint8_t *tier_dev, float *pose_dev,
                  void *stream) {
  if (!c) return CEM_E_ARG;
  if (pop < 0 || pop > MAX_POP) return fail(c, CEM_E_ARG, "pop out of range [0, 65536]");
  if (pop == 0) return CEM_OK;
  if (!Z_dev || !cost_dev || !tier_dev) return fail(c, CEM_E_ARG, "null buffer");
  return launch_rollout(c, Z_dev, pop, cost_dev, tier_dev, pose_dev, nullptr, 0, (hipStream_t)stream);
}

int rollout_trace(cem_ctx *c, const float *Z_dev, int32_t pop, int32_t n_steps, float *trace_dev, void *stream) {
  if (!c) return CEM_E_ARG;
  if (!Z_dev || !trace_dev) return fail(c, CEM_E_ARG, "null buffer");
  if (pop < 0 || pop > MAX_POP) return fail(c, CEM_E_ARG, "pop out of range [0, 65536]");
  if (n_steps < 1 || n_steps > c->scene.horizon) return fail(c, CEM_E_ARG, "n_steps out of range [1, horizon]");
  if (scenarios(c->scene) > 1) return fail(c, CEM_E_ARG, "traces are per environment: no domain randomisation");
  if (pop == 0) return CEM_OK;
  return launch_rollout(c, Z_dev, pop, nullptr, nullptr, nullptr, trace_dev, n_steps, (hipStream_t)stream);
}

int cem_refit(cem_ctx *c, const float *Z_dev, const float *cost_dev, const uint8_t *tier_dev, int32_t pop,
              int32_t *elite_idx_dev, int32_t *sel_info_dev, void *stream) {
  if (!c) return CEM_E_ARG;
  if (!Z_dev || !cost_dev || !tier_dev) return fail(c, CEM_E_ARG, "null buffer");
  if (pop < 1 || pop > MAX_POP) return fail(c, CEM_E_ARG, "pop out of range [1, 65536]");
  HIPCHK(c, launch_select_refit(c->st, Z_dev, cost_dev, tier_dev, pop, elite_idx_dev, sel_info_dev, c->stats,
                                MAX_STATS_ITERS, 1, (hipStream_t)stream));
  return CEM_OK;
}

int plan_solve(cem_ctx *c, int32_t iters, cem_result *res, float *stats_host, void *stream) {
  if (!c) return CEM_E_ARG;
  if (!res || iters < 0) return fail(c, CEM_E_ARG, "null result or iters < 0");
  hipStream_t s = (hipStream_t)stream;
  int32_t it0 = 0;
  HIPCHK(c, hipMemcpyAsync(&it0, &c->st->iter, sizeof it0, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (it0 + iters > MAX_STATS_ITERS) return fail(c, CEM_E_ARG, "iteration counter would exceed 4096");
  if (c->pop_final > 0) {
    // n_env schedule: each iteration launched with its own row count (the
    // sampler reads the iteration from the device counter, which the refit
    // advances)
    for (int j = 0; j < iters; ++j) {
      const int n = pop_at(c, it0 + j);
      HIPCHK(c, launch_sample(c->seed, c->inst, -1, c->st, n, c->D, c->Z, s));
      const int r = launch_rollout(c, c->Z, n, c->cost, c->tier, c->pose, nullptr, 0, s);
      if (r != CEM_OK) return r;
      HIPCHK(c, launch_select_refit(c->st, c->Z, c->cost, c->tier, n, nullptr, nullptr, c->stats, MAX_STATS_ITERS,
                                    1, s));
    }
  } else if (!c->iter_graph) {
    // one CE iteration: sample (iteration read from the device counter) ->
    // rollout -> select/refit (advances the counter), captured once
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = launch_sample(c->seed, c->inst, -1, c->st, c->pop, c->D, c->Z, c->own);
    int r2 = launch_rollout(c, c->Z, c->pop, c->cost, c->tier, c->pose, nullptr, 0, c->own);
    hipError_t e3 = launch_select_refit(c->st, c->Z, c->cost, c->tier, c->pop, nullptr, nullptr, c->stats,
                                        MAX_STATS_ITERS, 1, c->own);
    hipError_t e4 = hipStreamEndCapture(c->own, &g);
    if (e1 != hipSuccess || r2 != CEM_OK || e3 != hipSuccess || e4 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, CEM_E_HIP, "graph capture of the CE iteration failed");
    }
    hipError_t e5 = hipGraphInstantiate(&c->iter_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e5 != hipSuccess) {
      c->iter_graph = nullptr;
      return hip_fail(c, e5, "hipGraphInstantiate");
    }
  }
  if (c->pop_final <= 0)
    for (int j = 0; j < iters; ++j) HIPCHK(c, hipGraphLaunch(c->iter_graph, s));
  DevState h;
  HIPCHK(c, hipMemcpyAsync(&h, c->st, sizeof h, hipMemcpyDeviceToHost, s));
  if (stats_host && iters > 0)
    HIPCHK(c, hipMemcpyAsync(stats_host, c->stats + (size_t)it0 * CEM_STATS_COLS,
                             sizeof(float) * iters * CEM_STATS_COLS, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::memset(res, 0, sizeof *res);
  res->dim = c->D;
  for (int d = 0; d < c->D; ++d) {
    res->best_z[d] = h.best_z[d];
    res->mu[d] = h.mu[d];
  }
  for (int t = 0; t < c->D * c->D; ++t) res->cov[t] = h.S[t];
  res->best_cost = h.best_cost;
  res->best_tier = h.best_tier;
  res->iters_done = h.iter;
  return h.factor_status ? fail(c, CEM_E_NUMERIC, "diagonal fallback used in the last refit") : CEM_OK;
}

int cem_get_theta(cem_ctx *c, double *mu, double *cov) {
  if (!c) return CEM_E_ARG;
  if (!mu || !cov) return fail(c, CEM_E_ARG, "null output");
  HIPCHK(c, hipMemcpyAsync(mu, c->st->mu, sizeof(double) * c->D, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipMemcpyAsync(cov, c->st->S, sizeof(double) * c->D * c->D, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipStreamSynchronize(c->own));
  return CEM_OK;
}

int cem_set_theta(cem_ctx *c, const double *mu, const double *cov) {
  if (!c) return CEM_E_ARG;
  if (!mu || !cov) return fail(c, CEM_E_ARG, "null input");
  HIPCHK(c, hipDeviceSynchronize());
  int rc = upload_theta(c, mu, cov, false, c->own);
  if (rc != CEM_OK) return rc;
  return factor_and_check(c, c->own);
}

int cem_get_factor(cem_ctx *c, double *L) {
  if (!c) return CEM_E_ARG;
  if (!L) return fail(c, CEM_E_ARG, "null output");
  HIPCHK(c, hipMemcpyAsync(L, c->st->L, sizeof(double) * c->D * c->D, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipStreamSynchronize(c->own));
  return CEM_OK;
}

int cem_pop_at(const cem_ctx *c, int32_t iter) { return (c && iter >= 0) ? pop_at(c, iter) : 0; }

int cem_get_instance(cem_ctx *c, double *draws) {
  if (!c) return CEM_E_ARG;
  if (!draws) return fail(c, CEM_E_ARG, "null output");
  float mu = 0.0f;
  HIPCHK(c, hipMemcpyAsync(draws, c->st->goal, sizeof(double) * 2, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipMemcpyAsync(&mu, &c->st->obj_mu, sizeof(float), hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipStreamSynchronize(c->own));
  draws[2] = (double)mu;
  return CEM_OK;
}

int cem_get_scenarios(cem_ctx *c, float *mu, float *mass) {
  if (!c) return CEM_E_ARG;
  if (!mu || !mass) return fail(c, CEM_E_ARG, "null output");
  HIPCHK(c, hipMemcpyAsync(mu, c->st->dr_mu, sizeof(float) * CEM_MAX_DR, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipMemcpyAsync(mass, c->st->dr_mass, sizeof(float) * CEM_MAX_DR, hipMemcpyDeviceToHost, c->own));
  HIPCHK(c, hipStreamSynchronize(c->own));
  return CEM_OK;
}

int cem_env_steps(cem_ctx *c, uint64_t *steps) {
  if (!c) return CEM_E_ARG;
  if (!steps) return fail(c, CEM_E_ARG, "null output");
  HIPCHK(c, hipDeviceSynchronize());
  unsigned long long n = 0;
  HIPCHK(c, hipMemcpy(&n, &c->st->env_steps, sizeof n, hipMemcpyDeviceToHost));
  *steps = (uint64_t)n;
  return CEM_OK;
}

int cem_get_outcomes(cem_ctx *c, int32_t n, float *cost, uint8_t *tier, float *pose) {
  if (!c) return CEM_E_ARG;
  if (n < 0 || n > c->pop) return fail(c, CEM_E_ARG, "n out of range [0, pop]");
  if (!cost || !tier) return fail(c, CEM_E_ARG, "null output");
  HIPCHK(c, hipDeviceSynchronize());
  if (n == 0) return CEM_OK;
  HIPCHK(c, hipMemcpy(cost, c->cost, sizeof(float) * n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(tier, c->tier, n, hipMemcpyDeviceToHost));
  if (pose) HIPCHK(c, hipMemcpy(pose, c->pose, sizeof(float) * 7 * n, hipMemcpyDeviceToHost));
  return CEM_OK;
}

int cem_reset(cem_ctx *c) {
  if (!c) return CEM_E_ARG;
  HIPCHK(c, hipDeviceSynchronize());
  return reset_best(c, c->own);
}

}  // extern "C"

// ---- batched instances -------------------------------------------------------

struct cem_batch {
  std::vector<cem_ctx *> ctx;
  std::vector<int32_t> iters;
  InstDesc *insts = nullptr;
  WorkItem *items = nullptr;
  int n_items = 0, max_pop = 0, item_envs = 64, grid = 0, n_cu = 0;
  int *queue = nullptr;
  int *pool = nullptr;  // per instance: the next unstarted plan of its rollout (batched launch)
  hipStream_t own = nullptr;
  hipGraphExec_t graph = nullptr;
  std::string err;
};

namespace {

int bfail(cem_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

// The batch takes the rollout instance specialised to the robot model when
// every robot instance's robot is the model.
bool batch_spec(const cem_batch *b) {
  for (const cem_ctx *c : b->ctx)
    if (c->scene.kind != CEM_SCENE_PUSH && !robot_spec_for(c->scene)) return false;
  return true;
}

#define BHIPCHK(b, expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return bfail(b, CEM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Work list: every instance cut into items of `envs` environments, the most
// expensive first (horizon x substeps x a per-substep weight of the scene kind),
// so the long items start early and the short ones fill in behind them.
int build_items(cem_batch *b, int envs) {
  struct Key {
    double cost;
    WorkItem w;
  };
  std::vector<Key> keys;
  for (int i = 0; i < (int)b->ctx.size(); ++i) {
    const cem_ctx *c = b->ctx[i];
    const double weight = c->scene.kind == CEM_SCENE_PUSH ? 1.0 : 28.0;
    const double per_env = (double)c->scene.horizon * c->scene.substeps * weight;
    // a row's scenarios (a power of two <= 64) never straddle two items
    const int R = scenarios(c->scene), step = std::max(envs, R), n_env = c->pop * R;
    for (int e0 = 0; e0 < n_env; e0 += step) {
      Key k;
      k.w.inst = i;
      k.w.env0 = e0;
      k.w.n = std::min(step, n_env - e0);
      k.w.pad = 0;
      k.cost = per_env;
      keys.push_back(k);
    }
  }
  std::stable_sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) { return a.cost > b.cost; });
  std::vector<WorkItem> h(keys.size());
  for (size_t i = 0; i < keys.size(); ++i) h[i] = keys[i].w;
  if (b->items) (void)hipFree(b->items);
  b->items = nullptr;
  BHIPCHK(b, hipMalloc(&b->items, sizeof(WorkItem) * std::max<size_t>(1, h.size())));
  BHIPCHK(b, hipMemcpy(b->items, h.data(), sizeof(WorkItem) * h.size(), hipMemcpyHostToDevice));
  b->n_items = (int)h.size();
  b->item_envs = envs;
  return CEM_OK;
}

// One CE iteration of every instance still under its cap: batched sampling,
// one persistent rollout launch over the work list, one refit workgroup per instance.
int build_graph(cem_batch *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  hipGraph_t g = nullptr;
  BHIPCHK(b, hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
  const int n = (int)b->ctx.size();
  hipError_t e1 = launch_sample_batch(b->insts, n, b->max_pop, b->own);
  hipError_t e2 = launch_rollout_batch(b->insts, n, b->items, b->n_items, b->queue, b->pool, b->grid, batch_spec(b),
                                       b->own);
  hipError_t e3 = launch_select_refit_batch(b->insts, n, MAX_STATS_ITERS, b->own);
  hipError_t e4 = hipStreamEndCapture(b->own, &g);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, CEM_E_HIP, "graph capture of the batched CE iteration failed");
  }
  hipError_t e5 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e5 != hipSuccess) {
    b->graph = nullptr;
    return bfail(b, CEM_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e5));
  }
  return CEM_OK;
}

void batch_release(cem_batch *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->own) (void)hipStreamDestroy(b->own);
  (void)hipFree(b->insts);
  (void)hipFree(b->items);
  (void)hipFree(b->queue);
  (void)hipFree(b->pool);
  for (cem_ctx *c : b->ctx) cem_free(c);
}

}  // namespace

extern "C" {

int cem_batch_init(const cem_problem *problems, const int32_t *iters, int32_t n, cem_batch **out) {
  if (!out) return CEM_E_ARG;
  *out = nullptr;
  if (!problems || !iters || n < 1 || n > 4096) return CEM_E_ARG;
  for (int i = 0; i < n; ++i)
    if (iters[i] < 0 || iters[i] > MAX_STATS_ITERS || problems[i].pop_final != 0 || problems[i].lanes_per_env > 1)
      return CEM_E_ARG;
  cem_batch *b = new (std::nothrow) cem_batch();
  if (!b) return CEM_E_ALLOC;
  int rc = CEM_OK;
  for (int i = 0; i < n && rc == CEM_OK; ++i) {
    cem_ctx *c = nullptr;
    rc = cem_init(&problems[i], &c);
    if (rc == CEM_OK) b->ctx.push_back(c);
    else b->err = "cem_init failed for instance " + std::to_string(i);
  }
  if (rc == CEM_OK) {
    b->iters.assign(iters, iters + n);
    std::vector<InstDesc> h(n);
    for (int i = 0; i < n; ++i) {
      cem_ctx *c = b->ctx[i];
      h[i] = desc_of(c, c->Z, c->pop, c->cost, c->tier, c->pose);
      h[i].iters = iters[i];
      b->max_pop = std::max(b->max_pop, c->pop);
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&b->insts, sizeof(InstDesc) * n) != hipSuccess || hipMalloc(&b->queue, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->pool, sizeof(int) * n) != hipSuccess ||
        hipMemcpy(b->insts, h.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice) != hipSuccess) {
      rc = CEM_E_HIP;
      b->err = "batch set-up";
    }
  }
  if (rc == CEM_OK) {
    b->grid = 2 * b->n_cu;
    rc = build_items(b, 64);
  }
  if (rc == CEM_OK) rc = build_graph(b);
  if (rc != CEM_OK) {
    batch_release(b);
    delete b;
    return rc;
  }
  *out = b;
  return CEM_OK;
}

void cem_batch_free(cem_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->own);
  batch_release(b);
  delete b;
}

const char *cem_batch_last_error(const cem_batch *b) { return b ? b->err.c_str() : "null batch"; }

int cem_batch_size(const cem_batch *b) { return b ? (int)b->ctx.size() : 0; }

cem_ctx *cem_batch_instance(cem_batch *b, int32_t i) {
  if (!b || i < 0 || i >= (int)b->ctx.size()) return nullptr;
  return b->ctx[i];
}

int cem_batch_autotune(cem_batch *b, int32_t *config_out) {
  if (!b) return CEM_E_ARG;
  const int mults[3] = {1, 2, 4};
  const int envs_opts[2] = {64, 32};
  float best = INFINITY;
  int best_grid = b->grid, best_envs = b->item_envs;
  // the trial passes roll out the instances' current iteration's samples (the
  // sampling does not advance the iteration counter, so the next step draws
  // the same rows again); their simulated steps are not the CE run's, so each
  // instance's step counter is put back afterwards
  const int n = (int)b->ctx.size();
  std::vector<unsigned long long> steps0(n);
  BHIPCHK(b, hipStreamSynchronize(b->own));
  BHIPCHK(b, hipDeviceSynchronize());
  for (int i = 0; i < n; ++i)
    BHIPCHK(b, hipMemcpy(&steps0[i], &b->ctx[i]->st->env_steps, sizeof(unsigned long long), hipMemcpyDeviceToHost));
  BHIPCHK(b, launch_sample_batch(b->insts, n, b->max_pop, b->own));
  hipEvent_t e0, e1;
  BHIPCHK(b, hipEventCreate(&e0));
  BHIPCHK(b, hipEventCreate(&e1));
  for (int ei = 0; ei < 2; ++ei) {
    int rc = build_items(b, envs_opts[ei]);
    if (rc != CEM_OK) return rc;
    for (int mi = 0; mi < 3; ++mi) {
      const int grid = mults[mi] * b->n_cu;
      BHIPCHK(b, hipEventRecord(e0, b->own));
      BHIPCHK(b, launch_rollout_batch(b->insts, n, b->items, b->n_items, b->queue, b->pool, grid, batch_spec(b),
                                      b->own));
      BHIPCHK(b, hipEventRecord(e1, b->own));
      BHIPCHK(b, hipEventSynchronize(e1));
      float ms = 0.0f;
      BHIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_grid = grid;
        best_envs = envs_opts[ei];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < n; ++i)
    BHIPCHK(b, hipMemcpyAsync(&b->ctx[i]->st->env_steps, &steps0[i], sizeof(unsigned long long),
                              hipMemcpyHostToDevice, b->own));
  BHIPCHK(b, hipStreamSynchronize(b->own));
  b->grid = best_grid;
  int rc = build_items(b, best_envs);
  if (rc == CEM_OK) rc = build_graph(b);
  if (config_out) {
    config_out[0] = b->grid;
    config_out[1] = b->item_envs;
    config_out[2] = (int32_t)(best * 1000.0f);  // microseconds of the fastest rollout pass
  }
  return rc;
}

int cem_batch_step(cem_batch *b, void *stream) {
  if (!b) return CEM_E_ARG;
  BHIPCHK(b, hipGraphLaunch(b->graph, (hipStream_t)stream));
  return CEM_OK;
}

int cem_batch_record(cem_batch *b, int32_t iters, float *X_dev, float *Y_dev, int64_t capacity, int64_t *n_out,
                     void *stream) {
  if (!b) return CEM_E_ARG;
  if (iters < 0 || !X_dev || !Y_dev || !n_out) return bfail(b, CEM_E_ARG, "bad arguments");
  for (cem_ctx *c : b->ctx)
    if (c->D != b->ctx[0]->D) return bfail(b, CEM_E_ARG, "recording needs one parameter dimension");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> it(b->ctx.size());
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    BHIPCHK(b, hipMemcpyAsync(&it[i], &b->ctx[i]->st->iter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  BHIPCHK(b, hipStreamSynchronize(s));
  int64_t n = 0;
  const int D = b->ctx[0]->D;
  for (int j = 0; j < iters; ++j) {
    BHIPCHK(b, hipGraphLaunch(b->graph, s));
    for (size_t i = 0; i < b->ctx.size(); ++i) {
      cem_ctx *c = b->ctx[i];
      if (it[i] >= b->iters[i]) continue;  // this instance did not run in this step
      ++it[i];
      if (n + c->pop > capacity) return bfail(b, CEM_E_ARG, "dataset capacity exceeded");
      const float cap = c->scene.time_weight * c->scene.dt * (float)c->scene.horizon;
      BHIPCHK(b, launch_pack_dataset(desc_of(c, c->Z, c->pop, c->cost, c->tier, c->pose), cap, X_dev + n * D,
                                     Y_dev + n * 8, s));
      n += c->pop;
    }
  }
  BHIPCHK(b, hipStreamSynchronize(s));
  *n_out = n;
  return CEM_OK;
}

int cem_batch_solve(cem_batch *b, int32_t iters, cem_result *results, void *stream) {
  if (!b) return CEM_E_ARG;
  if (iters < 0) return bfail(b, CEM_E_ARG, "iters < 0");
  hipStream_t s = (hipStream_t)stream;
  for (int j = 0; j < iters; ++j) BHIPCHK(b, hipGraphLaunch(b->graph, s));
  BHIPCHK(b, hipStreamSynchronize(s));
  if (!results) return CEM_OK;
  int rc = CEM_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    cem_ctx *c = b->ctx[i];
    DevState h;
    BHIPCHK(b, hipMemcpy(&h, c->st, sizeof h, hipMemcpyDeviceToHost));
    cem_result &r = results[i];
    std::memset(&r, 0, sizeof r);
    r.dim = c->D;
    for (int d = 0; d < c->D; ++d) {
      r.best_z[d] = h.best_z[d];
      r.mu[d] = h.mu[d];
    }
    for (int t = 0; t < c->D * c->D; ++t) r.cov[t] = h.S[t];
    r.best_cost = h.best_cost;
    r.best_tier = h.best_tier;
    r.iters_done = h.iter;
    if (h.factor_status) rc = CEM_E_NUMERIC;
  }
  return rc;
}

}  // extern "C"
