// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/cemtamp.h"

namespace cem {

constexpr int MAX_D = CEM_MAX_D;
constexpr int MAX_ELITE = 256;
constexpr int MAX_POP = 65536;
constexpr int MAX_STATS_ITERS = 4096;

// Per-context constants derived from the scene once at set-up (by a device
// kernel), so the rollout does not recompute them every substep.
struct SceneConsts {
  float st_R[CEM_MAX_STATIC][9];       // static box rotations (box -> world), row-major
  int32_t st_axis[CEM_MAX_STATIC];     // 1 where that rotation is exactly the identity (no yaw, no pitch)
  float I_body[CEM_MAX_JOINTS][21];    // spatial inertia of body j about its frame origin: A(6) B(9) C(6)
};

// Device-resident CE state of one context (one task instance).
struct DevState {
  double mu[MAX_D];
  double S[MAX_D * MAX_D];     // covariance
  double L[MAX_D * MAX_D];     // its Cholesky factor (lower, row-major)
  double cov0[MAX_D * MAX_D];  // initial covariance (its diagonal feeds the single-elite noise)
  double goal[2];              // per-instance draw: the push goal
  float obj_mu;                // per-instance draw: the object's friction (0: per-class values)
  float dr_mu[CEM_MAX_DR];     // domain-randomisation scenarios: object friction and mass
  float dr_mass[CEM_MAX_DR];
  int32_t iter;                // CE iteration counter for the replayed iteration
  int32_t D, cov_mode, n_elite;
  float best_z[MAX_D];
  float best_cost;
  int32_t best_tier;
  int32_t factor_status;       // 0 ok, 1 diagonal fallback used
  int32_t sel_info[6];         // n_e, mode, n_tier0..3 of the last refit
  uint64_t seed;               // Philox key
  uint32_t inst_id;            // Philox counter word 3
  int32_t pop;
  cem_init_region region;      // iteration-0 region (used when region_on)
  int32_t region_on;
  cem_scene scene;             // device copy of the scene (read by the rollout kernels)
  SceneConsts sk;              // derived from scene by launch_scene_consts
  // Control steps the rollouts of this context have simulated (summed over
  // environments).  The only field a rollout writes: one atomic add per work
  // item through a generic pointer, never read by device code.
  unsigned long long env_steps;
};

// One task instance as the launches see it: its device state and buffers.
struct InstDesc {
  DevState *st;
  const float *Z;   // pop x D parameter rows
  float *cost;
  uint8_t *tier;
  float *pose;      // pop x 7, nullable
  float *stats;     // iteration stats rows (batched refit), nullable
  int32_t kind, pop, D, iters;  // iters: iteration cap in batched runs
  int32_t scen;                 // scenarios per row (1: no domain randomisation); pop * scen environments
  int32_t lanes;                // lanes per environment (1, 2, 4); pop * scen * lanes lanes
  int32_t spec;                 // 1: the robot is the compiled-in model (robot_spec_for), use its instance
  int32_t *perm;                // robot scene at one lane per environment: the order in which the launch hands
                                // plans to lanes (pop entries, written by the launch); nullptr: index order
};
// Up to 64 environments [env0, env0 + n) of instance `inst`.
struct WorkItem {
  int32_t inst, env0, n, pad;
};

// Domain-randomisation scenarios per parameter row (1: none).
inline int scenarios(const cem_scene &s) { return s.dr_scenarios > 1 ? s.dr_scenarios : 1; }

// Read-only views for the device code.  The scene, its derived constants and
// the rest of a context's state do not change while a rollout runs; reading
// them through the constant address space lets the compiler issue scalar
// loads for the wave-uniform accesses.
typedef const __attribute__((address_space(4))) cem_scene CScene;
typedef const __attribute__((address_space(4))) SceneConsts CConsts;
typedef const __attribute__((address_space(4))) DevState CDevState;
typedef const __attribute__((address_space(4))) InstDesc CInstDesc;
typedef const __attribute__((address_space(4))) WorkItem CWorkItem;

// Launchers (each file owns its kernels).
hipError_t launch_instance_draw(const cem_scene &sc, uint64_t seed, uint32_t inst, DevState *st, hipStream_t s);
hipError_t launch_sample(uint64_t seed, uint32_t inst, int32_t iter, const DevState *st, int pop, int D, float *Z,
                         hipStream_t s);
hipError_t launch_sample_batch(const InstDesc *insts, int n_inst, int max_pop, hipStream_t s);
hipError_t launch_mlp_init(uint64_t seed, const long *w0, const long *nw, const int *fan_in, long n_params,
                           float *P, hipStream_t s);
hipError_t launch_factor(DevState *st, hipStream_t s);
hipError_t launch_select_refit(DevState *st, const float *Z, const float *cost, const uint8_t *tier, int pop,
                               int32_t *elite_idx, int32_t *sel_info, float *stats, int stats_cap,
                               int advance_iter, hipStream_t s);
hipError_t launch_select_refit_batch(const InstDesc *insts, int n_inst, int stats_cap, hipStream_t s);
hipError_t launch_rollout_single(const InstDesc &d, float *trace, int trace_steps, hipStream_t s);
hipError_t launch_rollout_batch(const InstDesc *insts, int n_inst, const WorkItem *items, int n_items, int *queue,
                                int *pool, int grid, bool spec, hipStream_t s);
// Whether the scene's robot is the compiled-in model (every joint and body
// field equal) and the specialised rollout instance is switched on.
bool robot_spec_for(const cem_scene &sc);
hipError_t launch_scene_consts(DevState *st, hipStream_t s);
hipError_t launch_pack_dataset(const InstDesc &d, float cost_cap, float *X, float *Y, hipStream_t s);

}  // namespace cem

// Host-side context of one CE problem (the opaque cem_ctx of the ABI).
struct cem_ctx {
  cem_scene scene;
  int D = 0, pop = 0, n_elite = 0, cov_mode = 0;
  uint64_t seed = 0;
  uint32_t inst = 0;
  int device = 0;
  cem::DevState *st = nullptr;
  float *Z = nullptr, *cost = nullptr, *pose = nullptr, *stats = nullptr;
  uint8_t *tier = nullptr;
  hipStream_t own = nullptr;
  hipGraphExec_t iter_graph = nullptr;
  int pop_final = 0, pop_ramp = 0;  // n_env schedule (pop_final 0: none)
  int lanes = 1;                    // lanes per environment
  int32_t *perm = nullptr;          // robot scenes: the order of a launch's plans over the lanes (pop entries)
  uint64_t serial = 0;  // unique per context in the process (host addresses are reused after cem_free)
  std::string err;
};
