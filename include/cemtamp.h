/* cemtamp: cross-entropy optimisation of the controller parameters of a fixed
 * task-and-motion plan, rolled out in parallel through contact-rich rigid-body
 * dynamics on an AMD Instinct MI355X (gfx950).
 *
 * The method (Sec. III-B, Alg. 1 of "Cross-Entropy Optimization of Physically
 * Grounded Task and Motion Plans"): given a symbolic plan pi = (a_1..a_k) whose
 * actions carry continuous controller parameters Z_pi, repeat
 *   sample n_env parameter vectors Z ~ phi(theta)          -> cem_sample
 *   roll every plan out through the dynamics, scoring the
 *   per-step action costs, final cost and feasibility        -> rollout_batch
 *   refit theta to the top N_e feasible samples              -> cem_refit
 * and return the best sample and the final theta             -> plan_solve.
 * phi is a Gaussian N(mu, Sigma): independent normals (cov_mode 0, as in the
 * paper's experiments, Sec. IV-A "Algorithm setting") or a full covariance
 * (cov_mode 1).
 *
 * Conventions for every call:
 *  - Return value: CEM_OK (0) or a CEM_E_* code; nothing aborts or throws.
 *    cem_last_error(ctx) gives a text for the last failure on that context.
 *  - "_dev" pointers are device (HBM) pointers owned by the caller; the library
 *    never frees them.  "stream" is a hipStream_t passed as void* (NULL = the
 *    null stream).  Calls taking a stream are asynchronous on it; faults of the
 *    asynchronous work surface at the next synchronous call.
 *  - The context owns theta, its Cholesky factor, the per-instance scene draws,
 *    the elite scratch, the best-so-far record and the replay graph; all of it
 *    is allocated by cem_init, so the per-iteration calls never allocate.
 *  - One host thread at a time per context; separate contexts are independent.
 *    Work of one context that overlaps on several streams races on the
 *    context's device scratch (the elite scratch, and the order in which a
 *    robot scene's rollout hands plans to lanes): keep it on one stream.
 */
#ifndef CEMTAMP_H
#define CEMTAMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CEM_OK = 0,
  CEM_E_ARG = 1,      /* invalid argument (size, pointer, mode)            */
  CEM_E_SCENE = 2,    /* invalid scene description                          */
  CEM_E_ALLOC = 3,    /* device allocation failed                           */
  CEM_E_HIP = 4,      /* a HIP runtime call failed                          */
  CEM_E_NUMERIC = 5,  /* covariance not factorable: diagonal fallback used  */
  CEM_E_STATE = 6     /* call not valid in the context's current state      */
};

enum { CEM_SCENE_PUSH = 1, CEM_SCENE_PICKPLACE = 2, CEM_SCENE_MOVEPUSH = 3 };

#define CEM_MAX_STATIC 8
#define CEM_MAX_D 16
#define CEM_MAX_ANNULI 4
#define CEM_MAX_DR 64
#define CEM_STATS_COLS 8
#define CEM_TRACE_FREE 13
#define CEM_MAX_JOINTS 12
#define CEM_TRACE_ROBOT 35   /* object p q v w (13), robot q (11), robot qd (11) */

/* The physical scene and the plan's controllers (Problem 1: state space
 * X = Q x SE(3)^m, dynamics x_{t+1} = f(x_t, c_i, z_i), horizon T).
 * Units SI, z up, gravity along -z.  Copied by cem_init. */
typedef struct cem_scene {
  int32_t kind;                 /* CEM_SCENE_*                                     */
  int32_t substeps;             /* physics substeps per control step dt            */
  int32_t horizon;              /* control steps T                                 */
  float dt, gravity, k_contact, c_contact, eps_v;
  float mu_ground, mu_tool, mu_static, mu_ramp;   /* friction per contact class  */
  float obj_half[3], obj_mass, obj_pos0[3], obj_yaw0;  /* the free object (a box) */
  int32_t n_static;             /* static boxes: centre, half extents, yaw, pitch */
  float st_center[CEM_MAX_STATIC][3], st_half[CEM_MAX_STATIC][3];
  float st_yaw[CEM_MAX_STATIC], st_pitch[CEM_MAX_STATIC];
  int32_t st_ramp[CEM_MAX_STATIC];              /* 1: friction class mu_ramp      */
  float pusher_radius, pusher_standoff, pusher_height, pusher_vmax;
  int32_t pusher_steps;         /* control steps the pusher moves                  */
  float goal_rho_lo, goal_rho_hi, goal_phi_lo, goal_phi_hi;  /* seeded goal draw  */
  float goal_tol, time_weight;  /* success radius; weight of the time cost         */
  /* Articulated mobile manipulator (pick-place, move-push).  Fixed topology:
   * joints 0, 1, 2 move the base along world x, y and about z (bodies 0, 1
   * massless); 3..8 a serial arm; 9, 10 the two fingers, children of body 8.
   * Joint j moves body j relative to body j_parent[j]: its frame sits at
   * j_origin (parent body frame, no fixed rotation), rotating (type 0) about
   * or sliding (type 1) along axis 0..5 = +x,+y,+z,-x,-y,-z.  Body j: mass,
   * COM (body frame), half extents of a solid box about the COM (inertia, and
   * the collision box of the base and the fingers).  j_inom: nominal inertia
   * scaling the joint PD gains; q0: initial configuration. */
  int32_t n_joints;
  int32_t j_type[CEM_MAX_JOINTS], j_axis[CEM_MAX_JOINTS], j_parent[CEM_MAX_JOINTS];
  float j_origin[CEM_MAX_JOINTS][3], b_mass[CEM_MAX_JOINTS], b_com[CEM_MAX_JOINTS][3];
  float b_half[CEM_MAX_JOINTS][3], j_inom[CEM_MAX_JOINTS], q0[CEM_MAX_JOINTS];
  int32_t ee_body;              /* end-effector body and offset of the EE point   */
  float ee_offset[3];
  /* controllers: joint PD tau = inom (omega_c^2 e - 2 zeta omega_c qd),
   * |tau| <= inom * accel_max; DLS IK (ik_iters steps, damping ik_lambda);
   * base speed clamp [base_vmin, base_vmax], yaw rate base_wmax; success
   * tolerances; phase durations (s) stretched so no arm reference moves
   * faster than joint_speed_max; action timeouts (s); pre-grasp distance;
   * finger open / closed targets; goal table (static box index) and the
   * object speed below which it is at rest. */
  int32_t ik_iters;
  float omega_c, zeta, ik_lambda;
  float base_vmin, base_vmax, base_wmax, base_tol, yaw_tol, ee_tol;
  float t_approach, t_descend, t_close, t_lift, t_transfer, t_release;
  float timeout_move, timeout_pick, timeout_place;
  float pregrasp, finger_open, finger_closed, rest_speed;
  int32_t goal_static;
  float joint_speed_max, accel_max;
  /* move-push (Sec. IV-A, plan pi_m&p): the push action's speed clamp
   * [push_vmin, push_vmax] (m/s), longest push push_dmax (m) and timeout (s);
   * the friction coefficient of every contact of the object, drawn per
   * instance as U[obj_mu_lo, obj_mu_hi] on the scene stream when
   * obj_mu_hi > 0 (otherwise the per-class coefficients apply); and, when
   * goal_static < 0, the goal region psi_g: the object's centre inside the
   * axis-aligned box goal_box_center +- goal_box_half, at rest. */
  float push_vmin, push_vmax, push_dmax, timeout_push;
  float obj_mu_lo, obj_mu_hi;
  float goal_box_center[3], goal_box_half[3];
  /* Early stop of a robot rollout (0: off, every rollout runs T steps).  When
   * > 0, a rollout ends after the control step at which, for settle_steps
   * consecutive steps, every action has ended and the object has moved slower
   * than rest_speed; psi_g is then read at that step.  The cost is final once
   * the last action has ended, so only psi_g of an object that would start
   * moving again afterwards can differ from the full-horizon result.  The
   * push scene ignores it. */
  int32_t settle_steps;
  /* Stop of a robot rollout on a failed action (0: off).  When 1, a rollout
   * ends at the control step at which an action ends without success (its
   * timeout): the plan can no longer be feasible, since Problem 2 needs every
   * action to succeed, and Alg. 1 evaluates only the costs of successful
   * plans.  The stopped plan reports tier 2, the cost of the steps before the
   * stop and the object's pose there; plans whose actions all succeed run as
   * without the option.  The push scene ignores it. */
  int32_t fail_stop;
  /* Domain randomisation (Sec. IV-C: plans made robust to bounded uncertainty
   * in friction or mass).  dr_scenarios R in {0, 1}: off.  R in {2, 4, ..., 64}
   * (robot scenes): every parameter row is rolled out under R scenarios.
   * Scenario r draws the object's friction U[dr_mu_lo, dr_mu_hi] (when
   * dr_mu_hi > 0; else the instance's value) and its mass U[dr_mass_lo,
   * dr_mass_hi] (when dr_mass_hi > 0; else obj_mass) from the scene stream
   * (block 1, sample r, iteration 0): the same R scenarios for every row and
   * iteration of an instance.  A row's tier is the worst over its scenarios,
   * its cost the mean (dr_reduce 0) or the maximum (1), its pose scenario 0's.
   * rollout_trace rejects such scenes. */
  int32_t dr_scenarios, dr_reduce;
  float dr_mu_lo, dr_mu_hi, dr_mass_lo, dr_mass_hi;
} cem_scene;

/* Initial distribution phi(theta^0) as a region (Sec. III-B: iteration 0
 * draws uniformly inside each parameter's region h(z) <= 0; Sec. IV-A gives
 * rings around the tables for the base positions and boxes for the others).
 * Every dimension d draws z_d ~ U[lo_d, hi_d] except the pairs (d, d+1) named
 * by ann_dim, which draw a point uniform by area in the ring
 * ann_radius[k][0] <= |(z_d, z_d+1) - ann_center[k]| <= ann_radius[k][1].
 * The uniforms are the Philox words of the CE stream at iteration 0 (word
 * d mod 4 of block d / 4 of the sample), so the draw is bit-reproducible:
 *   box:  z_d = fma(hi_d - lo_d, u_d, lo_d)
 *   ring: r = sqrt(fma(r1*r1 - r0*r0, u_d, r0*r0)), (s, c) = sincos(2 pi u_d+1),
 *         z_d = fma(r, c, cx), z_d+1 = fma(r, s, cy)
 * with every operation in FP32, correctly rounded. */
typedef struct cem_init_region {
  float lo[CEM_MAX_D], hi[CEM_MAX_D];
  int32_t n_annuli;
  int32_t ann_dim[CEM_MAX_ANNULI];
  float ann_center[CEM_MAX_ANNULI][2];
  float ann_radius[CEM_MAX_ANNULI][2];
} cem_init_region;

/* One CE problem (Alg. 1 inputs).  mu0 has D entries, cov0 D x D row-major
 * (cov_mode 0 reads its diagonal only).  D is fixed by the scene kind
 * (push 3, pick-place 16, move-push 12).  Pointers are host pointers, copied. */
typedef struct cem_problem {
  const cem_scene *scene;
  int32_t pop;                  /* n_env: samples per iteration, 1..65536          */
  int32_t n_elite;              /* N_e, 1..min(pop, 256)                           */
  int32_t cov_mode;             /* 0 diagonal, 1 full                              */
  /* Lanes of a wave that share one environment of a robot scene (0 or 1: one
   * lane each; 2, 4, 8 or 16: the lanes split the environment's contact tests
   * and sum their forces).  An implementation choice, not part of Alg. 1: it
   * fills more of the device when pop is small, and moves the FP32 rounding
   * of the contact sums.  Push scenes and batches take 0 or 1 only;
   * lanes_per_env * dr_scenarios <= 64.  Else CEM_E_ARG. */
  int32_t lanes_per_env;
  const double *mu0, *cov0;
  uint64_t seed;                /* Philox key                                      */
  uint32_t instance;            /* Philox counter word 3 (task instance id)        */
  /* n_env(j), the samples of iteration j (an input of Alg. 1; Sec. IV-A
   * lowers it linearly over the first iterations, then holds it).  0 keeps
   * n_env = pop; otherwise n_elite <= pop_final <= pop, pop_ramp_iters >= 1 and
   *   n_env(j) = pop - floor((pop - pop_final) * min(j, pop_ramp_iters) / pop_ramp_iters).
   * plan_solve follows it (launching each iteration directly rather than
   * replaying a captured graph); batches reject it. */
  int32_t pop_final, pop_ramp_iters;
  /* nullable: iteration 0 draws from N(mu0, cov0) like every other */
  const cem_init_region *init_region;
} cem_problem;

/* Output of plan_solve (host memory, filled on return). */
typedef struct cem_result {
  float best_z[CEM_MAX_D];      /* best sample over all iterations                 */
  float best_cost;
  int32_t best_tier;            /* 0 feasible, 1 actions ok / goal missed, 2 other, 3 diverged */
  int32_t iters_done;
  int32_t dim;
  double mu[CEM_MAX_D];         /* final theta                                     */
  double cov[CEM_MAX_D * CEM_MAX_D];
} cem_result;

typedef struct cem_ctx cem_ctx;

/* Validates the problem, allocates the context's device state on the current
 * device, draws the per-instance scene quantities (the push goal) on the GPU
 * and factors cov0.  Synchronous.  *out is NULL on failure. */
int cem_init(const cem_problem *p, cem_ctx **out);
void cem_free(cem_ctx *c);

int cem_dim(const cem_ctx *c);
/* Measurement aid, not part of the method: the device's FP32 vector FMA rate
 * (FLOP/s, an FMA counting 2) on the current device, from a kernel of
 * independent unpacked FMA chains at eight waves per SIMD, best of three timed
 * launches on `stream` (NULL: the null stream).  The ceiling of unpacked FP32
 * arithmetic, beside the published packed peak.  Synchronous; allocates and
 * frees an 8 MiB output buffer. */
int cem_valu_fma_rate(double *flops_per_s, void *stream);
/* sizeof of the ABI structs (0 cem_scene, 1 cem_problem, 2 cem_result,
 * 3 cem_init_region; else 0),
 * for bindings to check their layouts. */
int cem_sizeof(int which);
/* The rollout kernel has an instance compiled for one robot: the mobile
 * manipulator of the robot scenes (joint types and axes, joint origins, body
 * masses, centres of mass and half extents; robot_model.hpp), with the
 * articulated-body passes unrolled and the products with the robot's
 * structural zeros left out (Problem 1's dynamics, Featherstone's algorithm;
 * the same arithmetic otherwise, so its results differ from the generic
 * instance's only by rounding).  A launch takes it when its scene's robot
 * equals the model field for field, the generic instance otherwise.
 * enable = 0 makes every launch prepared after the call (a context's
 * rollout, a batch's captured iteration) take the generic instance; nonzero
 * restores the default.  Process-wide; no error. */
void cem_set_robot_specialization(int32_t enable);
const char *cem_strerror(int code);
const char *cem_last_error(const cem_ctx *c);

/* Alg. 1, sampling step: Z_dev (pop x D row-major, FP32) = mu + L eps with
 * eps ~ N(0, I) from Philox-4x32-10 counters (tag 0, sample i, iteration
 * iter, instance) and Box-Muller; accumulated in FP64, rounded once.  At
 * iter 0 of a problem with an init_region, the region's uniform draw instead.
 * Row i depends only on (seed, instance, iter, i), so the first n rows are
 * the rows of a population of n. */
int cem_sample(cem_ctx *c, int32_t iter, float *Z_dev, void *stream);

/* Alg. 1, evaluation step: roll every row of Z_dev (pop x D) out for the
 * horizon and write cost_dev[pop] (plan cost, Problem 2 objective),
 * tier_dev[pop] (0 feasible, 1 all actions succeeded but goal missed,
 * 2 other, 3 diverged) and, if pose_dev is non-NULL, the final object pose
 * pose_dev[pop][7] = (p, q).  pop may differ from the problem's pop.  For a
 * robot scene at one lane per environment and pop up to the problem's, the
 * launch first orders the rows by their first move's duration in the
 * context's scratch, so that a wave's lanes run similar plans; each row's
 * outcome is the same in any order. */
int rollout_batch(cem_ctx *c, const float *Z_dev, int32_t pop, float *cost_dev, uint8_t *tier_dev,
                  float *pose_dev, void *stream);

/* Same dynamics, recording the state after each of the first n_steps control
 * steps: trace_dev[pop][n_steps][W] with W = CEM_TRACE_FREE (13: the free
 * object's p q v w) for the push scene and W = CEM_TRACE_ROBOT (35: object
 * p q v w, then robot q[11] and qd[11]) for the robot scenes.  Steps after a
 * rollout stopped (early stop, divergence) are left unwritten.  Scenes with
 * domain-randomisation scenarios are rejected (CEM_E_ARG). */
int rollout_trace(cem_ctx *c, const float *Z_dev, int32_t pop, int32_t n_steps, float *trace_dev, void *stream);

/* Alg. 1, update step: order the samples by (tier, cost, index), NaN cost as
 * tier 3; take the top N_e feasible, or all feasible if fewer, or - with
 * none feasible - the best whose actions all succeeded (Sec. III-B); refit
 * mu and Sigma (maximum likelihood, FP64) and factor Sigma in FP64.  A
 * single selected sample gives mu = that sample, Sigma = diag((0.1 sigma0)^2);
 * nothing selectable leaves theta unchanged.  Optional outputs:
 * elite_idx_dev[n_elite] (-1 padded), sel_info_dev[6] = (n_e, mode,
 * n_tier0..3).  Also updates the best-so-far record. */
int cem_refit(cem_ctx *c, const float *Z_dev, const float *cost_dev, const uint8_t *tier_dev, int32_t pop,
              int32_t *elite_idx_dev, int32_t *sel_info_dev, void *stream);

/* Alg. 1 end to end: iters iterations of sample -> rollout -> refit on the
 * context's own buffers, replayed from one captured HIP graph per iteration
 * (launched directly, n_env(j) rows each, when the problem has an n_env
 * schedule).  Continues from the context's current theta and iteration
 * counter.
 * Synchronous.  stats_host (nullable) gets iters rows of CEM_STATS_COLS floats:
 * best cost of the iteration, n_tier0..3, n_e, mode, best cost so far. */
int plan_solve(cem_ctx *c, int32_t iters, cem_result *res, float *stats_host, void *stream);

/* theta access (host arrays mu[D], cov[D*D]); set refactors.  Synchronous. */
int cem_get_theta(cem_ctx *c, double *mu, double *cov);
int cem_set_theta(cem_ctx *c, const double *mu, const double *cov);
/* Cholesky factor currently used by cem_sample (host L[D*D]). Synchronous. */
int cem_get_factor(cem_ctx *c, double *L);
/* n_env(iter) of the context's schedule (pop when it has none); 0 for a
 * null context or iter < 0. */
int cem_pop_at(const cem_ctx *c, int32_t iter);
/* Per-instance scene draws (Philox scene stream, counter word 3 = instance),
 * host draws[3] = (goal x, goal y, object friction coefficient or 0 when the
 * scene does not draw one). Synchronous. */
int cem_get_instance(cem_ctx *c, double *draws);
/* The instance's domain-randomisation scenarios (scene dr_*): host
 * mu[CEM_MAX_DR], mass[CEM_MAX_DR] get each scenario's object friction and
 * mass as drawn (0 where the scene draws none).  Synchronous. */
int cem_get_scenarios(cem_ctx *c, float *mu, float *mass);
/* Control steps simulated by this context's rollouts since cem_init, summed
 * over environments: T per rollout, fewer for one that stopped early or
 * diverged.  Batched runs count into each instance's context.  Waits for all
 * work on the device first.  Synchronous. */
int cem_env_steps(cem_ctx *c, uint64_t *steps);
/* Outcomes of the rollouts into the context's own buffers (the iterations of
 * plan_solve and of batched steps write them; the last iteration's remain):
 * host cost[n], tier[n] and, if pose is non-NULL, pose[n][7] of rows 0..n-1,
 * n <= pop.  Waits for all work on the device first.  Synchronous. */
int cem_get_outcomes(cem_ctx *c, int32_t n, float *cost, uint8_t *tier, float *pose);
/* Reset the best-so-far record and the iteration counter. Synchronous. */
int cem_reset(cem_ctx *c);

/* ---- Many task instances in one launch ------------------------------------
 * n independent CE problems (each its own scene kind, population, horizon,
 * seed and instance id) iterated together: every CE iteration is one captured
 * graph of a batched sampling launch, ONE persistent rollout launch whose
 * workgroups pull (instance, 64-environment chunk) items, most expensive
 * first, from an atomic queue, and one refit workgroup per instance.
 * Instances stop at their own iteration cap iters[b].  Results per instance
 * are the same bits as running that instance alone with plan_solve. */
typedef struct cem_batch cem_batch;
/* problems[n], iters[n] (host, copied).  Synchronous.  *out NULL on failure. */
int cem_batch_init(const cem_problem *problems, const int32_t *iters, int32_t n, cem_batch **out);
void cem_batch_free(cem_batch *b);
int cem_batch_size(const cem_batch *b);
const char *cem_batch_last_error(const cem_batch *b);
/* The context of instance i (owned by the batch: theta, factor, instance draws). */
cem_ctx *cem_batch_instance(cem_batch *b, int32_t i);
/* Times one rollout pass for each persistent grid (1, 2, 4 workgroups per CU)
 * and work-item size (64 or 32 environments) and keeps the fastest.  The
 * passes roll out each instance's samples of its current iteration (drawn
 * first; the same rows its next step draws).  config_out (nullable, 3 ints):
 * grid, environments per item, microseconds of that pass.  Leaves the CE
 * state and the step counters (cem_env_steps) as they were.  Synchronous. */
int cem_batch_autotune(cem_batch *b, int32_t *config_out);
/* One CE iteration of every instance under its cap, asynchronous on stream. */
int cem_batch_step(cem_batch *b, void *stream);
/* iters iterations, then results[n] (host) for every instance.  Synchronous. */
int cem_batch_solve(cem_batch *b, int32_t iters, cem_result *results, void *stream);
/* Runs iters iterations and after each appends every instance that ran its
 * (parameter row, outcome) pairs to X_dev (rows x D, one D for all instances)
 * and Y_dev (rows x 8: cost, final object position, orientation w >= 0; a
 * diverged rollout gets the horizon cost and the start pose).  *n_out = rows
 * written (at most capacity, else CEM_E_ARG).  Synchronous. */
int cem_batch_record(cem_batch *b, int32_t iters, float *X_dev, float *Y_dev, int64_t capacity, int64_t *n_out,
                     void *stream);

/* ---- Learned surrogate for screening ----------------------------------------
 * Not in the paper (whose limitation is the cost of full rollouts): a
 * 16 -> 256 -> 256 -> 256 -> 8 perceptron with GELU (tanh form) predicting
 * (cost, final object pose) from the 16 pick-and-place parameters, trained on
 * simulated rollouts.  Products run as BF16 MFMA with FP32 accumulation;
 * master weights and Adam moments are FP32.  Inputs and targets are
 * standardised per column (cem_mlp_fit_norm / set_norm).  The flat parameter
 * vector is W1 (256x16, row = output unit), b1, W2, b2, W3, b3, W4 (8x256), b4. */
typedef struct cem_mlp cem_mlp;
/* He-normal weights from Philox stream 2, zero biases, identity
 * standardisation; work buffers for up to max_rows rows.  Synchronous. */
int cem_mlp_init(uint64_t seed, int32_t max_rows, cem_mlp **out);
void cem_mlp_free(cem_mlp *m);
int cem_mlp_n_params(void);
const char *cem_mlp_last_error(const cem_mlp *m);
/* host copies of the FP32 master parameters (cem_mlp_n_params floats) */
int cem_mlp_get_params(cem_mlp *m, float *host);
int cem_mlp_set_params(cem_mlp *m, const float *host);
/* standardisation, 48 host floats: x_mean[16] x_std[16] y_mean[8] y_std[8] */
int cem_mlp_get_norm(cem_mlp *m, float *host48);
int cem_mlp_set_norm(cem_mlp *m, const float *host48);
/* column means / standard deviations of a dataset (n rows), on the GPU */
int cem_mlp_fit_norm(cem_mlp *m, const float *X_dev, const float *Y_dev, int64_t n, void *stream);
/* predictions Y_dev (n x 8, de-standardised) of raw parameter rows X_dev (n x 16) */
int cem_mlp_forward(cem_mlp *m, const float *X_dev, int32_t n, float *Y_dev, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cem_mlp_forward with its work buffers - standardised inputs, two hidden
 * layers, standardised outputs, 8.5 MiB in all - in a fixed array that the
 * library holds on each device it runs on until the process ends, instead
 * of the network's own buffers.  Same kernels, same results as
 * cem_mlp_forward; calls no allocating routine.  X_dev (n x 16) and Y_dev
 * (n x 8) as in cem_mlp_forward; n <= CEM_MLP_STATIC_ROWS, else CEM_E_ARG.
 * Asynchronous on stream.  Every call on one device shares that device's
 * array: calls ordered on one stream are safe, calls that overlap on one
 * device (other streams, other host threads) race. */
#define CEM_MLP_STATIC_ROWS 8192
int cem_mlp_forward_static(cem_mlp *m, const float *X_dev, int32_t n, float *Y_dev, void *stream);
/* mean squared error over n rows and 8 standardised outputs, and its gradient
 * w.r.t. the parameters (grad_dev, nullable) */
int cem_mlp_loss_grad(cem_mlp *m, const float *X_dev, const float *Y_dev, int32_t n, float *grad_dev, float *loss_dev,
                      void *stream);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the rows given */
int cem_mlp_train_step(cem_mlp *m, const float *X_dev, const float *Y_dev, int32_t n, float lr, float *loss_dev,
                       void *stream);
/* epochs over n rows in shuffled minibatches of `batch` (an affine
 * permutation per epoch, from seed); mean minibatch loss per epoch to
 * epoch_loss_host (nullable).  Runs on the null stream, after the caller's
 * earlier work there.  Synchronous. */
int cem_mlp_train(cem_mlp *m, const float *X_dev, const float *Y_dev, int64_t n, int32_t batch, int32_t epochs,
                  float lr, uint64_t seed, float *epoch_loss_host);
/* Screening: sample the context's population (iteration iter), predict every
 * candidate and keep the n_sim smallest (goal predicted to fail, predicted
 * cost, index) keys - the goal test is the plan's psi_g on the predicted
 * pose - written in index order: Zsim_dev (n_sim x 16), pred_dev (n_sim x 8,
 * nullable). */
int cem_screen(cem_ctx *c, cem_mlp *m, int32_t iter, int32_t n_sim, float *Zsim_dev, float *pred_dev, void *stream);
/* Surrogate-screened CE: each iteration samples the context's population,
 * screens it down to n_sim candidates, simulates those in full and refits
 * from the simulated costs (the surrogate never decides a cost that enters
 * the refit).  One captured graph per iteration.  surrogate_err_host
 * (nullable, iters floats): mean |predicted - simulated| cost of each
 * iteration's simulated candidates.  Synchronous. */
int plan_solve_screened(cem_ctx *c, cem_mlp *m, int32_t iters, int32_t n_sim, cem_result *res, float *stats_host,
                        float *surrogate_err_host, void *stream);

#ifdef __cplusplus
}
#endif
#endif
