// The rollout launch (evaluation step of Alg. 1) for one or many task instances.
//
// Work is cut into items of up to 64 environments of one instance (one wave,
// one environment per lane; a single robot instance may give each environment
// 2, 4, 8 or 16 adjacent lanes, which split its contact tests).  A single instance runs one workgroup per item.
// A batch of instances (independent CE problems with their own scene kind,
// population and horizon) runs as one persistent launch: each workgroup pulls
// the next item from an atomic queue until the list is exhausted, so the items
// of long-horizon instances, put first in the list, overlap with the many short
// ones and no workgroup idles while work remains.  In a batch, the plans of a
// robot instance (without domain randomisation) come from a per-instance pool
// instead of the item's fixed range: an item's wave takes the next 64
// unstarted plans of its instance, and each lane whose rollout ends early
// (settled, failed, diverged) takes the instance's next unstarted plan, so the
// lanes stay busy while the instance has plans left.  Both modes execute the
// same per-environment code in the same kernel, so an instance's results do
// not depend on whether it ran alone or in a batch.
#include <atomic>

#include "internal.hpp"
#include "robot_env.hpp"
#include "push_env.hpp"

namespace cem {
namespace {

template <bool TRACE, bool MULTI, bool SPEC>
__global__ void __launch_bounds__(64) rollout_items_kernel(InstDesc single, const InstDesc *__restrict__ insts,
                                                           const WorkItem *__restrict__ items, int n_items,
                                                           int *__restrict__ queue, int *__restrict__ pool,
                                                           int check_iter, float *__restrict__ trace,
                                                           int trace_steps) {
  __shared__ float lds[R_ROWS * PP_LANES];
  const int lane = threadIdx.x;
  int it = blockIdx.x;
  for (;;) {
    if (queue) {
      int v = 0;
      if (lane == 0) v = atomicAdd(queue, 1);
      it = __builtin_amdgcn_readfirstlane(v);  // lane 0's ticket, provably wave-uniform
    }
    if (it >= n_items) break;  // every wave of the grid reaches this once the queue is drained
    InstDesc d;
    int env0, n, inst = 0;
    if (insts) {
      const CWorkItem &w = ((CWorkItem *)items)[it];
      inst = w.inst;
      const CInstDesc &di = ((CInstDesc *)insts)[w.inst];
      d.st = di.st;
      d.Z = di.Z;
      d.cost = di.cost;
      d.tier = di.tier;
      d.pose = di.pose;
      d.kind = di.kind;
      d.pop = di.pop;
      d.iters = di.iters;
      d.scen = di.scen;
      d.lanes = 1;
      d.perm = di.perm;
      env0 = w.env0;
      n = w.n;
    } else {
      d = single;
      env0 = it * 64;
      n = min(64, d.pop * d.scen * d.lanes - env0);
    }
    CDevState *st = (CDevState *)d.st;
    const bool active = !(check_iter && st->iter >= d.iters);  // wave-uniform
    const bool robot = d.kind != CEM_SCENE_PUSH;                // wave-uniform
    const int R = d.scen;  // scenarios per row: a power of two <= 64, aligned to the item (wave-uniform)
    // lanes per environment: 1, 2, 4, 8 or 16, with R * G <= 64 (wave-uniform; 1 unless MULTI)
    const int G = MULTI ? d.lanes : 1;
    int steps = 0;
    EnvOut o{0.0f, 0, 0, {0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f}};
    // lane layout: ((row * R) + scenario) * G + g, g the lane's place in its environment's group
    const int lg = G == 16 ? 4 : G == 8 ? 3 : G == 4 ? 2 : G == 2 ? 1 : 0;
    const long vl = env0 + lane, env = vl >> lg;
    // the item's environments hold the plans in the order the launch set
    const long row = d.perm && env / R < d.pop ? d.perm[env / R] : env / R;
    const int g = (int)(vl & (G - 1));
    const bool pooled = pool && robot && R == 1;  // wave-uniform
    if (active && robot && (pooled || lane < n)) {
      // One inlined copy of the environment code serves both modes, so an
      // instance's outcomes are bit for bit the same whether it ran alone or
      // pooled in a batch.  Pooled: the item's plans are the next 64 of the
      // instance's pool; then, lane by lane as rollouts end, one more each
      // (one atomic add per wave).  Alone: this lane's one rollout (its
      // group's, with G lanes per environment) with its scenario's draws.
      const int pop = d.pop;
      long row0 = row;
      bool live0 = true;
      float mu = st->obj_mu, m = st->scene.obj_mass;
      // the pool's k-th plan: plan perm[k] where the launch ordered the plans
      const int32_t *perm = d.perm;
      if (pooled) {
        int e0 = 0;
        if (lane == 0) e0 = atomicAdd(&pool[inst], 64);
        e0 = __builtin_amdgcn_readfirstlane(e0);
        row0 = (long)e0 + lane;
        live0 = row0 < pop;
        if (live0 && perm) row0 = perm[row0];
      } else if (R > 1) {
        const int r = (int)(env & (R - 1));
        if (st->scene.dr_mu_hi > 0.0f) mu = st->dr_mu[r];
        if (st->scene.dr_mass_hi > 0.0f) m = st->dr_mass[r];
      }
      auto claim = [&](bool need, long &r, bool &live) {
        if (!pooled) {
          if (need) live = false;
          return;
        }
        const unsigned long long want = __ballot(need);
        if (want == 0ull) return;
        const int leader = __builtin_ctzll(want);
        int base = 0;
        if (lane == leader) base = atomicAdd(&pool[inst], __popcll(want));
        base = __shfl(base, leader);
        if (need) {
          r = (long)base + __popcll(want & ((1ull << lane) - 1ull));
          live = r < pop;
          if (live && perm) r = perm[r];
        }
      };
      auto finish = [&](const EnvOut &e, long r) {
        if (!pooled) {
          o = e;
          return;
        }
        if (d.cost) d.cost[r] = e.cost;
        if (d.tier) d.tier[r] = (uint8_t)e.tier;
        if (d.pose)
#pragma unroll
          for (int i = 0; i < 7; ++i) d.pose[r * 7 + i] = e.pose[i];
      };
      const int s = robot_env<TRACE, MULTI, SPEC>(st, d.Z, row0, live0, mu, m, lds, lane, pooled ? 0 : g,
                                                  pooled ? 1 : G, pooled ? nullptr : trace, pooled ? 0 : trace_steps,
                                                  claim, finish);
      steps = (pooled || g == 0) ? s : 0;
    } else if (active && !robot && lane < n) {
      push_env<TRACE>(st->scene, st, d.Z, env, d.cost, d.tier, d.pose, trace, trace_steps);
      steps = st->scene.horizon;
    }
    if (active && robot && !pooled) {
      // a row's scenarios sit in R adjacent lanes: the worst tier, and the
      // mean or the largest cost, by a fixed butterfly over the group
      const bool use_max = st->scene.dr_reduce != 0;
      for (int m = G; m < R * G; m <<= 1) {
        const float oc = __shfl_xor(o.cost, m);
        const int ot = __shfl_xor(o.tier, m);
        o.cost = use_max ? fmaxf(o.cost, oc) : o.cost + oc;
        o.tier = max(o.tier, ot);
      }
      if (R > 1 && !use_max) o.cost = o.cost * (1.0f / (float)R);
      if (lane < n && (env & (R - 1)) == 0 && g == 0) {
        if (d.cost) d.cost[row] = o.cost;
        if (d.tier) d.tier[row] = (uint8_t)o.tier;
        if (d.pose)
#pragma unroll
          for (int i = 0; i < 7; ++i) d.pose[row * 7 + i] = o.pose[i];
      }
    }
    if (active) {
      // the item's simulated control steps, one atomic add per wave
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) steps += __shfl_xor(steps, m);
      if (lane == 0) atomicAdd(&d.st->env_steps, (unsigned long long)steps);
    }
    if (!queue) break;
  }
}

using RolloutKernel = void (*)(InstDesc, const InstDesc *, const WorkItem *, int, int *, int *, int, float *, int);

// Scene constants used every substep, derived once per context: the static
// boxes' rotations Rz(yaw) Ry(pitch) and each body's spatial inertia about its
// frame origin (a solid box of the body's mass about its centre of mass).
__global__ void scene_consts_kernel(DevState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  CScene &sc = *(CScene *)&st->scene;
  SceneConsts &k = st->sk;
  for (int b = 0; b < CEM_MAX_STATIC; ++b) {
    const M3f R = static_rot(sc, b);
    const float m[9] = {R.r0.x, R.r0.y, R.r0.z, R.r1.x, R.r1.y, R.r1.z, R.r2.x, R.r2.y, R.r2.z};
    for (int i = 0; i < 9; ++i) k.st_R[b][i] = m[i];
    k.st_axis[b] = m[0] == 1.0f && m[4] == 1.0f && m[8] == 1.0f && m[1] == 0.0f && m[2] == 0.0f && m[3] == 0.0f &&
                   m[5] == 0.0f && m[6] == 0.0f && m[7] == 0.0f;
  }
  for (int j = 0; j < CEM_MAX_JOINTS; ++j) {
    const Sym6 I = body_inertia(sc, j);
    for (int i = 0; i < 6; ++i) {
      k.I_body[j][i] = I.A[i];
      k.I_body[j][15 + i] = I.C[i];
    }
    for (int i = 0; i < 9; ++i) k.I_body[j][6 + i] = I.B[i];
  }
}

// The order in which a launch hands a robot instance's plans to its lanes (one
// lane per environment): by the duration of the plan's first action (a base
// move from the start pose, as the controller times it), in 64 bins of 0.1 s,
// so that the lanes of a wave reach their next actions at similar steps and
// their contact passes coincide more often.  A plan's rollout does not depend
// on the lane or the wave that runs it, so every order gives the same
// outcomes; within a bin the order is whatever the atomics give.  One
// workgroup per instance writes d.perm[0 .. pop).
__device__ void order_plans(const InstDesc &d) {
  constexpr int NB = 64;
  constexpr float BIN = 0.1f;
  __shared__ int hist[NB];
  const cem_scene &sc = d.st->scene;
  const float x0 = sc.q0[0], y0 = sc.q0[1], p0 = sc.q0[2];
  const float vlo = sc.base_vmin, vhi = sc.base_vmax, wmax = sc.base_wmax;
  auto bin_of = [&](int i) {
    const float *z = d.Z + (long)i * d.D;
    const float dx = z[0] - x0, dy = z[1] - y0;
    const float dpsi = remainderf(z[2] - p0, 6.283185307179586f);
    const float t = fmaxf(sqrtf(dx * dx + dy * dy) / fmaxf(vlo, fminf(vhi, z[3])), fabsf(dpsi) / wmax);
    return t >= 0.0f && t < NB * BIN ? (int)(t * (1.0f / BIN)) : NB - 1;  // NaN and long moves last
  };
  for (int k = threadIdx.x; k < NB; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < d.pop; i += blockDim.x) atomicAdd(&hist[bin_of(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < NB; ++k) {
      const int c = hist[k];
      hist[k] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d.pop; i += blockDim.x) d.perm[atomicAdd(&hist[bin_of(i)], 1)] = i;
}
// A batch's instances, one workgroup each; and one instance.
__global__ void plan_order_kernel(const InstDesc *__restrict__ insts) {
  if (insts[blockIdx.x].perm) order_plans(insts[blockIdx.x]);
}
__global__ void plan_order_single_kernel(InstDesc d) { order_plans(d); }

// Clears the work queue's ticket and the instances' plan pools before a
// batched launch (a kernel rather than a memset, so the clearing can sit in a
// captured graph).
__global__ void reset_counters_kernel(int *q, int *pool, int n_pool) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *q = 0;
  if (pool && i < n_pool) pool[i] = 0;
}

// Training pairs of one instance: X row = its parameter row, Y row = (cost,
// final object position, orientation with w >= 0).  A diverged rollout (non
// finite cost or pose) is recorded with cost_cap and the object's start pose.
__global__ void pack_dataset_kernel(const float *__restrict__ Z, const float *__restrict__ cost,
                                    const float *__restrict__ pose, int pop, int D, float cost_cap,
                                    const DevState *__restrict__ st, float *__restrict__ X, float *__restrict__ Y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= pop) return;
  for (int d = 0; d < D; ++d) X[(long)r * D + d] = Z[(long)r * D + d];
  float p[7];
  bool fin = isfinite(cost[r]);
  for (int j = 0; j < 7; ++j) {
    p[j] = pose[(long)r * 7 + j];
    fin = fin && isfinite(p[j]);
  }
  const float s = p[3] < 0.0f ? -1.0f : 1.0f;
  float *y = Y + (long)r * 8;
  if (fin) {
    y[0] = cost[r];
    for (int j = 0; j < 3; ++j) y[1 + j] = p[j];
    for (int j = 3; j < 7; ++j) y[1 + j] = s * p[j];
  } else {
    y[0] = cost_cap;
    y[1] = st->scene.obj_pos0[0];
    y[2] = st->scene.obj_pos0[1];
    y[3] = st->scene.obj_pos0[2];
    y[4] = 1.0f;
    y[5] = 0.0f;
    y[6] = 0.0f;
    y[7] = 0.0f;
  }
}

}  // namespace

// Library-wide switch of the rollout instance specialised to the robot model
// (on unless cem_set_robot_specialization turned it off).
std::atomic<int> g_robot_spec{1};

bool robot_spec_for(const cem_scene &sc) {
  if (!g_robot_spec.load() || (sc.kind != CEM_SCENE_PICKPLACE && sc.kind != CEM_SCENE_MOVEPUSH)) return false;
  if (sc.n_joints != rm::N) return false;
  for (int j = 0; j < rm::N; ++j) {
    if (sc.j_type[j] != rm::TYPE[j] || sc.j_axis[j] != rm::AXIS[j] || sc.b_mass[j] != rm::MASS[j]) return false;
    for (int c = 0; c < 3; ++c)
      if (sc.j_origin[j][c] != rm::ORIGIN[j][c] || sc.b_com[j][c] != rm::COM[j][c] || sc.b_half[j][c] != rm::HALF[j][c])
        return false;
  }
  return true;
}

hipError_t launch_rollout_single(const InstDesc &d, float *trace, int trace_steps, hipStream_t s) {
  if (d.scen < 1 || d.scen > 64 || (d.scen & (d.scen - 1))) return hipErrorInvalidValue;
  if ((d.lanes != 1 && d.lanes != 2 && d.lanes != 4 && d.lanes != 8 && d.lanes != 16) || d.scen * d.lanes > 64 ||
      (d.lanes > 1 && d.kind == CEM_SCENE_PUSH))
    return hipErrorInvalidValue;
  const int n_items = (d.pop * d.scen * d.lanes + 63) / 64;
  if (n_items == 0) return hipSuccess;
  const bool multi = d.lanes > 1;
  if (d.perm) hipLaunchKernelGGL(plan_order_single_kernel, dim3(1), dim3(256), 0, s, d);
  const RolloutKernel k =
      d.spec ? (trace ? (multi ? rollout_items_kernel<true, true, true> : rollout_items_kernel<true, false, true>)
                      : (multi ? rollout_items_kernel<false, true, true> : rollout_items_kernel<false, false, true>))
             : (trace ? (multi ? rollout_items_kernel<true, true, false> : rollout_items_kernel<true, false, false>)
                      : (multi ? rollout_items_kernel<false, true, false> : rollout_items_kernel<false, false, false>));
  hipLaunchKernelGGL(k, dim3(n_items), dim3(64), 0, s, d, nullptr, nullptr, n_items, nullptr, nullptr, 0, trace,
                     trace ? trace_steps : 0);
  return hipGetLastError();
}

hipError_t launch_scene_consts(DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(scene_consts_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_pack_dataset(const InstDesc &d, float cost_cap, float *X, float *Y, hipStream_t s) {
  if (d.pop <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_dataset_kernel, dim3((d.pop + 255) / 256), dim3(256), 0, s, d.Z, d.cost, d.pose, d.pop, d.D,
                     cost_cap, d.st, X, Y);
  return hipGetLastError();
}

hipError_t launch_rollout_batch(const InstDesc *insts, int n_inst, const WorkItem *items, int n_items, int *queue,
                                int *pool, int grid, bool spec, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3((n_inst + 255) / 256 + 1), dim3(256), 0, s, queue, pool, n_inst);
  hipLaunchKernelGGL(plan_order_kernel, dim3(n_inst), dim3(256), 0, s, insts);
  InstDesc none{};
  const RolloutKernel k = spec ? rollout_items_kernel<false, false, true> : rollout_items_kernel<false, false, false>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64), 0, s, none, insts, items, n_items, queue, pool, 1, nullptr, 0);
  return hipGetLastError();
}

}  // namespace cem

void cem_set_robot_specialization(int32_t enable) { cem::g_robot_spec.store(enable ? 1 : 0); }
