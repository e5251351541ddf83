// Update step of CE optimisation (Alg. 1) and the FP64 factorisation of theta.
//
// Elites (Sec. III-B): samples ordered by (tier, cost, index); the top N_e
// feasible (tier 0), or all feasible when fewer, or - none feasible - the best
// whose actions all succeeded (tier 1).  New theta = maximum-likelihood
// Gaussian of the elites (the KL-minimising CE update); one selected sample ->
// that sample with artificial noise diag((0.1 sigma0)^2); none -> unchanged.
//
// One workgroup of 1024 threads does the whole update: a 64-bit key per
// sample (tier:2 | order-preserving cost bits:32 | index:30) is unique, so the
// N_e-th smallest key is found by an 8-pass MSB radix select with LDS
// histograms, the <= 256 keys at or below it are gathered and bitonic-sorted
// in LDS, and the sorted elite list drives the refit.  Mean and covariance
// sums run in FP64 in elite order and the Cholesky factor column by column,
// each sum in ascending order, so every run gives the same bits.  This
// translation unit is compiled with -ffp-contract=off.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace cem {
namespace {

constexpr int BS = 1024;
constexpr uint64_t IDX_MASK = (1ull << 30) - 1;

enum : int32_t { SEL_TOP = 0, SEL_ALL_FEAS = 1, SEL_ONE = 2, SEL_TIER1 = 3, SEL_NONE = 4 };

__device__ __forceinline__ uint64_t make_key(const float *cost, const uint8_t *tier, int i, int *tier_out) {
  float c = cost[i];
  int t = tier[i];
  t = t > 3 ? 3 : t;
  if (c != c) {  // NaN
    t = 3;
    c = __int_as_float(0x7F800000);
  }
  if (c == 0.0f) c = 0.0f;  // -0 -> +0
  const uint32_t b = __float_as_uint(c);
  const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  *tier_out = t;
  return ((uint64_t)t << 62) | ((uint64_t)ord << 30) | (uint64_t)i;
}

__device__ __forceinline__ float key_cost(uint64_t k) {
  const uint32_t ord = (uint32_t)(k >> 30);
  const uint32_t b = (ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord;
  return __uint_as_float(b);
}

// Cholesky of S + delta I into L (row-major, stride D), column by column;
// thread j-loop is shared, rows below the pivot in parallel; every sum runs
// over ascending k exactly as the sequential definition.  Returns ok flag.
__device__ bool chol_block(int D, const double *S, double delta, double *A, double *L, int *bad) {
  const int tid = threadIdx.x;
  for (int t = tid; t < D * D; t += BS) {
    A[t] = S[t];
    L[t] = 0.0;
  }
  __syncthreads();
  if (tid < D) A[tid * D + tid] = A[tid * D + tid] + delta;
  if (tid == 0) *bad = 0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    if (tid == 0) {
      double s = A[j * D + j];
      for (int k = 0; k < j; ++k) s = s - L[j * D + k] * L[j * D + k];
      if (!(s > 0.0) || !isfinite(s)) *bad = 1;
      L[j * D + j] = sqrt(s);
    }
    __syncthreads();
    if (*bad) return false;
    const int i = j + 1 + tid;
    if (i < D) {
      double t = A[i * D + j];
      for (int k = 0; k < j; ++k) t = t - L[i * D + k] * L[j * D + k];
      L[i * D + j] = t / L[j * D + j];
    }
    __syncthreads();
  }
  return true;
}

// delta = 1e-9 tr(S)/D + 1e-12, x10 per failed try, six tries, then the
// diagonal fallback sqrt(max(S_dd, 1e-12)).  Writes st->L, st->factor_status.
__device__ void factor_into(DevState *st, double *A, double *L, int *bad) {
  const int D = st->D;
  __shared__ double delta_s;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int d = 0; d < D; ++d) tr = tr + st->S[d * D + d];
    delta_s = 1e-9 * tr / (double)D + 1e-12;
  }
  __syncthreads();
  double delta = delta_s;
  bool ok = false;
  for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
    ok = chol_block(D, st->S, delta, A, L, bad);
    delta = delta * 10.0;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < D * D; t += BS) {
    const int r = t / D, c = t % D;
    double v;
    if (ok) v = L[t];
    else v = (r == c) ? sqrt(fmax(st->S[t], 1e-12)) : 0.0;
    st->L[t] = v;
  }
  if (threadIdx.x == 0) st->factor_status = ok ? 0 : 1;
  __syncthreads();
}

__device__ __forceinline__ void select_refit_block(DevState *__restrict__ st, const float *__restrict__ Z,
                                                   const float *__restrict__ cost, const uint8_t *__restrict__ tier,
                                                   int pop, int32_t *__restrict__ elite_out,
                                                   int32_t *__restrict__ sel_out, float *__restrict__ stats,
                                                   int stats_cap, int advance_iter) {
  __shared__ int cnt[4];
  __shared__ unsigned hist[256];
  __shared__ uint64_t sel[MAX_ELITE];
  __shared__ uint64_t wmin[BS / 64];
  __shared__ int ne_s, mode_s, nsel_s, rank_s, bad_s;
  __shared__ uint64_t prefix_s, mask_s, minkey_s;
  __shared__ double A[MAX_D * MAX_D], Lw[MAX_D * MAX_D];
  const int tid = threadIdx.x;
  const int D = st->D;
  const int n_elite = st->n_elite;

  if (tid < 4) cnt[tid] = 0;
  __syncthreads();
  // tier counts and the overall minimum key
  int lc[4] = {0, 0, 0, 0};
  uint64_t mk = ~0ull;
  for (int i = tid; i < pop; i += BS) {
    int t;
    const uint64_t k = make_key(cost, tier, i, &t);
    lc[t]++;
    mk = k < mk ? k : mk;
  }
  for (int t = 0; t < 4; ++t)
    if (lc[t]) atomicAdd(&cnt[t], lc[t]);
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_down(mk, off, 64);
    mk = o < mk ? o : mk;
  }
  if ((tid & 63) == 0) wmin[tid >> 6] = mk;
  __syncthreads();
  if (tid == 0) {
    uint64_t m = ~0ull;
    for (int w = 0; w < BS / 64; ++w) m = wmin[w] < m ? wmin[w] : m;
    minkey_s = m;
    const int n0 = cnt[0], n1 = cnt[1];
    int ne, mode;
    if (n0 >= n_elite) { ne = n_elite; mode = SEL_TOP; }
    else if (n0 >= 2) { ne = n0; mode = SEL_ALL_FEAS; }
    else if (n0 == 1) { ne = 1; mode = SEL_ONE; }
    else if (n1 >= 1) { ne = n1 < n_elite ? n1 : n_elite; mode = ne == 1 ? SEL_ONE : SEL_TIER1; }
    else { ne = 0; mode = SEL_NONE; }
    ne_s = ne;
    mode_s = mode;
    prefix_s = 0;
    mask_s = 0;
    rank_s = ne;
    nsel_s = 0;
  }
  __syncthreads();
  const int ne = ne_s;

  if (ne > 0) {
    // radix select of the ne-th smallest key (keys are unique)
    for (int shift = 56; shift >= 0; shift -= 8) {
      if (tid < 256) hist[tid] = 0;
      __syncthreads();
      const uint64_t prefix = prefix_s, mask = mask_s;
      for (int i = tid; i < pop; i += BS) {
        int t;
        const uint64_t k = make_key(cost, tier, i, &t);
        if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (tid == 0) {
        int rank = rank_s;
        unsigned cum = 0;
        for (int b = 0; b < 256; ++b) {
          if (cum + hist[b] >= (unsigned)rank) {
            prefix_s = prefix | ((uint64_t)b << shift);
            rank_s = rank - (int)cum;
            break;
          }
          cum += hist[b];
        }
        mask_s = mask | (255ull << shift);
      }
      __syncthreads();
    }
    const uint64_t thr = prefix_s;
    for (int i = tid; i < pop; i += BS) {
      int t;
      const uint64_t k = make_key(cost, tier, i, &t);
      if (k <= thr) {
        const int slot = atomicAdd(&nsel_s, 1);
        if (slot < MAX_ELITE) sel[slot] = k;
      }
    }
    __syncthreads();
    for (int t = nsel_s + tid; t < MAX_ELITE; t += BS) sel[t] = ~0ull;
    __syncthreads();
    // bitonic sort of the 256 gathered keys
    for (int size = 2; size <= MAX_ELITE; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        if (tid < MAX_ELITE / 2) {
          const int lo = 2 * tid - (tid & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const uint64_t a = sel[lo], b = sel[hi];
          if ((a > b) == up) {
            sel[lo] = b;
            sel[hi] = a;
          }
        }
        __syncthreads();
      }
    }
  }

  const int mode = mode_s;
  if (elite_out)
    for (int e = tid; e < n_elite; e += BS) elite_out[e] = e < ne ? (int32_t)(sel[e] & IDX_MASK) : -1;

  // refit
  if (ne == 1) {
    const long r0 = (long)(sel[0] & IDX_MASK) * D;
    if (tid < D) st->mu[tid] = (double)Z[r0 + tid];
    for (int t = tid; t < D * D; t += BS) {
      const int a = t / D, b = t % D;
      double v = 0.0;
      if (a == b) {
        const double s = 0.1 * sqrt(st->cov0[t]);
        v = s * s;
      }
      st->S[t] = v;
    }
  } else if (ne >= 2) {
    if (tid < D) {
      double acc = 0.0;
      for (int e = 0; e < ne; ++e) acc = acc + (double)Z[(long)(sel[e] & IDX_MASK) * D + tid];
      st->mu[tid] = acc / (double)ne;
    }
    __syncthreads();
    if (tid < D * D) {
      const int a = tid / D, b = tid % D;
      double v = 0.0;
      if (st->cov_mode != 0 || a == b) {
        const double ma = st->mu[a], mb = st->mu[b];
        double acc = 0.0;
        for (int e = 0; e < ne; ++e) {
          const long r = (long)(sel[e] & IDX_MASK) * D;
          const double da = (double)Z[r + a] - ma;
          const double db = (double)Z[r + b] - mb;
          acc = acc + da * db;
        }
        v = acc / (double)ne;
      }
      st->S[tid] = v;
    }
  }
  __syncthreads();
  if (ne >= 1) factor_into(st, A, Lw, &bad_s);

  // best-so-far record, stats, selection info
  if (tid == 0) {
    const uint64_t k = minkey_s;
    const int bt = (int)(k >> 62);
    const float bc = key_cost(k);
    const int bi = (int)(k & IDX_MASK);
    if (pop > 0 && (bt < st->best_tier || (bt == st->best_tier && bc < st->best_cost))) {
      st->best_tier = bt;
      st->best_cost = bc;
      for (int d = 0; d < D; ++d) st->best_z[d] = Z[(long)bi * D + d];
    }
    st->sel_info[0] = ne;
    st->sel_info[1] = mode;
    for (int t = 0; t < 4; ++t) st->sel_info[2 + t] = cnt[t];
    if (sel_out)
      for (int t = 0; t < 6; ++t) sel_out[t] = st->sel_info[t];
    const int it = st->iter;
    if (stats && it >= 0 && it < stats_cap) {
      float *row = stats + (long)it * CEM_STATS_COLS;
      row[0] = pop > 0 ? bc : __int_as_float(0x7F800000);
      for (int t = 0; t < 4; ++t) row[1 + t] = (float)cnt[t];
      row[5] = (float)ne;
      row[6] = (float)mode;
      row[7] = st->best_cost;
    }
    if (advance_iter) st->iter = it + 1;
  }
}

__global__ void __launch_bounds__(BS) select_refit_kernel(DevState *__restrict__ st, const float *__restrict__ Z,
                                                          const float *__restrict__ cost,
                                                          const uint8_t *__restrict__ tier, int pop,
                                                          int32_t *__restrict__ elite_out,
                                                          int32_t *__restrict__ sel_out, float *__restrict__ stats,
                                                          int stats_cap, int advance_iter) {
  select_refit_block(st, Z, cost, tier, pop, elite_out, sel_out, stats, stats_cap, advance_iter);
}

// Batched: one workgroup per instance; instances past their iteration cap are skipped.
__global__ void __launch_bounds__(BS) select_refit_batch_kernel(const InstDesc *__restrict__ insts, int stats_cap) {
  const InstDesc d = insts[blockIdx.x];
  if (d.st->iter >= d.iters) return;  // uniform over the workgroup
  select_refit_block(d.st, d.Z, d.cost, d.tier, d.pop, nullptr, nullptr, d.stats, stats_cap, 1);
}

__global__ void __launch_bounds__(BS) factor_kernel(DevState *st) {
  __shared__ double A[MAX_D * MAX_D], Lw[MAX_D * MAX_D];
  __shared__ int bad;
  factor_into(st, A, Lw, &bad);
}

}  // namespace

hipError_t launch_select_refit(DevState *st, const float *Z, const float *cost, const uint8_t *tier, int pop,
                               int32_t *elite_idx, int32_t *sel_info, float *stats, int stats_cap,
                               int advance_iter, hipStream_t s) {
  hipLaunchKernelGGL(select_refit_kernel, dim3(1), dim3(BS), 0, s, st, Z, cost, tier, pop, elite_idx, sel_info,
                     stats, stats_cap, advance_iter);
  return hipGetLastError();
}

hipError_t launch_select_refit_batch(const InstDesc *insts, int n_inst, int stats_cap, hipStream_t s) {
  hipLaunchKernelGGL(select_refit_batch_kernel, dim3(n_inst), dim3(BS), 0, s, insts, stats_cap);
  return hipGetLastError();
}

hipError_t launch_factor(DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(factor_kernel, dim3(1), dim3(BS), 0, s, st);
  return hipGetLastError();
}

}  // namespace cem
