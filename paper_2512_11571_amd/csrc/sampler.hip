// Sampling step of CE optimisation (Alg. 1: draw n_env parameter vectors
// Z ~ phi(theta), phi Gaussian per Sec. IV-A) and the per-instance scene draws.
//
// Philox-4x32-10 (Salmon et al., SC'11): 4-word counter, 2-word key, ten
// rounds of two 32x32->64 multiplies that remix the halves with the other
// words and the key, the key bumped by two Weyl constants between rounds.
// Normals by Box-Muller with ln / sin / cos evaluated by the routines below,
// built only from correctly rounded FP32 operations so every GPU produces the
// same bits.  This translation unit is compiled with -ffp-contract=off: no
// multiply-add is fused unless written as fmaf.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace cem {
namespace {

constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;

struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox10(U4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = M0 * x.a, hi0 = __umulhi(M0, x.a);
    const uint32_t lo1 = M1 * x.c, hi1 = __umulhi(M1, x.c);
    U4 y;
    y.a = hi1 ^ x.b ^ k0;
    y.b = lo1;
    y.c = hi0 ^ x.d ^ k1;
    y.d = lo0;
    x = y;
    k0 += W0;
    k1 += W1;
  }
  return x;
}

__device__ __forceinline__ U4 draw(uint64_t seed, uint32_t tag, uint32_t block, uint32_t sample, uint32_t iter,
                                   uint32_t inst) {
  U4 c{(tag << 24) | (block & 0x00FFFFFFu), sample, iter, inst};
  return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// (0,1): top 23 bits b -> (2b + 1) 2^-24, exact.
__device__ __forceinline__ float unit(uint32_t x) { return (float)(2u * (x >> 9) + 1u) * 0x1p-24f; }

// ln u for positive normal u: u = m 2^e, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^11/11), s = (m - 1)/(m + 1);
// e ln 2 with ln 2 split so that e * hi is exact.
__device__ __forceinline__ float ln_f32(float u) {
  const uint32_t bits = __float_as_uint(u);
  int e = (int)((bits >> 23) & 0xFFu) - 127;
  float m = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);
  if (m > 1.41421353816986083984375f) {
    m = m * 0.5f;
    e += 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float s2 = s * s;
  float p = __builtin_fmaf(s2, 1.0f / 11.0f, 1.0f / 9.0f);
  p = __builtin_fmaf(s2, p, 1.0f / 7.0f);
  p = __builtin_fmaf(s2, p, 1.0f / 5.0f);
  p = __builtin_fmaf(s2, p, 1.0f / 3.0f);
  const float lm = 2.0f * __builtin_fmaf(s * s2, p, s);
  const float ef = (float)e;
  const float hi = ef * 0.693145751953125f;
  const float lo = __builtin_fmaf(ef, 1.428606765330187e-06f, lm);
  return hi + lo;
}

// sin, cos of 2 pi u (u with <= 24 fraction bits): quarter-turn reduction is
// exact; Taylor polynomials on |x| <= pi/4; quadrant rotation.
__device__ __forceinline__ void sincos_2pi(float u, float &s, float &c) {
  const float t = 4.0f * u;
  const float k = __builtin_rintf(t);
  const float x = (t - k) * 1.57079637050628662109375f;
  const float x2 = x * x;
  float ps = __builtin_fmaf(x2, -1.0f / 39916800.0f, 1.0f / 362880.0f);
  ps = __builtin_fmaf(x2, ps, -1.0f / 5040.0f);
  ps = __builtin_fmaf(x2, ps, 1.0f / 120.0f);
  ps = __builtin_fmaf(x2, ps, -1.0f / 6.0f);
  const float sx = __builtin_fmaf(x * x2, ps, x);
  float pc = __builtin_fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = __builtin_fmaf(x2, pc, -1.0f / 720.0f);
  pc = __builtin_fmaf(x2, pc, 1.0f / 24.0f);
  pc = __builtin_fmaf(x2, pc, -0.5f);
  const float cx = __builtin_fmaf(x2, pc, 1.0f);
  const int q = ((int)k) & 3;
  s = q == 0 ? sx : (q == 1 ? cx : (q == 2 ? -sx : -cx));
  c = q == 0 ? cx : (q == 1 ? -sx : (q == 2 ? -cx : sx));
}

// Iteration 0 from the region (Sec. III-B: uniform inside each parameter's
// region): u_d is word d mod 4 of the CE-stream block d / 4; a ring pair
// (d, d+1) takes its radius uniform in r^2 (uniform by area) from u_d and its
// angle 2 pi u_{d+1}; every other dimension is uniform on [lo_d, hi_d].
__device__ __forceinline__ void region_row(uint64_t seed, uint32_t inst, const cem_init_region &R, int D, int i,
                                           float *__restrict__ Z) {
  float u[MAX_D];
#pragma unroll
  for (int blk = 0; blk < MAX_D / 4; ++blk) {
    u[blk * 4 + 0] = u[blk * 4 + 1] = u[blk * 4 + 2] = u[blk * 4 + 3] = 0.0f;
    if (blk * 4 < D) {
      const U4 w = draw(seed, 0u, (uint32_t)blk, (uint32_t)i, 0u, inst);
      u[blk * 4 + 0] = unit(w.a);
      u[blk * 4 + 1] = unit(w.b);
      u[blk * 4 + 2] = unit(w.c);
      u[blk * 4 + 3] = unit(w.d);
    }
  }
  float z[MAX_D];
#pragma unroll
  for (int d = 0; d < MAX_D; ++d) z[d] = __builtin_fmaf(R.hi[d] - R.lo[d], u[d], R.lo[d]);
  for (int k = 0; k < R.n_annuli; ++k) {
    const int d = R.ann_dim[k];
    const float r0 = R.ann_radius[k][0], r1 = R.ann_radius[k][1];
    const float a0 = r0 * r0, a1 = r1 * r1;
    float ud = 0.0f, ue = 0.0f;
#pragma unroll
    for (int e = 0; e < MAX_D; ++e) {
      ud = e == d ? u[e] : ud;
      ue = e == d + 1 ? u[e] : ue;
    }
    const float r = sqrtf(__builtin_fmaf(a1 - a0, ud, a0));
    float sn, cs;
    sincos_2pi(ue, sn, cs);
    const float x = __builtin_fmaf(r, cs, R.ann_center[k][0]);
    const float y = __builtin_fmaf(r, sn, R.ann_center[k][1]);
#pragma unroll
    for (int e = 0; e < MAX_D; ++e) {
      z[e] = e == d ? x : z[e];
      z[e] = e == d + 1 ? y : z[e];
    }
  }
  float *row = Z + (long)i * D;
  for (int d = 0; d < D; ++d) row[d] = z[d];
}

// One sample row: D normals from ceil(D/4) Philox blocks, then
// z_d = fl32(mu_d + sum_{e<=d} L_de eps_e) in FP64, ascending e.
__device__ __forceinline__ void sample_row(uint64_t seed, uint32_t inst, uint32_t iter,
                                           const DevState *__restrict__ st, int D, int i, float *__restrict__ Z) {
  if (iter == 0 && st->region_on) {
    region_row(seed, inst, st->region, D, i, Z);
    return;
  }
  float eps[MAX_D];
#pragma unroll
  for (int blk = 0; blk < MAX_D / 4; ++blk) {
    if (blk * 4 < D) {
      const U4 w = draw(seed, 0u, (uint32_t)blk, (uint32_t)i, iter, inst);
      const uint32_t ws[4] = {w.a, w.b, w.c, w.d};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float r = sqrtf(-2.0f * ln_f32(unit(ws[2 * h])));
        float sn, cs;
        sincos_2pi(unit(ws[2 * h + 1]), sn, cs);
        eps[blk * 4 + 2 * h] = r * cs;
        eps[blk * 4 + 2 * h + 1] = r * sn;
      }
    }
  }
  float *row = Z + (long)i * D;
  for (int d = 0; d < D; ++d) {
    double acc = 0.0;
    for (int e = 0; e <= d; ++e) acc = acc + st->L[d * D + e] * (double)eps[e];
    row[d] = (float)(st->mu[d] + acc);
  }
}

// One thread per row of one instance; the iteration is the argument or, when
// negative, the instance's device counter (the replayed iteration).
__global__ void __launch_bounds__(256) sample_kernel(uint64_t seed, uint32_t inst, int32_t iter_arg,
                                                     const DevState *__restrict__ st, int pop, int D,
                                                     float *__restrict__ Z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pop) return;
  const uint32_t iter = iter_arg >= 0 ? (uint32_t)iter_arg : (uint32_t)st->iter;
  sample_row(seed, inst, iter, st, D, i, Z);
}

// Batched: grid.y = instance; instances past their iteration cap are skipped.
__global__ void __launch_bounds__(256) sample_batch_kernel(const InstDesc *__restrict__ insts) {
  const InstDesc d = insts[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.pop || d.st->iter >= d.iters) return;
  sample_row(d.st->seed, d.st->inst_id, (uint32_t)d.st->iter, d.st, d.D, i, const_cast<float *>(d.Z));
}

// He-normal initial weights of the surrogate network: entry p of a weight
// matrix with fan-in f is eps_p sqrt(2 / f), eps_p the normal p % 4 of Philox
// stream 2 block p / 4 (sample 0, iteration 0, instance 0), computed in FP64
// and rounded once to FP32; biases are zero.  Layers: [w0, w0 + nw) weights.
struct InitLayers {
  long w0[4], nw[4];
  int fan_in[4];
  long n_params;
};
__global__ void __launch_bounds__(256) mlp_init_kernel(uint64_t seed, InitLayers L, float *__restrict__ P) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L.n_params) return;
  int layer = -1;
  for (int l = 0; l < 4; ++l)
    if (p >= L.w0[l] && p < L.w0[l] + L.nw[l]) layer = l;
  if (layer < 0) {
    P[p] = 0.0f;
    return;
  }
  const U4 w = draw(seed, 2u, (uint32_t)(p / 4), 0u, 0u, 0u);
  const uint32_t ws[4] = {w.a, w.b, w.c, w.d};
  const int h = (int)(p % 4) / 2;
  const float r = sqrtf(-2.0f * ln_f32(unit(ws[2 * h])));
  float sn, cs;
  sincos_2pi(unit(ws[2 * h + 1]), sn, cs);
  const float e = (p % 2 == 0) ? r * cs : r * sn;
  P[p] = (float)((double)e * sqrt(2.0 / (double)L.fan_in[layer]));
}

// Per-instance draws on the scene stream (tag 1), one Philox block: the push
// goal g = start + rho (cos phi, sin phi), rho and phi uniform in their ranges
// (words 0, 1), and the object's friction coefficient U[obj_mu_lo, obj_mu_hi]
// when obj_mu_hi > 0 (word 2).
__global__ void instance_draw_kernel(cem_scene sc, uint64_t seed, uint32_t inst, DevState *st) {
  const int t = threadIdx.x;
  if (blockIdx.x != 0) return;
  if (t < CEM_MAX_DR) {
    // domain-randomisation scenario t: object friction (word 0) and mass (word 1)
    const U4 v = draw(seed, 1u, 1u, (uint32_t)t, 0u, inst);
    st->dr_mu[t] = sc.dr_mu_hi > 0.0f
                       ? (float)((double)sc.dr_mu_lo + ((double)sc.dr_mu_hi - (double)sc.dr_mu_lo) * (double)unit(v.a))
                       : 0.0f;
    st->dr_mass[t] =
        sc.dr_mass_hi > 0.0f
            ? (float)((double)sc.dr_mass_lo + ((double)sc.dr_mass_hi - (double)sc.dr_mass_lo) * (double)unit(v.b))
            : 0.0f;
  }
  if (t != 0) return;
  const U4 w = draw(seed, 1u, 0u, 0u, 0u, inst);
  const double u0 = (double)unit(w.a), u1 = (double)unit(w.b);
  const double rho = (double)sc.goal_rho_lo + ((double)sc.goal_rho_hi - (double)sc.goal_rho_lo) * u0;
  const double phi = (double)sc.goal_phi_lo + ((double)sc.goal_phi_hi - (double)sc.goal_phi_lo) * u1;
  st->goal[0] = (double)sc.obj_pos0[0] + rho * cos(phi);
  st->goal[1] = (double)sc.obj_pos0[1] + rho * sin(phi);
  st->obj_mu = sc.obj_mu_hi > 0.0f
                   ? (float)((double)sc.obj_mu_lo + ((double)sc.obj_mu_hi - (double)sc.obj_mu_lo) * (double)unit(w.c))
                   : 0.0f;
}

}  // namespace

hipError_t launch_sample(uint64_t seed, uint32_t inst, int32_t iter, const DevState *st, int pop, int D, float *Z,
                         hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(sample_kernel, dim3((pop + bs - 1) / bs), dim3(bs), 0, s, seed, inst, iter, st, pop, D, Z);
  return hipGetLastError();
}

hipError_t launch_mlp_init(uint64_t seed, const long *w0, const long *nw, const int *fan_in, long n_params,
                           float *P, hipStream_t s) {
  InitLayers L;
  for (int l = 0; l < 4; ++l) {
    L.w0[l] = w0[l];
    L.nw[l] = nw[l];
    L.fan_in[l] = fan_in[l];
  }
  L.n_params = n_params;
  hipLaunchKernelGGL(mlp_init_kernel, dim3((unsigned)((n_params + 255) / 256)), dim3(256), 0, s, seed, L, P);
  return hipGetLastError();
}

hipError_t launch_sample_batch(const InstDesc *insts, int n_inst, int max_pop, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(sample_batch_kernel, dim3((max_pop + bs - 1) / bs, n_inst), dim3(bs), 0, s, insts);
  return hipGetLastError();
}

hipError_t launch_instance_draw(const cem_scene &sc, uint64_t seed, uint32_t inst, DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(instance_draw_kernel, dim3(1), dim3(64), 0, s, sc, seed, inst, st);
  return hipGetLastError();
}

}  // namespace cem
