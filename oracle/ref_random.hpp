// Oracle: counter-based sampling. TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Sec. III-B, Alg. 1 (sampling step): every CE iteration draws n_env parameter
// vectors Z ~ phi(theta).  phi is a Gaussian (Sec. IV-A, "Algorithm setting":
// independent normals; a full covariance is the generalisation).
//
// Generator: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), written from its published definition:
// a 4-word counter and a 2-word key; ten rounds, each round multiplying words 0
// and 2 by the constants M0, M1 to 64-bit products and re-mixing the halves
// with the other two words and the key; the key is bumped by the Weyl
// constants W0, W1 between rounds.
//
// Normals: Box-Muller on pairs of uniforms.  So that the CPU and the GPU give
// bit-identical normals, ln, sin and cos are computed here by explicit FP32
// routines built only from correctly rounded IEEE operations (+ - * / fma),
// with polynomial coefficients that are plain Taylor coefficients (1/n!,
// 1/(2k+1)); no vendor libm is involved.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

namespace ref {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

struct Word4 { uint32_t w[4]; };

// One Philox-4x32 round on counter x with key (k0, k1).
inline Word4 philox_round(const Word4 &x, uint32_t k0, uint32_t k1) {
  uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x.w[0];
  uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x.w[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  Word4 y;
  y.w[0] = hi1 ^ x.w[1] ^ k0;
  y.w[1] = lo1;
  y.w[2] = hi0 ^ x.w[3] ^ k1;
  y.w[3] = lo0;
  return y;
}

// Philox-4x32-10: ten rounds, key bumped after every round but the last.
inline Word4 philox4x32_10(Word4 ctr, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    ctr = philox_round(ctr, k0, k1);
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  return ctr;
}

// Stream tags (the top byte of counter word 0).
constexpr uint32_t STREAM_CEM = 0, STREAM_SCENE = 1, STREAM_MLP_INIT = 2, STREAM_SHUFFLE = 3;

// Counter layout: c0 = tag<<24 | block, c1 = sample, c2 = iteration, c3 = instance.
inline Word4 philox_draw(uint64_t seed, uint32_t tag, uint32_t block, uint32_t sample,
                         uint32_t iter, uint32_t instance) {
  Word4 c;
  c.w[0] = (tag << 24) | (block & 0x00FFFFFFu);
  c.w[1] = sample;
  c.w[2] = iter;
  c.w[3] = instance;
  return philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
}

// Uniform in (0,1): the top 23 bits b give u = (2b + 1) * 2^-24, exact in FP32.
inline float u01(uint32_t x) {
  uint32_t b = x >> 9;
  return (float)(2u * b + 1u) * 0x1p-24f;
}

// Natural log of a positive normal FP32 number.  u = m * 2^e with
// m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1), by the odd
// series s + s^3/3 + ... + s^11/11 (|s| <= 0.1716, truncation < 2^-27 rel);
// ln 2 is split hi/lo (Cody-Waite) so e*ln2_hi is exact for |e| < 2^8.
inline float ref_logf(float u) {
  uint32_t bits;
  std::memcpy(&bits, &u, 4);
  int e = (int)((bits >> 23) & 0xFFu) - 127;
  uint32_t mb = (bits & 0x007FFFFFu) | 0x3F800000u;  // m in [1, 2)
  float m;
  std::memcpy(&m, &mb, 4);
  if (m > 1.41421353816986083984375f) {  // fl32(sqrt 2)
    m = m * 0.5f;
    e += 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float s2 = s * s;
  float p = std::fma(s2, 1.0f / 11.0f, 1.0f / 9.0f);
  p = std::fma(s2, p, 1.0f / 7.0f);
  p = std::fma(s2, p, 1.0f / 5.0f);
  p = std::fma(s2, p, 1.0f / 3.0f);
  const float s3 = s * s2;
  const float lm = 2.0f * std::fma(s3, p, s);
  const float LN2_HI = 0.693145751953125f;   // 0x3F317200: 15 trailing zero bits
  const float LN2_LO = 1.428606765330187e-06f;  // fl32(ln 2 - LN2_HI)
  const float ef = (float)e;
  const float hi = ef * LN2_HI;
  const float lo = std::fma(ef, LN2_LO, lm);
  return hi + lo;
}

// sin and cos of 2*pi*u for u in (0,1) with at most 24 fraction bits.
// 4u is exact; k = nearest integer; f = 4u - k is exact with |f| <= 1/2;
// x = f * pi/2 (|x| <= pi/4); Taylor polynomials through x^11 / x^10;
// the quadrant k mod 4 rotates (sin x, cos x).
inline void ref_sincos2pi(float u, float *s_out, float *c_out) {
  const float t = 4.0f * u;
  const float k = std::nearbyint(t);
  const float f = t - k;
  const float x = f * 1.57079637050628662109375f;  // fl32(pi/2)
  const float x2 = x * x;
  float ps = std::fma(x2, -1.0f / 39916800.0f, 1.0f / 362880.0f);
  ps = std::fma(x2, ps, -1.0f / 5040.0f);
  ps = std::fma(x2, ps, 1.0f / 120.0f);
  ps = std::fma(x2, ps, -1.0f / 6.0f);
  const float sx = std::fma(x * x2, ps, x);
  float pc = std::fma(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = std::fma(x2, pc, -1.0f / 720.0f);
  pc = std::fma(x2, pc, 1.0f / 24.0f);
  pc = std::fma(x2, pc, -0.5f);
  const float cx = std::fma(x2, pc, 1.0f);
  const int q = ((int)k) & 3;
  float s, c;
  if (q == 0) { s = sx; c = cx; }
  else if (q == 1) { s = cx; c = -sx; }
  else if (q == 2) { s = -sx; c = -cx; }
  else { s = -cx; c = sx; }
  *s_out = s;
  *c_out = c;
}

// Four standard normals from one Philox block: Box-Muller on (u0,u1), (u2,u3):
// r = sqrt(-2 ln u_a); n = (r cos 2 pi u_b, r sin 2 pi u_b).
inline void normals4(const Word4 &x, float out[4]) {
  for (int h = 0; h < 2; ++h) {
    const float ua = u01(x.w[2 * h]);
    const float ub = u01(x.w[2 * h + 1]);
    const float r = std::sqrt(-2.0f * ref_logf(ua));
    float s, c;
    ref_sincos2pi(ub, &s, &c);
    out[2 * h] = r * c;
    out[2 * h + 1] = r * s;
  }
}

// epsilon_d of sample i in iteration j of instance b.
inline float cem_normal(uint64_t seed, int d, uint32_t i, uint32_t j, uint32_t b) {
  Word4 x = philox_draw(seed, STREAM_CEM, (uint32_t)(d / 4), i, j, b);
  float n[4];
  normals4(x, n);
  return n[d % 4];
}

// z = mu + L eps (L lower triangular), accumulated in FP64 with separate
// multiply and add in ascending column order, then rounded once to FP32.
inline void cem_sample_row(uint64_t seed, uint32_t i, uint32_t j, uint32_t b, int D,
                           const double *mu, const double *L, float *z_out, float *eps_out) {
  float eps[64];
  for (int d = 0; d < D; ++d) eps[d] = cem_normal(seed, d, i, j, b);
  for (int d = 0; d < D; ++d) {
    double acc = 0.0;
    for (int e = 0; e <= d; ++e) {
      volatile double prod = L[d * D + e] * (double)eps[e];
      acc = acc + prod;
    }
    volatile double zz = mu[d] + acc;
    z_out[d] = (float)zz;
    if (eps_out) eps_out[d] = eps[d];
  }
}

// Initial distribution as a region (Sec. III-B: iteration 0 samples uniformly
// inside each parameter's region h(z) <= 0; Sec. IV-A: rings around the tables
// for the base positions, boxes for the others).  The uniforms are the words
// of the same Philox blocks the normals of iteration 0 would use: u_d is word
// d mod 4 of block d / 4.  A box dimension maps u to lo + (hi - lo) u.  A ring
// pair (d, d+1) with centre c and radii r0 <= r1 must be uniform by area: the
// fraction of the ring's area within radius r is (r^2 - r0^2) / (r1^2 - r0^2),
// so r^2 is uniform on [r0^2, r1^2]; the angle is uniform on [0, 2 pi).
// Every step is one correctly rounded FP32 operation (fma where written), so
// the GPU's draw is reproducible bit for bit.
struct RefRegion {
  const float *lo, *hi;  // D each
  int n_rings;
  const int *ring_dim;   // first dimension of each pair
  const float *ring;     // n_rings x (cx, cy, r0, r1)
};

inline void region_sample_row(uint64_t seed, uint32_t i, uint32_t b, int D, const RefRegion &R, float *z_out) {
  float u[64];
  for (int d = 0; d < D; ++d) u[d] = u01(philox_draw(seed, STREAM_CEM, (uint32_t)(d / 4), i, 0u, b).w[d % 4]);
  for (int d = 0; d < D; ++d) z_out[d] = std::fma(R.hi[d] - R.lo[d], u[d], R.lo[d]);
  for (int k = 0; k < R.n_rings; ++k) {
    const int d = R.ring_dim[k];
    const float *g = R.ring + 4 * k;
    const float rr0 = g[2] * g[2], rr1 = g[3] * g[3];
    const float r = std::sqrt(std::fma(rr1 - rr0, u[d], rr0));
    float s, c;
    ref_sincos2pi(u[d + 1], &s, &c);
    z_out[d] = std::fma(r, c, g[0]);
    z_out[d + 1] = std::fma(r, s, g[1]);
  }
}

// n_env(j): pop, or with a schedule (pop_final > 0) a linear decrease to
// pop_final over the first `ramp` iterations, constant afterwards (Sec. IV-A,
// "Algorithm setting"), rounded down in the decrement.
inline int n_env_at(int pop, int pop_final, int ramp, int j) {
  if (pop_final <= 0) return pop;
  const long k = j < ramp ? j : ramp;
  return pop - (int)((long)(pop - pop_final) * k / ramp);
}

}  // namespace ref
