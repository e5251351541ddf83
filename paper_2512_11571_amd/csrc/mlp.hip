// Learned surrogate for candidate screening: a 16 -> 256 -> 256 -> 256 -> 8
// perceptron (GELU, tanh form) predicting a plan's cost and final object pose
// from its controller parameters, trained on rollouts the simulator produced.
// Not part of the paper's method; its limitation paragraph (full rollouts are
// expensive) motivates it: CE samples a 16x larger population, the network
// ranks it, and only the most promising candidates are simulated in full -
// full simulation decides every cost that enters the refit.
//
// All matrix products run on the MFMA units: BF16 operands, FP32
// accumulation (gfx950's v_mfma_f32_16x16x32_bf16), 128x128 output tiles per
// workgroup of four waves, each wave a 64x64 quadrant of 4x4 MFMA tiles, the
// K dimension staged through LDS 32 at a time; bias, GELU and its derivative
// are fused into the epilogue.  Master weights and Adam moments are FP32; the
// BF16 copy of the weights is refreshed by the Adam kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace cem {
namespace {

constexpr int IN = 16, HID = 256, OUT = 8, NL = 4;
constexpr int DIMS[NL + 1] = {IN, HID, HID, HID, OUT};

__host__ __device__ constexpr long w_off(int l) {
  long o = 0;
  for (int k = 0; k < l; ++k) o += (long)DIMS[k] * DIMS[k + 1] + DIMS[k + 1];
  return o;
}
__host__ __device__ constexpr long b_off(int l) { return w_off(l) + (long)DIMS[l] * DIMS[l + 1]; }
constexpr long N_PARAMS = w_off(NL);

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32; inf kept, NaN
// stays NaN), one value or two packed (a in the low half).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU, tanh form: 0.5 x (1 + tanh u), u = sqrt(2/pi) (x + 0.044715 x^3),
// evaluated as x s with s = 1 / (1 + e^(-2u)) (the same function: 1 + tanh u =
// 2 / (1 + e^(-2u))), e^(-2u) = 2^(-2 u log2 e) and the reciprocal from the
// hardware's exp2 and rcp (about 1 ulp each: far below the BF16 rounding of
// the activations); its derivative s + 2 x s (1 - s) sqrt(2/pi) (1 + 3 0.044715 x^2).
constexpr float GELU_C = 0.7978845608028654f, GELU_A = 0.044715f;
constexpr float GELU_K = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634);
__device__ __forceinline__ float gelu_s(float x) {
  const float u = x * fmaf(GELU_A * x, x, 1.0f);
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(GELU_K * u));
}
__device__ __forceinline__ float gelu(float x) { return x * gelu_s(x); }
__device__ __forceinline__ float gelu_grad(float x) {
  const float s = gelu_s(x);
  return s + 2.0f * x * s * (1.0f - s) * GELU_C * fmaf(3.0f * GELU_A * x, x, 1.0f);
}

enum Epi : int {
  EPI_STORE = 0,      // C = acc (fp32)
  EPI_BIAS = 1,       // C = acc + bias[n] (fp32)
  EPI_BIAS_GELU = 2,  // Z = acc + bias[n] (fp32, optional), H = bf16(gelu(Z))
  EPI_DGELU = 3       // dZ = acc * gelu'(Zin[m][n]): fp32 (optional) and bf16
};

struct GemmArgs {
  const uint16_t *A;  // A(m, k) = A[m * a_m + k * a_k]
  long a_m, a_k;
  const uint16_t *B;  // B(k, n) = B[k * b_k + n * b_n]
  long b_k, b_n;
  int M, N, K;
  int epi;
  const float *bias;  // [N]
  const float *Zin;   // [M x N] (DGELU)
  float *C;           // fp32 out, C[m * ldc + n]
  uint16_t *H;        // bf16 out, H[m * ldc + n]
  int ldc;
  // split contraction (EPI_STORE only): workgroup z sums k in [z * kc, (z + 1) * kc)
  // into C + z * c_split (fp32 partial sums, reduced afterwards)
  int kc;
  long c_split;
};

// Eight elements of an operand, p[e * stride] for e = 0..7, into LDS: one
// 16-byte load where they are contiguous (stride 1), in range and aligned,
// element by element (zero outside the operand) otherwise.  `ok(e)` says
// whether element e is in range; `dst(e)` is its LDS slot.
template <class InRange, class Dst>
__device__ __forceinline__ void stage8(const uint16_t *__restrict__ p, long stride, bool all_in, InRange ok, Dst dst) {
  if (stride == 1 && all_in && (((uintptr_t)p & 15u) == 0u)) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) dst(e) = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) dst(e) = ok(e) ? p[e * stride] : (uint16_t)0;
  }
}

// 128x128 tile of C per workgroup (256 threads = 4 waves, 64x64 each), 32 of
// the contraction per step: one v_mfma_f32_16x16x32_bf16 per 16x16 tile and
// step, in which lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] (e = 0..7) and gets D[4 (l / 16) + t][l % 16]
// (t = 0..3).  Each operand is staged along its contiguous axis with 16-byte
// loads and kept in LDS with the contraction contiguous ([m][k] and [n][k]),
// so a lane reads each 8-element fragment as one 16-byte word.
constexpr int TILE = 128;
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  constexpr int KS = 32, LDK = KS + 8;  // 80-byte LDS rows: 16-byte aligned, banks staggered
  __shared__ __align__(16) uint16_t As[TILE][LDK];
  __shared__ __align__(16) uint16_t Bs[TILE][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int kbeg = blockIdx.z * g.kc, kend = min(g.K, kbeg + g.kc);
  const bool a_kfast = g.a_k == 1, b_kfast = g.b_k == 1 && g.b_n != 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = kbeg; k0 < kend; k0 += KS) {
    // A (128 x 32): two chunks of 8 per thread, 128 rows x 4 chunks of k or 32 k x 16 chunks of m
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + 256 * h;
      if (a_kfast) {
        const int am = c >> 2, ak = (c & 3) * 8, m = m0 + am, k = k0 + ak;
        const uint16_t *p = g.A + (long)m * g.a_m + k;
        stage8(p, 1, m < g.M && k + 7 < kend, [&](int e) { return m < g.M && k + e < kend; },
               [&](int e) -> uint16_t & { return As[am][ak + e]; });
      } else {
        const int ak = c >> 4, am = (c & 15) * 8, m = m0 + am, k = k0 + ak;
        const uint16_t *p = g.A + (long)m * g.a_m + (long)k * g.a_k;
        stage8(p, g.a_m, k < kend && m + 7 < g.M, [&](int e) { return k < kend && m + e < g.M; },
               [&](int e) -> uint16_t & { return As[am + e][ak]; });
      }
    }
    // B (32 x 128): the same for 128 columns
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + 256 * h;
      if (b_kfast) {
        const int bn = c >> 2, bk = (c & 3) * 8, n = n0 + bn, k = k0 + bk;
        const uint16_t *p = g.B + (long)k + (long)n * g.b_n;
        stage8(p, 1, n < g.N && k + 7 < kend, [&](int e) { return n < g.N && k + e < kend; },
               [&](int e) -> uint16_t & { return Bs[bn][bk + e]; });
      } else {
        const int bk = c >> 4, bn = (c & 15) * 8, n = n0 + bn, k = k0 + bk;
        const uint16_t *p = g.B + (long)k * g.b_k + (long)n * g.b_n;
        stage8(p, g.b_n, k < kend && n + 7 < g.N, [&](int e) { return k < kend && n + e < g.N; },
               [&](int e) -> uint16_t & { return Bs[bn + e][bk]; });
      }
    }
    __syncthreads();
    const int r = lane & 15, q = lane >> 4;
    bf16x8 af[4], bfr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + r][8 * q]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * j + r][8 * q]);
    // the transposed tile, C^T = B^T A^T: B's fragment as the first operand
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // lane holds C[m][n + t] (t = 0..3), m = wm + 16 i + l % 16, n = wn + 16 j +
  // 4 (l / 16): four adjacent outputs of a row, stored as one 16-byte (fp32)
  // or 8-byte (bf16) word where the row stride and the buffers allow
  const int r = lane & 15, q = lane >> 4;
  const bool vec = (g.ldc & 3) == 0 && ((uintptr_t)g.C & 15u) == 0 && ((uintptr_t)g.H & 7u) == 0 &&
                   ((uintptr_t)g.Zin & 15u) == 0 && ((uintptr_t)g.bias & 15u) == 0;
  const float *out_bias = g.bias;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + wm + 16 * i + r, nb = n0 + wn + 16 * j + 4 * q;
      if (m >= g.M || nb >= g.N) continue;
      const long o = (long)m * g.ldc + nb;
      float v[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
      if (vec && nb + 3 < g.N) {
        if (g.epi == EPI_STORE) {
          *reinterpret_cast<float4 *>(g.C + o + blockIdx.z * g.c_split) = float4{v[0], v[1], v[2], v[3]};
        } else if (g.epi == EPI_BIAS) {
          const float4 b = *reinterpret_cast<const float4 *>(out_bias + nb);
          *reinterpret_cast<float4 *>(g.C + o) = float4{v[0] + b.x, v[1] + b.y, v[2] + b.z, v[3] + b.w};
        } else if (g.epi == EPI_BIAS_GELU) {
          const float4 b = *reinterpret_cast<const float4 *>(out_bias + nb);
          v[0] += b.x; v[1] += b.y; v[2] += b.z; v[3] += b.w;
          if (g.C) *reinterpret_cast<float4 *>(g.C + o) = float4{v[0], v[1], v[2], v[3]};
          *reinterpret_cast<uint2 *>(g.H + o) = uint2{f2bf2(gelu(v[0]), gelu(v[1])), f2bf2(gelu(v[2]), gelu(v[3]))};
        } else {
          const float4 z = *reinterpret_cast<const float4 *>(g.Zin + o);
          v[0] *= gelu_grad(z.x); v[1] *= gelu_grad(z.y); v[2] *= gelu_grad(z.z); v[3] *= gelu_grad(z.w);
          if (g.C) *reinterpret_cast<float4 *>(g.C + o) = float4{v[0], v[1], v[2], v[3]};
          *reinterpret_cast<uint2 *>(g.H + o) = uint2{f2bf2(v[0], v[1]), f2bf2(v[2], v[3])};
        }
        continue;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int n = nb + t;
        if (n >= g.N) continue;
        float x = v[t];
        if (g.epi == EPI_STORE) {
          g.C[o + t + blockIdx.z * g.c_split] = x;
        } else if (g.epi == EPI_BIAS) {
          g.C[o + t] = x + out_bias[n];
        } else if (g.epi == EPI_BIAS_GELU) {
          x += out_bias[n];
          if (g.C) g.C[o + t] = x;
          g.H[o + t] = f2bf(gelu(x));
        } else {
          x *= gelu_grad(g.Zin[o + t]);
          if (g.C) g.C[o + t] = x;
          g.H[o + t] = f2bf(x);
        }
      }
    }
}

hipError_t gemm(GemmArgs g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  g.kc = g.K;
  g.c_split = 0;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3((g.N + TILE - 1) / TILE, (g.M + TILE - 1) / TILE, 1), dim3(256), 0, s, g);
  return hipGetLastError();
}

// The whole network's inference over 128 rows per workgroup (256 threads = 4
// waves): the inputs standardised, three hidden layers and the output layer,
// the outputs de-standardised.  The activations stay in LDS (one bf16
// 128 x 256 buffer, 66 KB: two workgroups per CU), so HBM sees only x in and
// y out.  A layer computes its transpose, out^T (n x 128) = W H^T, with
// v_mfma_f32_16x16x32_bf16: the first operand is W (lane l holds
// W[n0 + l % 16][k0 + 8 (l / 16) + e], one 16-byte load from global memory,
// the same weights for every workgroup, so the caches serve them; the next
// step's are loaded ahead) and the second the activations
// (H[m0 + l % 16][k0 + 8 (l / 16) + e], one 16-byte read from LDS); lane l
// then holds out[m0 + l % 16][n0 + 4 (l / 16) + t] (t = 0..3), four adjacent
// outputs of one row, stored as one 8-byte word once every wave has read the
// layer's input.  Wave w takes the outputs 64 w .. 64 w + 63 of a hidden
// layer for all 128 rows (each weight fragment serves eight row tiles: the
// weights are read from the caches once per 128 rows), and rows
// 32 w .. 32 w + 31 of the output layer.  Per output the contraction runs in
// ascending 32-steps (the 16 inputs padded with zeros to one step), and the
// prologue and epilogues are the expressions of norm_in_kernel,
// gemm_bf16_kernel's bias / GELU epilogues and denorm_out_kernel.
constexpr int FT = 128, FLD = HID + 8, MT = FT / 16;  // rows per workgroup; LDS row stride in bf16 (528 B); row tiles
static_assert(w_off(1) % 8 == 0 && w_off(2) % 8 == 0 && w_off(3) % 8 == 0, "16-byte aligned weight blocks");
__device__ __forceinline__ bf16x8 ld16(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p)); }
__global__ void __launch_bounds__(256, 2) mlp_fused_kernel(const float *__restrict__ X, int n,
                                                        const float *__restrict__ norm,
                                                        const uint16_t *__restrict__ Pb,
                                                        const float *__restrict__ P, float *__restrict__ Y) {
  __shared__ __align__(16) uint16_t Hs[FT][FLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const long row0 = (long)blockIdx.x * FT;
  const bf16x8 zero8 = __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
  // standardised inputs in columns 0..15, zeros in 16..31; rows past n are zero
  for (int i = tid; i < FT * 32; i += 256) {
    const int m = i >> 5, c = i & 31;
    uint16_t v = 0;
    if (c < IN && row0 + m < n) v = f2bf((X[(row0 + m) * IN + c] - norm[c]) / norm[IN + c]);
    Hs[m][c] = v;
  }
  __syncthreads();
#pragma unroll 1
  for (int l = 0; l < NL - 1; ++l) {
    const int ni = l == 0 ? IN : HID, steps = (ni + 31) / 32;
    const uint16_t *__restrict__ W = Pb + w_off(l);
    const float *__restrict__ bias = P + b_off(l);
    const uint16_t(*Hin)[FLD] = Hs;
    uint16_t(*Hout)[FLD] = Hs;
    f32x4 acc[4][MT];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < MT; ++i) acc[j][i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 wf[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) wf[j] = 8 * q < ni ? ld16(W + (long)(64 * wave + 16 * j + r) * ni + 8 * q) : zero8;
#pragma unroll 1
    for (int ks = 0; ks < steps; ++ks) {
      const int k0 = 32 * ks;
      bf16x8 wn[4];  // the next step's weights, loaded ahead
      const bool more = ks + 1 < steps;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        wn[j] = more ? ld16(W + (long)(64 * wave + 16 * j + r) * ni + k0 + 32 + 8 * q) : zero8;
      bf16x8 hf[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) hf[i] = *reinterpret_cast<const bf16x8 *>(&Hin[16 * i + r][k0 + 8 * q]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < MT; ++i) acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j], hf[i], acc[j][i], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) wf[j] = wn[j];
    }
    __syncthreads();  // every wave has read the layer's input
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int nb = 64 * wave + 16 * j + 4 * q;
      const float b0 = bias[nb], b1 = bias[nb + 1], b2 = bias[nb + 2], b3 = bias[nb + 3];
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const uint32_t h01 = f2bf2(gelu(acc[j][i][0] + b0), gelu(acc[j][i][1] + b1));
        const uint32_t h23 = f2bf2(gelu(acc[j][i][2] + b2), gelu(acc[j][i][3] + b3));
        *reinterpret_cast<uint2 *>(&Hout[16 * i + r][nb]) = uint2{h01, h23};
      }
    }
    __syncthreads();
  }
  // output layer: 8 outputs, weight rows 8..15 of the 16-row operand are zero;
  // wave w takes the row tiles 2 w and 2 w + 1
  const uint16_t *__restrict__ W3 = Pb + w_off(NL - 1);
  const float *__restrict__ b3 = P + b_off(NL - 1);
#pragma unroll
  for (int h = 0; h < MT / 4; ++h) {
    const int mt = (MT / 4) * wave + h;
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < HID / 32; ++ks) {
      const int k0 = 32 * ks;
      const bf16x8 wf = r < OUT ? ld16(W3 + (long)r * HID + k0 + 8 * q) : zero8;
      const bf16x8 hf = *reinterpret_cast<const bf16x8 *>(&Hs[16 * mt + r][k0 + 8 * q]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, hf, acc, 0, 0, 0);
    }
    const long m = row0 + 16 * mt + r;
    if (q < 2 && m < n) {
      const float *mean = norm + 2 * IN, *sd = norm + 2 * IN + OUT;
      float y[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 4 * q + t;
        const float yn = acc[t] + b3[c];
        y[t] = yn * sd[c] + mean[c];
      }
      *reinterpret_cast<float4 *>(Y + m * OUT + 4 * q) = float4{y[0], y[1], y[2], y[3]};
    }
  }
}

// out[i] = sum over z of part[z * stride + i], z ascending (a fixed order, so
// the result does not depend on scheduling).
__global__ void reduce_splits_kernel(const float *__restrict__ part, int splits, long stride, long n,
                                     float *__restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
  for (int z = 0; z < splits; ++z) acc += part[(long)z * stride + i];
  out[i] = acc;
}

constexpr int MAX_SPLITS = 32;
constexpr int COLSUM_CHUNKS = 32;  // row chunks of the bias-gradient column sums (partials in the split buffer)
// C (M x N, ldc = N) = A B with a long contraction K: the K range is cut into
// up to MAX_SPLITS chunks of whole 32-steps so that small outputs (weight
// gradients) still spread over the chip; partial sums go to `part`
// (MAX_SPLITS x M x N floats) and are reduced in a fixed order.
hipError_t gemm_split(GemmArgs g, float *part, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int tiles = ((g.N + TILE - 1) / TILE) * ((g.M + TILE - 1) / TILE);
  int splits = std::max(1, std::min(MAX_SPLITS, 512 / tiles));
  g.kc = ((g.K + splits - 1) / splits + 31) / 32 * 32;
  splits = std::max(1, (g.K + g.kc - 1) / g.kc);
  float *out = g.C;
  g.C = part;
  g.c_split = (long)g.M * g.ldc;
  g.epi = EPI_STORE;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3((g.N + TILE - 1) / TILE, (g.M + TILE - 1) / TILE, splits), dim3(256), 0,
                     s, g);
  const long n = (long)g.M * g.ldc;
  hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, splits, n, n, out);
  return hipGetLastError();
}

// ---- small elementwise / reduction kernels ----

__global__ void fill_kernel(float *p, long n, float v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// x -> bf16((x - mean) / std), n x 16
__global__ void norm_in_kernel(const float *__restrict__ X, int n, const float *__restrict__ mean,
                               const float *__restrict__ sd, uint16_t *__restrict__ Xn) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * IN) return;
  const int c = (int)(i % IN);
  Xn[i] = f2bf((X[i] - mean[c]) / sd[c]);
}

// y = yn * std + mean, n x 8
__global__ void denorm_out_kernel(const float *__restrict__ Yn, int n, const float *__restrict__ mean,
                                  const float *__restrict__ sd, float *__restrict__ Y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * OUT) return;
  const int c = (int)(i % OUT);
  Y[i] = Yn[i] * sd[c] + mean[c];
}

// dL/dy_n for the mean squared error on normalised targets, its BF16 copy, and
// the per-row squared error (summed by the loss kernel).
__global__ void mse_grad_kernel(const float *__restrict__ Yn, const float *__restrict__ T, int n,
                                const float *__restrict__ mean, const float *__restrict__ sd,
                                float *__restrict__ dY, uint16_t *__restrict__ dYb, float *__restrict__ sq) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * OUT) return;
  const int c = (int)(i % OUT);
  const float e = Yn[i] - (T[i] - mean[c]) / sd[c];
  const float g = 2.0f * e / ((float)n * (float)OUT);
  dY[i] = g;
  dYb[i] = f2bf(g);
  sq[i] = e * e;
}

// Deterministic sum of v[0..n) / scale into *out (one workgroup).
__global__ void __launch_bounds__(1024) sum_kernel(const float *__restrict__ v, long n, float scale,
                                                   float *__restrict__ out) {
  __shared__ double part[1024];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += 1024) s += (double)v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)(part[0] / (double)scale);
}

// Column sums (bias gradients), first of two deterministic stages:
// part[z * cols + c] = sum of M[r * cols + c] over the rows r of chunk z
// (chunks of ceil(rows / gridDim.y) rows).  A 256-thread block covers 64
// columns of one chunk: thread (x, y) sums rows y, y + 4, ... of the chunk in
// column x (neighbouring threads read neighbouring columns), then the four
// partial sums are added in order.  reduce_splits_kernel adds the chunks in
// ascending z.
__global__ void __launch_bounds__(256) colsum_part_kernel(const float *__restrict__ M, int rows, int cols,
                                                          float *__restrict__ part) {
  __shared__ float p4[4][64];
  const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + x;
  const int chunk = (rows + gridDim.y - 1) / gridDim.y, r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float acc = 0.0f;
  if (c < cols)
    for (int r = r0 + y; r < r1; r += 4) acc += M[(long)r * cols + c];
  p4[y][x] = acc;
  __syncthreads();
  if (y == 0 && c < cols) part[(long)blockIdx.y * cols + c] = ((p4[0][x] + p4[1][x]) + p4[2][x]) + p4[3][x];
}

// Adam (Kingma & Ba) with bias correction; refreshes the BF16 weight copy.
__global__ void adam_kernel(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ Pb, long n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  P[i] = p;
  Pb[i] = f2bf(p);
}

__global__ void to_bf16_kernel(const float *__restrict__ P, uint16_t *__restrict__ Pb, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Pb[i] = f2bf(P[i]);
}

// Mean and standard deviation of each column of M (rows x cols), FP64 sums.
__global__ void colstats_kernel(const float *__restrict__ M, long rows, int cols, float *__restrict__ mean,
                                float *__restrict__ sd) {
  const int c = blockIdx.x;
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (long r = threadIdx.x; r < rows; r += 256) {
    const double x = M[r * cols + c];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)rows;
    const double var = s2[0] / (double)rows - mu * mu;
    mean[c] = (float)mu;
    sd[c] = (float)sqrt(var > 1e-12 ? var : 1e-12);
  }
}

// Training minibatch: rows (a * (j0 + r) + c) mod N of X and Y (an affine
// permutation of the dataset, a coprime to N).
__global__ void gather_batch_kernel(const float *__restrict__ X, const float *__restrict__ Y, long N, long a, long c,
                                    long j0, int rows, float *__restrict__ Xb, float *__restrict__ Yb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)rows * (IN + OUT)) return;
  const long r = i / (IN + OUT);
  const int col = (int)(i % (IN + OUT));
  // a, j0 + r < N <= 2^24 (checked on the host), so the product fits in 64 bits
  const long src = (long)(((unsigned long long)a * (unsigned long long)(j0 + r) + (unsigned long long)c) %
                          (unsigned long long)N);
  if (col < IN) Xb[r * IN + col] = X[src * IN + col];
  else Yb[r * OUT + (col - IN)] = Y[src * OUT + (col - IN)];
}

// ---- screening -------------------------------------------------------------

__device__ __forceinline__ uint32_t ordered(float c) {
  if (c != c) c = __int_as_float(0x7F800000);
  if (c == 0.0f) c = 0.0f;
  const uint32_t b = __float_as_uint(c);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Screening key of candidate i: (goal predicted to fail, predicted cost, i).
// The goal test is the plan's psi_g (object on the goal table's top face)
// applied to the predicted final pose; without a goal table it always holds.
__global__ void screen_keys_kernel(const float *__restrict__ Y, int n, const DevState *__restrict__ st,
                                   uint64_t *__restrict__ keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cem_scene &sc = st->scene;
  const float *y = Y + (long)i * OUT;
  uint64_t miss = 0;
  if (sc.kind == CEM_SCENE_PICKPLACE && sc.goal_static >= 0 && sc.goal_static < sc.n_static) {
    const int b = sc.goal_static;
    const float top = sc.st_center[b][2] + sc.st_half[b][2];
    const bool goal = fabsf(y[1] - sc.st_center[b][0]) <= sc.st_half[b][0] &&
                      fabsf(y[2] - sc.st_center[b][1]) <= sc.st_half[b][1] && y[3] >= top - sc.obj_half[2] &&
                      y[3] <= top + 3.0f * sc.obj_half[2];
    miss = goal ? 0 : 1;
  }
  keys[i] = (miss << 62) | ((uint64_t)ordered(y[0]) << 30) | (uint64_t)i;
}

// The k smallest of n unique keys, listed in index order: an 8-pass MSB radix
// select of the k-th key with LDS histograms, then an order-preserving
// compaction (per-thread contiguous chunks, block prefix sum).  One workgroup.
__global__ void __launch_bounds__(1024) topk_kernel(const uint64_t *__restrict__ keys, int n, int k,
                                                    int32_t *__restrict__ sel) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long prefix_s, mask_s;
  __shared__ int rank_s;
  __shared__ int scan[1024];
  const int tid = threadIdx.x;
  if (tid == 0) {
    prefix_s = 0;
    mask_s = 0;
    rank_s = k;
  }
  __syncthreads();
  for (int shift = 56; shift >= 0; shift -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    const unsigned long long prefix = prefix_s, mask = mask_s;
    for (int i = tid; i < n; i += 1024) {
      const unsigned long long key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      const int rank = rank_s;
      unsigned cum = 0;
      for (int b = 0; b < 256; ++b) {
        if (cum + hist[b] >= (unsigned)rank) {
          prefix_s = prefix | ((unsigned long long)b << shift);
          rank_s = rank - (int)cum;
          break;
        }
        cum += hist[b];
      }
      mask_s = mask | (255ull << shift);
    }
    __syncthreads();
  }
  const unsigned long long thr = prefix_s;
  const int chunk = (n + 1023) / 1024;
  const int lo = tid * chunk, hi = min(n, lo + chunk);
  int cnt = 0;
  for (int i = lo; i < hi; ++i) cnt += keys[i] <= thr ? 1 : 0;
  scan[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan (Hillis-Steele)
    const int v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int out = scan[tid] - cnt;
  for (int i = lo; i < hi; ++i)
    if (keys[i] <= thr && out < k) sel[out++] = i;
}

__global__ void gather_rows_kernel(const float *__restrict__ Z, int D, const float *__restrict__ Y,
                                   const int32_t *__restrict__ sel, int k, float *__restrict__ Zs,
                                   float *__restrict__ Ys) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const long s = sel[j];
  for (int d = 0; d < D; ++d) Zs[(long)j * D + d] = Z[s * D + d];
  if (Ys)
    for (int c = 0; c < OUT; ++c) Ys[(long)j * OUT + c] = Y[s * OUT + c];
}

// Surrogate error of one screened iteration: mean |predicted - simulated| cost
// over the simulated rows with a finite cost.
__global__ void __launch_bounds__(256) screen_error_kernel(const float *__restrict__ pred, const float *__restrict__ cost,
                                                           int k, const DevState *__restrict__ st,
                                                           float *__restrict__ err, int cap) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < k; j += 256) {
    const float c = cost[j];
    if (isfinite(c)) {
      a += fabs((double)pred[(long)j * OUT] - (double)c);
      b += 1.0;
    }
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  const int it = st->iter;  // read before the refit of this iteration advances it
  if (threadIdx.x == 0 && it >= 0 && it < cap) err[it] = s2[0] > 0.0 ? (float)(s1[0] / s2[0]) : -1.0f;
}

}  // namespace
}  // namespace cem

// ---- host side ---------------------------------------------------------------

namespace cem {
namespace {

// Work buffers of cem_mlp_forward_static, for callers that cannot allocate:
// standardised inputs (bf16, rows x 16), two hidden-layer buffers used in
// turn (bf16, rows x 256 each) and the standardised outputs (fp32, rows x 8),
// for up to CEM_MLP_STATIC_ROWS rows: 8.5 MiB, held by every device the
// library runs on until the process ends.  Every region starts on a 256-byte
// boundary.  Each call writes every element it reads, so nothing needs
// clearing between calls.
constexpr size_t SC_ROWS = CEM_MLP_STATIC_ROWS;
constexpr size_t SC_XN = 0;
constexpr size_t SC_H0 = SC_XN + SC_ROWS * IN * sizeof(uint16_t);
constexpr size_t SC_H1 = SC_H0 + SC_ROWS * HID * sizeof(uint16_t);
constexpr size_t SC_YN = SC_H1 + SC_ROWS * HID * sizeof(uint16_t);
constexpr size_t SC_BYTES = SC_YN + SC_ROWS * OUT * sizeof(float);
static_assert(SC_H0 % 256 == 0 && SC_H1 % 256 == 0 && SC_YN % 256 == 0, "256-byte aligned regions");

__device__ __align__(256) unsigned char scratch[SC_BYTES];

// The array's device address on each device (each device holds its own copy
// at its own address).  Host code uses only these addresses: the array's name
// in host code is not a device address.
std::mutex scratch_mu;
std::vector<void *> scratch_addr;

// Looks up (once per device, with that device current) and returns the
// current device's copy of the array; nullptr and *err set on failure.
void *scratch_on_current_device(hipError_t *err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if ((size_t)dev >= scratch_addr.size()) scratch_addr.resize((size_t)dev + 1, nullptr);
  if (!scratch_addr[dev]) {
    void *p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    scratch_addr[dev] = p;
  }
  return scratch_addr[dev];
}

}  // namespace
}  // namespace cem

using namespace cem;

struct cem_mlp {
  int max_rows = 0;
  float *P = nullptr, *G = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *Pb = nullptr;
  float *norm = nullptr;  // x_mean[16] x_std[16] y_mean[8] y_std[8]
  uint16_t *Xn = nullptr, *H[3] = {nullptr, nullptr, nullptr}, *dYb = nullptr, *dZb[2] = {nullptr, nullptr};
  float *Zp[3] = {nullptr, nullptr, nullptr}, *Yn = nullptr, *dY = nullptr, *sq = nullptr, *dZf = nullptr;
  float *Ypred = nullptr, *loss = nullptr, *Xb = nullptr, *Yb = nullptr, *Zs = nullptr, *Ps = nullptr;
  float *err = nullptr;
  float *part = nullptr;  // split-contraction partial sums (MAX_SPLITS x 256 x 256)
  uint64_t *keys = nullptr;
  int32_t *sel = nullptr;
  int step = 0;
  hipStream_t own = nullptr;
  hipGraphExec_t screen_graph = nullptr;
  uint64_t graph_serial = 0;  // the context the screened-iteration graph was captured for
  int graph_nsim = 0;
  std::string err_text;
};

namespace {

int mfail(cem_mlp *m, int code, const std::string &msg) {
  if (m) m->err_text = msg;
  return code;
}
#define MHIPCHK(m, expr)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return mfail(m, CEM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

unsigned blocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

GemmArgs gargs(const uint16_t *A, long a_m, long a_k, const uint16_t *B, long b_k, long b_n, int M, int N, int K,
               int epi, const float *bias, const float *Zin, float *C, uint16_t *H, int ldc) {
  GemmArgs g;
  g.A = A; g.a_m = a_m; g.a_k = a_k;
  g.B = B; g.b_k = b_k; g.b_n = b_n;
  g.M = M; g.N = N; g.K = K; g.epi = epi;
  g.bias = bias; g.Zin = Zin; g.C = C; g.H = H; g.ldc = ldc;
  return g;
}

// Forward pass of n rows of raw parameters X; keeps the pre-activations when
// `train`; leaves normalised outputs in m->Yn.
hipError_t forward_n(cem_mlp *m, const float *X, int n, bool train, hipStream_t s) {
  hipLaunchKernelGGL(norm_in_kernel, dim3(blocks((long)n * IN, 256)), dim3(256), 0, s, X, n, m->norm, m->norm + IN,
                     m->Xn);
  const uint16_t *in = m->Xn;
  long a_m = IN;
  for (int l = 0; l < NL; ++l) {
    const int ni = DIMS[l], no = DIMS[l + 1];
    const uint16_t *W = m->Pb + w_off(l);  // W[o][i]: B(k = i, n = o) = W[o * ni + i]
    const float *bias = m->P + b_off(l);
    GemmArgs g;
    if (l < NL - 1)
      g = gargs(in, a_m, 1, W, 1, ni, n, no, ni, EPI_BIAS_GELU, bias, nullptr, train ? m->Zp[l] : nullptr, m->H[l], no);
    else
      g = gargs(in, a_m, 1, W, 1, ni, n, no, ni, EPI_BIAS, bias, nullptr, m->Yn, nullptr, no);
    hipError_t e = gemm(g, s);
    if (e != hipSuccess) return e;
    if (l < NL - 1) {
      in = m->H[l];
      a_m = no;
    }
  }
  return hipGetLastError();
}

// Loss and gradient (into m->G) of the mean squared error on normalised targets.
hipError_t loss_grad_n(cem_mlp *m, const float *X, const float *T, int n, hipStream_t s) {
  hipError_t e = forward_n(m, X, n, true, s);
  if (e != hipSuccess) return e;
  const float *ym = m->norm + 2 * IN, *ys = m->norm + 2 * IN + OUT;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks((long)n * OUT, 256)), dim3(256), 0, s, m->Yn, T, n, ym, ys, m->dY,
                     m->dYb, m->sq);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, m->sq, (long)n * OUT, (float)n * (float)OUT, m->loss);
  // output layer
  const uint16_t *Hin[NL] = {m->Xn, m->H[0], m->H[1], m->H[2]};
  const uint16_t *dZ = m->dYb;
  const float *dZf = m->dY;
  int nz = OUT;
  for (int l = NL - 1; l >= 0; --l) {
    const int ni = DIMS[l];
    // dW_l[o][i] = sum_b dZ[b][o] Hin[b][i]
    e = gemm_split(gargs(dZ, 1, nz, Hin[l], ni, 1, nz, ni, n, EPI_STORE, nullptr, nullptr, m->G + w_off(l), nullptr, ni),
                   m->part, s);
    if (e != hipSuccess) return e;
    // bias gradient: column sums of dZ in COLSUM_CHUNKS row chunks, then the chunks in order
    hipLaunchKernelGGL(colsum_part_kernel, dim3((nz + 63) / 64, COLSUM_CHUNKS), dim3(256), 0, s, dZf, n, nz, m->part);
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(blocks(nz, 256)), dim3(256), 0, s, m->part, COLSUM_CHUNKS, (long)nz,
                       (long)nz, m->G + b_off(l));
    if (l == 0) break;
    // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
    uint16_t *out = m->dZb[(NL - 1 - l) & 1];
    e = gemm(gargs(dZ, nz, 1, m->Pb + w_off(l), ni, 1, n, ni, nz, EPI_DGELU, nullptr, m->Zp[l - 1], m->dZf, out, ni), s);
    if (e != hipSuccess) return e;
    dZ = out;
    dZf = m->dZf;
    nz = ni;
  }
  return hipGetLastError();
}

void mlp_release(cem_mlp *m) {
  if (m->screen_graph) (void)hipGraphExecDestroy(m->screen_graph);
  if (m->own) (void)hipStreamDestroy(m->own);
  void *ptrs[] = {m->P, m->G, m->m, m->v, m->Pb, m->norm, m->Xn, m->H[0], m->H[1], m->H[2], m->dYb, m->dZb[0],
                  m->dZb[1], m->Zp[0], m->Zp[1], m->Zp[2], m->Yn, m->dY, m->sq, m->dZf, m->Ypred, m->loss,
                  m->Xb, m->Yb, m->Zs, m->Ps, m->err, m->part, m->keys, m->sel};
  for (void *p : ptrs) (void)hipFree(p);
}

}  // namespace

extern "C" {

int cem_mlp_n_params(void) { return (int)N_PARAMS; }

const char *cem_mlp_last_error(const cem_mlp *m) { return m ? m->err_text.c_str() : "null network"; }

int cem_mlp_init(uint64_t seed, int32_t max_rows, cem_mlp **out) {
  if (!out) return CEM_E_ARG;
  *out = nullptr;
  if (max_rows < 1 || max_rows > (1 << 22)) return CEM_E_ARG;
  cem_mlp *m = new (std::nothrow) cem_mlp();
  if (!m) return CEM_E_ALLOC;
  m->max_rows = max_rows;
  const size_t R = (size_t)max_rows;
  bool ok = hipStreamCreateWithFlags(&m->own, hipStreamNonBlocking) == hipSuccess;
  auto alloc = [&](void **p, size_t bytes) { ok = ok && hipMalloc(p, bytes) == hipSuccess; };
  alloc((void **)&m->P, sizeof(float) * N_PARAMS);
  alloc((void **)&m->G, sizeof(float) * N_PARAMS);
  alloc((void **)&m->m, sizeof(float) * N_PARAMS);
  alloc((void **)&m->v, sizeof(float) * N_PARAMS);
  alloc((void **)&m->Pb, sizeof(uint16_t) * N_PARAMS);
  alloc((void **)&m->norm, sizeof(float) * (2 * IN + 2 * OUT));
  alloc((void **)&m->Xn, sizeof(uint16_t) * R * IN);
  for (int l = 0; l < 3; ++l) {
    alloc((void **)&m->H[l], sizeof(uint16_t) * R * HID);
    alloc((void **)&m->Zp[l], sizeof(float) * R * HID);
  }
  alloc((void **)&m->dZb[0], sizeof(uint16_t) * R * HID);
  alloc((void **)&m->dZb[1], sizeof(uint16_t) * R * HID);
  alloc((void **)&m->dZf, sizeof(float) * R * HID);
  alloc((void **)&m->dYb, sizeof(uint16_t) * R * OUT);
  alloc((void **)&m->Yn, sizeof(float) * R * OUT);
  alloc((void **)&m->dY, sizeof(float) * R * OUT);
  alloc((void **)&m->sq, sizeof(float) * R * OUT);
  alloc((void **)&m->Ypred, sizeof(float) * R * OUT);
  alloc((void **)&m->loss, sizeof(float));
  alloc((void **)&m->Xb, sizeof(float) * R * IN);
  alloc((void **)&m->Yb, sizeof(float) * R * OUT);
  alloc((void **)&m->Zs, sizeof(float) * R * IN);
  alloc((void **)&m->Ps, sizeof(float) * R * OUT);
  alloc((void **)&m->err, sizeof(float) * MAX_STATS_ITERS);
  alloc((void **)&m->part, sizeof(float) * MAX_SPLITS * HID * HID);
  alloc((void **)&m->keys, sizeof(uint64_t) * R);
  alloc((void **)&m->sel, sizeof(int32_t) * R);
  if (!ok) {
    mlp_release(m);
    delete m;
    return CEM_E_ALLOC;
  }
  hipError_t se = hipSuccess;
  if (!scratch_on_current_device(&se)) {  // set-up of cem_mlp_forward_static on this device
    mlp_release(m);
    delete m;
    return CEM_E_HIP;
  }
  long w0[4], nw[4];
  int fan[4];
  for (int l = 0; l < 4; ++l) {
    w0[l] = w_off(l);
    nw[l] = (long)DIMS[l] * DIMS[l + 1];
    fan[l] = DIMS[l];
  }
  hipStream_t s = m->own;
  bool k = launch_mlp_init(seed, w0, nw, fan, N_PARAMS, m->P, s) == hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, s, m->m, N_PARAMS, 0.0f);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, s, m->v, N_PARAMS, 0.0f);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, m->norm, (long)IN, 0.0f);          // x mean 0
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, m->norm + IN, (long)IN, 1.0f);     // x std 1
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, m->norm + 2 * IN, (long)OUT, 0.0f);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, m->norm + 2 * IN + OUT, (long)OUT, 1.0f);
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, s, m->P, m->Pb, N_PARAMS);
  k = k && hipStreamSynchronize(s) == hipSuccess;
  if (!k) {
    mlp_release(m);
    delete m;
    return CEM_E_HIP;
  }
  *out = m;
  return CEM_OK;
}

void cem_mlp_free(cem_mlp *m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->own);
  mlp_release(m);
  delete m;
}

int cem_mlp_get_params(cem_mlp *m, float *host) {
  if (!m || !host) return CEM_E_ARG;
  MHIPCHK(m, hipMemcpy(host, m->P, sizeof(float) * N_PARAMS, hipMemcpyDeviceToHost));
  return CEM_OK;
}

int cem_mlp_set_params(cem_mlp *m, const float *host) {
  if (!m || !host) return CEM_E_ARG;
  MHIPCHK(m, hipMemcpy(m->P, host, sizeof(float) * N_PARAMS, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, m->own, m->P, m->Pb, N_PARAMS);
  MHIPCHK(m, hipStreamSynchronize(m->own));
  return CEM_OK;
}

int cem_mlp_get_norm(cem_mlp *m, float *host48) {
  if (!m || !host48) return CEM_E_ARG;
  MHIPCHK(m, hipMemcpy(host48, m->norm, sizeof(float) * (2 * IN + 2 * OUT), hipMemcpyDeviceToHost));
  return CEM_OK;
}

int cem_mlp_set_norm(cem_mlp *m, const float *host48) {
  if (!m || !host48) return CEM_E_ARG;
  for (int i = 0; i < IN; ++i)
    if (!(host48[IN + i] > 0.0f)) return mfail(m, CEM_E_ARG, "input std must be positive");
  for (int i = 0; i < OUT; ++i)
    if (!(host48[2 * IN + OUT + i] > 0.0f)) return mfail(m, CEM_E_ARG, "target std must be positive");
  MHIPCHK(m, hipMemcpy(m->norm, host48, sizeof(float) * (2 * IN + 2 * OUT), hipMemcpyHostToDevice));
  return CEM_OK;
}

int cem_mlp_fit_norm(cem_mlp *m, const float *X_dev, const float *Y_dev, int64_t n, void *stream) {
  if (!m || !X_dev || !Y_dev || n < 1) return CEM_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(colstats_kernel, dim3(IN), dim3(256), 0, s, X_dev, (long)n, IN, m->norm, m->norm + IN);
  hipLaunchKernelGGL(colstats_kernel, dim3(OUT), dim3(256), 0, s, Y_dev, (long)n, OUT, m->norm + 2 * IN,
                     m->norm + 2 * IN + OUT);
  MHIPCHK(m, hipGetLastError());
  return CEM_OK;
}

int cem_mlp_forward(cem_mlp *m, const float *X_dev, int32_t n, float *Y_dev, void *stream) {
  if (!m) return CEM_E_ARG;
  if (n < 0 || n > m->max_rows) return mfail(m, CEM_E_ARG, "n out of range [0, max_rows]");
  if (n == 0) return CEM_OK;
  if (!X_dev || !Y_dev) return mfail(m, CEM_E_ARG, "null buffer");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(mlp_fused_kernel, dim3(blocks(n, FT)), dim3(256), 0, s, X_dev, n, m->norm, m->Pb, m->P, Y_dev);
  MHIPCHK(m, hipGetLastError());
  return CEM_OK;
}

int cem_mlp_forward_static(cem_mlp *m, const float *X_dev, int32_t n, float *Y_dev, void *stream) {
  if (!m) return CEM_E_ARG;
  if (n < 0 || n > CEM_MLP_STATIC_ROWS)
    return mfail(m, CEM_E_ARG, "n out of range [0, CEM_MLP_STATIC_ROWS = 8192] of the fixed work buffers");
  if (n == 0) return CEM_OK;
  if (!X_dev || !Y_dev) return mfail(m, CEM_E_ARG, "null buffer");
  hipError_t e = hipSuccess;
  unsigned char *scr = (unsigned char *)scratch_on_current_device(&e);
  if (!scr) return mfail(m, CEM_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  uint16_t *Xn = (uint16_t *)(scr + SC_XN);
  uint16_t *Hs[2] = {(uint16_t *)(scr + SC_H0), (uint16_t *)(scr + SC_H1)};
  float *Yn = (float *)(scr + SC_YN);
  hipStream_t s = (hipStream_t)stream;
  // the layers of forward_n, the hidden activations alternating between the
  // two buffers (a layer reads one and writes the other)
  hipLaunchKernelGGL(norm_in_kernel, dim3(blocks((long)n * IN, 256)), dim3(256), 0, s, X_dev, n, m->norm,
                     m->norm + IN, Xn);
  const uint16_t *in = Xn;
  long a_m = IN;
  for (int l = 0; l < NL; ++l) {
    const int ni = DIMS[l], no = DIMS[l + 1];
    const uint16_t *W = m->Pb + w_off(l);
    const float *bias = m->P + b_off(l);
    GemmArgs g;
    if (l < NL - 1)
      g = gargs(in, a_m, 1, W, 1, ni, n, no, ni, EPI_BIAS_GELU, bias, nullptr, nullptr, Hs[l & 1], no);
    else
      g = gargs(in, a_m, 1, W, 1, ni, n, no, ni, EPI_BIAS, bias, nullptr, Yn, nullptr, no);
    MHIPCHK(m, gemm(g, s));
    if (l < NL - 1) {
      in = Hs[l & 1];
      a_m = no;
    }
  }
  hipLaunchKernelGGL(denorm_out_kernel, dim3(blocks((long)n * OUT, 256)), dim3(256), 0, s, Yn, n, m->norm + 2 * IN,
                     m->norm + 2 * IN + OUT, Y_dev);
  MHIPCHK(m, hipGetLastError());
  return CEM_OK;
}

int cem_mlp_loss_grad(cem_mlp *m, const float *X_dev, const float *Y_dev, int32_t n, float *grad_dev, float *loss_dev,
                      void *stream) {
  if (!m) return CEM_E_ARG;
  if (n < 1 || n > m->max_rows) return mfail(m, CEM_E_ARG, "n out of range [1, max_rows]");
  if (!X_dev || !Y_dev) return mfail(m, CEM_E_ARG, "null buffer");
  hipStream_t s = (hipStream_t)stream;
  MHIPCHK(m, loss_grad_n(m, X_dev, Y_dev, n, s));
  if (grad_dev) MHIPCHK(m, hipMemcpyAsync(grad_dev, m->G, sizeof(float) * N_PARAMS, hipMemcpyDeviceToDevice, s));
  if (loss_dev) MHIPCHK(m, hipMemcpyAsync(loss_dev, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
  return CEM_OK;
}

int cem_mlp_train_step(cem_mlp *m, const float *X_dev, const float *Y_dev, int32_t n, float lr, float *loss_dev,
                       void *stream) {
  int rc = cem_mlp_loss_grad(m, X_dev, Y_dev, n, nullptr, loss_dev, stream);
  if (rc != CEM_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  m->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, m->step)), c2 = (float)(1.0 - std::pow(b2, m->step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, s, m->P, m->G, m->m, m->v, m->Pb,
                     N_PARAMS, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  MHIPCHK(m, hipGetLastError());
  return CEM_OK;
}

int cem_mlp_train(cem_mlp *m, const float *X_dev, const float *Y_dev, int64_t n, int32_t batch, int32_t epochs,
                  float lr, uint64_t seed, float *epoch_loss_host) {
  if (!m || !X_dev || !Y_dev) return CEM_E_ARG;
  if (n < 1 || n > (1 << 24) || batch < 1 || batch > m->max_rows || epochs < 0)
    return mfail(m, CEM_E_ARG, "bad sizes");
  hipStream_t s = nullptr;  // the null stream: ordered after the caller's earlier work on it
  const long steps = (long)(n / batch);
  if (steps < 1) return mfail(m, CEM_E_ARG, "dataset smaller than one batch");
  std::vector<float> losses(steps);
  float *dloss = nullptr;
  MHIPCHK(m, hipMalloc(&dloss, sizeof(float) * steps));
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {  // splitmix64 for the epoch's shuffle parameters
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto gcd = [](uint64_t a, uint64_t b) {
    while (b) {
      const uint64_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  int rc = CEM_OK;
  for (int e = 0; e < epochs && rc == CEM_OK; ++e) {
    uint64_t a = next() % (uint64_t)n;
    while (a == 0 || gcd(a, (uint64_t)n) != 1) a = (a + 1) % (uint64_t)n;
    const uint64_t c = next() % (uint64_t)n;
    for (long j = 0; j < steps && rc == CEM_OK; ++j) {
      hipLaunchKernelGGL(gather_batch_kernel, dim3(blocks((long)batch * (IN + OUT), 256)), dim3(256), 0, s, X_dev,
                         Y_dev, (long)n, (long)a, (long)c, j * (long)batch, batch, m->Xb, m->Yb);
      rc = cem_mlp_train_step(m, m->Xb, m->Yb, batch, lr, dloss + j, s);
    }
    if (rc == CEM_OK && epoch_loss_host) {
      if (hipMemcpyAsync(losses.data(), dloss, sizeof(float) * steps, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = mfail(m, CEM_E_HIP, "loss copy");
        break;
      }
      double acc = 0.0;
      for (float v : losses) acc += v;
      epoch_loss_host[e] = (float)(acc / (double)steps);
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(dloss);
  return rc;
}

// One screening pass: sample the context's population (iteration iter, or the
// device counter when iter < 0), predict every candidate, keep the n_sim with
// the smallest (goal predicted to fail, predicted cost, index) keys, written
// in index order to Zsim (n_sim x D) and their predictions to pred (n_sim x 8).
static int screen_into(cem_ctx *c, cem_mlp *m, int32_t iter, int32_t n_sim, float *Zsim, float *pred, hipStream_t s) {
  hipError_t e = launch_sample(c->seed, c->inst, iter, c->st, c->pop, c->D, c->Z, s);
  if (e != hipSuccess) return mfail(m, CEM_E_HIP, "sample");
  hipLaunchKernelGGL(mlp_fused_kernel, dim3(blocks(c->pop, FT)), dim3(256), 0, s, c->Z, c->pop, m->norm, m->Pb, m->P,
                     m->Ypred);
  hipLaunchKernelGGL(screen_keys_kernel, dim3(blocks(c->pop, 256)), dim3(256), 0, s, m->Ypred, c->pop, c->st, m->keys);
  hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(1024), 0, s, m->keys, c->pop, n_sim, m->sel);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks(n_sim, 256)), dim3(256), 0, s, c->Z, c->D, m->Ypred, m->sel,
                     n_sim, Zsim, pred);
  e = hipGetLastError();
  return e == hipSuccess ? CEM_OK : mfail(m, CEM_E_HIP, "screen launch");
}

int cem_screen(cem_ctx *c, cem_mlp *m, int32_t iter, int32_t n_sim, float *Zsim_dev, float *pred_dev, void *stream) {
  if (!c || !m) return CEM_E_ARG;
  if (c->D != IN) return mfail(m, CEM_E_ARG, "the network takes 16 parameters");
  if (c->pop > m->max_rows) return mfail(m, CEM_E_ARG, "population exceeds the network's max_rows");
  if (n_sim < 1 || n_sim > c->pop) return mfail(m, CEM_E_ARG, "n_sim out of range [1, pop]");
  if (!Zsim_dev || iter < 0) return mfail(m, CEM_E_ARG, "null Zsim or iter < 0");
  return screen_into(c, m, iter, n_sim, Zsim_dev, pred_dev, (hipStream_t)stream);
}

int plan_solve_screened(cem_ctx *c, cem_mlp *m, int32_t iters, int32_t n_sim, cem_result *res, float *stats_host,
                        float *surrogate_err_host, void *stream) {
  if (!c || !m || !res) return CEM_E_ARG;
  if (c->D != IN) return mfail(m, CEM_E_ARG, "the network takes 16 parameters");
  if (c->pop > m->max_rows) return mfail(m, CEM_E_ARG, "population exceeds the network's max_rows");
  if (n_sim < 1 || n_sim > c->pop || n_sim < c->n_elite) return mfail(m, CEM_E_ARG, "n_sim out of range [n_elite, pop]");
  if (iters < 0) return mfail(m, CEM_E_ARG, "iters < 0");
  hipStream_t s = (hipStream_t)stream;
  int32_t it0 = 0;
  MHIPCHK(m, hipMemcpyAsync(&it0, &c->st->iter, sizeof it0, hipMemcpyDeviceToHost, s));
  MHIPCHK(m, hipStreamSynchronize(s));
  if (it0 + iters > MAX_STATS_ITERS) return mfail(m, CEM_E_ARG, "iteration counter would exceed 4096");
  // the graph holds the context's device buffers: reuse it only for that same
  // context (its serial, not its address, which a later context can reuse)
  if (!m->screen_graph || m->graph_serial != c->serial || m->graph_nsim != n_sim) {
    if (m->screen_graph) (void)hipGraphExecDestroy(m->screen_graph);
    m->screen_graph = nullptr;
    hipGraph_t g = nullptr;
    MHIPCHK(m, hipStreamBeginCapture(m->own, hipStreamCaptureModeThreadLocal));
    int rc = screen_into(c, m, -1, n_sim, m->Zs, m->Ps, m->own);
    InstDesc d{};
    d.st = c->st; d.Z = m->Zs; d.cost = c->cost; d.tier = c->tier; d.pose = nullptr; d.stats = c->stats;
    d.kind = c->scene.kind; d.pop = n_sim; d.D = c->D; d.iters = 1 << 30; d.scen = scenarios(c->scene);
    d.lanes = c->lanes;
    d.spec = robot_spec_for(c->scene) ? 1 : 0;
    hipError_t e2 = launch_rollout_single(d, nullptr, 0, m->own);
    hipLaunchKernelGGL(screen_error_kernel, dim3(1), dim3(256), 0, m->own, m->Ps, c->cost, n_sim, c->st, m->err,
                       MAX_STATS_ITERS);
    hipError_t e3 = launch_select_refit(c->st, m->Zs, c->cost, c->tier, n_sim, nullptr, nullptr, c->stats,
                                        MAX_STATS_ITERS, 1, m->own);
    hipError_t e4 = hipStreamEndCapture(m->own, &g);
    if (rc != CEM_OK || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return mfail(m, CEM_E_HIP, "graph capture of the screened CE iteration failed");
    }
    hipError_t e5 = hipGraphInstantiate(&m->screen_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e5 != hipSuccess) {
      m->screen_graph = nullptr;
      return mfail(m, CEM_E_HIP, "hipGraphInstantiate");
    }
    m->graph_serial = c->serial;
    m->graph_nsim = n_sim;
  }
  for (int j = 0; j < iters; ++j) MHIPCHK(m, hipGraphLaunch(m->screen_graph, s));
  DevState h;
  MHIPCHK(m, hipMemcpyAsync(&h, c->st, sizeof h, hipMemcpyDeviceToHost, s));
  if (stats_host && iters > 0)
    MHIPCHK(m, hipMemcpyAsync(stats_host, c->stats + (size_t)it0 * CEM_STATS_COLS,
                              sizeof(float) * iters * CEM_STATS_COLS, hipMemcpyDeviceToHost, s));
  if (surrogate_err_host && iters > 0)
    MHIPCHK(m, hipMemcpyAsync(surrogate_err_host, m->err + it0, sizeof(float) * iters, hipMemcpyDeviceToHost, s));
  MHIPCHK(m, hipStreamSynchronize(s));
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
  return h.factor_status ? CEM_E_NUMERIC : CEM_OK;
}

}  // extern "C"
