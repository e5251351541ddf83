// Oracle: the learned surrogate that screens candidate plans before full
// simulation.  TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Not part of the paper's method (its limitation paragraph notes that full
// rollouts are expensive): a multilayer perceptron 16 -> 256 -> 256 -> 256 -> 8
// predicts a plan's cost and final object pose from its 16 controller
// parameters.  Written from the textbook definitions:
//   forward   a_0 = x, z_l = W_l a_{l-1} + b_l, a_l = gelu(z_l) (hidden), y = z_4
//   gelu      the tanh form of Hendrycks & Gimpel (2016):
//             gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
//   loss      mean over the batch and the 8 outputs of (y - t)^2
//   backward  reverse-mode chain rule through the layers
//   Adam      Kingma & Ba (2015) with bias correction.
// Parameters are one flat vector: W1 (256x16, row = output unit), b1, W2
// (256x256), b2, W3 (256x256), b3, W4 (8x256), b4 -- 137,992 values.
// The "BF16" forward rounds inputs, weights and every hidden activation to
// bfloat16 (round to nearest even, through FP32) and accumulates in FP64: the
// arithmetic a BF16-input / FP32-accumulate matrix unit performs, up to the
// accumulation order.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace ref {

constexpr int MLP_L = 4;
constexpr int MLP_DIMS[MLP_L + 1] = {16, 256, 256, 256, 8};

inline long mlp_w_off(int l) {  // offset of W_{l+1}
  long o = 0;
  for (int k = 0; k < l; ++k) o += (long)MLP_DIMS[k] * MLP_DIMS[k + 1] + MLP_DIMS[k + 1];
  return o;
}
inline long mlp_b_off(int l) { return mlp_w_off(l) + (long)MLP_DIMS[l] * MLP_DIMS[l + 1]; }
inline long mlp_n_params() { return mlp_w_off(MLP_L); }

inline double gelu(double x) {
  const double c = std::sqrt(2.0 / 3.14159265358979323846);
  return 0.5 * x * (1.0 + std::tanh(c * (x + 0.044715 * x * x * x)));
}
inline double gelu_grad(double x) {
  const double c = std::sqrt(2.0 / 3.14159265358979323846);
  const double t = std::tanh(c * (x + 0.044715 * x * x * x));
  return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * c * (1.0 + 3.0 * 0.044715 * x * x);
}

// bfloat16 value of x: x rounded to FP32, then to the nearest bfloat16 (ties to even).
inline double to_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return x;  // inf / nan
  const uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

struct MlpCache {
  std::vector<double> z[MLP_L + 1], a[MLP_L + 1];  // per layer, batch-major
};

// Forward pass over n rows of x (n x 16); y (n x 8).  bf16: emulate BF16 operands.
inline void mlp_forward(const double *P, const double *x, int n, double *y, bool bf16, MlpCache *cache) {
  std::vector<double> in((size_t)n * MLP_DIMS[0]);
  for (size_t i = 0; i < in.size(); ++i) in[i] = bf16 ? to_bf16(x[i]) : x[i];
  if (cache) cache->a[0] = in;
  for (int l = 0; l < MLP_L; ++l) {
    const int ni = MLP_DIMS[l], no = MLP_DIMS[l + 1];
    const double *W = P + mlp_w_off(l), *b = P + mlp_b_off(l);
    std::vector<double> z((size_t)n * no), out((size_t)n * no);
    for (int r = 0; r < n; ++r)
      for (int o = 0; o < no; ++o) {
        double acc = 0.0;
        for (int i = 0; i < ni; ++i) {
          const double w = bf16 ? to_bf16(W[(long)o * ni + i]) : W[(long)o * ni + i];
          acc += w * in[(size_t)r * ni + i];
        }
        acc += b[o];
        z[(size_t)r * no + o] = acc;
        if (l < MLP_L - 1) {
          const double g = gelu(bf16 ? (double)(float)acc : acc);
          out[(size_t)r * no + o] = bf16 ? to_bf16(g) : g;
        } else {
          out[(size_t)r * no + o] = acc;
        }
      }
    if (cache) {
      cache->z[l + 1] = z;
      cache->a[l + 1] = out;
    }
    in.swap(out);
  }
  std::memcpy(y, in.data(), sizeof(double) * (size_t)n * MLP_DIMS[MLP_L]);
}

// Mean squared error over n rows and gradient dP (same layout as P).
// bf16: the backward of a BF16-operand / FP32-accumulate matrix unit, up to
// the accumulation order: the BF16 forward, and the operands of every product
// of the backward - the output gradients dL/dz of each layer, the weights
// and the activations - rounded to bfloat16, while the bias gradients sum the
// unrounded dL/dz and the GELU derivative takes the FP32 pre-activation.
inline double mlp_loss_grad(const double *P, const double *x, const double *t, int n, double *dP, bool bf16 = false) {
  MlpCache c;
  std::vector<double> y((size_t)n * MLP_DIMS[MLP_L]);
  mlp_forward(P, x, n, y.data(), bf16, &c);
  auto rnd = [&](double v) { return bf16 ? to_bf16(v) : v; };
  const int no = MLP_DIMS[MLP_L];
  const double scale = 1.0 / ((double)n * no);
  double loss = 0.0;
  std::vector<double> dz((size_t)n * no);
  for (size_t i = 0; i < dz.size(); ++i) {
    const double e = y[i] - t[i];
    loss += e * e;
    dz[i] = 2.0 * e * scale;
  }
  loss *= scale;
  if (!dP) return loss;
  for (long i = 0; i < mlp_n_params(); ++i) dP[i] = 0.0;
  for (int l = MLP_L - 1; l >= 0; --l) {
    const int ni = MLP_DIMS[l], nol = MLP_DIMS[l + 1];
    const double *W = P + mlp_w_off(l);
    double *dW = dP + mlp_w_off(l), *db = dP + mlp_b_off(l);
    const std::vector<double> &ain = c.a[l];
    for (int r = 0; r < n; ++r)
      for (int o = 0; o < nol; ++o) {
        const double g = dz[(size_t)r * nol + o];
        db[o] += g;
        const double gr = rnd(g);
        for (int i = 0; i < ni; ++i) dW[(long)o * ni + i] += gr * ain[(size_t)r * ni + i];
      }
    if (l == 0) break;
    std::vector<double> dprev((size_t)n * ni, 0.0);
    for (int r = 0; r < n; ++r)
      for (int i = 0; i < ni; ++i) {
        double acc = 0.0;
        for (int o = 0; o < nol; ++o) acc += rnd(dz[(size_t)r * nol + o]) * rnd(W[(long)o * ni + i]);
        const double zp = c.z[l][(size_t)r * ni + i];
        dprev[(size_t)r * ni + i] = acc * gelu_grad(bf16 ? (double)(float)zp : zp);
      }
    dz.swap(dprev);
  }
  return loss;
}

// One Adam step (t = step count after this step, from 1).
inline void adam_step(double *P, const double *g, double *m, double *v, long n, double lr, double b1, double b2,
                      double eps, int t) {
  const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
  for (long i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    P[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
  }
}

}  // namespace ref
