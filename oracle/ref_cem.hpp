// Oracle: cross-entropy select and refit. TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Sec. III-B and Alg. 1: after the rollouts, the top N_e samples are the
// feasible ones with the lowest cost; the new theta is the maximum-likelihood
// Gaussian of the elites (the KL-minimising update of CE optimisation, cited
// there to Botev et al.); independent normals in the experiments (Sec. IV-A,
// "Algorithm setting"), a full covariance as the general case.
// Fallbacks (Sec. III-B, text before Alg. 1): fewer feasible than N_e -> use
// the n_feasible ones; a single feasible sample -> that sample plus artificial
// noise; none feasible -> the plans whose actions all succeeded.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace ref {

enum SelectMode : int32_t {
  SEL_TOP = 0,        // n0 >= N_e: top N_e feasible
  SEL_ALL_FEAS = 1,   // 2 <= n0 < N_e: all feasible
  SEL_ONE = 2,        // exactly one sample selected: mean = it, noise covariance
  SEL_TIER1 = 3,      // no feasible: top min(N_e, n1) whose actions all succeeded
  SEL_NONE = 4        // nothing usable: theta unchanged
};

struct Key {
  int32_t tier;
  float cost;
  int32_t idx;
};

inline bool key_less(const Key &a, const Key &b) {
  if (a.tier != b.tier) return a.tier < b.tier;
  if (a.cost != b.cost) return a.cost < b.cost;
  return a.idx < b.idx;
}

// Sort the population by (tier, cost, index) ascending (NaN cost counts as
// tier 3) and pick the elite set.  Returns the number of elites written.
inline int select_elites(int pop, const float *cost, const uint8_t *tier, int n_elite, int32_t *elite_idx,
                         int32_t *mode_out, int32_t *tier_counts) {
  std::vector<Key> keys(pop);
  int counts[4] = {0, 0, 0, 0};
  for (int i = 0; i < pop; ++i) {
    Key k;
    k.tier = std::isnan(cost[i]) ? 3 : (tier[i] > 3 ? 3 : (int32_t)tier[i]);
    k.cost = std::isnan(cost[i]) ? INFINITY : (cost[i] == 0.0f ? 0.0f : cost[i]);
    k.idx = i;
    keys[i] = k;
    counts[k.tier]++;
  }
  std::sort(keys.begin(), keys.end(), key_less);
  if (tier_counts)
    for (int t = 0; t < 4; ++t) tier_counts[t] = counts[t];
  const int n0 = counts[0], n1 = counts[1];
  int ne;
  int32_t mode;
  if (n0 >= n_elite) { ne = n_elite; mode = SEL_TOP; }
  else if (n0 >= 2) { ne = n0; mode = SEL_ALL_FEAS; }
  else if (n0 == 1) { ne = 1; mode = SEL_ONE; }
  else if (n1 >= 1) { ne = std::min(n_elite, n1); mode = ne == 1 ? SEL_ONE : SEL_TIER1; }
  else { ne = 0; mode = SEL_NONE; }
  for (int e = 0; e < ne; ++e) elite_idx[e] = keys[e].idx;  // tier-1 block starts at 0 when n0 == 0
  *mode_out = mode;
  return ne;
}

// Cholesky factor of the symmetric D x D matrix A (row-major): for each column
// j, L_jj = sqrt(A_jj - sum_k<j L_jk^2), L_ij = (A_ij - sum_k<j L_ik L_jk) / L_jj,
// sums in ascending k.  Returns false on a non-positive or non-finite pivot.
inline bool cholesky(int D, const double *A, double *L) {
  for (int i = 0; i < D * D; ++i) L[i] = 0.0;
  for (int j = 0; j < D; ++j) {
    double s = A[j * D + j];
    for (int k = 0; k < j; ++k) s = s - L[j * D + k] * L[j * D + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    const double ljj = std::sqrt(s);
    L[j * D + j] = ljj;
    for (int i = j + 1; i < D; ++i) {
      double t = A[i * D + j];
      for (int k = 0; k < j; ++k) t = t - L[i * D + k] * L[j * D + k];
      L[i * D + j] = t / ljj;
    }
  }
  return true;
}

// Jittered factorisation: delta = 1e-9 tr(S)/D + 1e-12 on the diagonal; on
// failure delta x10, up to six tries; then the diagonal fallback
// L = diag(sqrt(max(S_dd, 1e-12))).  Returns 0 on success, 1 if the fallback was used.
inline int factor_cov(int D, const double *S, double *L) {
  double tr = 0.0;
  for (int d = 0; d < D; ++d) tr = tr + S[d * D + d];
  double delta = 1e-9 * tr / (double)D + 1e-12;
  std::vector<double> A(D * D);
  for (int attempt = 0; attempt < 6; ++attempt) {
    for (int i = 0; i < D * D; ++i) A[i] = S[i];
    for (int d = 0; d < D; ++d) A[d * D + d] = A[d * D + d] + delta;
    if (cholesky(D, A.data(), L)) return 0;
    delta = delta * 10.0;
  }
  for (int i = 0; i < D * D; ++i) L[i] = 0.0;
  for (int d = 0; d < D; ++d) L[d * D + d] = std::sqrt(std::max(S[d * D + d], 1e-12));
  return 1;
}

// Maximum-likelihood refit from the elite rows of Z (pop x D, FP32):
// mu = mean, S = (1/n) sum (z - mu)(z - mu)^T (diagonal only when cov_mode == 0).
// A single elite: mu = that row, S = diag((0.1 sigma0_d)^2).  No elites: unchanged.
// Updates mu, S (D x D) and L in place; returns the factor_cov status.
inline int refit(int D, int cov_mode, const float *Z, const int32_t *elite, int ne, int32_t mode,
                 const double *cov0, double *mu, double *S, double *L) {
  if (mode == SEL_NONE || ne == 0) return factor_cov(D, S, L);
  if (ne == 1) {
    for (int d = 0; d < D; ++d) mu[d] = (double)Z[(long)elite[0] * D + d];
    for (int i = 0; i < D * D; ++i) S[i] = 0.0;
    for (int d = 0; d < D; ++d) {
      const double s = 0.1 * std::sqrt(cov0[d * D + d]);
      S[d * D + d] = s * s;
    }
    return factor_cov(D, S, L);
  }
  for (int d = 0; d < D; ++d) {
    double acc = 0.0;
    for (int e = 0; e < ne; ++e) acc = acc + (double)Z[(long)elite[e] * D + d];
    mu[d] = acc / (double)ne;
  }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      if (cov_mode == 0 && a != b) { S[a * D + b] = 0.0; continue; }
      double acc = 0.0;
      for (int e = 0; e < ne; ++e) {
        const double da = (double)Z[(long)elite[e] * D + a] - mu[a];
        const double db = (double)Z[(long)elite[e] * D + b] - mu[b];
        acc = acc + da * db;
      }
      S[a * D + b] = acc / (double)ne;
    }
  return factor_cov(D, S, L);
}

}  // namespace ref
