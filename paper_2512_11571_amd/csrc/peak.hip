// FP32 vector FMA rate of the device, measured: the ceiling the rollout's
// arithmetic (unpacked FP32) can reach, reported beside the published packed
// peak.  Every thread runs eight independent FMA chains whose values stay
// finite; one store per thread keeps the chains live.
#include <hip/hip_runtime.h>

#include "cemtamp.h"

namespace {

constexpr int CHAINS = 8, ITERS = 4096;

__global__ void __launch_bounds__(256) fma_chains_kernel(float b, float c, float *__restrict__ out) {
  float a[CHAINS];
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) a[k] = (float)(threadIdx.x + k);
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) a[k] = fmaf(a[k], b, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) s += a[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int cem_valu_fma_rate(double *flops_per_s, void *stream) {
  if (!flops_per_s) return CEM_E_ARG;
  *flops_per_s = 0.0;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return CEM_E_HIP;
  const int blocks = n_cu * 32, threads = 256;  // eight 64-lane waves per SIMD
  float *out = nullptr;
  if (hipMalloc(&out, sizeof(float) * (size_t)blocks * threads) != hipSuccess) return CEM_E_ALLOC;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = CEM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = CEM_E_HIP;
  float best_ms = 0.0f;
  for (int rep = 0; rc == CEM_OK && rep < 4; ++rep) {  // the first launch warms up
    hipLaunchKernelGGL(fma_chains_kernel, dim3(blocks), dim3(threads), 0, s, 0.999999f, 1e-6f, out);
    if (hipEventRecord(e0, s) != hipSuccess) { rc = CEM_E_HIP; break; }
    hipLaunchKernelGGL(fma_chains_kernel, dim3(blocks), dim3(threads), 0, s, 0.999999f, 1e-6f, out);
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = CEM_E_HIP; break; }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = CEM_E_HIP; break; }
    if (rep > 0 && (best_ms == 0.0f || ms < best_ms)) best_ms = ms;
  }
  if (rc == CEM_OK && hipGetLastError() != hipSuccess) rc = CEM_E_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (rc == CEM_OK && best_ms > 0.0f)
    *flops_per_s = 2.0 * CHAINS * ITERS * (double)blocks * threads / (best_ms * 1e-3);
  return rc;
}
