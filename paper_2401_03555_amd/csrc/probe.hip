// Measurement support: an FP64 FMA throughput probe, so that rooflines can
// quote the FP64 vector rate this device reaches beside the published peak.
// Not a step of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "impact.h"

namespace {

constexpr int kChains = 16;  // independent FMA chains per thread (hide latency)

__global__ __launch_bounds__(256) void k_probe_fma(double* __restrict__ out, int32_t iters,
                                                   double a, double b) {
  double x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = 1e-3 * (double)(threadIdx.x + k);
  for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = __builtin_fma(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  // a store the compiler cannot drop, taken by no thread for these a and b
  if (s < -1.0) out[0] = s;
}

}  // namespace

extern "C" int impact_probe_fp64_fma(int64_t n_blocks, int32_t iters, double* out, void* stream) {
  if (n_blocks < 1 || n_blocks > (1 << 24) || iters < 1 || !out) return IMPACT_E_INVAL;
  hipLaunchKernelGGL(k_probe_fma, dim3((unsigned)n_blocks), dim3(256), 0, (hipStream_t)stream, out,
                     iters, 0.999999, 1e-7);
  return hipGetLastError() == hipSuccess ? IMPACT_OK : IMPACT_E_HIP;
}
