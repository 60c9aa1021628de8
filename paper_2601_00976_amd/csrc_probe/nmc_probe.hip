// Measurement library, not part of the solve: the FP64 FMA throughput probe
// behind the measured roofline denominator (declared in include/nmc_probe.h,
// built as libnmc_probe.so beside the solver library).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nmc_probe.h"

namespace {

// 16 independent FMA chains per lane, 8 rounds per loop trip
__global__ __launch_bounds__(64) void probe_fma_kernel(int iters, double* __restrict__ out) {
  const int64_t l = (int64_t)blockIdx.x * 64 + threadIdx.x;
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = 1.0 + 1e-3 * k + 1e-9 * (double)threadIdx.x;
  const double a = 0.9999999, b = 1e-7;
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = __builtin_fma(x[k], a, b);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += x[k];
  out[l] = s;
}

}  // namespace

extern "C" int nmc_probe_fma_f64(int64_t waves, int iters, double* out, void* stream) {
  if (waves < 1 || waves > (int64_t(1) << 20) || iters < 1 || iters > (1 << 24) || !out)
    return NMC_PROBE_E_INVALID_ARG;
  const int rounds = (iters + 7) / 8 * 8;
  hipLaunchKernelGGL(probe_fma_kernel, dim3((unsigned)waves), dim3(64), 0, (hipStream_t)stream, rounds, out);
  return hipGetLastError() == hipSuccess ? NMC_PROBE_OK : NMC_PROBE_E_HIP;
}
