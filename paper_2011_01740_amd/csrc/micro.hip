// Measurement helper: the FP64 FMA rate the chip sustains, measured with
// independent FMA chains on every lane (the "FMA-chain" peak beside the
// published 78.6 TFLOP/s, which assumes every VALU slot is an FP64 FMA at the
// 2.4 GHz peak engine clock).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ens.h"

namespace {

constexpr int kChains = 8;  // independent chains per lane: enough to cover FMA latency

// a_k <- a_k * m + c for `iters` rounds; m slightly below 1 keeps the values
// bounded; the sum is stored so that nothing is dead code.
__global__ __launch_bounds__(256) void k_fma_chain(int64_t iters, double m, double c,
                                                   double *out) {
  double a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = 1.0 + 1e-3 * (threadIdx.x + k);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int ens_micro_fma(int32_t device, int64_t iters, double *tflops, float *ms) {
  if (iters <= 0 || !tflops) return ENS_E_INVAL;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return ENS_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return ENS_E_INVAL;
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  // 8 blocks of 256 per CU: 8 waves per SIMD
  const int blocks = 8 * (cus > 0 ? cus : 256);
  double *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float t = 0.f;
  if (e == hipSuccess) e = hipMalloc((void **)&out, (size_t)blocks * 256 * sizeof(double));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    // warm-up, then the timed launch
    hipLaunchKernelGGL(k_fma_chain, dim3(blocks), dim3(256), 0, 0, iters / 8 + 1,
                       1.0 - 1.0 / 1024.0, 1.0 / 1024.0, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, 0);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fma_chain, dim3(blocks), dim3(256), 0, 0, iters, 1.0 - 1.0 / 1024.0,
                       1.0 / 1024.0, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return ENS_E_HIP;
  const double flop = 2.0 * kChains * (double)iters * blocks * 256.0;
  *tflops = flop / (t * 1e-3) / 1e12;
  if (ms) *ms = t;
  return ENS_OK;
}
