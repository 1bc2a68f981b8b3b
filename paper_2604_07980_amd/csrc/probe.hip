// Measurement of the device's int32 vector-ALU rate, the peak the matching and census
// kernels are priced against. Every lane runs kChains independent chains of the
// matching kernels' cost arithmetic, b <- acc ^ b; acc <- popcount(b) + acc (one
// v_xor_b32 and one accumulating v_bcnt_u32_b32 per step; feeding the sum back into the
// next operand keeps the chain from having a closed form the compiler could use), with
// enough workgroups to fill every SIMD. The rate is lane-operations per second over one
// timed launch.
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

constexpr int kChains = 8;

// written only when the result takes a value no input produces, which the compiler
// cannot rule out, so the chains are not optimised away
__device__ uint32_t g_probe_sink[256];

__global__ __launch_bounds__(256) void int_rate_kernel(int iters, uint32_t seed) {
  uint32_t b[kChains], acc[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    acc[i] = seed * (threadIdx.x + 13u * i + 1u);
    b[i] = acc[i] * 7u + 3u;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      b[i] = acc[i] ^ b[i];
      asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc[i]) : "v"(b[i]));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += acc[i] ^ b[i];
  if (s == 0xFFFFFFFFu) g_probe_sink[threadIdx.x] = s;
}

}  // namespace
}  // namespace ocsr

extern "C" int32_t ocsr_measure_int_rate(ocsr_ctx* ctx, int32_t iters, double* ops_per_s,
                                         double* ms) {
  using namespace ocsr;
  if (!ctx || !ops_per_s || iters < 1 || iters > (1 << 20))
    return report_error(OCSR_E_INVALID, "measure_int_rate: null argument or iters outside 1..2^20");
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return report_error(OCSR_E_HIP, "measure_int_rate: device query failed");
  const int wgs = n_cu * 16;   // 64 waves per CU: 16 per SIMD
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return report_error(OCSR_E_HIP, "measure_int_rate: hipEventCreate failed");
  int32_t rc = OCSR_OK;
  for (int w = 0; w < 3 && rc == OCSR_OK; ++w) {
    hipLaunchKernelGGL(int_rate_kernel, dim3(wgs), dim3(256), 0, nullptr, iters, 3u);
    if (hipGetLastError() != hipSuccess) rc = OCSR_E_HIP;
  }
  float t = 0.0f;
  if (rc == OCSR_OK) {
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(int_rate_kernel, dim3(wgs), dim3(256), 0, nullptr, iters, 5u);
    hipEventRecord(e1, nullptr);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      rc = OCSR_E_HIP;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != OCSR_OK) return report_error(rc, "measure_int_rate: launch or timing failed");
  // lanes x iterations x chains x 2 operations (xor, popcount-add)
  const double ops = (double)wgs * 256.0 * iters * kChains * 2.0;
  *ops_per_s = ops / (t * 1e-3);
  if (ms) *ms = t;
  return OCSR_OK;
}
