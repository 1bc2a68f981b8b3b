// Measures the int32 vector-ALU rate of the GPU: every lane runs 8 independent chains of
// v_xor_b32 + v_bcnt_u32_b32 + v_add3_u32 (the matching kernels' cost arithmetic), with
// enough waves to fill every SIMD. Prints lane-operations per second.
//
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         int_peak.hip -o int_peak && ./int_peak
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

__global__ __launch_bounds__(256) void int_chains(uint32_t* out, int iters, uint32_t seed) {
  uint32_t a[8], b[8], acc[8];
  for (int i = 0; i < 8; ++i) { a[i] = seed * (threadIdx.x + 7 * i + 1); b[i] = a[i] * 3u + 1u; acc[i] = 0; }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t x = a[i] ^ b[i];
      acc[i] = __builtin_amdgcn_mbcnt_lo(0, 0) + __popc(x) + acc[i];
      b[i] = x;
    }
  }
  uint32_t s = 0;
  for (int i = 0; i < 8; ++i) s += acc[i] + b[i];
  if (s == 0x12345678u) out[threadIdx.x] = s;
}
int main() {
  uint32_t* out = nullptr;
  if (hipMalloc(&out, 4096) != hipSuccess) return 1;
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return 1;
  const int iters = 4096, wgs = pr.multiProcessorCount * 16;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  for (int w = 0; w < 3; ++w) int_chains<<<wgs, 256>>>(out, iters, 3);
  hipEventRecord(e0);
  int_chains<<<wgs, 256>>>(out, iters, 5);
  hipEventRecord(e1);
  hipEventSynchronize(e1);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  const double ops = (double)wgs * 4 * iters * 8 * 3 * 64;   // waves x iters x chains x 3 ops x lanes
  printf("%d CUs at %d MHz: %.3f ms, %.2f T int32 lane-ops/s\n", pr.multiProcessorCount,
         pr.clockRate / 1000, ms, ops / (ms * 1e-3) / 1e12);
  hipFree(out);
  return 0;
}
