// Device helpers shared by the census and matching code.
#pragma once

#include "ocsr_internal.hpp"

namespace ocsr {
namespace dev {

__device__ __forceinline__ int cdiv_nonneg(int a, int s) { return (a + s - 1) / s; }

// A value the whole wave holds, moved to scalar registers (the compiler cannot always
// tell that a value read through a uniformly computed index is uniform).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A pointer to global memory that the whole wave holds (the result stays a global-memory
// pointer, so accesses through it remain global rather than flat instructions).
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  typedef __attribute__((address_space(1))) T GlobalT;
  return (T*)(GlobalT*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v, int from = 1) {
  for (int o = 32; o >= from; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

// XCD-aware dealing of n work units over a launch's workgroups. The GPU hands out
// workgroups round-robin over its 8 XCDs (workgroup b runs on XCD b mod 8), and each
// XCD has its own L2. When the grid is a multiple of 8, XCD x takes the contiguous
// units [n x / 8, n (x + 1) / 8), dealt over its workgroups b = x, x + 8, ..., so
// neighbouring units, which read neighbouring data, share one L2; otherwise every
// workgroup strides over all units. first / step: the workgroup's first unit and stride;
// end: one past its last.
struct Deal {
  int first, step, end;
};
__device__ __forceinline__ Deal xcd_deal(int n) {
  const int G = gridDim.x, b = blockIdx.x;
  if ((G & 7) != 0 || G < 8) return Deal{b, G, n};
  const int x = b & 7, per = G >> 3;
  const int lo = (int)((long long)n * x / 8), hi = (int)((long long)n * (x + 1) / 8);
  return Deal{lo + (b >> 3), per, hi};
}

// First unit of share w of n units cut into G equal consecutive shares, floor(n w / G),
// in 32-bit arithmetic (n < 2^31, G < 46341).
__device__ __forceinline__ int share_start(int n, int w, int G) {
  return (n / G) * w + (n % G) * w / G;
}

// Two lists dealt together (the close and the far work items of a call): each XCD
// takes its contiguous share of list A and its share of list B and deals them, A's
// first, over its workgroups as one local list. Every XCD thus holds an equal share of
// each list, and a workgroup that gets no A unit takes a B unit. Local position i is
// the unit at(i) of the concatenation [A, B].
struct Deal2 {
  int first, step, end;   // the workgroup's positions in its XCD's local list
  int a_lo, a_n, b_at;    // the XCD's A share [a_lo, a_lo + a_n); its B share at b_at
  __device__ __forceinline__ int at(int i) const { return i < a_n ? a_lo + i : b_at + (i - a_n); }
};
__device__ __forceinline__ Deal2 xcd_deal2(int na, int nb) {
  const int G = gridDim.x, b = blockIdx.x;
  if ((G & 7) != 0 || G < 8) return Deal2{b, G, na + nb, 0, na, na};
  const int x = b & 7, per = G >> 3;
  const int alo = (int)((long long)na * x / 8), ahi = (int)((long long)na * (x + 1) / 8);
  const int blo = (int)((long long)nb * x / 8), bhi = (int)((long long)nb * (x + 1) / 8);
  return Deal2{b >> 3, per, (ahi - alo) + (bhi - blo), alo, ahi - alo, na + blo};
}

// Orders the LDS traffic of one wave: every lane's earlier LDS writes are seen by the
// wave's later LDS reads (a wave's LDS instructions complete in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ld_word(const uint64_t* __restrict__ row, int x, int W) {
  return (x >= 0 && x < W) ? row[x] : 0ull;
}

// device-scope counters
__device__ __forceinline__ int add_release(int32_t* p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bound on the spin of a grid barrier: the arrivals come from resident workgroups, so
// the wait ends; the bound only guards against a defect.
constexpr int kSpinLimit = 1 << 22;

// Readies a workgroup's global writes for one thread's device-scope release: every wave
// waits until its own stores are complete in the L2 (vmcnt 0: the vector L1 writes
// through), then the workgroup meets at a barrier. The one release that follows (an L2
// write-back on this multi-XCD GPU) then covers every wave's writes, where a release
// fence in each wave would cost one write-back per wave.
__device__ __forceinline__ void publish_workgroup() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// Grid-wide barrier of a launch whose workgroups are all resident: every workgroup
// publishes its writes, counts itself in one of kBarSlots counters (one device-scope
// release per workgroup) and waits (bounded) until the slots add up to the grid size.
__device__ __forceinline__ void grid_barrier(int32_t* slots, int n_groups, int32_t* timeout_flag) {
  publish_workgroup();
  if (threadIdx.x == 0) {
    add_release(slots + (blockIdx.x % kBarSlots), 1);
    int spins = 0;
    for (;;) {
      int sum = 0;
#pragma unroll
      for (int k = 0; k < kBarSlots; ++k) sum += load_relaxed(slots + k);
      if (sum >= n_groups) break;
      if (++spins > kSpinLimit) {
        __hip_atomic_store(timeout_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

}  // namespace dev
}  // namespace ocsr
