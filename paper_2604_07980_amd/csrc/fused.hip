// Fused persistent launch: census, planning, matching and aggregation of up to
// kMaxFrames frames in one kernel (Alg. 2 end to end).
//
// The grid holds exactly as many 256-thread workgroups as fit on the device at once, so
// all of them are resident, and the launch runs in three phases split by grid barriers:
//   1. the plan of every frame, then every census tile (64 x 32 level pixels of one view
//      at one level), dealt round-robin to the workgroups;
//   2. the work items of every frame (all close items first, then all far items), up to
//      item_blocks blocks of one box per item, spread over the four waves;
//   3. one box per workgroup: aggregation and depth.
// Work is dealt by workgroup index, so no shared counter is touched per item; each
// barrier costs one atomic per workgroup, spread over kBarSlots counters. Its wait is
// bounded: an expired wait (which needs a workgroup that was not resident) marks every
// box of the call with OCSR_REASON_INTERNAL_TIMEOUT instead of hanging.
#include "dev_census.hpp"
#include "dev_match.hpp"

namespace ocsr {
namespace {

template <int ROWS, int NX, int CPL>
struct VTiled {
  static constexpr int rows = ROWS, nx = NX, cpl = CPL;
  static constexpr size_t kLdsBytes = dev::Tiled<ROWS, NX, CPL>::kLdsBytes;
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

__global__ __launch_bounds__(64) void reset_kernel(MatchWs ws) {
  if (threadIdx.x < GC_N) ws.gcount[threadIdx.x] = 0;
}

template <int CSX, int CSY, class FV, class CV>
__global__ __launch_bounds__(256) void fused_kernel(MatchParamsDev P, FramesDev FR,
                                                    const ocsr_box* boxes, MatchWs ws,
                                                    ocsr_box_result* out, int sentinel,
                                                    int n_census) {
  constexpr size_t kWave = (cmax(FV::kLdsBytes, CV::kLdsBytes) + 15) & ~(size_t)15;
  constexpr size_t kLds = cmax(cmax(dev::CensusTile<CSX, CSY>::kLdsBytes, 4 * kWave),
                               sizeof(dev::AggLds));
  __shared__ uint64_t lds[(kLds + 7) / 8];
  __shared__ int mprefix[2 * kMaxFrames + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int G = gridDim.x, w = blockIdx.x;
  const int F = FR.n;
  int32_t* timeout = ws.gcount + GC_TIMEOUT;

  // ---- phase 1: plans, then census tiles
  for (int a = w; a < F + n_census; a += G) {
    if (a < F) {
      if (wave == 0) dev::plan_frame(P, FR.f[a], a, FR.n_boxes_total, boxes, ws, lane);
    } else {
      dev::frame_census_tile<CSX, CSY>(P, FR, boxes, a - F, CSX, CSY, sentinel, (uint32_t*)lds);
    }
    __syncthreads();   // the next item reuses the LDS
  }
  dev::grid_barrier(ws.gcount + GC_BAR0, G, timeout);
  bool timed_out = dev::load_relaxed(timeout) != 0;

  // ---- phase 2: work items; close items of every frame, then far items
  if (tid < 64) {
    // mprefix[j] = items before slot j, slot j < F: close items of frame j, else far
    // items of frame j - F
    const int j = lane < F ? lane : lane - F;
    const int cnt = lane < 2 * F ? ws.fcount[j * FC_N + (lane < F ? FC_CLOSE_ITEMS : FC_FAR_ITEMS)] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < 2 * F) mprefix[lane + 1] = incl;
    if (lane == 0) mprefix[0] = 0;
  }
  __syncthreads();
  const int n_items = timed_out ? 0 : mprefix[2 * F];
  void* wl = (char*)lds + wave * kWave;
  for (int m = w; m < n_items; m += G) {
    int slot = 0;
    for (int k = 1; k < 2 * F; ++k)
      if (m >= mprefix[k]) slot = k;
    const int f = slot < F ? slot : slot - F;
    const FrameDev& fr = FR.f[f];
    const int q = m - mprefix[slot];
    if (slot < F) {
      dev::run_item(P, fr, f, FR.n_boxes_total, ws, 1, q, wave, lane, [&](const dev::BlockCtx& c) {
        dev::match_block_tiled<CV::rows, CV::nx, CV::cpl>(P, fr, ws, DebugDev{}, c, lane, wl);
      });
    } else {
      dev::run_item(P, fr, f, FR.n_boxes_total, ws, 0, q, wave, lane, [&](const dev::BlockCtx& c) {
        dev::match_block_tiled<FV::rows, FV::nx, FV::cpl>(P, fr, ws, DebugDev{}, c, lane, wl);
      });
    }
  }
  dev::grid_barrier(ws.gcount + GC_BAR1, G, timeout);
  timed_out = dev::load_relaxed(timeout) != 0;

  // ---- phase 3: aggregation, one box per workgroup
  for (int k = w; k < FR.n_boxes_total; k += G) {
    dev::aggregate_box(P, ws, k, out, timed_out, *(dev::AggLds*)lds);
    __syncthreads();
  }
}

enum class FusedPair { kNone, k4_2__8_12, k4_2__8_8, k4_2__8_16, k8_8__8_12 };

FusedPair fused_pair(const MatchParamsDev& P, int sx, int sy) {
  // the persistent kernel has no vertical search: such calls take the multi-launch path
  if (sx != 3 || sy != 4 || P.vertical) return FusedPair::kNone;
  const PathDev& f = P.path[0];
  const PathDev& c = P.path[1];
  if (c.rows != 8 || f.passes != 1 || c.passes != 1) return FusedPair::kNone;
  if (f.rows == 4 && f.cpl == 2) {
    if (c.cpl == 12) return FusedPair::k4_2__8_12;
    if (c.cpl == 8) return FusedPair::k4_2__8_8;
    if (c.cpl == 16) return FusedPair::k4_2__8_16;
  }
  if (f.rows == 8 && f.cpl == 8 && c.cpl == 12) return FusedPair::k8_8__8_12;
  return FusedPair::kNone;
}

template <class K>
hipError_t launch_one(K kernel, const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                      const MatchWs& ws, ocsr_box_result* out, int sentinel, int n_census,
                      int n_cu, int wgs_per_cu, hipStream_t stream) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kernel, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorNotSupported;
  if (wgs_per_cu > 0) per_cu = per_cu < wgs_per_cu ? per_cu : wgs_per_cu;
  kernel<<<per_cu * n_cu, 256, 0, stream>>>(P, FR, boxes, ws, out, sentinel, n_census);
  return hipGetLastError();
}

}  // namespace

bool fused_available(const MatchParamsDev& p, int sx, int sy) {
  return fused_pair(p, sx, sy) != FusedPair::kNone;
}

hipError_t launch_fused(const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, int sx, int sy, int sentinel,
                        int n_census_tiles, int n_cu, int wgs_per_cu, hipStream_t stream,
                        const LaunchTimer* timer) {
  const FusedPair pair = fused_pair(P, sx, sy);
  if (pair == FusedPair::kNone) return hipErrorNotSupported;
  if (timer) timer->before(timer->ctx, "reset", stream);
  reset_kernel<<<1, 64, 0, stream>>>(ws);
  if (timer) timer->after(timer->ctx, "reset", stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "fused", stream);
  switch (pair) {
    case FusedPair::k4_2__8_12:
      e = launch_one(fused_kernel<3, 4, VTiled<4, 4, 2>, VTiled<8, 8, 12>>, P, FR, boxes, ws, out,
                     sentinel, n_census_tiles, n_cu, wgs_per_cu, stream);
      break;
    case FusedPair::k4_2__8_8:
      e = launch_one(fused_kernel<3, 4, VTiled<4, 4, 2>, VTiled<8, 8, 8>>, P, FR, boxes, ws, out,
                     sentinel, n_census_tiles, n_cu, wgs_per_cu, stream);
      break;
    case FusedPair::k4_2__8_16:
      e = launch_one(fused_kernel<3, 4, VTiled<4, 4, 2>, VTiled<8, 8, 16>>, P, FR, boxes, ws, out,
                     sentinel, n_census_tiles, n_cu, wgs_per_cu, stream);
      break;
    case FusedPair::k8_8__8_12:
      e = launch_one(fused_kernel<3, 4, VTiled<8, 8, 8>, VTiled<8, 8, 12>>, P, FR, boxes, ws, out,
                     sentinel, n_census_tiles, n_cu, wgs_per_cu, stream);
      break;
    default:
      e = hipErrorNotSupported;
  }
  if (timer) timer->after(timer->ctx, "fused", stream);
  return e;
}

}  // namespace ocsr
