// Fused persistent launch: census, planning, matching and aggregation of up to
// kMaxFrames frames in one kernel (Alg. 2 end to end).
//
// The grid holds exactly as many 256-thread workgroups as fit on the device at once, so
// all of them are resident, and the launch runs in phases split by grid barriers:
//   1. the plan of every frame with the list of the census tiles its boxes' searches
//      read (workgroups 0 .. F - 1), then, after a grid barrier, the census of the
//      listed tiles, the shares of one XCD's workgroups consecutive in the list;
//   2. the work items of every frame (all close items first, then all far items), each
//      list dealt XCD by XCD, in the same matchers as the multi-launch kernels;
//   3. one box per workgroup: aggregation and depth.
// Work is dealt by workgroup index, so no shared counter is touched per item; each
// barrier costs one atomic per workgroup, spread over kBarSlots counters. Its wait is
// bounded: an expired wait (which needs a workgroup that was not resident) marks every
// box of the call with OCSR_REASON_INTERNAL_TIMEOUT instead of hanging.
#include "dev_census.hpp"
#include "dev_match.hpp"

namespace ocsr {
namespace {

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

__global__ __launch_bounds__(64) void reset_kernel(MatchWs ws) {
  if (threadIdx.x < GC_N) ws.gcount[threadIdx.x] = 0;
}

template <int CSX, int CSY, class FM, class CM>
__global__ __launch_bounds__(256) void fused_kernel(MatchParamsDev P, FramesDev FR,
                                                    const ocsr_box* boxes, MatchWs ws,
                                                    ocsr_box_result* out, int sentinel) {
  constexpr size_t kWave = cmax(FM::kLds, CM::kLds);
  constexpr size_t kPlan = sizeof(uint32_t) * kFrameTileWords + sizeof(int) * 8;
  constexpr size_t kLds = cmax(cmax(cmax(dev::CensusTile<CSX, CSY>::kLdsBytes, kPlan), kItemWaves * kWave),
                               sizeof(dev::AggLds));
  __shared__ uint64_t lds[(kLds + 7) / 8];
  __shared__ int mprefix[2 * kMaxFrames + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int G = gridDim.x, w = blockIdx.x;
  const int F = FR.n;
  int32_t* timeout = ws.gcount + GC_TIMEOUT;

  // ---- phase 1: the plan of every frame with its list of census tiles, then the census
  // of the listed tiles, the shares of one XCD's workgroups consecutive in the list
  if (w < F) {
    uint32_t* bits = (uint32_t*)lds;
    int* sc = (int*)(bits + kFrameTileWords);
    if (wave == 0) dev::plan_frame(P, FR.f[w], w, FR.n_boxes_total, boxes, ws, lane, false);
    dev::list_frame_tiles(P, FR.f[w], w, boxes, ws, bits, sc);
    dev::write_frame_items(P, FR.f[w], w, FR.n_boxes_total, ws, tid, 256, (int32_t*)bits,
                           kFrameTileWords);
    __syncthreads();   // the LDS is reused below
  }
  dev::grid_barrier(ws.gcount + GC_BAR0, G, timeout);
  {
    int* pre = mprefix;   // the frames' list lengths, then reused for the items
    if (tid < 64) {
      const int cnt = lane < F ? ws.fcount[lane * FC_N + FC_TILES] : 0;
      const int incl = dev::wave_incl_scan(cnt, lane);
      if (lane < F) pre[lane + 1] = incl;
      if (lane == 0) pre[0] = 0;
    }
    __syncthreads();
    const int N = pre[F];
    const int x = w & 7;
    int r = 0;
    for (int y = 0; y < x; ++y) r += (G - y + 7) >> 3;
    r += w >> 3;
    const int lo = dev::share_start(N, r, G), hi = dev::share_start(N, r + 1, G);
    int f = 0;
    for (int q = lo; q < hi; ++q) {
      while (q >= pre[f + 1]) ++f;
      const FrameDev& fr = FR.f[f];
      const dev::FrameTile ft = dev::frame_tile_local(fr, f, fr.tile_list[q - pre[f]]);
      dev::make_census_tile<CSX, CSY>(ft.job, CSX, CSY, sentinel, (uint32_t*)lds);
      __syncthreads();   // the next tile reuses the LDS
    }
  }
  dev::grid_barrier(ws.gcount + GC_BAR2, G, timeout);
  bool timed_out = dev::load_relaxed(timeout) != 0;

  // ---- phase 2: work items; close items of every frame, then far items
  if (tid < 64) {
    const int j = lane < F ? lane : lane - F;
    const int cnt = lane < 2 * F ? ws.fcount[j * FC_N + (lane < F ? FC_CLOSE_ITEMS : FC_FAR_ITEMS)] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < 2 * F) mprefix[lane + 1] = incl;
    if (lane == 0) mprefix[0] = 0;
  }
  __syncthreads();
  if (!timed_out) {
    void* wl = (char*)lds + wave * kWave;
    const int n_close = mprefix[F];
    const dev::Deal2 dl = dev::xcd_deal2(n_close, mprefix[2 * F] - n_close);
    for (int i = dl.first; i < dl.end; i += dl.step) {
      const int m = dl.at(i);
      int slot = 0;
      for (int k = 1; k < 2 * F; ++k)
        if (m >= mprefix[k]) slot = k;
      const int f = slot < F ? slot : slot - F;
      const FrameDev& fr = FR.f[f];
      const int q = m - mprefix[slot];
      const int at = q + (slot < F ? 0 : mprefix[f + 1] - mprefix[f]);
      const ItemRec* rp = ws.items + (size_t)f * ws.items_cap + at;
      // per-lane indexing formed afresh per item (as in match_pair2_kernel)
      int il = lane;
      asm volatile("" : "+v"(il));
      if (slot < F) {
        const typename CM::State st = CM::frame_state(ws, fr, il);
        const ItemRec rec = *rp;
        CM::run_item(P, fr, ws, DebugDev{}, f, 1, rec, wave, il, wl, st);
      } else {
        const typename FM::State st = FM::frame_state(ws, fr, il);
        const ItemRec rec = *rp;
        FM::run_item(P, fr, ws, DebugDev{}, f, 0, rec, wave, il, wl, st);
      }
    }
  }
  __syncthreads();
  dev::grid_barrier(ws.gcount + GC_BAR1, G, timeout);
  timed_out = dev::load_relaxed(timeout) != 0;

  // ---- phase 3: aggregation, one box per workgroup
  for (int k = w; k < FR.n_boxes_total; k += G) {
    dev::aggregate_box(P, ws, k, out, timed_out, *(dev::AggLds*)lds);
    __syncthreads();
  }
}

// matcher pairs with a fused kernel: far (rows, cpl) and close (rows, cpl)
enum class FusedPair { kNone, kQ2H3, kQ2H4, kQ2H2, kQ4H4, kH2H3 };

FusedPair fused_pair(const MatchParamsDev& P, int sx, int sy) {
  // the persistent kernel has no vertical search: such calls take the multi-launch path
  if (sx != 3 || sy != 4 || P.vertical) return FusedPair::kNone;
  const PathDev& f = P.path[0];
  const PathDev& c = P.path[1];
  if (c.rows != 2 || f.passes != 1 || c.passes != 1) return FusedPair::kNone;
  if (f.rows == 1 && f.cpl == 2) {
    if (c.cpl == 3) return FusedPair::kQ2H3;
    if (c.cpl == 4) return FusedPair::kQ2H4;
    if (c.cpl == 2) return FusedPair::kQ2H2;
  }
  if (f.rows == 1 && f.cpl == 4 && c.cpl == 4) return FusedPair::kQ4H4;
  if (f.rows == 2 && f.cpl == 2 && c.cpl == 3) return FusedPair::kH2H3;
  return FusedPair::kNone;
}

constexpr int kFusedDefaultWgsPerCu = 2;

template <class K>
hipError_t launch_one(K kernel, const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                      const MatchWs& ws, ocsr_box_result* out, int sentinel, int n_cu,
                      int wgs_per_cu, hipStream_t stream) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kernel, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorNotSupported;
  // default 2 per CU: every workgroup pays an L2 write-back and an invalidation at each
  // grid barrier, which outweighs the waves more workgroups add (16-frame batch: 0.42 ms
  // at 2 per CU, 0.57 ms at the 4 that fit)
  const int cap = wgs_per_cu > 0 ? wgs_per_cu : kFusedDefaultWgsPerCu;
  per_cu = per_cu < cap ? per_cu : cap;
  kernel<<<per_cu * n_cu, 256, 0, stream>>>(P, FR, boxes, ws, out, sentinel);
  return hipGetLastError();
}

// the plan step lists a frame's census tiles in an LDS bitmap of kFrameTileWords words
bool frames_listable(const FramesDev& FR) {
  for (int f = 0; f < FR.n; ++f)
    if (2 * (FR.f[f].tiles0 + FR.f[f].tiles1) > 32 * kFrameTileWords) return false;
  return true;
}

}  // namespace

bool fused_available(const MatchParamsDev& p, const FramesDev& FR, int sx, int sy) {
  return fused_pair(p, sx, sy) != FusedPair::kNone && frames_listable(FR);
}

hipError_t launch_fused(const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, int sx, int sy, int sentinel,
                        int n_cu, int wgs_per_cu, hipStream_t stream, const LaunchTimer* timer) {
  const FusedPair pair = fused_pair(P, sx, sy);
  if (pair == FusedPair::kNone || !frames_listable(FR)) return hipErrorNotSupported;
  if (timer) timer->before(timer->ctx, "reset", stream);
  reset_kernel<<<1, 64, 0, stream>>>(ws);
  if (timer) timer->after(timer->ctx, "reset", stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "fused", stream);
  switch (pair) {
#define OCSR_FUSED(K, FMT, CMT)                                                              \
    case FusedPair::K:                                                                       \
      e = launch_one(fused_kernel<3, 4, dev::FMT, dev::CMT>, P, FR, boxes, ws, out, sentinel,  \
                     n_cu, wgs_per_cu, stream);                                              \
      break;
    OCSR_FUSED(kQ2H3, QuadMatcher<2>, HalfMatcher<3>)
    OCSR_FUSED(kQ2H4, QuadMatcher<2>, HalfMatcher<4>)
    OCSR_FUSED(kQ2H2, QuadMatcher<2>, HalfMatcher<2>)
    OCSR_FUSED(kQ4H4, QuadMatcher<4>, HalfMatcher<4>)
    OCSR_FUSED(kH2H3, HalfMatcher<2>, HalfMatcher<3>)
#undef OCSR_FUSED
    default:
      e = hipErrorNotSupported;
  }
  if (timer) timer->after(timer->ctx, "fused", stream);
  return e;
}

}  // namespace ocsr
