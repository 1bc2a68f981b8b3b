// Multi-launch path (Alg. 2): census and plan of every frame in one launch, one
// matching launch per level, one aggregation launch. A matching launch deals work items
// (up to item_blocks blocks of one box, spread over the four waves of a workgroup)
// over its grid; the aggregation launch gives each box a workgroup that forms its
// disparity (Sec. 4.3.4) and depth (Eq. 1). Results cross workgroups only at kernel
// boundaries. The device steps are in dev_census.hpp and dev_match.hpp, shared with
// the fused persistent kernel.
#include "dev_census.hpp"
#include "dev_match.hpp"

namespace ocsr {
namespace {

// one wave per frame (descriptor-level calls, whose census is the caller's)
__global__ __launch_bounds__(64) void plan_kernel(MatchParamsDev P, FramesDev FR,
                                                  const ocsr_box* boxes, MatchWs ws) {
  const int f = blockIdx.x;
  dev::plan_frame(P, FR.f[f], f, FR.n_boxes_total, boxes, ws, threadIdx.x);
}

// workgroups 0 .. n_frames - 1 plan a frame each (one wave); the rest make the census, one
// tile each (a workgroup tests whether some box's search reads its tile)
template <int SX, int SY>
__global__ __launch_bounds__(256) void frame_census_kernel(MatchParamsDev P, FramesDev FR,
                                                           const ocsr_box* boxes, MatchWs ws,
                                                           int sx, int sy, int sentinel) {
  __shared__ uint32_t lds[SX >= 0 ? dev::CensusTile<(SX > 0 ? SX : 0), (SY > 0 ? SY : 0)>::kLdsBytes / 4 : 1];
  __shared__ int tsc[4];
  if ((int)blockIdx.x < FR.n) {
    if (threadIdx.x < 64)
      dev::plan_frame(P, FR.f[blockIdx.x], blockIdx.x, FR.n_boxes_total, boxes, ws, threadIdx.x);
    return;
  }
  dev::frame_census_tile<SX, SY>(P, FR, boxes, blockIdx.x - FR.n, sx, sy, sentinel, lds, true,
                                 &tsc[0]);
}

// Plan of frame blockIdx.x and the list of its census tiles. Wave 0 plans the boxes while
// waves 1-3 mark the tiles their searches read, each wave in a tile map of its own (so
// the marking waits for no workgroup barrier, and the plan and the marking overlap);
// then all four waves list the tiles of the three maps and write the work items, from
// the plans wave 0 also left in LDS.
__global__ __launch_bounds__(256) void plan_tiles_kernel(MatchParamsDev P, FramesDev FR,
                                                         const ocsr_box* boxes, MatchWs ws) {
  constexpr int kMaps = kItemWaves - 1;
  constexpr int kPlanCap = 128;   // frames of at most this many boxes keep their plans in LDS
  __shared__ uint32_t bits[kMaps * kFrameTileWords];
  __shared__ BoxPlan lplan[kPlanCap];
  __shared__ int32_t lend[2 * kPlanCap + 2];
  __shared__ int sc[8];
  const int f = blockIdx.x;
  const FrameDev& fr = FR.f[f];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (wave == 0) {
    dev::plan_frame(P, fr, f, FR.n_boxes_total, boxes, ws, lane, false, lplan, lend, kPlanCap);
  } else {
    uint32_t* map = bits + (wave - 1) * kFrameTileWords;
    const int n_tiles = 2 * (fr.tiles0 + fr.tiles1);
    const int n_words = (n_tiles + 31) >> 5;
    for (int i = lane; i < n_words; i += 64) map[i] = dev::tile_map_init(P, n_tiles, i);
    dev::wave_sync();
    if (!P.full_census) dev::mark_frame_tiles(P, fr, boxes, map, (int)threadIdx.x - 64, 192);
  }
  __syncthreads();
  dev::compact_frame_tiles(fr, f, ws, bits, kMaps, kFrameTileWords, sc);
  dev::write_frame_items(P, fr, f, FR.n_boxes_total, ws, threadIdx.x, 256, (int32_t*)bits,
                         kMaps * kFrameTileWords, lplan, lend, kPlanCap);
}

// Census of the listed tiles of every frame by persistent workgroups: the frames' lists,
// concatenated, are shared out in equal consecutive parts, the parts of one XCD's
// workgroups adjacent (neighbouring tiles read overlapping source rows).
template <int SX, int SY>
__global__ __launch_bounds__(256) void census_list_kernel(MatchParamsDev P, FramesDev FR,
                                                          const ocsr_box* boxes, MatchWs ws,
                                                          int sx, int sy, int sentinel) {
  __shared__ uint32_t lds[SX >= 0 ? dev::CensusTile<(SX > 0 ? SX : 0), (SY > 0 ? SY : 0)>::kLdsBytes / 4 : 1];
  __shared__ int pre[kMaxFrames + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    const int cnt = lane < FR.n ? ws.fcount[lane * FC_N + FC_TILES] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < FR.n) pre[lane + 1] = incl;
    if (lane == 0) pre[0] = 0;
  }
  __syncthreads();
  const int N = pre[FR.n];
  const int G = gridDim.x, b = blockIdx.x, x = b & 7;
  int w = 0;   // this workgroup's rank when the workgroups of XCD 0 come first, then XCD 1, ...
  for (int y = 0; y < x; ++y) w += (G - y + 7) >> 3;
  w += b >> 3;
  const int lo = dev::share_start(N, w, G), hi = dev::share_start(N, w + 1, G);
  int f = 0;
  auto job = [&](int q) {
    while (q >= pre[f + 1]) ++f;
    const FrameDev& fr = FR.f[f];
    return dev::frame_tile_local(fr, f, fr.tile_list[q - pre[f]]).job;
  };
  if constexpr (SX >= 0) {
    // software-pipelined: the next tile's source bytes are loaded into registers while
    // the current tile's comparisons run from LDS
    if (lo >= hi) return;
    dev::CensusRegs<SX, SY> g;
    dev::CensusJob jq = job(lo);
    dev::census_load<SX, SY>(jq, g);
    for (int q = lo; q < hi; ++q) {
      dev::census_put<SX, SY>(g, lds);
      __syncthreads();
      dev::CensusJob jn = jq;
      if (q + 1 < hi) {
        jn = job(q + 1);
        dev::census_load<SX, SY>(jn, g);
      }
      dev::census_compute<SX, SY>(jq, sentinel, lds);
      __syncthreads();   // the next tile reuses the LDS
      jq = jn;
    }
  } else {
    for (int q = lo; q < hi; ++q) {
      dev::make_census_tile<SX, SY>(job(q), sx, sy, sentinel, lds);
      __syncthreads();
    }
  }
}

// Waves per SIMD a single-level kernel is compiled for (as many as its registers allow
// without spilling, checked in the built code).
template <int ROWS, int CPL, int PASSES>
constexpr int tiled_waves() {
  return ROWS == 4 ? ((CPL <= 2 || (CPL <= 4 && PASSES == 1)) ? 6 : CPL <= 8 ? 4 : 2)
                   : (CPL <= 4 && PASSES == 1) ? 5
                   : ((CPL <= 4 && PASSES <= 3) || (CPL <= 6 && PASSES <= 2)) ? 4
                   : CPL <= 12 ? 3 : CPL <= 16 ? 2 : 1;
}

template <int ROWS, int NX, int CPL, int PASSES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tiled_waves<ROWS, CPL, PASSES>()))) void match_tiled_kernel(MatchParamsDev P, FramesDev FR,
                                                          MatchWs ws, DebugDev dbg, int level) {
  constexpr size_t kWave = (dev::Tiled<ROWS, NX, CPL, PASSES>::kLdsBytes + 15) & ~(size_t)15;
  __shared__ uint64_t lds[(kItemWaves * kWave + 7) / 8];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  void* wl = (char*)lds + wave * kWave;
  dev::level_items(FR, ws, level, [&](int f, int, int at) {
    const FrameDev& fr = FR.f[f];
    const ItemRec r = ws.items[(size_t)f * ws.items_cap + at];
    dev::run_item_rec(P, fr, f, level, r, wave, [&](const dev::BlockCtx& c) {
      dev::match_block_tiled<ROWS, NX, CPL, PASSES>(P, fr, ws, dbg, c, lane, wl);
    });
  });
}

// Waves per SIMD the paired kernel is compiled for: three where both variants fit in a
// third of the register file without spilling (checked in the built code), else two.
template <int FR_, int FC, int CC, int CP>
constexpr int pair_waves() {
  return CP > 1 ? (CC <= 6 ? 4 : 3)
         : ((FR_ == 4 && FC <= 2 && CC <= 12) || (FC <= 8 && CC <= 8)) ? 3 : 2;
}

// Both levels in one launch: work items of every frame's close level first, then of
// every far level (FV / CV: the far and close kernel variants).
template <int FR_, int FX, int FC, int CR_, int CX, int CC, int CP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(pair_waves<FR_, FC, CC, CP>()))) void match_pair_kernel(MatchParamsDev P, FramesDev FR,
                                                         MatchWs ws, DebugDev dbg) {
  constexpr size_t kF = (dev::Tiled<FR_, FX, FC>::kLdsBytes + 15) & ~(size_t)15;
  constexpr size_t kC = (dev::Tiled<CR_, CX, CC, CP>::kLdsBytes + 15) & ~(size_t)15;
  constexpr size_t kWave = kF > kC ? kF : kC;
  __shared__ uint64_t lds[(kItemWaves * kWave + 7) / 8];
  __shared__ int prefix[2 * kMaxFrames + 1];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int F = FR.n;
  if (threadIdx.x < 64) {
    // prefix[j]: items before slot j; slot j < F is frame j's close level, else frame
    // j - F's far level
    const int j = lane < F ? lane : lane - F;
    const int cnt = lane < 2 * F ? ws.fcount[j * FC_N + (lane < F ? FC_CLOSE_ITEMS : FC_FAR_ITEMS)] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < 2 * F) prefix[lane + 1] = incl;
    if (lane == 0) prefix[0] = 0;
  }
  __syncthreads();
  void* wl = (char*)lds + wave * kWave;
  const int n_close = prefix[F];
  const dev::Deal2 dl = dev::xcd_deal2(n_close, prefix[2 * F] - n_close);
  for (int i = dl.first; i < dl.end; i += dl.step) {
    const int m = dl.at(i);
    int slot = 0;
    for (int k = 1; k < 2 * F; ++k)
      if (m >= prefix[k]) slot = k;
    const int f = slot < F ? slot : slot - F;
    const FrameDev& fr = FR.f[f];
    const int q = m - prefix[slot];
    // the frame's far items follow its close items (slot f) in the records
    const int at = q + (slot < F ? 0 : prefix[f + 1] - prefix[f]);
    const ItemRec r = ws.items[(size_t)f * ws.items_cap + at];
    if (slot < F) {
      dev::run_item_rec(P, fr, f, 1, r, wave, [&](const dev::BlockCtx& c) {
        dev::match_block_tiled<CR_, CX, CC, CP>(P, fr, ws, dbg, c, lane, wl);
      });
    } else {
      dev::run_item_rec(P, fr, f, 0, r, wave, [&](const dev::BlockCtx& c) {
        dev::match_block_tiled<FR_, FX, FC>(P, fr, ws, dbg, c, lane, wl);
      });
    }
  }
}

// Both levels in one launch with any pair of matchers (FM far, CM close): work items of
// every frame's close level first, then of every far level. Compiled for WAVES waves per
// SIMD.
template <class FM, class CM, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void match_pair2_kernel(
    MatchParamsDev P, FramesDev FR, MatchWs ws, DebugDev dbg) {
  constexpr size_t kWave = FM::kLds > CM::kLds ? FM::kLds : CM::kLds;
  __shared__ uint64_t lds[(kItemWaves * kWave + 7) / 8];
  __shared__ int prefix[2 * kMaxFrames + 1];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int F = FR.n;
  if (threadIdx.x < 64) {
    const int j = lane < F ? lane : lane - F;
    const int cnt = lane < 2 * F ? ws.fcount[j * FC_N + (lane < F ? FC_CLOSE_ITEMS : FC_FAR_ITEMS)] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < 2 * F) prefix[lane + 1] = incl;
    if (lane == 0) prefix[0] = 0;
  }
  __syncthreads();
  void* wl = (char*)lds + wave * kWave;
  // the close items of every frame, then the far ones, dealt XCD by XCD as two lists
  const int n_close = prefix[F];
  const dev::Deal2 dl = dev::xcd_deal2(n_close, prefix[2 * F] - n_close);
  for (int i = dl.first; i < dl.end; i += dl.step) {
    const int m = dl.at(i);
    int slot = 0;
    for (int k = 1; k < 2 * F; ++k)
      if (m >= prefix[k]) slot = k;
    const int f = slot < F ? slot : slot - F;
    const FrameDev& fr = FR.f[f];
    const int q = m - prefix[slot];
    const int at = q + (slot < F ? 0 : prefix[f + 1] - prefix[f]);
    const ItemRec* rp = ws.items + (size_t)f * ws.items_cap + at;
    // the lane index passes through an empty asm statement per item, so that neither
    // matcher's per-lane indexing is held in registers across the loop (both would be)
    int il = lane;
    asm volatile("" : "+v"(il));
    if (slot < F) {
      const typename CM::State st = CM::frame_state(ws, fr, il);
      const ItemRec r = *rp;
      CM::run_item(P, fr, ws, dbg, f, 1, r, wave, il, wl, st);
    } else {
      const typename FM::State st = FM::frame_state(ws, fr, il);
      const ItemRec r = *rp;
      FM::run_item(P, fr, ws, dbg, f, 0, r, wave, il, wl, st);
    }
  }
}

// One level with any matcher.
template <class M, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void match_level_kernel(
    MatchParamsDev P, FramesDev FR, MatchWs ws, DebugDev dbg, int level) {
  __shared__ uint64_t lds[(kItemWaves * M::kLds + 7) / 8];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  void* wl = (char*)lds + wave * M::kLds;
  dev::level_items(FR, ws, level, [&](int f, int, int at) {
    const FrameDev& fr = FR.f[f];
    const typename M::State st = M::frame_state(ws, fr, lane);
    const ItemRec r = ws.items[(size_t)f * ws.items_cap + at];
    M::run_item(P, fr, ws, dbg, f, level, r, wave, lane, wl, st);
  });
}

// Both levels with a vertical range in one launch: work items of every frame's close
// level first, then of every far level (as match_pair_kernel), each wave with an LDS
// share of wave_bytes (the larger of the two levels' needs). The two levels' blocks
// overlap on the GPU, which outweighs the registers the combined kernel takes (measured
// against one launch per level).
template <int FROWS, int CROWS>
__global__ __launch_bounds__(256) void match_dy_pair_kernel(MatchParamsDev P, FramesDev FR, MatchWs ws,
                                                            DebugDev dbg, int wave_bytes) {
  extern __shared__ uint64_t dy_lds[];
  __shared__ int prefix[2 * kMaxFrames + 1];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int F = FR.n;
  if (threadIdx.x < 64) {
    // prefix[j]: items before slot j; slot j < F is frame j's close level, else frame
    // j - F's far level
    const int j = lane < F ? lane : lane - F;
    const int cnt = lane < 2 * F ? ws.fcount[j * FC_N + (lane < F ? FC_CLOSE_ITEMS : FC_FAR_ITEMS)] : 0;
    const int incl = dev::wave_incl_scan(cnt, lane);
    if (lane < 2 * F) prefix[lane + 1] = incl;
    if (lane == 0) prefix[0] = 0;
  }
  __syncthreads();
  void* wl = (char*)dy_lds + (size_t)wave * wave_bytes;
  const int total = prefix[2 * F];
  for (int m = blockIdx.x; m < total; m += gridDim.x) {
    int slot = 0;
    for (int k = 1; k < 2 * F; ++k)
      if (m >= prefix[k]) slot = k;
    const int f = slot < F ? slot : slot - F;
    const FrameDev& fr = FR.f[f];
    const int q = m - prefix[slot];
    // the frame's far items follow its close items in the records
    const int at = q + (slot < F ? 0 : prefix[f + 1] - prefix[f]);
    const ItemRec r = ws.items[(size_t)f * ws.items_cap + at];
    if constexpr (FROWS == CROWS) {
      // one matcher for both levels: a single inlined copy keeps the register count of
      // the one-level kernel
      dev::run_item_rec(P, fr, f, slot < F ? 1 : 0, r, wave, [&](const dev::BlockCtx& c) {
        dev::match_block_dy<CROWS, CROWS>(P, fr, ws, dbg, c, lane, wl);
      });
    } else if (slot < F) {
      dev::run_item_rec(P, fr, f, 1, r, wave, [&](const dev::BlockCtx& c) {
        dev::match_block_dy<CROWS, CROWS>(P, fr, ws, dbg, c, lane, wl);
      });
    } else {
      dev::run_item_rec(P, fr, f, 0, r, wave, [&](const dev::BlockCtx& c) {
        dev::match_block_dy<FROWS, FROWS>(P, fr, ws, dbg, c, lane, wl);
      });
    }
  }
}

__global__ __launch_bounds__(256) void aggregate_kernel(MatchParamsDev P, MatchWs ws,
                                                        ocsr_box_result* out) {
  __shared__ dev::AggLds sm;
  dev::aggregate_box(P, ws, blockIdx.x, out, false, sm);
}

}  // namespace

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t match_ws_bytes(int n_frames, int n_boxes_total, int cap_blocks) {
  const size_t n = (size_t)(n_boxes_total > 0 ? n_boxes_total : 1);
  const size_t c = (size_t)(cap_blocks > 0 ? cap_blocks : 1) * (size_t)(n_frames > 0 ? n_frames : 1);
  return align256(n * sizeof(BoxPlan)) + align256(n * sizeof(BoxClip)) +
         align256(2 * n * sizeof(int32_t)) +
         align256((size_t)kMaxFrames * FC_N * sizeof(int32_t)) + align256(GC_N * sizeof(int32_t)) +
         2 * align256(c * sizeof(float)) + align256(c * sizeof(uint8_t)) +
         (size_t)(n_frames > 0 ? n_frames : 1) * items_capacity(n_boxes_total, cap_blocks) * sizeof(ItemRec);
}

MatchWs match_ws_carve(void* base, int n_frames, int n_boxes_total, int cap_blocks) {
  const size_t n = (size_t)(n_boxes_total > 0 ? n_boxes_total : 1);
  const size_t c = (size_t)(cap_blocks > 0 ? cap_blocks : 1) * (size_t)(n_frames > 0 ? n_frames : 1);
  char* b = (char*)base;
  MatchWs ws;
  ws.plan = (BoxPlan*)b;        b += align256(n * sizeof(BoxPlan));
  ws.clip = (BoxClip*)b;        b += align256(n * sizeof(BoxClip));
  ws.litem_end = (int32_t*)b;   b += align256(2 * n * sizeof(int32_t));
  ws.fcount = (int32_t*)b;      b += align256((size_t)kMaxFrames * FC_N * sizeof(int32_t));
  ws.gcount = (int32_t*)b;      b += align256(GC_N * sizeof(int32_t));
  ws.blk_val = (float*)b;       b += align256(c * sizeof(float));
  ws.agg_tmp = (float*)b;       b += align256(c * sizeof(float));
  ws.blk_flag = (uint8_t*)b;    b += align256(c * sizeof(uint8_t));
  ws.items = (ItemRec*)b;
  ws.items_cap = items_capacity(n_boxes_total, cap_blocks);
  return ws;
}

namespace {
// the built kernels, as in launch_level, in order of preference for the default
struct BuiltVariant { int rows, nx, cpl, passes; };
// rows = 2: the row-half kernel (lanes over 32 candidate groups x 2 row halves of an
// up to 8 x 8 block, cpl candidates per group)
// rows = 1: the four-block kernel (lanes over 4 blocks of up to 4 x 4 points x 16
// candidate groups, cpl candidates per group)
constexpr BuiltVariant kBuilt[] = {
    {1, 4, 2, 1},  {1, 4, 4, 1},
    {4, 4, 2, 1},  {2, 8, 1, 1},  {2, 8, 2, 1},  {2, 8, 3, 1},  {2, 8, 4, 1},
    {4, 4, 4, 1},  {4, 4, 8, 1},  {4, 4, 16, 1}, {8, 8, 4, 1},  {8, 8, 8, 1},
    {8, 8, 6, 2},  {8, 8, 12, 1}, {8, 8, 16, 1}, {8, 8, 24, 1}, {8, 8, 32, 1}, {8, 8, 4, 2},
    {8, 8, 4, 3},  {8, 8, 4, 4},  {8, 8, 8, 2},  {4, 4, 2, 2},  {4, 4, 4, 2},
    {0, 8, 4, 1}};
}  // namespace

bool variant_valid(const PathDev& ph, int rows, int cpl, int passes) {
  // rows = 0: the generic kernel, any TILED block of up to 64 points or a GRID block
  if (rows == 0 && cpl == 4 && passes == 1)
    return ph.nd <= 256 && (ph.mode == OCSR_MODE_GRID ? ph.n_side <= 8 : ph.bw * ph.bh <= 64);
  if (ph.mode != OCSR_MODE_TILED) return false;
  for (const BuiltVariant& b : kBuilt)
    if (b.rows == rows && b.cpl == cpl && b.passes == passes)
      return b.rows == 0   ? false
             : b.rows == 1 ? ph.bw <= 4 && ph.bh <= 4 && 16 * b.cpl >= ph.nd
             : b.rows == 2 ? ph.bw <= 8 && ph.bh <= 8 && 32 * b.cpl >= ph.nd
                           : ph.bw <= b.nx && ph.bh <= b.rows && (64 / b.rows) * b.cpl * b.passes >= ph.nd;
  return false;
}

int variant_candidates(const PathDev& ph, int* rows, int* cpl, int* passes, int cap) {
  int n = 0;
  for (const BuiltVariant& b : kBuilt) {
    if (!variant_valid(ph, b.rows, b.cpl, b.passes)) continue;
    if (n < cap) {
      rows[n] = b.rows;
      cpl[n] = b.cpl;
      passes[n] = b.passes;
    }
    ++n;
  }
  return n;
}

MatchVariant pick_variant(const PathDev& ph) {
  for (const BuiltVariant& b : kBuilt)
    if (variant_valid(ph, b.rows, b.cpl, b.passes)) return MatchVariant{1, b.rows, b.cpl, b.passes};
  return MatchVariant{0, 0, 0, 0};
}

static hipError_t launch_level(const MatchParamsDev& P, const FramesDev& FR, const MatchWs& ws,
                               const DebugDev& dbg, int level, int grid, hipStream_t stream,
                               const LaunchTimer* timer, const char* name) {
  const PathDev& v = P.path[level];
#define OCSR_TILED(R, X, C, PS)                                                             \
  if (v.rows == R && v.cpl == C && v.passes == PS)                                          \
    return timed_launch(timer, name, match_tiled_kernel<R, X, C, PS>, dim3(grid), dim3(256), 0, \
                        stream, P, FR, ws, dbg, level);
  OCSR_TILED(4, 4, 2, 1)
  OCSR_TILED(4, 4, 4, 1)
  OCSR_TILED(4, 4, 8, 1)
  OCSR_TILED(4, 4, 16, 1)
  OCSR_TILED(8, 8, 4, 1)
  OCSR_TILED(8, 8, 8, 1)
  OCSR_TILED(8, 8, 12, 1)
  OCSR_TILED(8, 8, 16, 1)
  OCSR_TILED(8, 8, 24, 1)
  OCSR_TILED(8, 8, 32, 1)
  OCSR_TILED(8, 8, 4, 2)
  OCSR_TILED(8, 8, 4, 3)
  OCSR_TILED(8, 8, 4, 4)
  OCSR_TILED(8, 8, 6, 2)
  OCSR_TILED(8, 8, 8, 2)
  OCSR_TILED(4, 4, 2, 2)
  OCSR_TILED(4, 4, 4, 2)
#undef OCSR_TILED
#define OCSR_HALF(C)                                                                        \
  if (v.rows == 2 && v.cpl == C)                                                             \
    return timed_launch(timer, name, match_level_kernel<dev::HalfMatcher<C>, 4>, dim3(grid), dim3(256), \
                        0, stream, P, FR, ws, dbg, level);
  OCSR_HALF(1)
  OCSR_HALF(2)
  OCSR_HALF(3)
  OCSR_HALF(4)
#undef OCSR_HALF
  if (v.rows == 0)
    return timed_launch(timer, name, match_level_kernel<dev::GenericMatcher, 4>, dim3(grid), dim3(256), 0,
                        stream, P, FR, ws, dbg, level);
  if (v.rows == 1 && v.cpl == 2)
    return timed_launch(timer, name, match_level_kernel<dev::QuadMatcher<2>, 4>, dim3(grid), dim3(256), 0,
                        stream, P, FR, ws, dbg, level);
  if (v.rows == 1 && v.cpl == 4)
    return timed_launch(timer, name, match_level_kernel<dev::QuadMatcher<4>, 4>, dim3(grid), dim3(256), 0,
                        stream, P, FR, ws, dbg, level);
  return hipErrorNotSupported;   // rejected by the argument checks before any launch
}

// One launch for both levels when a kernel for the pair of variants is built (with
// launch == false: only whether it is built).
#define COMMA ,
static bool launch_pair(const MatchParamsDev& P, const FramesDev& FR, const MatchWs& ws,
                        const DebugDev& dbg, int grid, hipStream_t stream, const LaunchTimer* timer,
                        bool launch) {
  const PathDev& f = P.path[0];
  const PathDev& c = P.path[1];
  if (f.passes != 1) return false;
#define OCSR_PAIR(FRW, FXW, FCP, CRW, CXW, CCP, CPS)                                     \
  if (f.rows == FRW && f.cpl == FCP && c.rows == CRW && c.cpl == CCP && c.passes == CPS) { \
    if (launch)                                                                          \
      timed_launch(timer, "match", match_pair_kernel<FRW, FXW, FCP, CRW, CXW, CCP, CPS>,    \
                   dim3(grid), dim3(256), 0, stream, P, FR, ws, dbg);                     \
    return true;                                                                         \
  }
  OCSR_PAIR(4, 4, 2, 8, 8, 8, 1)
  OCSR_PAIR(4, 4, 2, 8, 8, 12, 1)
  OCSR_PAIR(4, 4, 2, 8, 8, 16, 1)
  OCSR_PAIR(4, 4, 4, 8, 8, 8, 1)
  OCSR_PAIR(4, 4, 4, 8, 8, 12, 1)
  OCSR_PAIR(8, 8, 8, 8, 8, 8, 1)
  OCSR_PAIR(8, 8, 8, 8, 8, 12, 1)
  OCSR_PAIR(8, 8, 8, 8, 8, 16, 1)
  OCSR_PAIR(4, 4, 2, 8, 8, 4, 3)
  OCSR_PAIR(4, 4, 2, 8, 8, 6, 2)
  OCSR_PAIR(4, 4, 2, 8, 8, 4, 2)
#undef OCSR_PAIR
#define OCSR_PAIR2(FM, FRW, FCP, FPS, CCP)                                                  \
  if (f.rows == FRW && f.cpl == FCP && f.passes == FPS && c.rows == 2 && c.cpl == CCP) {    \
    if (launch)                                                                          \
      timed_launch(timer, "match", match_pair2_kernel<FM, dev::HalfMatcher<CCP>, 4>, dim3(grid),  \
                   dim3(256), 0, stream, P, FR, ws, dbg);                                 \
    return true;                                                                         \
  }
  OCSR_PAIR2(dev::TiledMatcher<4 COMMA 4 COMMA 2 COMMA 1>, 4, 2, 1, 2)
  OCSR_PAIR2(dev::TiledMatcher<4 COMMA 4 COMMA 2 COMMA 1>, 4, 2, 1, 3)
  OCSR_PAIR2(dev::TiledMatcher<4 COMMA 4 COMMA 2 COMMA 1>, 4, 2, 1, 4)
  OCSR_PAIR2(dev::HalfMatcher<1>, 2, 1, 1, 3)
  OCSR_PAIR2(dev::HalfMatcher<2>, 2, 2, 1, 3)
  OCSR_PAIR2(dev::HalfMatcher<2>, 2, 2, 1, 4)
  OCSR_PAIR2(dev::HalfMatcher<3>, 2, 3, 1, 3)
  OCSR_PAIR2(dev::QuadMatcher<2>, 1, 2, 1, 3)
  OCSR_PAIR2(dev::QuadMatcher<2>, 1, 2, 1, 4)
  OCSR_PAIR2(dev::GenericMatcher, 0, 4, 1, 3)
#undef OCSR_PAIR2
  return false;
}

hipError_t launch_frame_census(const MatchParamsDev& P, const FramesDev& FR,
                               const ocsr_box* boxes, const MatchWs& ws, int sx, int sy,
                               int sentinel, int n_census_tiles, hipStream_t stream,
                               const LaunchTimer* timer) {
  const dim3 grid(FR.n + n_census_tiles), block(256);
  auto kernel = sx == 3 && sy == 4   ? frame_census_kernel<3, 4>
                : sx == 2 && sy == 2 ? frame_census_kernel<2, 2>
                : sx == 4 && sy == 3 ? frame_census_kernel<4, 3>
                                     : frame_census_kernel<-1, -1>;
  return timed_launch(timer, "census", kernel, grid, block, 0, stream, P, FR, boxes, ws, sx, sy,
                      sentinel);
}

template <int SX, int SY>
static int census_list_occupancy() {
  static const int occ = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, census_list_kernel<SX, SY>, 256, 0) != hipSuccess)
      n = 1;
    return n > 0 ? n : 1;
  }();
  return occ;
}

hipError_t launch_plan_and_census(const MatchParamsDev& P, const FramesDev& FR,
                                  const ocsr_box* boxes, const MatchWs& ws, int sx, int sy,
                                  int sentinel, int n_cu, hipStream_t stream,
                                  const LaunchTimer* timer) {
  int n_tiles = 0;
  for (int f = 0; f < FR.n; ++f) {
    const int t = 2 * (FR.f[f].tiles0 + FR.f[f].tiles1);
    if (t > 32 * kFrameTileWords) return hipErrorNotSupported;
    n_tiles += t;
  }
  const bool w34 = sx == 3 && sy == 4, w22 = sx == 2 && sy == 2, w43 = sx == 4 && sy == 3;
  const int occ = w34 ? census_list_occupancy<3, 4>() : w22 ? census_list_occupancy<2, 2>()
                  : w43 ? census_list_occupancy<4, 3>() : census_list_occupancy<-1, -1>();
  // lists pay off once every persistent workgroup has several tiles to consider (a
  // 1080p frame's 2550 tiles run faster one workgroup per tile, a 16-frame batch's
  // 45600 listed)
  if (8 * std::max(1, n_cu) * occ > n_tiles) return hipErrorNotSupported;
  hipError_t e = timed_launch(timer, "plan", plan_tiles_kernel, dim3(FR.n), dim3(256), 0, stream, P,
                              FR, boxes, ws);
  if (e != hipSuccess) return e;
  auto kernel = w34 ? census_list_kernel<3, 4> : w22 ? census_list_kernel<2, 2>
                : w43 ? census_list_kernel<4, 3> : census_list_kernel<-1, -1>;
  // (shares are cut in 32-bit arithmetic, which takes grids below 46341)
  return timed_launch(timer, "census", kernel, dim3(std::min(std::max(1, n_cu) * occ, 46340)), dim3(256), 0, stream,
                      P, FR, boxes, ws, sx, sy, sentinel);
}

hipError_t launch_match(const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, const DebugDev& dbg,
                        bool plan_done, int n_match_wgs, int level_launches, hipStream_t stream,
                        const LaunchTimer* timer) {
  if (FR.n_boxes_total <= 0) return hipSuccess;
  hipError_t e;
  if (!plan_done) {
    if (timer) timer->before(timer->ctx, "plan", stream);
    plan_kernel<<<FR.n, 64, 0, stream>>>(P, FR, boxes, ws);
    if (timer) timer->after(timer->ctx, "plan", stream);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (P.vertical) {
    // both levels in one launch; when both fit the wider matcher (ROWS = 8, which also
    // takes 4 x 4 blocks, half its lanes idle) it serves both levels
    int fr_rows = dy_rows(P.path[0].bw, P.path[0].bh), cr_rows = dy_rows(P.path[1].bw, P.path[1].bh);
    auto fits8 = [](const PathDev& ph) {
      return dy_strip_words(8, ph.nd) <= 64 * dy_chunks(8) &&
             kItemWaves * dy_wave_lds_bytes(8, ph.nd, ph.ndy) <= kDyMaxWgLds;
    };
    if (fr_rows != cr_rows && fits8(P.path[0]) && fits8(P.path[1])) fr_rows = cr_rows = 8;
    const size_t wave_bytes = std::max(dy_wave_lds_bytes(fr_rows, P.path[0].nd, P.path[0].ndy),
                                       dy_wave_lds_bytes(cr_rows, P.path[1].nd, P.path[1].ndy));
    const size_t bytes = kItemWaves * wave_bytes;
    if (bytes > kDyMaxWgLds) return hipErrorInvalidValue;   // rejected by the argument checks
    const int wb = (int)wave_bytes;
    auto kernel = fr_rows == 4 && cr_rows == 8   ? match_dy_pair_kernel<4, 8>
                  : fr_rows == 8 && cr_rows == 8 ? match_dy_pair_kernel<8, 8>
                  : fr_rows == 4 && cr_rows == 4 ? match_dy_pair_kernel<4, 4>
                                                 : match_dy_pair_kernel<8, 4>;
    e = timed_launch(timer, "match", kernel, dim3(n_match_wgs), dim3(256), bytes, stream, P, FR, ws,
                     dbg, wb);
    if (e != hipSuccess) return e;
  } else if ((level_launches == 2 || (level_launches == 0 && FR.n == 1)) &&
             launch_pair(P, FR, ws, dbg, n_match_wgs, stream, nullptr, false)) {
    // one launch for both levels: in a one-frame call the far level alone cannot fill
    // the GPU, and its blocks fill the close level's tail (whole 1080p frame: 31 against
    // 38 us per frame); each level of a batch fills the GPU by itself, and there the two
    // forms are about even (16 frames: 117.5 against 10.3 + 109.2 us)
    e = launch_pair(P, FR, ws, dbg, n_match_wgs, stream, timer, true) ? hipGetLastError() : hipErrorNotSupported;
    if (e != hipSuccess) return e;
  } else {
    // close blocks first: they carry most of the work
    for (int level = 1; level >= 0; --level) {
      e = launch_level(P, FR, ws, dbg, level, n_match_wgs, stream, timer,
                       level == 0 ? "match_far" : "match_close");
      if (e != hipSuccess) return e;
    }
  }
  return timed_launch(timer, "aggregate", aggregate_kernel, dim3(FR.n_boxes_total), dim3(256), 0,
                      stream, P, ws, out);
}

}  // namespace ocsr
