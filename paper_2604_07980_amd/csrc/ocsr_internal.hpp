// Internal declarations shared by the HIP translation units of libocsr.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>

#include "ocsr.h"

namespace ocsr {

// Records msg as the calling thread's last error message and returns code.
int32_t report_error(int32_t code, const char* msg);

// ---------------------------------------------------------------------------------
// census
// ---------------------------------------------------------------------------------
struct CensusJobDev {
  const uint8_t* img;
  uint64_t* out;
  int32_t W, H, pitch, out_pitch;  // source size and pitch (bytes), output pitch (words)
  int32_t scale;
  int32_t tiles_x;                 // tiles along x of this job
  int32_t tile_begin;              // first global tile index of this job
  int32_t pad;
};

struct CensusJobsDev {
  CensusJobDev job[OCSR_MAX_CENSUS_JOBS];
  int32_t n;
};

// census tile: 64 columns x 32 rows of level pixels per workgroup of 256 threads
constexpr int kCensusTileX = 64;
constexpr int kCensusTileY = 32;
// plan step of whole-frame calls: the census tiles of one frame it can list (bitmap
// words in LDS); frames with more tiles take the per-tile census
constexpr int kFrameTileWords = 4096;

hipError_t launch_census(const CensusJobsDev& jobs, int total_tiles, int sx, int sy,
                         int sentinel, hipStream_t stream);

// ---------------------------------------------------------------------------------
// matching
// ---------------------------------------------------------------------------------
constexpr int kMaxFrames = OCSR_MAX_BATCH_FRAMES;

struct LevelDev {
  const uint64_t* L;
  const uint64_t* R;
  int32_t W, H, pitch, scale, sx, sy;
};

struct PathDev {
  int32_t mode, bw, bh, n_side;
  int32_t dlo, nd;                 // level search range [dlo, dlo + nd)
  int32_t rows, cpl, passes;       // matching kernel variant (chosen on the host)
  int32_t dylo, ndy;               // level vertical offsets [dylo, dylo + ndy)
};

// Matching parameters shared by every frame of a call.
struct MatchParamsDev {
  PathDev path[2];                 // 0: far path (scale 1), 1: close path (close scale)
  int32_t tau_s;
  int32_t lr_tol, min_point_pct, agg_mode;
  float tau_d;
  int32_t n_min, trim_pct;
  float fb;                        // focal_px * baseline_m, one fp32 multiply
  float d_eps;
  int32_t cap_blocks;              // block capacity of one frame
  int32_t item_blocks[2];          // blocks per work item of each level: kItemWaves x
                                   // the blocks one wave takes
  int32_t full_census;             // whole-frame calls: 1 = census of every tile, 0 = only
                                   // of the tiles some box's search reads
  int32_t vertical;                // 1: a vertical range is searched (the dy kernels run)
};

// Kernel of a path with a vertical range: one wave per block, NX x ROWS points, lanes
// (row, group of dy_cpl(ROWS) consecutive candidates), the candidates in runtime passes
// of kDyPass; per wave an LDS ring of ROWS + 1 strip rows of dy_strip_words words (each
// vertical step loads one new row), the template, and the forward and backward costs of
// every (d, dy) as uint16. A strip row is loaded in at most dy_chunks(ROWS) 64-word
// chunks per lane.
constexpr int kDyPass = 32;
inline int dy_rows(int bw, int bh) { return bw <= 4 && bh <= 4 ? 4 : 8; }
constexpr int dy_cpl(int rows) { return rows == 4 ? 2 : 4; }
constexpr int dy_chunks(int rows) { return rows == 4 ? 5 : 3; }
constexpr int dy_strip_words(int rows, int nd) { return (nd + kDyPass - 1) / kDyPass * kDyPass + rows - 1; }
// When all ROWS + ndy - 1 strip rows of a direction fit kDyFullLoads loads per lane they
// are staged at once (one round trip), else the ring of ROWS + 1 rows is used.
constexpr int kDyFullLoads = 16;
constexpr bool dy_full(int rows, int nd, int ndy) {
  return (rows + ndy - 1) * dy_strip_words(rows, nd) <= 64 * kDyFullLoads;
}
constexpr int dy_lds_rows(int rows, int nd, int ndy) { return dy_full(rows, nd, ndy) ? rows + ndy - 1 : rows + 1; }
inline size_t dy_wave_lds_bytes(int rows, int nd, int ndy) {
  auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
  return r16(sizeof(uint64_t) * dy_lds_rows(rows, nd, ndy) * dy_strip_words(rows, nd)) +
         r16(sizeof(uint64_t) * rows * rows) + 2 * r16(sizeof(uint16_t) * (size_t)nd * ndy);
}
constexpr size_t kDyMaxWgLds = 65536;   // LDS of one dy workgroup (kItemWaves waves)

// One frame of a call: descriptor levels, its boxes and (whole-frame calls) its images.
struct FrameDev {
  LevelDev lv[2];
  const uint8_t* imgL;             // whole-frame calls: the images the census is made from
  const uint8_t* imgR;
  int32_t W, H, pitch;             // full-resolution image size and pitch (bytes)
  int32_t box_off, n_boxes;        // the frame's boxes: [box_off, box_off + n_boxes)
  int32_t tile_begin;              // first census tile of the frame in the call's numbering
  int32_t* tile_list;              // whole-frame calls: the frame's tiles to make (frame-local
                                   // numbers), written by the plan step
  int32_t tiles0_x, tiles0, tiles1_x, tiles1;   // census tiles per view at levels 0 / 1
  uint64_t tx_recip[2];            // ceil(2^40 / tiles_x) of levels 0 / 1: t / tiles_x is
                                   // (t * tx_recip) >> 40, exactly, for t < 2^30
};

struct FramesDev {
  FrameDev f[kMaxFrames];
  int32_t n;
  int32_t n_boxes_total;
};

// Per-box plan, written by the plan step (one 64-byte record per box).
struct BoxPlan {
  int32_t status;                  // -1: to be matched; else an OCSR_REASON_* code
  int32_t level;                   // 0 far, 1 close
  int32_t lx0, ly0, lw, lh;        // level box
  int32_t nbx, nby;                // blocks along x / y
  int32_t bw, bh;                  // points per block along x / y
  int32_t ox, oy;                  // TILED: origin of block (0, 0)
  int32_t off;                     // first block number within the frame
  int32_t nblk;                    // blocks matched (0 if not matched)
  int32_t ioff;                    // first work item among the frame's boxes of its level
  int32_t frame;
};

struct BoxClip {
  int32_t cx0, cy0, cx1, cy1;      // clipped box; empty boxes are all zero
};

// Matching work is dealt in items of up to item_blocks consecutive blocks of one box
// (blocks per wave x the 4 waves of a 256-thread workgroup).
constexpr int kItemWaves = 4;
constexpr int kMaxBlocksPerWave = 8;

// per-frame counters: blocks numbered, block end of the matched boxes, work items of
// the far and close levels
enum { FC_NUMBERED = 0, FC_MATCHED = 1, FC_FAR_ITEMS = 2, FC_CLOSE_ITEMS = 3, FC_TILES = 4, FC_N = 8 };
// call-wide counters: the timeout flag, and the arrival slots of the fused launch's two
// grid barriers (arrivals spread over kBarSlots counters to keep atomics uncontended)
constexpr int kBarSlots = 8;
enum { GC_TIMEOUT = 0, GC_BAR0 = 8, GC_BAR1 = 16, GC_BAR2 = 24, GC_N = 32 };

// A work item as the plan writes it: the box, the item's first block and the box's
// block geometry, so that a matching workgroup reads one record (one cache line) and
// can stage its blocks' strips at once.
struct ItemRec {
  int32_t k;                       // box within the frame
  int32_t first;                   // the item's first block (0-based within the box)
  int32_t nblk, off;               // the box's blocks and its first block number
  int32_t nbx, bw, bh, ox, oy;     // block grid
  int32_t lx0, ly0, lw, lh;        // level box
  int32_t pad[3];
};
static_assert(sizeof(ItemRec) == 64, "one cache line per record");

struct MatchWs {
  BoxPlan* plan;       // [n_boxes_total]
  BoxClip* clip;       // [n_boxes_total]
  int32_t* litem_end;  // [2][n_boxes_total] per level and frame: running work-item end
  int32_t* fcount;     // [kMaxFrames][FC_N]
  int32_t* gcount;     // [GC_N]
  float* blk_val;      // [n_frames][cap_blocks] full-res disparity of a valid block
  float* agg_tmp;      // [n_frames][cap_blocks] sort buffer of the aggregation of boxes
                       // with more blocks than it keeps in LDS
  uint8_t* blk_flag;   // [n_frames][cap_blocks] bit 0 eligible, bit 1 valid
  ItemRec* items;      // [n_frames][items_cap]: a frame's close items, then its far items
  int32_t items_cap;   // records per frame
};

// Work items of a frame of at most cap_blocks blocks: items hold at least kItemWaves
// blocks of one box, so there are at most cap_blocks / kItemWaves + one per box.
inline int32_t items_capacity(int n_boxes_total, int cap_blocks) {
  return (cap_blocks > 0 ? cap_blocks : 1) / kItemWaves + (n_boxes_total > 0 ? n_boxes_total : 1);
}

size_t match_ws_bytes(int n_frames, int n_boxes_total, int cap_blocks);
MatchWs match_ws_carve(void* base, int n_frames, int n_boxes_total, int cap_blocks);

struct DebugDev {
  int32_t cap_blocks, cap_nd;
  int32_t* n_blocks;
  ocsr_block_record* blocks;
  uint16_t* cost_fwd;
  uint16_t* cost_bwd;
};

// launch hooks: a callback that brackets each kernel with timing events
struct LaunchTimer {
  void* ctx;
  void (*before)(void* ctx, const char* name, hipStream_t s);
  void (*after)(void* ctx, const char* name, hipStream_t s);
  // two events for one launch to carry, registered under `name` (false: none left)
  bool (*pair)(void* ctx, const char* name, hipEvent_t* start, hipEvent_t* stop);
};

// kernel<<<grid, block, shmem, s>>>(args...). With a timer the launch carries its own
// start and stop events, which the GPU stamps when the kernel starts and ends, so the
// time is the kernel's own, not the dispatch gap around it as with events recorded on the
// stream before and after.
template <typename... KArgs, typename... Args>
hipError_t timed_launch(const LaunchTimer* timer, const char* name, void (*kernel)(KArgs...),
                        dim3 grid, dim3 block, size_t shmem, hipStream_t s, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (timer && timer->pair && timer->pair(timer->ctx, name, &a, &b))
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, s, a, b, 0, static_cast<KArgs>(args)...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, static_cast<KArgs>(args)...);
  return hipGetLastError();
}

// Kernel variant of one level's blocks: the register-blocked TILED kernel with `rows`
// block rows per wave (4: blocks up to 4 x 4, 8: up to 8 x 8), `cpl` consecutive
// candidates per lane and `passes` passes over the candidates, which covers
// (64 / rows) * cpl * passes level candidates. Other shapes (GRID mode, wider blocks,
// wider ranges) have no register-blocked kernel; the generic kernel takes those it covers.
struct MatchVariant {
  int tiled;           // 1: a register-blocked TILED kernel exists
  int rows, cpl, passes;
};
// the default: the first built variant (in launch order) that covers the block and range
MatchVariant pick_variant(const PathDev& ph);
// whether the (rows, cpl, passes) kernel is built and covers the path's blocks and range
bool variant_valid(const PathDev& ph, int rows, int cpl, int passes);
// every built variant that covers the path, up to cap of them; returns the count
int variant_candidates(const PathDev& ph, int* rows, int* cpl, int* passes, int cap);

// Census of every view and level of every frame, and the plan of every frame, in one
// launch (frames whose images are given).
// Census (and plan) launch of a whole-frame call: one workgroup per census tile tests
// whether some box's search reads its tile and makes it if so; one more per frame plans it.
hipError_t launch_frame_census(const MatchParamsDev& p, const FramesDev& fr,
                               const ocsr_box* boxes, const MatchWs& ws, int sx, int sy,
                               int sentinel, int n_census_tiles, hipStream_t stream,
                               const LaunchTimer* timer);

// Plan of every frame of a whole-frame call, with the list of the census tiles its boxes'
// searches read (one workgroup per frame), then the census of the listed tiles by
// persistent workgroups. Returns hipErrorNotSupported (nothing launched) when a frame has
// more tiles than the plan step can list.
hipError_t launch_plan_and_census(const MatchParamsDev& p, const FramesDev& fr,
                                  const ocsr_box* boxes, const MatchWs& ws, int sx, int sy,
                                  int sentinel, int n_cu, hipStream_t stream,
                                  const LaunchTimer* timer);

// Multi-launch matching: the plan (unless plan_done), the matching of both levels'
// blocks, then one aggregation workgroup per box. level_launches (OCSR_OPTION_LEVEL_LAUNCHES)
// decides between one launch for both levels, when a kernel for the pair of variants
// is built, and one launch per level.
hipError_t launch_match(const MatchParamsDev& p, const FramesDev& fr, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, const DebugDev& dbg,
                        bool plan_done, int n_match_wgs, int level_launches, hipStream_t stream,
                        const LaunchTimer* timer);

// Fused path: census of every frame, planning, matching and aggregation in one
// persistent launch of co-resident workgroups (after a counter reset). Returns
// hipErrorNotSupported when no fused kernel is built for this census window and pair of
// path variants, or when a frame has more census tiles than the plan step can list.
// wgs_per_cu caps the workgroups per compute unit (0: the library default, 2).
hipError_t launch_fused(const MatchParamsDev& p, const FramesDev& fr, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, int sx, int sy, int sentinel,
                        int n_cu, int wgs_per_cu, hipStream_t stream, const LaunchTimer* timer);
bool fused_available(const MatchParamsDev& p, const FramesDev& fr, int sx, int sy);

// Dense counterpart: left-view and right-view winner-take-all over [dmin, dmax] of the
// (2 radius + 1)^2 window sums of Hamming costs, then the left/right check. d_left and
// d_right: int16 [H][W] scratch (d_right also an output when the caller asks for it).
static_assert(sizeof(ocsr_box_point) == 64, "box point layout");
static_assert(sizeof(ocsr_block_record) == 80, "block record layout");

// fp32 copy of ocsr_point_params for the point kernel
struct PointParamsDev {
  int32_t width, height;
  float Q[16], R[9], t[3];
  float fb;                        // f * b, one fp32 multiply
  float var_d, var_x, var_y;
};
// Priority object selection: per frame its size, crop in px and box range.
struct SelectFrameDev {
  int32_t W, H, X0, Y0, X1, Y1;
  int32_t box_off, n_boxes;
};
struct SelectDev {
  int32_t n;
  int32_t max_objects;
  SelectFrameDev f[OCSR_MAX_BATCH_FRAMES];
};
hipError_t launch_select(const SelectDev& S, const ocsr_box* in, ocsr_box* out, int32_t* rank,
                         int max_boxes, hipStream_t stream, const LaunchTimer* timer);

hipError_t launch_box_points(const ocsr_box* boxes, const ocsr_box_result* res, int n,
                             const PointParamsDev& pp, ocsr_box_point* out, hipStream_t stream,
                             const LaunchTimer* timer);

bool dense_radius_supported(int radius);
hipError_t launch_dense_offsets(const uint64_t* CL0, const uint64_t* CR, int W, int H, int pitch,
                                int nz, int dmin, int dmax, int radius, int lr_tol, int d_min,
                                int16_t* disp, int16_t* d_left, int16_t* d_right, int32_t* partial,
                                int32_t* counts, hipStream_t stream, const LaunchTimer* timer);
hipError_t launch_dense(const uint64_t* CL, const uint64_t* CR, int W, int H, int pitch, int dmin,
                        int dmax, int radius, int lr_tol, int16_t* disp, int16_t* d_left,
                        int16_t* d_right, hipStream_t stream, const LaunchTimer* timer);

}  // namespace ocsr
