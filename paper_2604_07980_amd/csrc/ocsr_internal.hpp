// Internal declarations shared by the HIP translation units of libocsr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ocsr.h"

namespace ocsr {

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

hipError_t launch_census(const CensusJobsDev& jobs, int total_tiles, int sx, int sy,
                         int sentinel, hipStream_t stream);

// ---------------------------------------------------------------------------------
// matching
// ---------------------------------------------------------------------------------
struct LevelDev {
  const uint64_t* L;
  const uint64_t* R;
  int32_t W, H, pitch, scale, sx, sy;
};

struct PathDev {
  int32_t mode, bw, bh, n_side;
  int32_t dlo, nd;                 // level search range [dlo, dlo + nd)
};

struct MatchParamsDev {
  LevelDev lv[2];                  // 0: far level (scale 1), 1: close level
  PathDev path[2];
  int32_t tau_s;
  int32_t lr_tol, min_point_pct, agg_mode;
  float tau_d;
  int32_t n_min, trim_pct;
  float fb;                        // focal_px * baseline_m, one fp32 multiply
  float d_eps;
  int32_t cap_blocks;
  int32_t n_boxes;
};

// Per-box plan, written by the plan kernel (one 64-byte record per box).
struct BoxPlan {
  int32_t status;                  // -1: to be matched; else an OCSR_REASON_* code
  int32_t level;                   // 0 far, 1 close
  int32_t lx0, ly0, lw, lh;        // level box
  int32_t nbx, nby;                // blocks along x / y
  int32_t bw, bh;                  // points per block along x / y
  int32_t ox, oy;                  // TILED: origin of block (0, 0)
  int32_t off;                     // first block number
  int32_t nblk;                    // blocks matched (0 if not matched)
  int32_t cx0, cy0;                // clipped box (full res); cx1, cy1 in BoxClip
};

struct BoxClip {
  int32_t cx0, cy0, cx1, cy1;      // clipped box; empty boxes have cx0 >= cx1
};

struct MatchWs {
  BoxPlan* plan;       // [n_boxes]
  BoxClip* clip;       // [n_boxes]
  int32_t* box_end;    // [n_boxes] off + nblk (monotone)
  int32_t* counters;   // [4]: 0 blocks numbered, 1 blocks matched
  float* blk_val;      // [cap_blocks] full-res disparity of a valid block
  uint8_t* blk_flag;   // [cap_blocks] bit 0 eligible, bit 1 valid
};

size_t match_ws_bytes(int n_boxes, int cap_blocks);
MatchWs match_ws_carve(void* base, int n_boxes, int cap_blocks);

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
};

hipError_t launch_match(const MatchParamsDev& p, const ocsr_box* boxes, const MatchWs& ws,
                        ocsr_box_result* out, const DebugDev& dbg, int n_match_wgs,
                        hipStream_t stream, const LaunchTimer* timer);

}  // namespace ocsr
