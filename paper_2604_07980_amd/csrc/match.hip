// Multi-launch matching path (Sec. 4.3.2-4.3.6, Alg. 2): plan, one grid-stride launch per
// level (far blocks, close blocks), one aggregation workgroup per box. The steps are in
// dev_match.hpp, shared with the fused persistent kernel.
#include "dev_match.hpp"

namespace ocsr {
namespace {

// one wave per frame
__global__ __launch_bounds__(64) void plan_kernel(MatchParamsDev P, FramesDev FR,
                                                  const ocsr_box* boxes, MatchWs ws) {
  const int f = blockIdx.x;
  dev::plan_frame(P, FR.f[f], f, FR.n_boxes_total, boxes, ws, threadIdx.x);
}

__global__ __launch_bounds__(64) void match_generic_kernel(MatchParamsDev P, FramesDev FR,
                                                           MatchWs ws, DebugDev dbg, int level) {
  dev::level_blocks(FR, ws, level, [&](int f, int q) {
    dev::match_block_generic(P, FR.f[f], f, FR.n_boxes_total, ws, dbg, level, q, false,
                             threadIdx.x);
  });
}

template <int ROWS, int NX, int CPL>
__global__ __launch_bounds__(64) void match_tiled_kernel(MatchParamsDev P, FramesDev FR,
                                                         MatchWs ws, DebugDev dbg, int level) {
  __shared__ uint64_t lds[(dev::Tiled<ROWS, NX, CPL>::kLdsBytes + 7) / 8];
  dev::level_blocks(FR, ws, level, [&](int f, int q) {
    dev::match_block_tiled<ROWS, NX, CPL>(P, FR.f[f], f, FR.n_boxes_total, ws, dbg, level, q,
                                          false, threadIdx.x, lds);
  });
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
         align256(2 * n * sizeof(int32_t)) + align256(n * sizeof(int32_t)) +
         align256((size_t)kMaxFrames * FC_N * sizeof(int32_t)) + align256(GC_N * sizeof(int32_t)) +
         align256(c * sizeof(float)) + align256(c * sizeof(uint8_t));
}

MatchWs match_ws_carve(void* base, int n_frames, int n_boxes_total, int cap_blocks) {
  const size_t n = (size_t)(n_boxes_total > 0 ? n_boxes_total : 1);
  const size_t c = (size_t)(cap_blocks > 0 ? cap_blocks : 1) * (size_t)(n_frames > 0 ? n_frames : 1);
  char* b = (char*)base;
  MatchWs ws;
  ws.plan = (BoxPlan*)b;        b += align256(n * sizeof(BoxPlan));
  ws.clip = (BoxClip*)b;        b += align256(n * sizeof(BoxClip));
  ws.lbox_end = (int32_t*)b;    b += align256(2 * n * sizeof(int32_t));
  ws.box_done = (int32_t*)b;    b += align256(n * sizeof(int32_t));
  ws.fcount = (int32_t*)b;      b += align256((size_t)kMaxFrames * FC_N * sizeof(int32_t));
  ws.gcount = (int32_t*)b;      b += align256(GC_N * sizeof(int32_t));
  ws.blk_val = (float*)b;       b += align256(c * sizeof(float));
  ws.blk_flag = (uint8_t*)b;
  return ws;
}

MatchVariant pick_variant(const PathDev& ph) {
  MatchVariant v = {0, 0, 0};
  if (ph.mode != OCSR_MODE_TILED) return v;
  static const int cpl4[] = {2, 4, 8, 16};
  static const int cpl8[] = {4, 8, 12, 16, 24, 32};
  if (ph.bw <= 4 && ph.bh <= 4) {
    for (int c : cpl4)
      if (16 * c >= ph.nd) return MatchVariant{1, 4, c};
  } else if (ph.bw <= 8 && ph.bh <= 8) {
    for (int c : cpl8)
      if (8 * c >= ph.nd) return MatchVariant{1, 8, c};
  }
  return v;
}

static hipError_t launch_level(const MatchParamsDev& P, const FramesDev& FR, const MatchWs& ws,
                               const DebugDev& dbg, int level, int grid, hipStream_t stream) {
  const MatchVariant v = pick_variant(P.path[level]);
#define OCSR_TILED(R, X, C)                                                          \
  if (v.tiled && v.rows == R && v.cpl == C) {                                        \
    match_tiled_kernel<R, X, C><<<grid, 64, 0, stream>>>(P, FR, ws, dbg, level);    \
    return hipGetLastError();                                                        \
  }
  OCSR_TILED(4, 4, 2)
  OCSR_TILED(4, 4, 4)
  OCSR_TILED(4, 4, 8)
  OCSR_TILED(4, 4, 16)
  OCSR_TILED(8, 8, 4)
  OCSR_TILED(8, 8, 8)
  OCSR_TILED(8, 8, 12)
  OCSR_TILED(8, 8, 16)
  OCSR_TILED(8, 8, 24)
  OCSR_TILED(8, 8, 32)
#undef OCSR_TILED
  match_generic_kernel<<<grid, 64, 0, stream>>>(P, FR, ws, dbg, level);
  return hipGetLastError();
}

hipError_t launch_match(const MatchParamsDev& P, const FramesDev& FR, const ocsr_box* boxes,
                        const MatchWs& ws, ocsr_box_result* out, const DebugDev& dbg,
                        int n_match_wgs, hipStream_t stream, const LaunchTimer* timer) {
  if (FR.n_boxes_total <= 0) return hipSuccess;
  hipError_t e;
  if (timer) timer->before(timer->ctx, "plan", stream);
  plan_kernel<<<FR.n, 64, 0, stream>>>(P, FR, boxes, ws);
  if (timer) timer->after(timer->ctx, "plan", stream);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // close blocks first: they carry most of the work
  for (int level = 1; level >= 0; --level) {
    const char* name = level == 0 ? "match_far" : "match_close";
    if (timer) timer->before(timer->ctx, name, stream);
    e = launch_level(P, FR, ws, dbg, level, n_match_wgs, stream);
    if (timer) timer->after(timer->ctx, name, stream);
    if (e != hipSuccess) return e;
  }
  if (timer) timer->before(timer->ctx, "aggregate", stream);
  aggregate_kernel<<<FR.n_boxes_total, 256, 0, stream>>>(P, ws, out);
  if (timer) timer->after(timer->ctx, "aggregate", stream);
  return hipGetLastError();
}

}  // namespace ocsr
