// C ABI of libocsr: argument validation, workspace layout, launches and timing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <cstdlib>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ocsr_internal.hpp"

using namespace ocsr;

// Temporal filter of the auto-rectification offset: the last `window` estimates and the
// previous output.
struct ocsr_rect_filter {
  int window = 1, max_step = 0, prev = 0;
  std::deque<int> hist;
};

struct ocsr_ctx {
  int device = 0;
  int n_cu = 256;
  bool timing = false;
  int use_fused = 0;
  int wgs_per_cu = 0;
  struct Pending {
    std::string name;
    hipEvent_t start, stop;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  std::map<std::string, std::pair<int64_t, double>> stats;
  hipEvent_t open_start = nullptr;
  // graph submission: instantiated launch sequences of whole-frame calls, most
  // recently used first, keyed by everything the launches depend on
  int use_graph = 0;
  // matching kernel variants chosen for (bw, bh, level candidates), e.g. by a tuner
  std::map<std::array<int, 3>, std::array<int, 3>> variants;
  int match_wgs_per_cu = 16;
  int blocks_per_wave = 1;
  int full_census = 0;
  int census_list = 1;
  int level_launches = 0;   // OCSR_OPTION_LEVEL_LAUNCHES
  struct Graph {
    std::string key;
    hipGraphExec_t exec;
  };
  std::list<Graph> graphs;
  hipStream_t capture_stream = nullptr;
  int64_t graph_hits = 0, graph_builds = 0;
};

constexpr size_t kMaxGraphs = 128;

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

// a status with its message, for the other translation units
int32_t ocsr::report_error(int32_t code, const char* msg) { return fail(code, "%s", msg); }

namespace {

int32_t hip_fail(hipError_t e, const char* what) {
  return fail(OCSR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

hipEvent_t take_event(ocsr_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void timer_before(void* ctx, const char* name, hipStream_t s) {
  (void)name;
  ocsr_ctx* c = (ocsr_ctx*)ctx;
  c->open_start = take_event(c);
  if (c->open_start) hipEventRecord(c->open_start, s);
}

void timer_after(void* ctx, const char* name, hipStream_t s) {
  ocsr_ctx* c = (ocsr_ctx*)ctx;
  hipEvent_t stop = take_event(c);
  if (!c->open_start || !stop) return;
  hipEventRecord(stop, s);
  c->pending.push_back({name, c->open_start, stop});
  c->open_start = nullptr;
}

bool timer_pair(void* ctx, const char* name, hipEvent_t* start, hipEvent_t* stop) {
  ocsr_ctx* c = (ocsr_ctx*)ctx;
  hipEvent_t a = take_event(c);
  if (!a) return false;
  hipEvent_t b = take_event(c);
  if (!b) {
    c->free_events.push_back(a);
    return false;
  }
  c->pending.push_back({name, a, b});
  *start = a;
  *stop = b;
  return true;
}

LaunchTimer make_timer(ocsr_ctx* c) { return LaunchTimer{c, timer_before, timer_after, timer_pair}; }

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Replays the graph cached under `key`, or captures the call's launches (enqueue, on
// the context's own capture stream, so that capture never touches the caller's
// stream), instantiates them and replays that. The least recently used graph is
// dropped beyond kMaxGraphs. With timing on, the replay is timed as "graph".
int32_t graph_launch(ocsr_ctx* ctx, const std::string& key,
                     const std::function<int32_t(hipStream_t, const LaunchTimer*)>& enqueue,
                     hipStream_t stream) {
  hipError_t e;
  auto it = std::find_if(ctx->graphs.begin(), ctx->graphs.end(),
                         [&](const ocsr_ctx::Graph& g) { return g.key == key; });
  if (it != ctx->graphs.end()) {
    ctx->graphs.splice(ctx->graphs.begin(), ctx->graphs, it);
    ++ctx->graph_hits;
  } else {
    if (!ctx->capture_stream) {
      e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const int32_t rc = enqueue(ctx->capture_stream, nullptr);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (rc != OCSR_OK) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    ctx->graphs.push_front({key, exec});
    ++ctx->graph_builds;
    while (ctx->graphs.size() > kMaxGraphs) {
      hipGraphExecDestroy(ctx->graphs.back().exec);
      ctx->graphs.pop_back();
    }
  }
  LaunchTimer t = make_timer(ctx);
  if (ctx->timing) t.before(ctx, "graph", stream);
  e = hipGraphLaunch(ctx->graphs.front().exec, stream);
  if (ctx->timing) t.after(ctx, "graph", stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return OCSR_OK;
}

int32_t check_census_window(int sx, int sy, int sentinel) {
  if (sx < 0 || sy < 0 || sx > 32 || sy > 32)
    return fail(OCSR_E_INVALID, "census window half-sizes must be in 0..32 (sx=%d sy=%d)", sx, sy);
  const int bits = (2 * sx + 1) * (2 * sy + 1) + (sentinel ? 1 : 0);
  if (bits > 64)
    return fail(OCSR_E_UNSUPPORTED, "census window of %d bits does not fit 64 (sx=%d sy=%d)", bits, sx, sy);
  return OCSR_OK;
}

int32_t check_job(const ocsr_census_job& j, int k) {
  if (!j.img || !j.out) return fail(OCSR_E_INVALID, "census job %d: null image or output", k);
  if (j.width <= 0 || j.height <= 0 || j.width > (1 << 16) || j.height > (1 << 16))
    return fail(OCSR_E_INVALID, "census job %d: size %dx%d outside 1..65536", k, j.width, j.height);
  if (j.pitch_bytes < j.width) return fail(OCSR_E_INVALID, "census job %d: pitch < width", k);
  if (j.scale < 1 || j.scale > 16) return fail(OCSR_E_INVALID, "census job %d: scale %d outside 1..16", k, j.scale);
  if (j.out_pitch_elems < j.width / j.scale)
    return fail(OCSR_E_INVALID, "census job %d: output pitch %d < %d", k, j.out_pitch_elems, j.width / j.scale);
  return OCSR_OK;
}

int32_t enqueue_census(const ocsr_census_job* jobs, int n_jobs, int sx, int sy, int sentinel,
                       hipStream_t stream, const LaunchTimer* tp) {
  CensusJobsDev d;
  memset(&d, 0, sizeof(d));
  int64_t tiles = 0;
  for (int k = 0; k < n_jobs; ++k) {
    const ocsr_census_job& j = jobs[k];
    const int Ws = j.width / j.scale, Hs = j.height / j.scale;
    CensusJobDev& o = d.job[k];
    o.img = j.img; o.out = j.out; o.W = j.width; o.H = j.height; o.pitch = j.pitch_bytes;
    o.out_pitch = j.out_pitch_elems; o.scale = j.scale;
    o.tiles_x = (int)cdiv64(Ws, kCensusTileX);
    o.tile_begin = (int)tiles;
    tiles += (int64_t)o.tiles_x * cdiv64(Hs, kCensusTileY);
  }
  d.n = n_jobs;
  if (tiles > (1ll << 30)) return fail(OCSR_E_CAPACITY, "census: too many tiles");
  if (tp) tp->before(tp->ctx, "census", stream);
  hipError_t e = launch_census(d, (int)tiles, sx, sy, sentinel, stream);
  if (tp) tp->after(tp->ctx, "census", stream);
  if (e != hipSuccess) return hip_fail(e, "census launch");
  return OCSR_OK;
}

int32_t check_path(const ocsr_path& ph, const char* name, int scale, PathDev* out) {
  if (ph.mode != OCSR_MODE_TILED && ph.mode != OCSR_MODE_GRID)
    return fail(OCSR_E_INVALID, "%s path: unknown mode %d", name, ph.mode);
  if (ph.mode == OCSR_MODE_TILED && (ph.bw < 1 || ph.bh < 1 || ph.bw * ph.bh > 64))
    return fail(OCSR_E_INVALID, "%s path: TILED block %dx%d needs 1 <= bw*bh <= 64", name, ph.bw, ph.bh);
  if (ph.mode == OCSR_MODE_GRID && (ph.n_side < 1 || ph.n_side > 8))
    return fail(OCSR_E_INVALID, "%s path: GRID n_side %d outside 1..8", name, ph.n_side);
  if (ph.dmin < 0 || ph.dmax < ph.dmin || ph.dmax > (1 << 20))
    return fail(OCSR_E_INVALID, "%s path: disparity range [%d, %d] invalid", name, ph.dmin, ph.dmax);
  const int64_t nd = cdiv64((int64_t)ph.dmax - ph.dmin + 1, scale);
  if (nd > OCSR_MAX_CANDIDATES)
    return fail(OCSR_E_CAPACITY, "%s path: %lld level candidates > %d", name, (long long)nd,
                OCSR_MAX_CANDIDATES);
  out->mode = ph.mode;
  out->bw = ph.bw;
  out->bh = ph.bh;
  out->n_side = ph.n_side;
  out->dlo = ph.dmin / scale;
  out->nd = (int)nd;
  return OCSR_OK;
}

int32_t check_level(const ocsr_level* lv, const char* name, LevelDev* out) {
  if (!lv) return fail(OCSR_E_INVALID, "%s: null level", name);
  if (!lv->L || !lv->R) return fail(OCSR_E_INVALID, "%s: null descriptor pointer", name);
  if (lv->width <= 0 || lv->height <= 0 || lv->width > (1 << 16) || lv->height > (1 << 16))
    return fail(OCSR_E_INVALID, "%s: size %dx%d outside 1..65536", name, lv->width, lv->height);
  if (lv->pitch_elems < lv->width) return fail(OCSR_E_INVALID, "%s: pitch < width", name);
  if (lv->scale < 1 || lv->scale > 16) return fail(OCSR_E_INVALID, "%s: scale %d outside 1..16", name, lv->scale);
  if (lv->sx < 0 || lv->sy < 0) return fail(OCSR_E_INVALID, "%s: negative census window", name);
  *out = LevelDev{lv->L, lv->R, lv->width, lv->height, lv->pitch_elems, lv->scale, lv->sx, lv->sy};
  return OCSR_OK;
}

int32_t build_params(const ocsr_ctx* ctx, const ocsr_match_params* p, int close_scale,
                     int cap_blocks, MatchParamsDev* d) {
  if (!p) return fail(OCSR_E_INVALID, "null params");
  if (p->struct_size != sizeof(ocsr_match_params))
    return fail(OCSR_E_INVALID, "params.struct_size %u != %zu", p->struct_size, sizeof(ocsr_match_params));
  memset(d, 0, sizeof(*d));
  int32_t rc;
  if ((rc = check_path(p->far_path, "far", 1, &d->path[0])) != OCSR_OK) return rc;
  if ((rc = check_path(p->close_path, "close", close_scale, &d->path[1])) != OCSR_OK) return rc;
  // the kernel variant of each path: the first built one that covers it (every TILED
  // block of up to 64 points and every GRID block is covered up to 256 candidates)
  for (int l = 0; l < 2; ++l) {
    PathDev& ph = d->path[l];
    const MatchVariant v = pick_variant(ph);
    if (!v.tiled)
      return fail(OCSR_E_UNSUPPORTED, "%s path: no kernel covers this block shape and range",
                  l == 0 ? "far" : "close");
    ph.rows = v.rows;
    ph.cpl = v.cpl;
    ph.passes = v.passes;
    auto it = ctx->variants.find({ph.bw, ph.bh, ph.nd});
    if (it != ctx->variants.end() && variant_valid(ph, it->second[0], it->second[1], it->second[2])) {
      ph.rows = it->second[0];
      ph.cpl = it->second[1];
      ph.passes = it->second[2];
    }
  }
  // vertical range (a 2D offset search, Sec. 4.3.2): level offsets floor(dy_min / s) ..
  // ceil(dy_max / s) on a level of scale s
  if (p->dy_min < -OCSR_MAX_DY || p->dy_max > OCSR_MAX_DY || p->dy_min > p->dy_max)
    return fail(OCSR_E_INVALID, "vertical range [%d, %d] outside -%d <= dy_min <= dy_max <= %d",
                p->dy_min, p->dy_max, OCSR_MAX_DY, OCSR_MAX_DY);
  d->vertical = p->dy_min != 0 || p->dy_max != 0;
  for (int l = 0; l < 2; ++l) {
    PathDev& ph = d->path[l];
    const int s = l == 0 ? 1 : close_scale;
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    ph.dylo = fdiv(p->dy_min, s);
    ph.ndy = -fdiv(-p->dy_max, s) - ph.dylo + 1;
    if (!d->vertical) continue;
    if (ph.mode != OCSR_MODE_TILED || ph.bw > 8 || ph.bh > 8)
      return fail(OCSR_E_UNSUPPORTED, "%s path: a vertical range needs TILED blocks of at most "
                  "8 x 8 points", l == 0 ? "far" : "close");
    if (ph.nd * ph.ndy > OCSR_MAX_DY_CANDIDATES)
      return fail(OCSR_E_UNSUPPORTED, "%s path: %d x %d (d, dy) candidates > %d", l == 0 ? "far" : "close",
                  ph.nd, ph.ndy, OCSR_MAX_DY_CANDIDATES);
    const int rows = dy_rows(ph.bw, ph.bh);
    if (dy_strip_words(rows, ph.nd) > 64 * dy_chunks(rows))
      return fail(OCSR_E_UNSUPPORTED, "%s path: %d level disparities are more than a vertical search "
                  "with %dx%d blocks takes", l == 0 ? "far" : "close", ph.nd, ph.bw, ph.bh);
    const size_t lds = kItemWaves * dy_wave_lds_bytes(rows, ph.nd, ph.ndy);
    if (lds > kDyMaxWgLds)
      return fail(OCSR_E_UNSUPPORTED, "%s path: %d disparities x %d vertical offsets need %zu bytes of "
                  "LDS per workgroup > %zu", l == 0 ? "far" : "close", ph.nd, ph.ndy, lds, kDyMaxWgLds);
  }
  if (p->lr_tol < 0) return fail(OCSR_E_INVALID, "lr_tol < 0");
  if (p->min_point_pct < 0 || p->min_point_pct > 100) return fail(OCSR_E_INVALID, "min_point_pct outside 0..100");
  if (p->agg_mode != OCSR_AGG_SEGMENT_MEDIAN && p->agg_mode != OCSR_AGG_TRIMMED_MEDIAN)
    return fail(OCSR_E_INVALID, "unknown agg_mode %d", p->agg_mode);
  if (p->trim_pct < 0 || p->trim_pct > 49) return fail(OCSR_E_INVALID, "trim_pct outside 0..49");
  if (!(p->tau_d >= 0.0f) || !std::isfinite(p->tau_d)) return fail(OCSR_E_INVALID, "tau_d must be finite and >= 0");
  if (!std::isfinite(p->focal_px) || !std::isfinite(p->baseline_m) || !std::isfinite(p->d_eps))
    return fail(OCSR_E_INVALID, "focal, baseline and d_eps must be finite");
  if (cap_blocks < 1 || cap_blocks > (1 << 24)) return fail(OCSR_E_INVALID, "cap_blocks %d outside 1..2^24", cap_blocks);
  d->tau_s = p->tau_s;
  d->lr_tol = p->lr_tol;
  d->min_point_pct = p->min_point_pct;
  d->agg_mode = p->agg_mode;
  d->tau_d = p->tau_d;
  d->n_min = p->n_min;
  d->trim_pct = p->trim_pct;
  const volatile float f = p->focal_px, b = p->baseline_m;
  d->fb = f * b;
  d->d_eps = p->d_eps;
  d->cap_blocks = cap_blocks;
  // work items: four blocks per wave for the four-block kernel, else blocks per wave
  for (int l = 0; l < 2; ++l)
    d->item_blocks[l] = kItemWaves * (d->path[l].rows == 1 ? 4 : ctx->blocks_per_wave);
  d->full_census = ctx->full_census;
  return OCSR_OK;
}

DebugDev make_debug(const ocsr_debug* dbg) {
  DebugDev dd;
  memset(&dd, 0, sizeof(dd));
  if (dbg) {
    dd.cap_blocks = dbg->cap_blocks;
    dd.cap_nd = dbg->cap_nd;
    dd.n_blocks = dbg->n_blocks;
    dd.blocks = dbg->blocks;
    dd.cost_fwd = dbg->cost_fwd;
    dd.cost_bwd = dbg->cost_bwd;
  }
  return dd;
}

int32_t check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws || ((uintptr_t)ws & 255)) return fail(OCSR_E_INVALID, "workspace null or not 256-byte aligned");
  if (ws_bytes < need) return fail(OCSR_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
  return OCSR_OK;
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// descriptor images of one frame: L0, R0 at scale 1, L1, R1 at the close scale
// census tiles of both views at both levels of a frame
int64_t frame_tiles(int W, int H, int s) {
  return 2 * (cdiv64(W, kCensusTileX) * cdiv64(H, kCensusTileY) +
              cdiv64(W / s, kCensusTileX) * cdiv64(H / s, kCensusTileY));
}

// the four descriptor images of a frame, and the list of its census tiles (the lists of
// every frame follow the images of every frame)
size_t frame_census_bytes(int W, int H, int s) {
  return 2 * a256((size_t)W * H * 8) + 2 * a256((size_t)(W / s) * (H / s) * 8) +
         a256(sizeof(int32_t) * (size_t)frame_tiles(W, H, s));
}

int32_t check_frames(const ocsr_frame* frames, int n_frames, const ocsr_frame_params* fp,
                     int* n_boxes_total, bool need_images = true) {
  if (!fp) return fail(OCSR_E_INVALID, "null frame params");
  if (fp->close_scale < 1 || fp->close_scale > 16) return fail(OCSR_E_INVALID, "close_scale outside 1..16");
  int32_t rc;
  if ((rc = check_census_window(fp->sx, fp->sy, fp->sentinel)) != OCSR_OK) return rc;
  if (!frames || n_frames < 1 || n_frames > OCSR_MAX_BATCH_FRAMES)
    return fail(OCSR_E_INVALID, "n_frames %d outside 1..%d", n_frames, OCSR_MAX_BATCH_FRAMES);
  long long total = 0;
  for (int f = 0; f < n_frames; ++f) {
    const ocsr_frame& fr = frames[f];
    if (need_images && (!fr.imgL || !fr.imgR)) return fail(OCSR_E_INVALID, "frame %d: null image", f);
    if (fr.width <= 0 || fr.height <= 0 || fr.width > (1 << 15) || fr.height > (1 << 15))
      return fail(OCSR_E_INVALID, "frame %d: size %dx%d outside 1..32768", f, fr.width, fr.height);
    if (fr.pitch_bytes < fr.width) return fail(OCSR_E_INVALID, "frame %d: pitch < width", f);
    if (fr.width / fp->close_scale < 1 || fr.height / fp->close_scale < 1)
      return fail(OCSR_E_INVALID, "frame %d: smaller than the close scale", f);
    if (fr.n_boxes < 0 || fr.box_offset != total)
      return fail(OCSR_E_INVALID, "frame %d: boxes must follow the previous frame's (offset %d, expected %lld)",
                  f, fr.box_offset, total);
    total += fr.n_boxes;
  }
  if (total > (1 << 20)) return fail(OCSR_E_INVALID, "more than 2^20 boxes");
  *n_boxes_total = (int)total;
  return OCSR_OK;
}

size_t batch_ws_bytes(const ocsr_frame* frames, int n_frames, const ocsr_frame_params* fp,
                      int n_boxes_total, int cap_blocks) {
  size_t b = 0;
  for (int f = 0; f < n_frames; ++f) b += frame_census_bytes(frames[f].width, frames[f].height, fp->close_scale);
  return b + match_ws_bytes(n_frames, n_boxes_total, cap_blocks);
}

int32_t range_frames(ocsr_ctx* ctx, const ocsr_frame* frames, int n_frames,
                     const ocsr_frame_params* fp, const ocsr_box* boxes,
                     const ocsr_match_params* params, int cap_blocks, void* ws, size_t ws_bytes,
                     ocsr_box_result* out, hipStream_t stream) {
  int n_total = 0;
  int32_t rc;
  if ((rc = check_frames(frames, n_frames, fp, &n_total)) != OCSR_OK) return rc;
  MatchParamsDev P;
  if ((rc = build_params(ctx, params, fp->close_scale, cap_blocks, &P)) != OCSR_OK) return rc;
  if (n_total > 0 && (!boxes || !out)) return fail(OCSR_E_INVALID, "null boxes or output");
  if ((rc = check_ws(ws, ws_bytes, batch_ws_bytes(frames, n_frames, fp, n_total, cap_blocks))) != OCSR_OK)
    return rc;
  if (n_total == 0) return OCSR_OK;
  const int s = fp->close_scale;
  FramesDev FR;
  memset(&FR, 0, sizeof(FR));
  FR.n = n_frames;
  FR.n_boxes_total = n_total;
  char* base = (char*)ws;
  int tiles = 0;
  for (int f = 0; f < n_frames; ++f) {
    const ocsr_frame& fr = frames[f];
    const int W = fr.width, H = fr.height, W1 = W / s, H1 = H / s;
    uint64_t* dL0 = (uint64_t*)base; base += a256((size_t)W * H * 8);
    uint64_t* dR0 = (uint64_t*)base; base += a256((size_t)W * H * 8);
    uint64_t* dL1 = (uint64_t*)base; base += a256((size_t)W1 * H1 * 8);
    uint64_t* dR1 = (uint64_t*)base; base += a256((size_t)W1 * H1 * 8);
    FrameDev& d = FR.f[f];
    d.lv[0] = LevelDev{dL0, dR0, W, H, W, 1, fp->sx, fp->sy};
    d.lv[1] = LevelDev{dL1, dR1, W1, H1, W1, s, fp->sx, fp->sy};
    d.imgL = fr.imgL; d.imgR = fr.imgR;
    d.W = W; d.H = H; d.pitch = fr.pitch_bytes;
    d.box_off = fr.box_offset; d.n_boxes = fr.n_boxes;
    d.tiles0_x = (int)cdiv64(W, kCensusTileX);
    d.tiles0 = d.tiles0_x * (int)cdiv64(H, kCensusTileY);
    d.tiles1_x = (int)cdiv64(W1, kCensusTileX);
    d.tiles1 = d.tiles1_x * (int)cdiv64(H1, kCensusTileY);
    d.tx_recip[0] = ((1ull << 40) + (uint64_t)d.tiles0_x - 1) / (uint64_t)d.tiles0_x;
    d.tx_recip[1] = ((1ull << 40) + (uint64_t)d.tiles1_x - 1) / (uint64_t)d.tiles1_x;
    d.tile_begin = tiles;
    tiles += 2 * (d.tiles0 + d.tiles1);
  }
  // the frames' census tile lists, after the images of every frame
  for (int f = 0; f < n_frames; ++f) {
    FR.f[f].tile_list = (int32_t*)base;
    base += a256(sizeof(int32_t) * (size_t)frame_tiles(frames[f].width, frames[f].height, s));
  }
  MatchWs mws = match_ws_carve(base, n_frames, n_total, cap_blocks);
  const bool fused = ctx->use_fused && fused_available(P, FR, fp->sx, fp->sy);
  const int sentinel = fp->sentinel ? 1 : 0;
  // the whole launch sequence of the call, on stream s
  auto enqueue = [&](hipStream_t s, const LaunchTimer* tp) -> int32_t {
    if (fused) {
      hipError_t e = launch_fused(P, FR, boxes, mws, out, fp->sx, fp->sy, sentinel, ctx->n_cu,
                                  ctx->wgs_per_cu, s, tp);
      return e == hipSuccess ? OCSR_OK : hip_fail(e, "fused launch");
    }
    hipError_t e = ctx->census_list != 0
                       ? launch_plan_and_census(P, FR, boxes, mws, fp->sx, fp->sy, sentinel, ctx->n_cu, s, tp)
                       : hipErrorNotSupported;
    if (e == hipErrorNotSupported)
      e = launch_frame_census(P, FR, boxes, mws, fp->sx, fp->sy, sentinel, tiles, s, tp);
    if (e != hipSuccess) return hip_fail(e, "census launch");
    e = launch_match(P, FR, boxes, mws, out, make_debug(nullptr), true,
                     std::max(1, ctx->n_cu * ctx->match_wgs_per_cu), ctx->level_launches, s, tp);
    return e == hipSuccess ? OCSR_OK : hip_fail(e, "match launch");
  };
  if (ctx->use_graph) {
    // Everything the launches depend on: the host-side descriptions, every device
    // pointer and size, and the options that choose the kernels.
    std::string key;
    auto put = [&key](const void* p, size_t n) { key.append((const char*)p, n); };
    put(frames, sizeof(ocsr_frame) * n_frames);
    put(fp, sizeof(*fp));
    put(&boxes, sizeof(boxes));
    put(params, sizeof(*params));
    put(&cap_blocks, sizeof(cap_blocks));
    put(&ws, sizeof(ws));
    put(&out, sizeof(out));
    put(&P, sizeof(P));
    const int opts[6] = {fused ? 1 : 0, ctx->wgs_per_cu, ctx->n_cu, ctx->match_wgs_per_cu,
                         ctx->census_list, ctx->level_launches};
    put(opts, sizeof(opts));
    return graph_launch(ctx, key, enqueue, stream);
  }
  LaunchTimer t = make_timer(ctx);
  return enqueue(stream, ctx->timing ? &t : nullptr);
}

// Scratch of ocsr_match_boxes_noalloc: a file-scope device array, one copy on every
// device the library runs on, held until the process ends. Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device address); it uses
// the device address resolved once per device at context creation.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[OCSR_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Resolves the device address of `scratch` on `device`, which must be current.
int32_t resolve_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return OCSR_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!ptr || ((uintptr_t)ptr & 255)) return fail(OCSR_E_HIP, "scratch address not 256-byte aligned");
  g_scratch_ptr[device] = ptr;
  return OCSR_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// ocsr_match_boxes on a given workspace; `timed` lets the context's timing events in
int32_t match_boxes_impl(ocsr_ctx* ctx, const ocsr_level* lv0, const ocsr_level* lv1,
                         const ocsr_box* boxes, int32_t n_boxes, const ocsr_match_params* params,
                         int32_t cap_blocks, void* ws, size_t ws_bytes, ocsr_box_result* out,
                         const ocsr_debug* dbg, void* stream, bool timed) {
  int32_t rc;
  FramesDev FR;
  memset(&FR, 0, sizeof(FR));
  if ((rc = check_level(lv0, "lv0", &FR.f[0].lv[0])) != OCSR_OK) return rc;
  if ((rc = check_level(lv1, "lv1", &FR.f[0].lv[1])) != OCSR_OK) return rc;
  if (lv0->scale != 1) return fail(OCSR_E_INVALID, "lv0 must have scale 1 (got %d)", lv0->scale);
  MatchParamsDev P;
  if ((rc = build_params(ctx, params, lv1->scale, cap_blocks, &P)) != OCSR_OK) return rc;
  if (n_boxes < 0 || n_boxes > (1 << 20)) return fail(OCSR_E_INVALID, "n_boxes %d outside 0..2^20", n_boxes);
  if (n_boxes == 0) return OCSR_OK;
  if (!boxes || !out) return fail(OCSR_E_INVALID, "null boxes or output");
  if ((rc = check_ws(ws, ws_bytes, match_ws_bytes(1, n_boxes, cap_blocks))) != OCSR_OK) return rc;
  if (dbg && (dbg->cap_blocks < 0 || dbg->cap_nd < 0))
    return fail(OCSR_E_INVALID, "debug capacities must be >= 0");
  FR.n = 1;
  FR.n_boxes_total = n_boxes;
  FR.f[0].W = lv0->width;
  FR.f[0].H = lv0->height;
  FR.f[0].box_off = 0;
  FR.f[0].n_boxes = n_boxes;
  MatchWs mws = match_ws_carve(ws, 1, n_boxes, cap_blocks);
  LaunchTimer t = make_timer(ctx);
  hipError_t e = launch_match(P, FR, boxes, mws, out, make_debug(dbg), false,
                              std::max(1, ctx->n_cu * ctx->match_wgs_per_cu), ctx->level_launches,
                              (hipStream_t)stream,
                              timed && ctx->timing ? &t : nullptr);
  if (e != hipSuccess) return hip_fail(e, "match launch");
  if (dbg && dbg->n_blocks) {
    e = hipMemcpyAsync(dbg->n_blocks, mws.fcount + FC_NUMBERED, sizeof(int32_t),
                       hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "debug block count copy");
  }
  return OCSR_OK;
}

}  // namespace

extern "C" {

int32_t ocsr_abi_version(void) { return OCSR_ABI_VERSION; }

const char* ocsr_last_error(void) { return g_last_error.c_str(); }

int32_t ocsr_ctx_create(int32_t device, ocsr_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(OCSR_E_INVALID, "null output pointer");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(OCSR_E_INVALID, "device %d outside 0..%d", device, n - 1);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(OCSR_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  if (device >= kMaxDevices) return fail(OCSR_E_INVALID, "device %d beyond %d", device, kMaxDevices - 1);
  // the no-allocation entry point's scratch: its address on this device, once
  int32_t rs = resolve_scratch(device);
  if (rs != OCSR_OK) return rs;
  ocsr_ctx* c = new (std::nothrow) ocsr_ctx();
  if (!c) return fail(OCSR_E_INVALID, "out of host memory");
  c->device = device;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = c;
  return OCSR_OK;
}

void ocsr_ctx_destroy(ocsr_ctx* ctx) {
  if (!ctx) return;
  for (auto& p : ctx->pending) {
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  for (auto e : ctx->free_events) hipEventDestroy(e);
  for (auto& g : ctx->graphs) hipGraphExecDestroy(g.exec);
  if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
  delete ctx;
}

int32_t ocsr_census(ocsr_ctx* ctx, const uint8_t* img, int32_t width, int32_t height,
                    int32_t pitch_bytes, const ocsr_census_params* params, uint64_t* out,
                    int32_t out_pitch_elems, void* stream) {
  g_last_error.clear();
  if (!ctx || !params) return fail(OCSR_E_INVALID, "null context or params");
  ocsr_census_job j;
  j.img = img; j.out = out; j.width = width; j.height = height; j.pitch_bytes = pitch_bytes;
  j.out_pitch_elems = out_pitch_elems; j.scale = params->scale; j.reserved = 0;
  int32_t rc;
  if ((rc = check_census_window(params->sx, params->sy, params->sentinel)) != OCSR_OK) return rc;
  if ((rc = check_job(j, 0)) != OCSR_OK) return rc;
  LaunchTimer t = make_timer(ctx);
  return enqueue_census(&j, 1, params->sx, params->sy, params->sentinel ? 1 : 0,
                        (hipStream_t)stream, ctx->timing ? &t : nullptr);
}

size_t ocsr_rect_workspace_bytes(const ocsr_rect_params* p) {
  if (!p || p->roi_w <= 0 || p->roi_h <= 0 || (int64_t)p->roi_w * p->roi_h > (1 << 26)) return 0;
  const int64_t nz = (int64_t)p->delta_max - p->delta_min + 1;
  if (nz < 1 || nz > OCSR_MAX_RECT_OFFSETS) return 0;
  // per offset: the left and right winner maps and the checked map, then one partial
  // count per 256-pixel row segment
  const size_t maps = 3 * (size_t)nz * p->roi_w * p->roi_h * sizeof(int16_t);
  const size_t parts = (size_t)nz * p->roi_h * ((p->roi_w + 255) / 256) * sizeof(int32_t);
  return a256(maps) + a256(parts);
}

int32_t ocsr_rect_offset_counts(ocsr_ctx* ctx, const ocsr_level* lv, const ocsr_rect_params* p,
                                int32_t* counts, int16_t* disp, void* ws, size_t ws_bytes,
                                void* stream) {
  g_last_error.clear();
  if (!ctx || !p) return fail(OCSR_E_INVALID, "null context or rectification params");
  int32_t rc;
  LevelDev L;
  if ((rc = check_level(lv, "lv", &L)) != OCSR_OK) return rc;
  if (!counts) return fail(OCSR_E_INVALID, "null counts");
  if (p->delta_min > p->delta_max || (int64_t)p->delta_max - p->delta_min + 1 > OCSR_MAX_RECT_OFFSETS)
    return fail(OCSR_E_INVALID, "offsets [%d, %d]: 1..%d of them", p->delta_min, p->delta_max,
                OCSR_MAX_RECT_OFFSETS);
  if (p->roi_w <= 0 || p->roi_h <= 0 || (int64_t)p->roi_w * p->roi_h > (1 << 26))
    return fail(OCSR_E_INVALID, "ROI %dx%d: 1..2^26 pixels", p->roi_w, p->roi_h);
  if (p->roi_x0 < 0 || (int64_t)p->roi_x0 + p->roi_w > L.W || (int64_t)p->roi_y0 - p->delta_max < 0 ||
      (int64_t)p->roi_y0 + p->roi_h - p->delta_min > L.H || p->roi_y0 + p->roi_h > L.H || p->roi_y0 < 0)
    return fail(OCSR_E_INVALID, "ROI [%d, %d) x [%d, %d) moved by %d..%d leaves the %dx%d level",
                p->roi_x0, p->roi_x0 + p->roi_w, p->roi_y0, p->roi_y0 + p->roi_h, p->delta_min,
                p->delta_max, L.W, L.H);
  if (p->dmin < 0 || p->dmax < p->dmin) return fail(OCSR_E_INVALID, "disparity range [%d, %d] invalid", p->dmin, p->dmax);
  if ((int64_t)p->dmax - p->dmin + 1 > OCSR_MAX_CANDIDATES)
    return fail(OCSR_E_CAPACITY, "[%d, %d]: more than %d candidates", p->dmin, p->dmax, OCSR_MAX_CANDIDATES);
  if (!dense_radius_supported(p->radius))
    return fail(OCSR_E_UNSUPPORTED, "window radius %d: only 1..3 are built", p->radius);
  if (p->lr_tol < 0 || p->d_min < 0) return fail(OCSR_E_INVALID, "lr_tol and d_min must be >= 0");
  if ((rc = check_ws(ws, ws_bytes, ocsr_rect_workspace_bytes(p))) != OCSR_OK) return rc;
  const int nz = p->delta_max - p->delta_min + 1;
  // the maps of one kind are consecutive planes of roi_w * roi_h; the partial counts
  // follow the three kinds
  int16_t* d_left = (int16_t*)ws;
  int16_t* d_right = d_left + (size_t)nz * p->roi_w * p->roi_h;
  int16_t* d_chk = disp ? disp : d_right + (size_t)nz * p->roi_w * p->roi_h;
  int32_t* partial = (int32_t*)((char*)ws + a256(3 * (size_t)nz * p->roi_w * p->roi_h * sizeof(int16_t)));
  const uint64_t* CL0 = L.L + ((int64_t)p->roi_y0 - p->delta_min) * L.pitch + p->roi_x0;
  const uint64_t* CR = L.R + (int64_t)p->roi_y0 * L.pitch + p->roi_x0;
  LaunchTimer t = make_timer(ctx);
  const hipError_t e = launch_dense_offsets(CL0, CR, p->roi_w, p->roi_h, L.pitch, nz, p->dmin, p->dmax,
                                            p->radius, p->lr_tol, p->d_min, d_chk, d_left, d_right,
                                            partial, counts, (hipStream_t)stream,
                                            ctx->timing ? &t : nullptr);
  return e == hipSuccess ? OCSR_OK : hip_fail(e, "rectification launch");
}

int32_t ocsr_rect_filter_create(int32_t window, int32_t max_step, int32_t initial,
                                ocsr_rect_filter** out) {
  g_last_error.clear();
  if (!out) return fail(OCSR_E_INVALID, "null output pointer");
  *out = nullptr;
  if (window < 1 || window > 1024) return fail(OCSR_E_INVALID, "window %d outside 1..1024", window);
  if (max_step < 0) return fail(OCSR_E_INVALID, "max_step %d < 0", max_step);
  ocsr_rect_filter* f = new (std::nothrow) ocsr_rect_filter();
  if (!f) return fail(OCSR_E_INVALID, "out of host memory");
  f->window = window;
  f->max_step = max_step;
  f->prev = initial;
  *out = f;
  return OCSR_OK;
}

void ocsr_rect_filter_destroy(ocsr_rect_filter* f) { delete f; }

int32_t ocsr_rect_filter_update(ocsr_rect_filter* f, const int32_t* counts, int32_t n_offsets,
                                int32_t delta_min, int32_t* raw, int32_t* filtered) {
  g_last_error.clear();
  if (!f || !counts || !raw || !filtered) return fail(OCSR_E_INVALID, "null argument");
  if (n_offsets < 1 || n_offsets > OCSR_MAX_RECT_OFFSETS)
    return fail(OCSR_E_INVALID, "n_offsets %d outside 1..%d", n_offsets, OCSR_MAX_RECT_OFFSETS);
  // estimate: the largest count; ties to the smallest |delta|, then the smaller delta
  int best = 0;
  for (int k = 1; k < n_offsets; ++k) {
    const int dk = delta_min + k, db = delta_min + best;
    if (counts[k] > counts[best] ||
        (counts[k] == counts[best] && (std::abs(dk) < std::abs(db) || (std::abs(dk) == std::abs(db) && dk < db))))
      best = k;
  }
  const int est = delta_min + best;
  f->hist.push_back(est);
  if ((int)f->hist.size() > f->window) f->hist.pop_front();
  std::vector<int> v(f->hist.begin(), f->hist.end());
  std::sort(v.begin(), v.end());
  const int med = v[(v.size() - 1) / 2];
  const int step = std::max(-f->max_step, std::min(f->max_step, med - f->prev));
  f->prev += step;
  *raw = est;
  *filtered = f->prev;
  return OCSR_OK;
}

int32_t ocsr_select_boxes(ocsr_ctx* ctx, const ocsr_frame* frames, int32_t n_frames,
                          const ocsr_box* in, const ocsr_select_params* params, ocsr_box* out,
                          int32_t* rank, void* stream) {
  g_last_error.clear();
  if (!ctx || !params) return fail(OCSR_E_INVALID, "null context or select params");
  if (!frames || n_frames < 1 || n_frames > OCSR_MAX_BATCH_FRAMES)
    return fail(OCSR_E_INVALID, "n_frames %d outside 1..%d", n_frames, OCSR_MAX_BATCH_FRAMES);
  if (params->max_objects < 0) return fail(OCSR_E_INVALID, "max_objects %d < 0", params->max_objects);
  const int32_t* c = params->crop_permille;
  if (c[0] < 0 || c[1] < 0 || c[0] > c[2] || c[1] > c[3] || c[2] > 1000 || c[3] > 1000)
    return fail(OCSR_E_INVALID, "crop [%d, %d) x [%d, %d) permille outside 0..1000", c[0], c[2], c[1], c[3]);
  SelectDev S;
  memset(&S, 0, sizeof(S));
  S.n = n_frames;
  S.max_objects = params->max_objects;
  long long total = 0;
  int max_boxes = 0;
  for (int f = 0; f < n_frames; ++f) {
    const ocsr_frame& fr = frames[f];
    if (fr.width <= 0 || fr.height <= 0 || fr.width > (1 << 15) || fr.height > (1 << 15))
      return fail(OCSR_E_INVALID, "frame %d: size %dx%d outside 1..32768", f, fr.width, fr.height);
    if (fr.n_boxes < 0 || fr.box_offset != total)
      return fail(OCSR_E_INVALID, "frame %d: boxes must follow the previous frame's (offset %d, expected %lld)",
                  f, fr.box_offset, total);
    if (fr.n_boxes > OCSR_MAX_SELECT_BOXES)
      return fail(OCSR_E_CAPACITY, "frame %d: %d boxes > %d", f, fr.n_boxes, OCSR_MAX_SELECT_BOXES);
    SelectFrameDev& d = S.f[f];
    d.W = fr.width;
    d.H = fr.height;
    d.X0 = (int)((long long)fr.width * c[0] / 1000);
    d.Y0 = (int)((long long)fr.height * c[1] / 1000);
    d.X1 = (int)((long long)fr.width * c[2] / 1000);
    d.Y1 = (int)((long long)fr.height * c[3] / 1000);
    d.box_off = fr.box_offset;
    d.n_boxes = fr.n_boxes;
    total += fr.n_boxes;
    max_boxes = std::max(max_boxes, fr.n_boxes);
  }
  if (total == 0) return OCSR_OK;
  if (!in || !out) return fail(OCSR_E_INVALID, "null boxes");
  const uintptr_t a0 = (uintptr_t)in, a1 = a0 + (size_t)total * sizeof(ocsr_box);
  const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (size_t)total * sizeof(ocsr_box);
  if (a0 < b1 && b0 < a1) return fail(OCSR_E_INVALID, "out overlaps in");
  LaunchTimer t = make_timer(ctx);
  const hipError_t e = launch_select(S, in, out, rank, max_boxes, (hipStream_t)stream,
                                     ctx->timing ? &t : nullptr);
  return e == hipSuccess ? OCSR_OK : hip_fail(e, "select launch");
}

int32_t ocsr_box_points(ocsr_ctx* ctx, const ocsr_box* boxes, const ocsr_box_result* results,
                        int32_t n_boxes, const ocsr_point_params* pp, ocsr_box_point* out,
                        void* stream) {
  g_last_error.clear();
  if (!ctx || !pp) return fail(OCSR_E_INVALID, "null context or point params");
  if (n_boxes < 0) return fail(OCSR_E_INVALID, "n_boxes %d < 0", n_boxes);
  if (n_boxes > 0 && (!boxes || !results || !out)) return fail(OCSR_E_INVALID, "null boxes, results or output");
  if (pp->width <= 0 || pp->height <= 0) return fail(OCSR_E_INVALID, "image size %dx%d", pp->width, pp->height);
  if (!(pp->focal_px > 0) || !(pp->baseline_m > 0))
    return fail(OCSR_E_INVALID, "focal length and baseline must be positive");
  if (!(pp->var_d >= 0) || !(pp->var_x >= 0) || !(pp->var_y >= 0))
    return fail(OCSR_E_INVALID, "variances must be non-negative");
  PointParamsDev d;
  d.width = pp->width;
  d.height = pp->height;
  for (int k = 0; k < 16; ++k) d.Q[k] = (float)pp->Q[k];
  for (int k = 0; k < 9; ++k) d.R[k] = (float)pp->R[k];
  for (int k = 0; k < 3; ++k) d.t[k] = (float)pp->t[k];
  d.fb = (float)pp->focal_px * (float)pp->baseline_m;
  d.var_d = (float)pp->var_d;
  d.var_x = (float)pp->var_x;
  d.var_y = (float)pp->var_y;
  LaunchTimer t = make_timer(ctx);
  const hipError_t e = launch_box_points(boxes, results, n_boxes, d, out, (hipStream_t)stream,
                                         ctx->timing ? &t : nullptr);
  return e == hipSuccess ? OCSR_OK : hip_fail(e, "point launch");
}

int32_t ocsr_census_many(ocsr_ctx* ctx, const ocsr_census_job* jobs, int32_t n_jobs,
                         int32_t sx, int32_t sy, int32_t sentinel, void* stream) {
  g_last_error.clear();
  if (!ctx || (!jobs && n_jobs > 0)) return fail(OCSR_E_INVALID, "null context or jobs");
  if (n_jobs < 0 || n_jobs > OCSR_MAX_CENSUS_JOBS)
    return fail(OCSR_E_INVALID, "n_jobs %d outside 0..%d", n_jobs, OCSR_MAX_CENSUS_JOBS);
  int32_t rc;
  if ((rc = check_census_window(sx, sy, sentinel)) != OCSR_OK) return rc;
  for (int k = 0; k < n_jobs; ++k)
    if ((rc = check_job(jobs[k], k)) != OCSR_OK) return rc;
  if (n_jobs == 0) return OCSR_OK;
  LaunchTimer t = make_timer(ctx);
  return enqueue_census(jobs, n_jobs, sx, sy, sentinel ? 1 : 0, (hipStream_t)stream,
                        ctx->timing ? &t : nullptr);
}

size_t ocsr_match_workspace_bytes(int32_t n_boxes, int32_t cap_blocks) {
  return match_ws_bytes(1, n_boxes, cap_blocks);
}

int32_t ocsr_match_boxes(ocsr_ctx* ctx, const ocsr_level* lv0, const ocsr_level* lv1,
                         const ocsr_box* boxes, int32_t n_boxes, const ocsr_match_params* params,
                         int32_t cap_blocks, void* ws, size_t ws_bytes, ocsr_box_result* out,
                         const ocsr_debug* dbg, void* stream) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  return match_boxes_impl(ctx, lv0, lv1, boxes, n_boxes, params, cap_blocks, ws, ws_bytes, out,
                          dbg, stream, true);
}

int32_t ocsr_match_boxes_noalloc(ocsr_ctx* ctx, const ocsr_level* lv0, const ocsr_level* lv1,
                                 const ocsr_box* boxes, int32_t n_boxes,
                                 const ocsr_match_params* params, int32_t cap_blocks,
                                 ocsr_box_result* out, const ocsr_debug* dbg, void* stream) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  void* ptr = scratch_ptr(ctx->device);
  if (!ptr) return fail(OCSR_E_INVALID, "no scratch resolved for device %d", ctx->device);
  if (n_boxes < 0 || n_boxes > (1 << 20)) return fail(OCSR_E_INVALID, "n_boxes %d outside 0..2^20", n_boxes);
  if (cap_blocks < 1 || cap_blocks > (1 << 24)) return fail(OCSR_E_INVALID, "cap_blocks %d outside 1..2^24", cap_blocks);
  const size_t need = match_ws_bytes(1, n_boxes, cap_blocks);
  if (need > (size_t)OCSR_NOALLOC_SCRATCH_BYTES)
    return fail(OCSR_E_CAPACITY, "%d boxes and %d block slots need %zu bytes of scratch, more than "
                "the %u of OCSR_NOALLOC_SCRATCH_BYTES", n_boxes, cap_blocks, need,
                (unsigned)OCSR_NOALLOC_SCRATCH_BYTES);
  return match_boxes_impl(ctx, lv0, lv1, boxes, n_boxes, params, cap_blocks, ptr,
                          (size_t)OCSR_NOALLOC_SCRATCH_BYTES, out, dbg, stream, false);
}

size_t ocsr_frame_workspace_bytes(int32_t width, int32_t height, const ocsr_frame_params* fp,
                                  int32_t n_boxes, int32_t cap_blocks) {
  if (!fp || width <= 0 || height <= 0 || fp->close_scale < 1) return 0;
  return frame_census_bytes(width, height, fp->close_scale) + match_ws_bytes(1, n_boxes, cap_blocks);
}

int32_t ocsr_range_frame(ocsr_ctx* ctx, const uint8_t* imgL, const uint8_t* imgR,
                         int32_t width, int32_t height, int32_t pitch_bytes,
                         const ocsr_frame_params* fp, const ocsr_box* boxes, int32_t n_boxes,
                         const ocsr_match_params* params, int32_t cap_blocks, void* ws,
                         size_t ws_bytes, ocsr_box_result* out, void* stream) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  ocsr_frame fr = {imgL, imgR, width, height, pitch_bytes, 0, n_boxes, 0};
  return range_frames(ctx, &fr, 1, fp, boxes, params, cap_blocks, ws, ws_bytes, out,
                      (hipStream_t)stream);
}

size_t ocsr_batch_workspace_bytes(const ocsr_frame* frames, int32_t n_frames,
                                  const ocsr_frame_params* fp, int32_t cap_blocks) {
  int n_total = 0;
  const std::string saved = g_last_error;
  const int32_t rc = check_frames(frames, n_frames, fp, &n_total, false);
  g_last_error = saved;
  if (rc != OCSR_OK) return 0;
  return batch_ws_bytes(frames, n_frames, fp, n_total, cap_blocks);
}

int32_t ocsr_range_batch(ocsr_ctx* ctx, const ocsr_frame* frames, int32_t n_frames,
                         const ocsr_frame_params* fp, const ocsr_box* boxes,
                         const ocsr_match_params* params, int32_t cap_blocks, void* ws,
                         size_t ws_bytes, ocsr_box_result* out, void* stream) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  return range_frames(ctx, frames, n_frames, fp, boxes, params, cap_blocks, ws, ws_bytes, out,
                      (hipStream_t)stream);
}

int32_t ocsr_ctx_set_option(ocsr_ctx* ctx, int32_t option, int32_t value) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  switch (option) {
    case OCSR_OPTION_FUSED:
      ctx->use_fused = value != 0;
      return OCSR_OK;
    case OCSR_OPTION_GRAPH:
      ctx->use_graph = value != 0;
      return OCSR_OK;
    case OCSR_OPTION_MATCH_WGS_PER_CU:
      if (value < 1 || value > 64) return fail(OCSR_E_INVALID, "match workgroups per CU outside 1..64");
      ctx->match_wgs_per_cu = value;
      return OCSR_OK;
    case OCSR_OPTION_BLOCKS_PER_WAVE:
      if (value < 1 || value > kMaxBlocksPerWave)
        return fail(OCSR_E_INVALID, "blocks per wave outside 1..%d", kMaxBlocksPerWave);
      ctx->blocks_per_wave = value;
      return OCSR_OK;
    case OCSR_OPTION_FULL_CENSUS:
      ctx->full_census = value != 0;
      return OCSR_OK;
    case OCSR_OPTION_CENSUS_TILE_LIST:
      ctx->census_list = value != 0;
      return OCSR_OK;
    case OCSR_OPTION_LEVEL_LAUNCHES:
      if (value < 0 || value > 2) return fail(OCSR_E_INVALID, "level launches %d outside 0..2", value);
      ctx->level_launches = value;
      return OCSR_OK;
    case OCSR_OPTION_WAVES_PER_CU:
      if (value < 0 || value > 32) return fail(OCSR_E_INVALID, "workgroups per CU outside 0..32");
      ctx->wgs_per_cu = value;
      return OCSR_OK;
    default:
      return fail(OCSR_E_INVALID, "unknown option %d", option);
  }
}

size_t ocsr_dense_workspace_bytes(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0) return 0;
  return 2 * a256((size_t)width * height * sizeof(int16_t));
}

int32_t ocsr_dense_match(ocsr_ctx* ctx, const ocsr_level* lv, int32_t dmin, int32_t dmax,
                         int32_t radius, int32_t lr_tol, int16_t* disp, int16_t* disp_right,
                         void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  int32_t rc;
  LevelDev L;
  if ((rc = check_level(lv, "lv", &L)) != OCSR_OK) return rc;
  if (!disp) return fail(OCSR_E_INVALID, "null disparity output");
  if (dmin < 0 || dmax < dmin) return fail(OCSR_E_INVALID, "disparity range [%d, %d] invalid", dmin, dmax);
  if (dmax - dmin + 1 > OCSR_MAX_CANDIDATES)
    return fail(OCSR_E_CAPACITY, "%d candidates > %d", dmax - dmin + 1, OCSR_MAX_CANDIDATES);
  if (!dense_radius_supported(radius))
    return fail(OCSR_E_UNSUPPORTED, "window radius %d: only 1..3 are built", radius);
  if (lr_tol < 0) return fail(OCSR_E_INVALID, "lr_tol < 0");
  if ((rc = check_ws(ws, ws_bytes, ocsr_dense_workspace_bytes(L.W, L.H))) != OCSR_OK) return rc;
  int16_t* d_left = (int16_t*)ws;
  int16_t* d_right = disp_right ? disp_right
                                : (int16_t*)((char*)ws + a256((size_t)L.W * L.H * sizeof(int16_t)));
  LaunchTimer t = make_timer(ctx);
  hipError_t e = launch_dense(L.L, L.R, L.W, L.H, L.pitch, dmin, dmax, radius, lr_tol, disp, d_left,
                              d_right, (hipStream_t)stream, ctx->timing ? &t : nullptr);
  if (e != hipSuccess) return hip_fail(e, "dense launch");
  return OCSR_OK;
}

int32_t ocsr_variant_candidates(int32_t bw, int32_t bh, int32_t n_candidates, int32_t* rows,
                                int32_t* cpl, int32_t* passes, int32_t cap) {
  g_last_error.clear();
  if (cap < 0 || (cap > 0 && (!rows || !cpl || !passes))) return fail(OCSR_E_INVALID, "null output arrays");
  PathDev ph = {};
  ph.mode = OCSR_MODE_TILED;
  ph.bw = bw;
  ph.bh = bh;
  ph.nd = n_candidates;
  return variant_candidates(ph, rows, cpl, passes, cap);
}

int32_t ocsr_ctx_set_variant(ocsr_ctx* ctx, int32_t bw, int32_t bh, int32_t n_candidates,
                             int32_t rows, int32_t cpl, int32_t passes) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  if (rows == 0 && cpl == 0 && passes == 0) {   // (0, 0, 0): back to the default
    ctx->variants.erase({bw, bh, n_candidates});
    return OCSR_OK;
  }
  PathDev ph = {};
  ph.mode = OCSR_MODE_TILED;
  ph.bw = bw;
  ph.bh = bh;
  ph.nd = n_candidates;
  if (!variant_valid(ph, rows, cpl, passes))
    return fail(OCSR_E_INVALID, "no kernel with %d rows, %d candidates per lane and %d passes "
                "covers %dx%d blocks and %d candidates", rows, cpl, passes, bw, bh, n_candidates);
  ctx->variants[{bw, bh, n_candidates}] = {rows, cpl, passes};
  return OCSR_OK;
}

int32_t ocsr_ctx_graph_stats(ocsr_ctx* ctx, int64_t* hits, int64_t* builds) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  if (hits) *hits = ctx->graph_hits;
  if (builds) *builds = ctx->graph_builds;
  return OCSR_OK;
}

int32_t ocsr_ctx_set_timing(ocsr_ctx* ctx, int32_t enable) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  ctx->timing = enable != 0;
  return OCSR_OK;
}

static int32_t drain_pending(ocsr_ctx* ctx) {
  for (auto& p : ctx->pending) {
    hipError_t e = hipEventSynchronize(p.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    auto& st = ctx->stats[p.name];
    st.first += 1;
    st.second += ms;
    ctx->free_events.push_back(p.start);
    ctx->free_events.push_back(p.stop);
  }
  ctx->pending.clear();
  return OCSR_OK;
}

int32_t ocsr_ctx_kernel_time(ocsr_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms) {
  g_last_error.clear();
  if (!ctx || !kernel || !launches || !total_ms) return fail(OCSR_E_INVALID, "null argument");
  int32_t rc = drain_pending(ctx);
  if (rc != OCSR_OK) return rc;
  auto it = ctx->stats.find(kernel);
  *launches = it == ctx->stats.end() ? 0 : it->second.first;
  *total_ms = it == ctx->stats.end() ? 0.0 : it->second.second;
  return OCSR_OK;
}

int32_t ocsr_ctx_reset_timing(ocsr_ctx* ctx) {
  g_last_error.clear();
  if (!ctx) return fail(OCSR_E_INVALID, "null context");
  int32_t rc = drain_pending(ctx);
  ctx->stats.clear();
  return rc;
}

}  // extern "C"
