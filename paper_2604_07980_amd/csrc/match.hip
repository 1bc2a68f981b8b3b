// Object-centric block matching on gfx950 (Sec. 4.3.2-4.3.6, Alg. 2).
//
// Three kernels per call, all on the caller's stream:
//   plan       one workgroup; per box: clip, far/close type (Sec. 4.3.4 type
//              equation), level box, block grid; block numbers by a prefix over boxes;
//   match      persistent wave-per-block loop over the numbered blocks: occluder mask
//              (Sec. 4.3.5), forward Hamming search over the level disparity range
//              (census cost equation), winner-take-all, parabola (sub-pixel equation),
//              backward search from the matched right positions and the L/R check
//              (Sec. 4.3.3);
//   aggregate  one workgroup per box: sort of the valid block disparities in LDS,
//              longest-segment or trimmed median (Sec. 4.3.4), depth Z = f b / d (Eq. 1).
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

constexpr int kAggMax = OCSR_MAX_BLOCKS_PER_BOX;

__device__ __forceinline__ int cdiv_nonneg(int a, int s) { return (a + s - 1) / s; }

// ---------------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void plan_kernel(MatchParamsDev p, const ocsr_box* boxes,
                                                    int W, int H, MatchWs ws) {
  __shared__ int scan[1024];
  __shared__ int carry;
  __shared__ int matched_end;
  const int tid = threadIdx.x;
  if (tid == 0) { carry = 0; matched_end = 0; }
  __syncthreads();
  for (int base = 0; base < p.n_boxes; base += 1024) {
    const int i = base + tid;
    BoxPlan pl = {};
    BoxClip cl = {0, 0, 0, 0};
    int count = 0;
    if (i < p.n_boxes) {
      const ocsr_box b = boxes[i];
      const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
      const int cx1 = min(b.x1, W), cy1 = min(b.y1, H);
      const bool empty = !(cx0 < cx1 && cy0 < cy1);
      if (!empty) cl = BoxClip{cx0, cy0, cx1, cy1};   // empty boxes overlap nothing
      pl.cx0 = cl.cx0; pl.cy0 = cl.cy0;
      if (!(b.flags & OCSR_BOX_RANGE)) {
        pl.status = OCSR_REASON_NOT_RANGED;
      } else if (empty) {
        pl.status = OCSR_REASON_CLIPPED_EMPTY;
      } else {
        const bool far_box = max(cx1 - cx0, cy1 - cy0) < p.tau_s;
        const int level = far_box ? 0 : 1;
        const LevelDev& lv = p.lv[level];
        const PathDev& ph = p.path[level];
        const int s = lv.scale;
        pl.level = level;
        // level pixels whose full-res position s*x lies in the box and whose census
        // is defined
        const int x0 = max(cdiv_nonneg(cx0, s), lv.sx), x1 = min(cdiv_nonneg(cx1, s), lv.W - lv.sx);
        const int y0 = max(cdiv_nonneg(cy0, s), lv.sy), y1 = min(cdiv_nonneg(cy1, s), lv.H - lv.sy);
        if (x1 <= x0 || y1 <= y0) {
          pl.status = OCSR_REASON_NO_ELIGIBLE_BLOCKS;
        } else {
          pl.lx0 = x0; pl.ly0 = y0; pl.lw = x1 - x0; pl.lh = y1 - y0;
          if (ph.mode == OCSR_MODE_TILED) {
            pl.bw = min(ph.bw, pl.lw);
            pl.bh = min(ph.bh, pl.lh);
            pl.nbx = max(1, pl.lw / ph.bw);
            pl.nby = max(1, pl.lh / ph.bh);
            pl.ox = pl.lx0 + (pl.lw - pl.nbx * pl.bw) / 2;
            pl.oy = pl.ly0 + (pl.lh - pl.nby * pl.bh) / 2;
          } else {
            pl.nbx = pl.nby = 1;
            pl.bw = min(ph.n_side, pl.lw);
            pl.bh = min(ph.n_side, pl.lh);
          }
          const int n = pl.nbx * pl.nby;
          if (n > OCSR_MAX_BLOCKS_PER_BOX) {
            pl.status = OCSR_REASON_CAPACITY_OVERFLOW;
          } else {
            pl.status = -1;
            count = n;
          }
        }
      }
    }
    scan[tid] = count;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {       // inclusive Hillis-Steele scan
      const int v = tid >= d ? scan[tid - d] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    const int off = carry + scan[tid] - count;
    if (i < p.n_boxes) {
      int nblk = 0;
      if (pl.status == -1) {
        if ((long long)off + count > (long long)p.cap_blocks) pl.status = OCSR_REASON_CAPACITY_OVERFLOW;
        else nblk = count;
      }
      pl.off = off;
      pl.nblk = nblk;
      ws.plan[i] = pl;
      ws.clip[i] = cl;
      ws.box_end[i] = off + nblk;
      if (nblk > 0) atomicMax(&matched_end, off + nblk);
    }
    __syncthreads();
    if (tid == 1023) carry += scan[1023];
    __syncthreads();
  }
  if (tid == 0) {
    ws.counters[0] = carry;
    ws.counters[1] = matched_end;
  }
}

// ---------------------------------------------------------------------------------
// match: one wave per block
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ld_word(const uint64_t* __restrict__ row, int x, int W) {
  return (x >= 0 && x < W) ? row[x] : 0ull;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

__device__ __forceinline__ uint32_t pick4(const uint32_t a[4], int r) {
  return r == 0 ? a[0] : r == 1 ? a[1] : r == 2 ? a[2] : a[3];
}

struct BlockGeom {
  int nx, ny;
  int s;
  int tiled;
  int cx, lx0, lw;   // TILED: first column cx; GRID: lx0, lw
  int cy, ly0, lh;
};

__device__ __forceinline__ int geom_col(const BlockGeom& g, int i) {
  return g.tiled ? g.cx + i : g.lx0 + (2 * i + 1) * g.lw / (2 * g.nx);
}
__device__ __forceinline__ int geom_row(const BlockGeom& g, int j) {
  return g.tiled ? g.cy + j : g.ly0 + (2 * j + 1) * g.lh / (2 * g.ny);
}

// S(d) for the 64 * 4 candidates of a wave: forward (dir > 0) or backward.
__device__ __forceinline__ void block_costs(const LevelDev& lv, const BlockGeom& g, uint64_t mask,
                                            int dlo, int nd, int dir, int d_f, int lane,
                                            uint32_t acc[4]) {
  acc[0] = acc[1] = acc[2] = acc[3] = 0;
  const int npts = g.nx * g.ny;
  for (int t = 0; t < npts; ++t) {
    if (!((mask >> t) & 1ull)) continue;
    const int j = t / g.nx, i = t - j * g.nx;
    const int x = geom_col(g, i), y = geom_row(g, j);
    const uint64_t* __restrict__ rowL = lv.L + (size_t)y * lv.pitch;
    const uint64_t* __restrict__ rowR = lv.R + (size_t)y * lv.pitch;
    if (dir > 0) {
      const uint64_t tmpl = rowL[x];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kc = lane + 64 * r;
        if (kc < nd) acc[r] += __popcll(tmpl ^ ld_word(rowR, x - (dlo + kc), lv.W));
      }
    } else {
      const int q = x - d_f;
      const uint64_t tmpl = ld_word(rowR, q, lv.W);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kc = lane + 64 * r;
        if (kc < nd) acc[r] += __popcll(tmpl ^ ld_word(rowL, q + dlo + kc, lv.W));
      }
    }
  }
}

// smallest index attaining the minimum cost (key = cost << 16 | index)
__device__ __forceinline__ uint32_t wta(const uint32_t acc[4], int nd, int lane) {
  uint32_t key = 0xFFFFFFFFu;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int kc = lane + 64 * r;
    if (kc < nd) key = min(key, (acc[r] << 16) | (uint32_t)kc);
  }
  return wave_min_u32(key);
}

__device__ __forceinline__ uint32_t cost_at(const uint32_t acc[4], int k) {
  return (uint32_t)__shfl((int)pick4(acc, k >> 6), k & 63, 64);
}

__global__ __launch_bounds__(64) void match_kernel(MatchParamsDev p, MatchWs ws, DebugDev dbg) {
  const int lane = threadIdx.x;
  const int M = ws.counters[1];
  for (int b = blockIdx.x; b < M; b += gridDim.x) {
    // the box whose block range holds b
    int lo = 0, hi = p.n_boxes - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ws.box_end[mid] > b) hi = mid;
      else lo = mid + 1;
    }
    const int k = lo;
    const BoxPlan pl = ws.plan[k];
    const BoxClip ck = ws.clip[k];
    const LevelDev& lv = p.lv[pl.level];
    const PathDev& ph = p.path[pl.level];
    const int local = b - pl.off;
    const int v = local / pl.nbx, u = local - v * pl.nbx;

    BlockGeom g;
    g.nx = pl.bw; g.ny = pl.bh; g.s = lv.scale;
    g.tiled = ph.mode == OCSR_MODE_TILED;
    g.cx = pl.ox + u * pl.bw; g.lx0 = pl.lx0; g.lw = pl.lw;
    g.cy = pl.oy + v * pl.bh; g.ly0 = pl.ly0; g.lh = pl.lh;
    const int s = g.s;
    const int npts = g.nx * g.ny;

    // occlusion-aware sampling: drop points inside any overlapping box with a larger
    // bottom y (Sec. 4.3.5)
    const int pi = lane % g.nx, pj = lane / g.nx;
    const int fx = s * geom_col(g, pi), fy = s * geom_row(g, min(pj, g.ny - 1));
    const int bx0 = s * geom_col(g, 0), bx1 = s * geom_col(g, g.nx - 1);
    const int by0 = s * geom_row(g, 0), by1 = s * geom_row(g, g.ny - 1);
    bool hidden = false;
    for (int jb = 0; jb < p.n_boxes; jb += 64) {
      const int o = jb + lane;
      bool occ = false;
      if (o < p.n_boxes && o != k) {
        const BoxClip co = ws.clip[o];
        occ = ck.cx0 < co.cx1 && co.cx0 < ck.cx1 && ck.cy0 < co.cy1 && co.cy0 < ck.cy1 &&
              co.cy1 > ck.cy1 && co.cx0 <= bx1 && co.cx1 > bx0 && co.cy0 <= by1 && co.cy1 > by0;
      }
      uint64_t m = __ballot(occ);
      while (m) {
        const int oo = jb + __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const BoxClip co = ws.clip[oo];
        hidden |= fx >= co.cx0 && fx < co.cx1 && fy >= co.cy0 && fy < co.cy1;
      }
    }
    const uint64_t mask = __ballot(lane < npts && !hidden);
    const int nmask = __popcll(mask);
    const bool eligible = nmask > 0 && 100 * nmask >= p.min_point_pct * npts;

    int d_f = ph.dlo, d_b = ph.dlo, lr_ok = 0, valid = 0;
    float d_sub = (float)ph.dlo;
    uint32_t fwd[4] = {0, 0, 0, 0}, bwd[4] = {0, 0, 0, 0};
    if (eligible) {
      block_costs(lv, g, mask, ph.dlo, ph.nd, +1, 0, lane, fwd);
      const uint32_t key = wta(fwd, ph.nd, lane);
      const int best = (int)(key & 0xFFFFu);
      d_f = ph.dlo + best;
      const int cbest = (int)(key >> 16);
      const int ca = (int)cost_at(fwd, max(best - 1, 0));
      const int cb = (int)cost_at(fwd, min(best + 1, ph.nd - 1));
      if (best > 0 && best < ph.nd - 1) {
        const int num = ca - cb;
        const int den = 2 * (ca + cb - 2 * cbest);
        const float offs = (float)num / (float)den;
        d_sub = (float)d_f + offs;
      } else {
        d_sub = (float)d_f;
      }
      block_costs(lv, g, mask, ph.dlo, ph.nd, -1, d_f, lane, bwd);
      const uint32_t bkey = wta(bwd, ph.nd, lane);
      d_b = ph.dlo + (int)(bkey & 0xFFFFu);
      lr_ok = abs(d_b - d_f) <= p.lr_tol;
      valid = lr_ok;
    }
    if (lane == 0) {
      ws.blk_val[b] = (float)s * d_sub;
      ws.blk_flag[b] = (uint8_t)((eligible ? 1 : 0) | (valid ? 2 : 0));
    }
    if (dbg.blocks && b < dbg.cap_blocks && lane == 0) {
      ocsr_block_record rec;
      rec.box = k; rec.level_scale = s; rec.u = u; rec.v = v;
      rec.px0 = geom_col(g, 0); rec.py0 = geom_row(g, 0); rec.nx = g.nx; rec.ny = g.ny;
      rec.mask = mask; rec.eligible = eligible; rec.d_f = d_f; rec.d_b = d_b;
      rec.lr_ok = lr_ok; rec.d_sub = d_sub; rec.valid = valid;
      rec.dlo = ph.dlo; rec.nd = ph.nd;
      dbg.blocks[b] = rec;
    }
    if (eligible && b < dbg.cap_blocks) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kc = lane + 64 * r;
        if (kc < ph.nd && kc < dbg.cap_nd) {
          if (dbg.cost_fwd) dbg.cost_fwd[(size_t)b * dbg.cap_nd + kc] = (uint16_t)fwd[r];
          if (dbg.cost_bwd) dbg.cost_bwd[(size_t)b * dbg.cap_nd + kc] = (uint16_t)bwd[r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// aggregate: one workgroup per box
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float median_sorted(const float* v, int m) {
  if (m & 1) return v[(m - 1) / 2];
  return (v[m / 2 - 1] + v[m / 2]) * 0.5f;
}

__global__ __launch_bounds__(256) void aggregate_kernel(MatchParamsDev p, MatchWs ws,
                                                        ocsr_box_result* out) {
  __shared__ float vals[kAggMax];
  __shared__ int n_valid_s, n_elig_s;
  __shared__ int seg_start, seg_len;
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const BoxPlan pl = ws.plan[k];
  if (pl.status != -1) {
    if (tid == 0) {
      ocsr_box_result r = {};
      r.reason = pl.status;
      out[k] = r;
    }
    return;
  }
  if (tid == 0) { n_valid_s = 0; n_elig_s = 0; }
  __syncthreads();
  for (int i = tid; i < pl.nblk; i += 256) {
    const uint8_t f = ws.blk_flag[pl.off + i];
    if (f & 1) atomicAdd(&n_elig_s, 1);
    if (f & 2) vals[atomicAdd(&n_valid_s, 1)] = ws.blk_val[pl.off + i];
  }
  __syncthreads();
  const int nv = n_valid_s, ne = n_elig_s;
  ocsr_box_result r = {};
  r.n_blocks = pl.nblk;
  r.n_eligible = ne;
  r.n_valid = nv;
  if (ne == 0 || nv == 0) {
    if (tid == 0) {
      r.reason = ne == 0 ? OCSR_REASON_NO_ELIGIBLE_BLOCKS : OCSR_REASON_NO_VALID_BLOCKS;
      out[k] = r;
    }
    return;
  }
  float d_box = 0.0f;
  bool ok = true;
  if (pl.nblk == 1) {
    d_box = vals[0];   // a single-block object takes its block result (Alg. 2)
    r.n_used = 1;
  } else {
    // bitonic sort of the valid values, padded with +inf to a power of two
    int n2 = 1;
    while (n2 < nv) n2 <<= 1;
    for (int i = nv + tid; i < n2; i += 256) vals[i] = __builtin_inff();
    __syncthreads();
    for (int kk = 2; kk <= n2; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < n2; i += 256) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const float a = vals[i], c = vals[ixj];
            const bool up = (i & kk) == 0;
            if ((a > c) == up) { vals[i] = c; vals[ixj] = a; }
          }
        }
        __syncthreads();
      }
    }
    if (p.agg_mode == OCSR_AGG_SEGMENT_MEDIAN) {
      // longest run whose consecutive gaps stay below tau_d; first run on ties
      if (tid < 64) {
        int best_start = 0, best_len = 1, start = 0;
        for (int base = 0; base < nv; base += 64) {
          const int q = base + tid;
          const bool brk = q > 0 && q < nv && !(vals[q] - vals[q - 1] < p.tau_d);
          uint64_t m = __ballot(brk);
          while (m) {
            const int pos = base + __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int len = pos - start;
            if (len > best_len) { best_len = len; best_start = start; }
            start = pos;
          }
        }
        const int len = nv - start;
        if (len > best_len) { best_len = len; best_start = start; }
        if (tid == 0) { seg_start = best_start; seg_len = best_len; }
      }
      __syncthreads();
      r.n_used = seg_len;
      if (seg_len < p.n_min) ok = false;
      else d_box = median_sorted(vals + seg_start, seg_len);
    } else {
      const int t = p.trim_pct * nv / 100;
      const int m = nv - 2 * t;
      r.n_used = m > 0 ? m : 0;
      if (m <= 0 || m < p.n_min) ok = false;
      else d_box = median_sorted(vals + t, m);
    }
  }
  if (tid == 0) {
    if (!ok) {
      r.reason = OCSR_REASON_TOO_FEW_CONSISTENT;
    } else {
      r.disparity = d_box;
      if (!(d_box > p.d_eps)) {
        r.reason = OCSR_REASON_NONPOSITIVE_DISPARITY;
      } else {
        r.depth = p.fb / d_box;   // Eq. 1, IEEE fp32 division
        r.valid = 1;
        r.reason = OCSR_REASON_OK;
      }
    }
    out[k] = r;
  }
}

}  // namespace

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t match_ws_bytes(int n_boxes, int cap_blocks) {
  const size_t n = (size_t)(n_boxes > 0 ? n_boxes : 1);
  const size_t c = (size_t)(cap_blocks > 0 ? cap_blocks : 1);
  return align256(n * sizeof(BoxPlan)) + align256(n * sizeof(BoxClip)) +
         align256(n * sizeof(int32_t)) + align256(4 * sizeof(int32_t)) +
         align256(c * sizeof(float)) + align256(c * sizeof(uint8_t));
}

MatchWs match_ws_carve(void* base, int n_boxes, int cap_blocks) {
  const size_t n = (size_t)(n_boxes > 0 ? n_boxes : 1);
  const size_t c = (size_t)(cap_blocks > 0 ? cap_blocks : 1);
  char* b = (char*)base;
  MatchWs ws;
  ws.plan = (BoxPlan*)b;        b += align256(n * sizeof(BoxPlan));
  ws.clip = (BoxClip*)b;        b += align256(n * sizeof(BoxClip));
  ws.box_end = (int32_t*)b;     b += align256(n * sizeof(int32_t));
  ws.counters = (int32_t*)b;    b += align256(4 * sizeof(int32_t));
  ws.blk_val = (float*)b;       b += align256(c * sizeof(float));
  ws.blk_flag = (uint8_t*)b;
  return ws;
}

hipError_t launch_match(const MatchParamsDev& p, const ocsr_box* boxes, const MatchWs& ws,
                        ocsr_box_result* out, const DebugDev& dbg, int n_match_wgs,
                        hipStream_t stream, const LaunchTimer* timer) {
  if (p.n_boxes <= 0) return hipSuccess;
  hipError_t e;
  const int W = p.lv[0].W, H = p.lv[0].H;
  if (timer) timer->before(timer->ctx, "plan", stream);
  plan_kernel<<<1, 1024, 0, stream>>>(p, boxes, W, H, ws);
  if (timer) timer->after(timer->ctx, "plan", stream);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "match", stream);
  match_kernel<<<n_match_wgs, 64, 0, stream>>>(p, ws, dbg);
  if (timer) timer->after(timer->ctx, "match", stream);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "aggregate", stream);
  aggregate_kernel<<<p.n_boxes, 256, 0, stream>>>(p, ws, out);
  if (timer) timer->after(timer->ctx, "aggregate", stream);
  return hipGetLastError();
}

}  // namespace ocsr
