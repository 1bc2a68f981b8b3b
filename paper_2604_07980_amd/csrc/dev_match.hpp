// Device code of the object-centric matching steps (Sec. 4.3.2-4.3.6, Alg. 2), shared by
// the multi-launch kernels (match.hip) and the fused persistent kernel (fused.hip).
//
//   plan_frame        one wave per frame: clip, far/close type (Sec. 4.3.4 type
//                     equation), level box, block grid, block and work-item numbers
//   match_block_tiled one wave per block: occluder mask (Sec. 4.3.5), forward Hamming
//                     search (census cost equation), winner-take-all, parabola
//                     (sub-pixel equation), backward search and L/R check (Sec. 4.3.3)
//   aggregate_box     one workgroup per box: longest-segment or trimmed median of the
//                     valid block disparities (Sec. 4.3.4), depth Z = f b / d (Eq. 1)
#pragma once

#include "dev_common.hpp"

namespace ocsr {
namespace dev {

// valid block values of a box that the aggregation keeps in LDS; boxes with more
// blocks aggregate from global memory (the method sets no limit on a box's blocks)
constexpr int kAggMax = 4096;

// ---------------------------------------------------------------------------------
// plan: one wave walks the frame's boxes 64 at a time
// ---------------------------------------------------------------------------------
// With items == false the item records are left to write_frame_items. With lplan and a
// frame of at most lcap boxes, the plans also go to lplan[i] and the running item ends of
// the two levels to lend[i] (far) and lend[n + i] (close), and the two item counts to
// lend[2 n] (far) and lend[2 n + 1] (close), in LDS, for write_frame_items.
__device__ __forceinline__ void plan_frame(const MatchParamsDev& P, const FrameDev& fr, int f,
                                           int n_total, const ocsr_box* __restrict__ boxes,
                                           const MatchWs& ws, int lane, bool items = true,
                                           BoxPlan* lplan = nullptr, int32_t* lend = nullptr,
                                           int lcap = 0) {
  const int n = fr.n_boxes;
  const int W = fr.W, H = fr.H;
  int carry = 0, carry0 = 0, carry1 = 0, matched_end = 0;
  // the next 64 boxes are loaded while the current ones are planned
  ocsr_box next = {};
  if (lane < n) next = boxes[fr.box_off + lane];
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    BoxPlan pl = {};
    BoxClip cl = {0, 0, 0, 0};
    int count = 0;
    const ocsr_box b = next;
    if (i + 64 < n) next = boxes[fr.box_off + i + 64];
    if (i < n) {
      const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
      const int cx1 = min(b.x1, W), cy1 = min(b.y1, H);
      const bool empty = !(cx0 < cx1 && cy0 < cy1);
      if (!empty) cl = BoxClip{cx0, cy0, cx1, cy1};   // empty boxes overlap nothing
      if (!(b.flags & OCSR_BOX_RANGE)) {
        pl.status = OCSR_REASON_NOT_RANGED;
      } else if (empty) {
        pl.status = OCSR_REASON_CLIPPED_EMPTY;
      } else {
        // far/close type (Sec. 4.3.4): FAR iff the longer clipped side is below tau_s
        const bool far_box = max(cx1 - cx0, cy1 - cy0) < P.tau_s;
        const int level = far_box ? 0 : 1;
        const LevelDev& lv = fr.lv[level];
        const PathDev& ph = P.path[level];
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
            // centred grid of whole blocks; one shrunken block when the box is smaller
            pl.bw = min(ph.bw, pl.lw);
            pl.bh = min(ph.bh, pl.lh);
            pl.nbx = max(1, pl.lw / ph.bw);
            pl.nby = max(1, pl.lh / ph.bh);
            pl.ox = pl.lx0 + (pl.lw - pl.nbx * pl.bw) / 2;
            pl.oy = pl.ly0 + (pl.lh - pl.nby * pl.bh) / 2;
          } else {
            // the whole box is one block sampled on an n_side x n_side grid
            pl.nbx = pl.nby = 1;
            pl.bw = min(ph.n_side, pl.lw);
            pl.bh = min(ph.n_side, pl.lh);
          }
          // the method sets no limit on a box's blocks; only the call's capacity does.
          // A count past the capacity saturates at cap + 1 (the box, and every later box,
          // then passes the capacity), which keeps the prefix in 32 bits.
          const long long nb = (long long)pl.nbx * pl.nby;
          pl.status = -1;
          count = (int)min(nb, (long long)P.cap_blocks + 1);
        }
      }
    }
    // block numbers: prefix over the boxes; a range passing the capacity is dropped
    const int incl = wave_incl_scan(count, lane);
    const int off = carry + incl - count;
    int nblk = 0;
    if (pl.status == -1 && i < n) {
      if ((long long)off + count > (long long)P.cap_blocks) pl.status = OCSR_REASON_CAPACITY_OVERFLOW;
      else nblk = count;
    }
    // work items of item_blocks blocks of the box's level
    const int ib = P.item_blocks[pl.level];
    const int nitem = (nblk + ib - 1) / ib;
    const int c0 = (pl.status == -1 && pl.level == 0) ? nitem : 0;
    const int c1 = (pl.status == -1 && pl.level == 1) ? nitem : 0;
    const int incl0 = wave_incl_scan(c0, lane);
    const int incl1 = wave_incl_scan(c1, lane);
    if (i < n) {
      const int g = fr.box_off + i;
      pl.off = off;
      pl.nblk = nblk;
      pl.ioff = pl.level == 0 ? carry0 + incl0 - c0 : carry1 + incl1 - c1;
      pl.frame = f;
      ws.plan[g] = pl;
      ws.clip[g] = cl;
      ws.litem_end[g] = carry0 + incl0;
      ws.litem_end[n_total + g] = carry1 + incl1;
      if (lplan && n <= lcap) {
        lplan[i] = pl;
        lend[i] = carry0 + incl0;
        lend[n + i] = carry1 + incl1;
      }
    }
    matched_end = max(matched_end, wave_max(nblk > 0 ? off + nblk : 0));
    carry += __shfl(incl, 63, 64);
    carry0 += __shfl(incl0, 63, 64);
    carry1 += __shfl(incl1, 63, 64);
  }
  if (lane == 0) {
    int32_t* fc = ws.fcount + f * FC_N;
    fc[FC_NUMBERED] = carry;
    fc[FC_MATCHED] = matched_end;
    fc[FC_FAR_ITEMS] = carry0;
    fc[FC_CLOSE_ITEMS] = carry1;
    if (lplan && n <= lcap) {
      lend[2 * n] = carry0;
      lend[2 * n + 1] = carry1;
    }
  }
  if (!items) return;
  // item records: the frame's close items from 0, its far items after them; each lane
  // writes those of its box (re-reading the plan it stored above)
  ItemRec* rec = ws.items + (size_t)f * ws.items_cap;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    if (i >= n) continue;
    const BoxPlan pl = ws.plan[fr.box_off + i];
    if (pl.status != -1 || pl.nblk <= 0) continue;
    const int ib = P.item_blocks[pl.level];
    const int nitem = (pl.nblk + ib - 1) / ib;
    const int at = (pl.level == 1 ? 0 : carry1) + pl.ioff;
    for (int t = 0; t < nitem; ++t) {
      ItemRec r;
      r.k = i;
      r.first = t * ib;
      r.nblk = pl.nblk;
      r.off = pl.off;
      r.nbx = pl.nbx; r.bw = pl.bw; r.bh = pl.bh; r.ox = pl.ox; r.oy = pl.oy;
      r.lx0 = pl.lx0; r.ly0 = pl.ly0; r.lw = pl.lw; r.lh = pl.lh;
      r.pad[0] = r.pad[1] = r.pad[2] = 0;
      rec[at + t] = r;
    }
  }
}

// The item records of frame f (as plan_frame writes them) by the nthr threads of one
// workgroup, after plan_frame(..., items = false) has stored the frame's plans, running
// item ends and counters (and the threads have synchronised with it): thread tid writes
// items tid, tid + nthr, ...; the box of an item is found by binary search on the running
// item ends of its level. With lds (lds_cap words the caller is done with) holding both
// levels' ends of the frame, they are copied there first and searched in LDS. With
// lplan (a frame of at most lcap boxes), plan_frame's LDS copies of the plans and ends
// are used instead.
__device__ __forceinline__ void write_frame_items(const MatchParamsDev& P, const FrameDev& fr, int f,
                                                  int n_total, const MatchWs& ws, int tid, int nthr,
                                                  int32_t* lds = nullptr, int lds_cap = 0,
                                                  const BoxPlan* lplan = nullptr,
                                                  const int32_t* lend = nullptr, int lcap = 0) {
  const int n = fr.n_boxes;
  const bool from_plan = lplan && n <= lcap;
  const bool in_lds = !from_plan && lds && 2 * n <= lds_cap;
  if (from_plan) {
    lds = (int32_t*)lend;
  } else if (in_lds) {
    __syncthreads();   // every thread is done with the caller's use of the LDS
    for (int i = tid; i < n; i += nthr) {
      lds[i] = ws.litem_end[fr.box_off + i];
      lds[n + i] = ws.litem_end[(size_t)n_total + fr.box_off + i];
    }
    __syncthreads();
  }
  const int32_t* fc = ws.fcount + f * FC_N;
  const int n_close = from_plan ? lend[2 * n + 1] : fc[FC_CLOSE_ITEMS];
  const int n_far = from_plan ? lend[2 * n] : fc[FC_FAR_ITEMS];
  ItemRec* rec = ws.items + (size_t)f * ws.items_cap;
  for (int t = tid; t < n_close + n_far; t += nthr) {
    const int level = t < n_close ? 1 : 0;
    const int q = level ? t : t - n_close;
    const int32_t* end = in_lds || from_plan ? lds + level * n
                                             : ws.litem_end + (size_t)level * n_total + fr.box_off;
    int lo = 0, hi = n - 1;   // first box whose running end passes q
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (end[mid] > q) hi = mid;
      else lo = mid + 1;
    }
    const BoxPlan pl = from_plan ? lplan[lo] : ws.plan[fr.box_off + lo];
    ItemRec r;
    r.k = lo;
    r.first = (q - pl.ioff) * P.item_blocks[level];
    r.nblk = pl.nblk;
    r.off = pl.off;
    r.nbx = pl.nbx; r.bw = pl.bw; r.bh = pl.bh; r.ox = pl.ox; r.oy = pl.oy;
    r.lx0 = pl.lx0; r.ly0 = pl.ly0; r.lw = pl.lw; r.lh = pl.lh;
    r.pad[0] = r.pad[1] = r.pad[2] = 0;
    rec[t] = r;
  }
}

// ---------------------------------------------------------------------------------
// per-block steps
// ---------------------------------------------------------------------------------
// first of the frame's boxes whose running block end passes q (one vector load per 64)
__device__ __forceinline__ int find_box(const int32_t* __restrict__ end, int n, int q, int lane) {
  for (int base = 0; base < n; base += 64) {
    const int e = base + lane < n ? end[base + lane] : 0x7FFFFFFF;
    const uint64_t m = __ballot(e > q);
    if (m) return base + __ffsll((unsigned long long)m) - 1;
  }
  return n - 1;
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

// Occlusion-aware sampling (Sec. 4.3.5): bit j*nx+i is set iff point (i, j) lies in no
// box of the frame that overlaps box k and has a larger bottom y. Lanes scan the boxes
// 64 at a time; the few occluders found are then tested against one point per lane.
__device__ __forceinline__ uint64_t block_mask(const MatchWs& ws, int box_off, int n, int k,
                                               const BlockGeom& g, int lane) {
  const BoxClip ck = ws.clip[box_off + k];
  const int s = g.s;
  const int npts = g.nx * g.ny;
  const int pi = lane % g.nx, pj = min(lane / g.nx, g.ny - 1);
  const int fx = s * geom_col(g, pi), fy = s * geom_row(g, pj);
  const int bx0 = s * geom_col(g, 0), bx1 = s * geom_col(g, g.nx - 1);
  const int by0 = s * geom_row(g, 0), by1 = s * geom_row(g, g.ny - 1);
  bool hidden = false;
  for (int jb = 0; jb < n; jb += 64) {
    const int o = jb + lane;
    const BoxClip co = o < n ? ws.clip[box_off + o] : BoxClip{0, 0, 0, 0};
    const bool occ = o < n && o != k && ck.cx0 < co.cx1 && co.cx0 < ck.cx1 && ck.cy0 < co.cy1 &&
                     co.cy0 < ck.cy1 && co.cy1 > ck.cy1 && co.cx0 <= bx1 && co.cx1 > bx0 &&
                     co.cy0 <= by1 && co.cy1 > by0;
    uint64_t m = __ballot(occ);
    while (m) {
      // the occluder's box, read from the lane that loaded it
      const int src = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int x0 = __builtin_amdgcn_readlane(co.cx0, src), x1 = __builtin_amdgcn_readlane(co.cx1, src);
      const int y0 = __builtin_amdgcn_readlane(co.cy0, src), y1 = __builtin_amdgcn_readlane(co.cy1, src);
      hidden |= fx >= x0 && fx < x1 && fy >= y0 && fy < y1;
    }
  }
  return __ballot(lane < npts && !hidden);
}

__device__ __forceinline__ bool block_eligible(const MatchParamsDev& P, uint64_t mask, int npts) {
  const int nm = __popcll(mask);
  return nm > 0 && 100 * nm >= P.min_point_pct * npts;
}

// parabola through (d_f - 1, a), (d_f, c), (d_f + 1, b) (sub-pixel equation, in d = -dx);
// at either end of the range the integer disparity is kept
__device__ __forceinline__ float subpixel(int d_f, int best, int nd, int a, int c, int b) {
  if (best > 0 && best < nd - 1) {
    const int num = a - b;
    const int den = 2 * (a + b - 2 * c);
    const float offs = (float)num / (float)den;
    return (float)d_f + offs;
  }
  return (float)d_f;
}

struct BlockCtx {
  int f;            // frame index
  int level;
  int k;            // box index within the frame
  int kg;           // box index over the call
  int b;            // block number within the frame
  int slot;         // block storage index over the call
  int u, v;
  BoxPlan pl;
  BlockGeom g;
};

// block `local` (0-based, row-major over the box's block grid) of box k of frame f, at
// column u and row v of the grid
__device__ __forceinline__ BlockCtx block_ctx(const MatchParamsDev& P, const FrameDev& fr, int f,
                                              int k, const BoxPlan& pl, int local, int u, int v,
                                              int level) {
  BlockCtx c;
  c.f = f;
  c.level = level;
  c.k = k;
  c.kg = fr.box_off + k;
  c.pl = pl;
  c.b = pl.off + local;
  c.slot = f * P.cap_blocks + c.b;
  c.v = v;
  c.u = u;
  const LevelDev& lv = fr.lv[level];
  c.g.nx = pl.bw; c.g.ny = pl.bh; c.g.s = lv.scale;
  c.g.tiled = P.path[level].mode == OCSR_MODE_TILED;
  c.g.cx = pl.ox + c.u * pl.bw; c.g.lx0 = pl.lx0; c.g.lw = pl.lw;
  c.g.cy = pl.oy + c.v * pl.bh; c.g.ly0 = pl.ly0; c.g.lh = pl.lh;
  return c;
}
__device__ __forceinline__ BlockCtx block_ctx(const MatchParamsDev& P, const FrameDev& fr, int f,
                                              int k, const BoxPlan& pl, int local, int level) {
  const int v = local / pl.nbx;
  return block_ctx(P, fr, f, k, pl, local, local - v * pl.nbx, v, level);
}

// Stores the block's result (lane 0 of the wave).
__device__ __forceinline__ void write_block(const MatchWs& ws, const DebugDev& dbg,
                                            const BlockCtx& c, const PathDev& ph, uint64_t mask,
                                            bool eligible, int d_f, int d_b, int lr_ok,
                                            float d_sub, int valid, int lane, int dy_f = 0,
                                            int dy_b = 0) {
  if (lane == 0) {
    ws.blk_val[c.slot] = (float)c.g.s * d_sub;   // d_full = s * d (Sec. 4.1)
    ws.blk_flag[c.slot] = (uint8_t)((eligible ? 1 : 0) | (valid ? 2 : 0));
    if (dbg.blocks && c.b < dbg.cap_blocks) {
      ocsr_block_record rec;
      rec.box = c.k; rec.level_scale = c.g.s; rec.u = c.u; rec.v = c.v;
      rec.px0 = geom_col(c.g, 0); rec.py0 = geom_row(c.g, 0); rec.nx = c.g.nx; rec.ny = c.g.ny;
      rec.mask = mask; rec.eligible = eligible; rec.d_f = d_f; rec.d_b = d_b;
      rec.lr_ok = lr_ok; rec.d_sub = d_sub; rec.valid = valid;
      rec.dlo = ph.dlo; rec.nd = ph.nd;
      rec.dy_f = dy_f; rec.dy_b = dy_b;
      dbg.blocks[c.b] = rec;
    }
  }
}

// ---------------------------------------------------------------------------------
// TILED block, register-blocked. One wave per block of at most NX x ROWS points.
// Lane = (row j, candidate group g); group g owns CPL consecutive candidates. The
// block's template rows and its search strip (nd + nx - 1 words per row) are staged
// in LDS with coalesced loads; each lane then holds its row's NX template words and
// NX + CPL - 1 strip words in registers and forms NX * CPL costs from them
// (2 x v_xor_b32 + 2 x v_bcnt_u32_b32 each). Row sums are combined with DPP.
// ---------------------------------------------------------------------------------
// popcount of a 64-bit word added to acc as two v_bcnt_u32_b32 (each adds its popcount
// to its second operand). Written as instructions so that the compiler cannot regroup a
// chain of these sums into popcounts of zero plus v_add3_u32 adds, which costs a fifth
// instruction per term.
__device__ __forceinline__ uint32_t popc64_acc(uint64_t x, uint32_t acc) {
  asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc) : "v"((uint32_t)x));
  asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc) : "v"((uint32_t)(x >> 32)));
  return acc;
}

// acc[c] = sum over the row's unmasked points i of popcount(t[i] ^ srow[i + c]).
// col_all / col_any (wave-uniform): the block columns whose point is unmasked in every
// row / in some row. Columns masked in every row (occluded, or past the block's width)
// are skipped. When every other column is unmasked in every row, a cost is 4 ops;
// otherwise each difference is ANDed with the lane's own mask bit (6 ops).
template <int NX, int CPL>
__device__ __forceinline__ void row_costs(const uint64_t (&t)[NX], const uint64_t* __restrict__ srow,
                                          uint32_t rowmask, uint32_t col_all, uint32_t col_any,
                                          uint32_t (&acc)[CPL]) {
  uint64_t w[NX + CPL - 1];
#pragma unroll
  for (int m = 0; m < NX + CPL - 1; ++m) w[m] = srow[m];
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0;
  if (col_all == col_any) {
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      if (col_all & (1u << i)) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc(t[i] ^ w[i + c], acc[c]);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      if (col_any & (1u << i)) {
        const uint64_t keep = ((rowmask >> i) & 1u) ? ~0ull : 0ull;
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc((t[i] ^ w[i + c]) & keep, acc[c]);
      }
    }
  }
}

template <int ROWS>
__device__ __forceinline__ uint32_t row_sum(uint32_t v) {
  // lanes j = lane % ROWS of one group: quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  if (ROWS == 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
  return v;
}

// S[jj * SW + m] = row jj's word at x_first + m of the level image (0 outside the
// image, past the block's ny rows or past sw words), for ROWS x SW entries. All loads
// of a lane are issued before the first is waited for; an entry with no word reads
// the block's first row at column 0 instead and is zeroed.
template <int ROWS, int SW>
__device__ __forceinline__ void stage_strip(uint64_t* __restrict__ S, const uint64_t* __restrict__ rows,
                                            int pitch, int x_first, int ny, int sw, int W, int lane) {
  if constexpr ((SW & (SW - 1)) == 0) {
    // power-of-two rows: word idx = lane + 64 k of the ROWS x SW strip, row and column
    // by shift and mask
    constexpr int N = ROWS * SW, IT = (N + 63) / 64;
    uint64_t w[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = lane + 64 * k;
      const int jj = idx / SW, m = idx % SW, x = x_first + m;
      const bool ok = idx < N && jj < ny && m < sw && x >= 0 && x < W;
      w[k] = rows[ok ? (size_t)jj * pitch + x : 0];
      w[k] = ok ? w[k] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = lane + 64 * k;
      if (idx < N) S[idx] = w[k];
    }
  } else {
    // row by row in chunks of 64 words: the row is a constant and the column the lane,
    // so no per-lane division (whose results the compiler would keep live in registers
    // across the whole work-item loop)
    constexpr int CH = (SW + 63) / 64;
    uint64_t w[ROWS][CH];
#pragma unroll
    for (int jj = 0; jj < ROWS; ++jj)
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int m = 64 * c + lane, x = x_first + m;
        const bool ok = jj < ny && m < sw && x >= 0 && x < W;
        w[jj][c] = rows[ok ? (size_t)jj * pitch + x : 0];
        w[jj][c] = ok ? w[jj][c] : 0ull;
      }
#pragma unroll
    for (int jj = 0; jj < ROWS; ++jj)
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (64 * c + lane < SW) S[jj * SW + 64 * c + lane] = w[jj][c];
  }
}

template <int ROWS, int NX, int CPL, int PASSES = 1>
struct Tiled {
  static constexpr int G = 64 / ROWS;
  static constexpr int NC = G * CPL * PASSES;  // candidates one wave covers
  static constexpr int SW = NC + NX - 1;       // strip words per row
  static constexpr size_t kLdsBytes = sizeof(uint64_t) * (ROWS * SW + ROWS * NX) +
                                      sizeof(uint32_t) * 2 * NC;
  static_assert(ROWS == 4 || ROWS == 8, "rows");
};

template <int ROWS, int NX, int CPL, int PASSES = 1>
__device__ __forceinline__ void match_block_tiled(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg,
                                                  const BlockCtx& c, int lane, void* lds) {
  using TT = Tiled<ROWS, NX, CPL, PASSES>;
  constexpr int PC = TT::G * CPL;              // candidates of one pass
  constexpr int SW = TT::SW, NC = TT::NC;
  uint64_t* S = (uint64_t*)lds;
  uint64_t* T = S + ROWS * SW;
  uint32_t* costf = (uint32_t*)(T + ROWS * NX);
  uint32_t* costb = costf + NC;
  const int j = lane % ROWS, grp = lane / ROWS;
  const LevelDev& lv = fr.lv[c.level];
  const PathDev& ph = P.path[c.level];
  const int nd = ph.nd, dlo = ph.dlo, dhi = dlo + nd - 1;

  const int nx = c.g.nx, ny = c.g.ny;
  const int X0 = c.g.cx, Y0 = c.g.cy;
  const uint64_t* __restrict__ Lb = lv.L + (size_t)Y0 * lv.pitch;
  const uint64_t* __restrict__ Rb = lv.R + (size_t)Y0 * lv.pitch;
  const int sw = nd + nx - 1;
  // forward: template CL(X0 + i, Y0 + j); strip CR(X0 - dhi + m, Y0 + j). Issued before
  // the occluder scan so that both sets of loads are in flight together.
  stage_strip<ROWS, SW>(S, Rb, lv.pitch, X0 - dhi, ny, sw, lv.W, lane);
  stage_strip<ROWS, NX>(T, Lb, lv.pitch, X0, ny, nx, lv.W, lane);
  const uint64_t mask = block_mask(ws, fr.box_off, fr.n_boxes, c.k, c.g, lane);
  const bool eligible = block_eligible(P, mask, nx * ny);
  wave_sync();
  if (!eligible) {
    write_block(ws, dbg, c, ph, mask, false, dlo, dlo, 0, (float)dlo, 0, lane);
    wave_sync();
    return;
  }
  const uint32_t rowmask = j < ny ? (uint32_t)((mask >> (j * nx)) & ((1u << nx) - 1u)) : 0u;
  // columns unmasked in every row / in some row (the mask is wave-uniform)
  uint32_t col_all = (1u << nx) - 1u, col_any = 0;
  for (int jj = 0; jj < ny; ++jj) {
    const uint32_t r = (uint32_t)((mask >> (jj * nx)) & ((1u << nx) - 1u));
    col_all &= r;
    col_any |= r;
  }
  uint64_t t[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) t[i] = T[j * NX + i];
  uint32_t acc[CPL];
  uint32_t key = 0xFFFFFFFFu;
  // strip entry e + i (e = ps*PC + grp*CPL + c) holds CR(X0 + i - d) for d = dhi - e;
  // the candidates are covered in PASSES passes of PC
#pragma unroll 1
  for (int ps = 0; ps < PASSES; ++ps) {
    if (j < ny) row_costs<NX, CPL>(t, S + j * SW + ps * PC + grp * CPL, rowmask, col_all, col_any, acc);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
      if (j >= ny) acc[cc] = 0;
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const uint32_t tot = row_sum<ROWS>(acc[cc]);
      const int e = ps * PC + grp * CPL + cc;
      if (e < nd) {
        const int kc = nd - 1 - e;
        key = min(key, (tot << 16) | (uint32_t)kc);
        if (j == 0) costf[kc] = tot;
      }
    }
  }
  key = wave_min_u32(key, ROWS);
  const int best = (int)(key & 0xFFFFu);
  const int d_f = dlo + best;
  // backward template CR(X0 - d_f + i, Y0 + j) sits in the forward strip at dhi - d_f + i
#pragma unroll
  for (int i = 0; i < NX; ++i) t[i] = S[j * SW + (dhi - d_f) + i];
  wave_sync();
  const int ca = (int)costf[max(best - 1, 0)];
  const int cb = (int)costf[min(best + 1, nd - 1)];
  const float d_sub = subpixel(d_f, best, nd, ca, (int)(key >> 16), cb);
  // backward strip: CL(X0 - d_f + dlo + m, Y0 + j)
  stage_strip<ROWS, SW>(S, Lb, lv.pitch, X0 - d_f + dlo, ny, sw, lv.W, lane);
  wave_sync();
  uint32_t bkey = 0xFFFFFFFFu;
#pragma unroll 1
  for (int ps = 0; ps < PASSES; ++ps) {
    if (j < ny) row_costs<NX, CPL>(t, S + j * SW + ps * PC + grp * CPL, rowmask, col_all, col_any, acc);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
      if (j >= ny) acc[cc] = 0;
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const uint32_t tot = row_sum<ROWS>(acc[cc]);
      const int kc = ps * PC + grp * CPL + cc;   // candidate dlo + kc
      if (kc < nd) {
        bkey = min(bkey, (tot << 16) | (uint32_t)kc);
        if (j == 0) costb[kc] = tot;
      }
    }
  }
  bkey = wave_min_u32(bkey, ROWS);
  const int d_b = dlo + (int)(bkey & 0xFFFFu);
  const int lr_ok = abs(d_b - d_f) <= P.lr_tol;
  if (c.b < dbg.cap_blocks && (dbg.cost_fwd || dbg.cost_bwd)) {
    wave_sync();
    for (int kc = lane; kc < nd && kc < dbg.cap_nd; kc += 64) {
      if (dbg.cost_fwd) dbg.cost_fwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costf[kc];
      if (dbg.cost_bwd) dbg.cost_bwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costb[kc];
    }
  }
  write_block(ws, dbg, c, ph, mask, true, d_f, d_b, lr_ok, d_sub, lr_ok, lane);
  wave_sync();
}

// ---------------------------------------------------------------------------------
// TILED block of up to 8 x 8 points, lanes over (candidate group, row half): lane
// l = 2 g + h takes block rows 4h .. 4h + 3 and the CPL consecutive strip positions
// g CPL + c (c < CPL), so one wave covers 32 CPL candidates in one pass. For each of its
// rows a lane reads the 8 template words and CPL + 7 strip words from LDS and forms
// 8 CPL costs at 4 operations each; the two row halves of a candidate meet in one DPP
// add, and the winner is a DPP wave minimum of packed (cost << 16 | index) keys. A strip
// row is staged in 64-word chunks through a buffer resource per row (load_half_strip).
// ---------------------------------------------------------------------------------
// strip row stride beyond the candidates (see Half::SWP)
constexpr int kHalfStripPad = 10;

template <int CPL>
struct Half {
  static constexpr int NC = 32 * CPL;               // candidates one wave covers
  // LDS words per strip row (>= NC + 7). The two row halves are read by the same
  // instructions (lanes 2g and 2g + 1), so rows four apart must start in different LDS
  // banks: 4 SWP is an odd multiple of 8 words.
  static constexpr int SWP = NC + kHalfStripPad;
  static constexpr int TH = 40;                     // template: rows 4..7 start here
  static constexpr int TW = TH + 32;                // template words
  static constexpr int CH = (NC + 7 + 63) / 64;     // 64-word chunks of a strip row
  static constexpr size_t kLdsBytes =
      sizeof(uint64_t) * (8 * SWP + TW) + sizeof(uint16_t) * 2 * NC;
  static_assert(SWP >= NC + 7, "a strip row holds nd + 7 words");
};

// Whole-wave minimum of v (every lane gets it): DPP within rows of 16, then row
// broadcasts (lane 15 into the next row, lane 31 into rows 2 and 3), then lane 63.
__device__ __forceinline__ uint32_t wave_min_dpp(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Strip rows 0 .. 7 of a level image from `rows` (the block's first row), words
// [x_first, x_first + 64 CH) of each row, for S[jj * SWP + m], m < SWP; rows at or past
// ny (which no kept point reads) are 0. load_half_strip issues the loads and
// store_half_strip writes the words to LDS, so that a caller can put other loads in
// flight between the two. Each row is read through a buffer resource spanning exactly
// that row (W words; none for rows past ny), so a word outside the image, left or right,
// reads as 0 by the hardware's range check without a memory access: a column below 0
// gives a byte offset that wraps past the range. The rows' resources and offsets are
// wave-uniform (scalar instructions); lane l reads word l of each 64-word chunk at a
// byte offset fixed for the whole strip, so the loads take no per-lane address
// arithmetic.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <int CH>
struct HalfStrip {
  u32x2 w[8][CH];
};
template <int SWP, int CH>
__device__ __forceinline__ HalfStrip<CH> load_half_strip(const uint64_t* __restrict__ rows, int pitch,
                                                         int x_first, int ny, int W, int lane) {
  static_assert(SWP > 64 * (CH - 1) && SWP <= 64 * CH, "the strip row ends in the last chunk");
  uint32_t voff[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) voff[c] = (uint32_t)(x_first + 64 * c + lane) * 8u;
  HalfStrip<CH> st;
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    // W words for rows inside the block (jj < ny: the sign bit of jj - ny), else none
    const int nrec = W * 8 * (int)((uint32_t)(jj - ny) >> 31);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(rows + (size_t)jj * pitch), (short)0, nrec, 0x00020000);
#pragma unroll
    for (int c = 0; c < CH; ++c) st.w[jj][c] = __builtin_amdgcn_raw_buffer_load_b64(rs, voff[c], 0, 0);
  }
  return st;
}
// The last chunk goes first: its lanes past the row end write their chunk-0 word, which
// the chunk-0 stores that follow overwrite (a wave's LDS writes land in order), so no
// lane mask is needed and no load is held back behind one.
template <int SWP, int CH>
__device__ __forceinline__ void store_half_strip(uint64_t* __restrict__ S, const HalfStrip<CH>& st,
                                                 int lane) {
  auto word = [](u32x2 v) { return ((uint64_t)v.y << 32) | v.x; };
  if constexpr (CH == 1) {
    if (lane < SWP) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) S[jj * SWP + lane] = word(st.w[jj][0]);
    }
  } else {
    const int mlast = 64 * (CH - 1) + lane < SWP ? 64 * (CH - 1) + lane : lane;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) S[jj * SWP + mlast] = word(st.w[jj][CH - 1]);
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
#pragma unroll
      for (int c = 0; c < CH - 1; ++c) S[jj * SWP + 64 * c + lane] = word(st.w[jj][c]);
  }
}

// One direction of the search: acc[c] = cost of strip position g CPL + c over the lane's
// rows, summed with the other row half. keep: the lane's point mask (bit r 8 + i for
// row 4h + r, column i; 0 for points that do not exist). `full` (wave-uniform): every
// point of an 8 x 8 block is kept, and a cost is 4 operations; otherwise each
// difference is ANDed with its point's mask bit (6 operations), with no branch per row
// or column.
template <int CPL>
__device__ __forceinline__ void half_costs(const uint64_t* __restrict__ T, const uint64_t* __restrict__ S,
                                           int g, int h, bool full, uint32_t keep,
                                           uint32_t (&acc)[CPL]) {
  constexpr int SWP = Half<CPL>::SWP;
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0;
  const uint64_t* __restrict__ trow = T + Half<CPL>::TH * h;
  const uint64_t* __restrict__ srow = S + 4 * h * SWP + g * CPL;
  if (full) {
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
      uint64_t t[8], w[CPL + 7];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = trow[8 * r + i];
#pragma unroll
      for (int m = 0; m < CPL + 7; ++m) w[m] = srow[r * SWP + m];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc(t[i] ^ w[i + c], acc[c]);
    }
  } else {
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
      uint64_t t[8], w[CPL + 7];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = trow[8 * r + i];
#pragma unroll
      for (int m = 0; m < CPL + 7; ++m) w[m] = srow[r * SWP + m];
      const uint32_t kr = keep >> (8 * r);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint64_t k = ((kr >> i) & 1u) ? ~0ull : 0ull;
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc((t[i] ^ w[i + c]) & k, acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    acc[c] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)acc[c], 0xB1, 0xF, 0xF, false);
}

// Whether point (fx, fy) lies in one of the rectangles held by the lanes of m (each lane
// o holds the clipped box co).
__device__ __forceinline__ bool in_lane_rects(uint64_t m, const BoxClip& co, int fx, int fy) {
  bool hidden = false;
  while (m) {
    const int src = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int x0 = __builtin_amdgcn_readlane(co.cx0, src), x1 = __builtin_amdgcn_readlane(co.cx1, src);
    const int y0 = __builtin_amdgcn_readlane(co.cy0, src), y1 = __builtin_amdgcn_readlane(co.cy1, src);
    hidden |= fx >= x0 && fx < x1 && fy >= y0 && fy < y1;
  }
  return hidden;
}

// Occlusion mask of a TILED block (Sec. 4.3.5) in the 8-column layout: bit j*8 + i is
// set iff point (i, j) exists (i < nx, j < ny) and lies in no box of the frame that
// overlaps box k and has a larger bottom y. Lane l tests point (l & 7, l >> 3).
__device__ __forceinline__ uint64_t tiled_mask8(const MatchWs& ws, int box_off, int n, int k,
                                                int s, int cx, int cy, int nx, int ny, int lane) {
  const BoxClip ck = ws.clip[box_off + k];
  const int pi = lane & 7, pj = lane >> 3;
  const bool exists = pi < nx && pj < ny;
  const int fx = s * (cx + pi), fy = s * (cy + pj);
  const int bx0 = s * cx, bx1 = s * (cx + nx - 1);
  const int by0 = s * cy, by1 = s * (cy + ny - 1);
  bool hidden = false;
  for (int jb = 0; jb < n; jb += 64) {
    const int o = jb + lane;
    const BoxClip co = o < n ? ws.clip[box_off + o] : BoxClip{0, 0, 0, 0};
    const bool occ = o < n && o != k && ck.cx0 < co.cx1 && co.cx0 < ck.cx1 && ck.cy0 < co.cy1 &&
                     co.cy0 < ck.cy1 && co.cy1 > ck.cy1 && co.cx0 <= bx1 && co.cx1 > bx0 &&
                     co.cy0 <= by1 && co.cy1 > by0;
    hidden |= in_lane_rects(__ballot(occ), co, fx, fy);
  }
  return __ballot(exists && !hidden);
}

// The boxes that may hide points of box k, for all blocks of one work item of a frame of
// at most 64 boxes (in_lanes; otherwise each block scans the frame's boxes itself):
// lane o holds box o's clipped rectangle, and bit o of `cand` is set iff box o overlaps
// box k and has the larger bottom y, the part of tiled_mask8's test that does not depend
// on the block.
struct OccLanes {
  BoxClip co;
  uint64_t cand;
  bool in_lanes;
};
// The frame's part, which does not depend on k (so its load need not wait for an item
// record): lane o holds box o's clipped rectangle.
__device__ __forceinline__ OccLanes frame_lanes(const MatchWs& ws, int box_off, int n, int lane) {
  OccLanes oc{BoxClip{0, 0, 0, 0}, 0ull, n <= 64};
  if (oc.in_lanes && lane < n) oc.co = ws.clip[box_off + lane];
  return oc;
}
// Box k's candidates (box k's own rectangle from lane k).
__device__ __forceinline__ void box_candidates(OccLanes& oc, int n, int k, int lane) {
  if (!oc.in_lanes) return;
  const BoxClip co = oc.co;
  const BoxClip ck{__builtin_amdgcn_readlane(co.cx0, k), __builtin_amdgcn_readlane(co.cy0, k),
                   __builtin_amdgcn_readlane(co.cx1, k), __builtin_amdgcn_readlane(co.cy1, k)};
  oc.cand = __ballot(lane < n && lane != k && ck.cx0 < co.cx1 && co.cx0 < ck.cx1 &&
                     ck.cy0 < co.cy1 && co.cy0 < ck.cy1 && co.cy1 > ck.cy1);
}
// tiled_mask8 from the rectangles of frame_lanes and box_candidates
__device__ __forceinline__ uint64_t tiled_mask8_lanes(const OccLanes& oc, int s, int cx, int cy,
                                                      int nx, int ny, int lane) {
  const int pi = lane & 7, pj = lane >> 3;
  const bool exists = pi < nx && pj < ny;
  const int fx = s * (cx + pi), fy = s * (cy + pj);
  const int bx0 = s * cx, bx1 = s * (cx + nx - 1);
  const int by0 = s * cy, by1 = s * (cy + ny - 1);
  const BoxClip co = oc.co;
  const bool occ = ((oc.cand >> lane) & 1ull) && co.cx0 <= bx1 && co.cx1 > bx0 && co.cy0 <= by1 &&
                   co.cy1 > by0;
  // the ballot of candidates is taken by the whole wave (lanes past the block hold boxes too)
  const bool hidden = in_lane_rects(__ballot(occ), co, fx, fy);
  return __ballot(exists && !hidden);
}

// The 8-column mask in the record's layout (bit j * nx + i).
__device__ __forceinline__ uint64_t pack_mask8(uint64_t m8, int nx, int ny, int lane) {
  const int j = lane / nx, i = lane - j * nx;
  return __ballot(lane < nx * ny && ((m8 >> (8 * j + i)) & 1ull));
}

// oc: the box's occluders when the frame's boxes fit the lanes (frame_lanes,
// box_candidates). The occlusion mask comes first (from registers in that case), so that
// a block that is not eligible loads no strip.
template <int CPL>
__device__ __forceinline__ void match_block_half(const MatchParamsDev& P, const FrameDev& fr,
                                                 const MatchWs& ws, const DebugDev& dbg,
                                                 const BlockCtx& c, const OccLanes& oc, int lane,
                                                 void* lds) {
  using HH = Half<CPL>;
  constexpr int SWP = HH::SWP, CH = HH::CH, NC = HH::NC;
  uint64_t* S = (uint64_t*)lds;
  uint64_t* T = S + 8 * SWP;                   // row jj at 8 jj, rows 4..7 moved by TH - 32
  uint16_t* costf = (uint16_t*)(T + HH::TW);   // a cost is at most 64 x 64
  uint16_t* costb = costf + NC;
  const int tslot = lane + (lane >= 32 ? HH::TH - 32 : 0);   // lane (i, jj) = i + 8 jj
  const int g = lane >> 1, h = lane & 1;
  const LevelDev& lv = fr.lv[c.level];
  const PathDev& ph = P.path[c.level];
  const int nd = ph.nd, dlo = ph.dlo, dhi = dlo + nd - 1;
  const int nx = c.g.nx, ny = c.g.ny;
  const int X0 = c.g.cx, Y0 = c.g.cy;
  const int W = lv.W;
  const uint64_t* __restrict__ Lb = uniform(lv.L + (size_t)Y0 * lv.pitch);
  const uint64_t* __restrict__ Rb = uniform(lv.R + (size_t)Y0 * lv.pitch);
  const uint64_t m8 = oc.in_lanes ? tiled_mask8_lanes(oc, c.g.s, X0, Y0, nx, ny, lane)
                                  : tiled_mask8(ws, fr.box_off, fr.n_boxes, c.k, c.g.s, X0, Y0, nx, ny, lane);
  const int npts = __popcll(m8);
  const bool eligible = npts > 0 && 100 * npts >= P.min_point_pct * nx * ny;
  if (!eligible) {
    const uint64_t mask = dbg.blocks ? pack_mask8(m8, nx, ny, lane) : 0ull;
    write_block(ws, dbg, c, ph, mask, false, dlo, dlo, 0, (float)dlo, 0, lane);
    return;
  }
  // forward strip CR(X0 - dhi + m, Y0 + j) and template CL(X0 + i, Y0 + j), loaded together
  const HalfStrip<CH> fw = load_half_strip<SWP, CH>(Rb, lv.pitch, X0 - dhi, ny, W, lane);
  uint64_t tw;
  {
    const int i = lane & 7, jj = lane >> 3;
    const bool ok = i < nx && jj < ny;
    tw = Lb[ok ? (size_t)jj * lv.pitch + X0 + i : 0];
    tw = ok ? tw : 0ull;
  }
  store_half_strip<SWP, CH>(S, fw, lane);
  T[tslot] = tw;
  wave_sync();
  const bool full = m8 == ~0ull;   // an 8 x 8 block with every point kept
  const uint32_t keep = (uint32_t)(m8 >> (32 * h));
  uint32_t acc[CPL];
  half_costs<CPL>(T, S, g, h, full, keep, acc);
  // both lanes of a group hold the whole cost; a strip position past the range writes
  // its (unread) slot at index e >= nd instead of a branch
  uint32_t key = 0xFFFFFFFFu;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int e = g * CPL + cc;            // strip position: candidate d = dhi - e
    const bool in = e < nd;
    const int kc = nd - 1 - e;
    key = min(key, in ? (acc[cc] << 16) | (uint32_t)kc : 0xFFFFFFFFu);
    costf[in ? kc : e] = (uint16_t)acc[cc];
  }
  key = wave_min_dpp(key);
  const int best = (int)(key & 0xFFFFu);
  const int d_f = dlo + best;
  // backward template CR(X0 - d_f + i, Y0 + j): strip position dhi - d_f + i
  {
    const int i = lane & 7, jj = lane >> 3;
    const uint64_t t = S[jj * SWP + (dhi - d_f) + i];
    wave_sync();
    T[tslot] = t;
  }
  const int ca = (int)costf[max(best - 1, 0)];
  const int cb = (int)costf[min(best + 1, nd - 1)];
  const float d_sub = subpixel(d_f, best, nd, ca, (int)(key >> 16), cb);
  // backward strip CL(X0 - d_f + dlo + m, Y0 + j)
  wave_sync();
  store_half_strip<SWP, CH>(S, load_half_strip<SWP, CH>(Lb, lv.pitch, X0 - d_f + dlo, ny, W, lane), lane);
  wave_sync();
  half_costs<CPL>(T, S, g, h, full, keep, acc);
  uint32_t bkey = 0xFFFFFFFFu;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int kc = g * CPL + cc;           // candidate d' = dlo + kc (slots past nd unread)
    bkey = min(bkey, kc < nd ? (acc[cc] << 16) | (uint32_t)kc : 0xFFFFFFFFu);
  }
  // the backward costs are read only for the debug output
  if (dbg.cost_bwd) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) costb[g * CPL + cc] = (uint16_t)acc[cc];
  }
  bkey = wave_min_dpp(bkey);
  const int d_b = dlo + (int)(bkey & 0xFFFFu);
  const int lr_ok = abs(d_b - d_f) <= P.lr_tol;
  uint64_t mask = 0;
  if (dbg.blocks || dbg.cost_fwd || dbg.cost_bwd) {
    mask = pack_mask8(m8, nx, ny, lane);
    if (c.b < dbg.cap_blocks && (dbg.cost_fwd || dbg.cost_bwd)) {
      wave_sync();
      for (int kc = lane; kc < nd && kc < dbg.cap_nd; kc += 64) {
        if (dbg.cost_fwd) dbg.cost_fwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costf[kc];
        if (dbg.cost_bwd) dbg.cost_bwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costb[kc];
      }
    }
  }
  write_block(ws, dbg, c, ph, mask, true, d_f, d_b, lr_ok, d_sub, lr_ok, lane);
  wave_sync();
}

// ---------------------------------------------------------------------------------
// TILED blocks of up to 4 x 4 points, four blocks per wave: lane l = 16 q + g takes
// block q of the four (its 16 lanes a DPP row) and the CPL consecutive strip positions
// g CPL + c, so a row of lanes covers 16 CPL candidates and each lane forms the whole
// cost of its candidates over the block's points (no reduction across lanes). The
// winner of a block is a DPP minimum within its row of lanes. Each block has its own
// strip and template in LDS, staged by its 16 lanes.
// ---------------------------------------------------------------------------------
template <int CPL>
struct Quad {
  static constexpr int NC = 16 * CPL;               // candidates per block
  static constexpr int SWP = NC + 4;                // LDS words per strip row (>= NC + 3)
  static constexpr int BLK = 4 * SWP + 16;          // LDS words per block: strip, template
  static constexpr int CH = (NC + 3 + 15) / 16;     // 16-word chunks of a strip row
  static constexpr size_t kLdsBytes = sizeof(uint64_t) * 4 * BLK + sizeof(uint32_t) * 2 * 4 * NC;
};

// Minimum over each row of 16 lanes (every lane of the row gets it).
__device__ __forceinline__ uint32_t row16_min_dpp(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));
  return v;
}

// One quarter's strip: rows 0 .. ny - 1 from `rows` (its block's first row), words
// [x_first, x_first + sw) into S[jj * SWP + m], 0 outside the image; g: the lane's
// index in its quarter. All loads are issued before the first store.
template <int CPL>
__device__ __forceinline__ void stage_quad_strip(uint64_t* __restrict__ S, const uint64_t* __restrict__ rows,
                                                 int pitch, int x_first, int ny, int sw, int W,
                                                 bool live, int g) {
  constexpr int SWP = Quad<CPL>::SWP, CH = Quad<CPL>::CH;
  uint64_t w[4][CH];
#pragma unroll
  for (int jj = 0; jj < 4; ++jj)
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int m = 16 * c + g, x = x_first + m;
      const bool ok = live && jj < ny && m < sw && x >= 0 && x < W;
      w[jj][c] = rows[ok ? (size_t)jj * pitch + x : 0];
      w[jj][c] = ok ? w[jj][c] : 0ull;
    }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj)
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (16 * c + g < SWP) S[jj * SWP + 16 * c + g] = w[jj][c];
}

// acc[c] = cost of strip position g CPL + c over the block's points; keep: the block's
// point mask in the 4-column layout (bit j * 4 + i); `full`: every point of four 4 x 4
// blocks is kept (wave-uniform).
template <int CPL>
__device__ __forceinline__ void quad_costs(const uint64_t* __restrict__ T, const uint64_t* __restrict__ S,
                                           int g, bool full, uint32_t keep, uint32_t (&acc)[CPL]) {
  constexpr int SWP = Quad<CPL>::SWP;
#pragma unroll
  for (int c = 0; c < CPL; ++c) acc[c] = 0;
  const uint64_t* __restrict__ srow = S + g * CPL;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint64_t t[4], w[CPL + 3];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = T[4 * r + i];
#pragma unroll
    for (int m = 0; m < CPL + 3; ++m) w[m] = srow[r * SWP + m];
    if (full) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc(t[i] ^ w[i + c], acc[c]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t k = ((keep >> (4 * r + i)) & 1u) ? ~0ull : 0ull;
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = popc64_acc((t[i] ^ w[i + c]) & k, acc[c]);
      }
    }
  }
}

// Blocks first .. first + 3 (those below nblk) of one box, one per row of 16 lanes.
template <int CPL>
__device__ __forceinline__ void match_blocks_quad(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg, int f,
                                                  int level, const ItemRec& r, int first, int lane,
                                                  void* lds) {
  using QQ = Quad<CPL>;
  constexpr int SWP = QQ::SWP, NC = QQ::NC;
  const int q = lane >> 4, g = lane & 15;
  const int local = first + q;
  const bool live = local < r.nblk;
  uint64_t* S = (uint64_t*)lds + q * QQ::BLK;
  uint64_t* T = S + 4 * SWP;
  uint32_t* costf = (uint32_t*)((uint64_t*)lds + 4 * QQ::BLK) + q * NC;
  uint32_t* costb = costf + 4 * NC;
  const LevelDev& lv = fr.lv[level];
  const PathDev& ph = P.path[level];
  const int nd = ph.nd, dlo = ph.dlo, dhi = dlo + nd - 1;
  const int nx = r.bw, ny = r.bh, W = lv.W, s = lv.scale;
  const int vv = live ? local / r.nbx : 0;
  const int uu = live ? local - vv * r.nbx : 0;
  const int X0 = r.ox + uu * nx, Y0 = r.oy + vv * ny;
  const uint64_t* __restrict__ Lb = lv.L + (size_t)Y0 * lv.pitch;
  const uint64_t* __restrict__ Rb = lv.R + (size_t)Y0 * lv.pitch;
  const int sw = nd + nx - 1;
  // forward strip CR(X0 - dhi + m, Y0 + j) and template CL(X0 + i, Y0 + j) of this
  // lane's block, issued before the occluder scan
  stage_quad_strip<CPL>(S, Rb, lv.pitch, X0 - dhi, ny, sw, W, live, g);
  const int pi = g & 3, pj = g >> 2;
  const bool exists = live && pi < nx && pj < ny;
  {
    uint64_t t = Lb[exists ? (size_t)pj * lv.pitch + X0 + pi : 0];
    T[g] = exists ? t : 0ull;
  }
  // occlusion (Sec. 4.3.5): every block of the wave belongs to box k, so the boxes that
  // occlude it are found once; each lane tests its own point against them
  const BoxClip ck = ws.clip[fr.box_off + r.k];
  const int fx = s * (X0 + pi), fy = s * (Y0 + pj);
  bool hidden = false;
  for (int jb = 0; jb < fr.n_boxes; jb += 64) {
    const int o = jb + lane;
    const BoxClip co = o < fr.n_boxes ? ws.clip[fr.box_off + o] : BoxClip{0, 0, 0, 0};
    const bool occ = o < fr.n_boxes && o != r.k && ck.cx0 < co.cx1 && co.cx0 < ck.cx1 &&
                     ck.cy0 < co.cy1 && co.cy0 < ck.cy1 && co.cy1 > ck.cy1;
    uint64_t m = __ballot(occ);
    while (m) {
      const int src = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int x0 = __builtin_amdgcn_readlane(co.cx0, src), x1 = __builtin_amdgcn_readlane(co.cx1, src);
      const int y0 = __builtin_amdgcn_readlane(co.cy0, src), y1 = __builtin_amdgcn_readlane(co.cy1, src);
      hidden |= fx >= x0 && fx < x1 && fy >= y0 && fy < y1;
    }
  }
  const uint64_t m64 = __ballot(exists && !hidden);
  const uint32_t keep = (uint32_t)(m64 >> (16 * q)) & 0xFFFFu;
  const int npts = __popc(keep);
  const bool eligible = live && npts > 0 && 100 * npts >= P.min_point_pct * nx * ny;
  const bool full = m64 == ~0ull;
  const bool writer = live && g == 0;
  wave_sync();
  uint32_t acc[CPL];
  quad_costs<CPL>(T, S, g, full, keep, acc);
  uint32_t key = 0xFFFFFFFFu;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int e = g * CPL + cc;            // strip position: candidate d = dhi - e
    if (e < nd) {
      const int kc = nd - 1 - e;
      key = min(key, (acc[cc] << 16) | (uint32_t)kc);
      costf[kc] = acc[cc];
    }
  }
  key = row16_min_dpp(key);
  const int best = (int)(key & 0xFFFFu);
  const int d_f = dlo + best;
  // backward template CR(X0 - d_f + i, Y0 + j): strip position dhi - d_f + i
  const uint64_t tb = S[pj * SWP + (dhi - d_f) + pi];
  wave_sync();
  T[g] = exists ? tb : 0ull;
  const int ca = (int)costf[max(best - 1, 0)];
  const int cb = (int)costf[min(best + 1, nd - 1)];
  const float d_sub = subpixel(d_f, best, nd, ca, (int)(key >> 16), cb);
  wave_sync();
  stage_quad_strip<CPL>(S, Lb, lv.pitch, X0 - d_f + dlo, ny, sw, W, live, g);
  wave_sync();
  quad_costs<CPL>(T, S, g, full, keep, acc);
  uint32_t bkey = 0xFFFFFFFFu;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int kc = g * CPL + cc;           // candidate d' = dlo + kc
    if (kc < nd) {
      bkey = min(bkey, (acc[cc] << 16) | (uint32_t)kc);
      costb[kc] = acc[cc];
    }
  }
  bkey = row16_min_dpp(bkey);
  const int d_b = dlo + (int)(bkey & 0xFFFFu);
  const int lr_ok = abs(d_b - d_f) <= P.lr_tol;
  const int slot = f * P.cap_blocks + r.off + local;
  if (writer) {
    ws.blk_val[slot] = (float)s * (eligible ? d_sub : (float)dlo);   // d_full = s * d (Sec. 4.1)
    ws.blk_flag[slot] = (uint8_t)((eligible ? 1 : 0) | (eligible && lr_ok ? 2 : 0));
  }
  if (dbg.blocks || dbg.cost_fwd || dbg.cost_bwd) {
    // record mask in the record's layout (bit j * nx + i) from the 4-column layout
    const int jr = g / nx, ir = g - jr * nx;
    const uint64_t pm = __ballot(live && g < nx * ny && ((keep >> (4 * jr + ir)) & 1u));
    const uint64_t mask = (pm >> (16 * q)) & 0xFFFFull;
    const int b = r.off + local;
    if (writer && dbg.blocks && b < dbg.cap_blocks) {
      ocsr_block_record rec;
      rec.box = r.k; rec.level_scale = s; rec.u = uu; rec.v = vv;
      rec.px0 = X0; rec.py0 = Y0; rec.nx = nx; rec.ny = ny;
      rec.mask = mask; rec.eligible = eligible;
      rec.d_f = eligible ? d_f : dlo; rec.d_b = eligible ? d_b : dlo;
      rec.lr_ok = eligible ? lr_ok : 0; rec.d_sub = eligible ? d_sub : (float)dlo;
      rec.valid = eligible && lr_ok;
      rec.dlo = dlo; rec.nd = nd;
      rec.dy_f = 0; rec.dy_b = 0;
      dbg.blocks[b] = rec;
    }
    if (live && eligible && b < dbg.cap_blocks && (dbg.cost_fwd || dbg.cost_bwd)) {
      wave_sync();
      for (int kc = g; kc < nd && kc < dbg.cap_nd; kc += 16) {
        if (dbg.cost_fwd) dbg.cost_fwd[(size_t)b * dbg.cap_nd + kc] = (uint16_t)costf[kc];
        if (dbg.cost_bwd) dbg.cost_bwd[(size_t)b * dbg.cap_nd + kc] = (uint16_t)costb[kc];
      }
    }
  }
  wave_sync();
}

// ---------------------------------------------------------------------------------
// Any block of up to 64 points on any point grid (TILED, or the single GRID block of
// the paper's far path, Sec. 4.3.4 "Far Objects"), up to 256 candidates: one wave per
// block, lane l takes candidates l + 64 r (r < 4) and walks the block's unmasked points
// one at a time. A point's template word is the same for every lane; its candidate
// words are consecutive in the row, one per lane. Every read of the level images goes
// through ld_word, which returns 0 outside [0, W); point rows lie inside the level box.
// ---------------------------------------------------------------------------------
constexpr size_t kGenericLdsBytes = sizeof(uint32_t) * 2 * 256;

__device__ __forceinline__ void generic_costs(const LevelDev& lv, const BlockGeom& g, uint64_t mask,
                                              int dlo, int nd, bool fwd, int d_f, int lane,
                                              uint32_t (&acc)[4]) {
  acc[0] = acc[1] = acc[2] = acc[3] = 0;
  uint64_t m = mask;
  while (m) {
    const int t = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int j = t / g.nx, i = t - j * g.nx;
    const int x = geom_col(g, i), y = geom_row(g, j);
    const uint64_t* __restrict__ rowL = lv.L + (size_t)y * lv.pitch;
    const uint64_t* __restrict__ rowR = lv.R + (size_t)y * lv.pitch;
    // forward: CL(x) against CR(x - d); backward: CR(x - d_f) against CL(x - d_f + d')
    const uint64_t tmpl = fwd ? ld_word(rowL, x, lv.W) : ld_word(rowR, x - d_f, lv.W);
    const uint64_t* __restrict__ other = fwd ? rowR : rowL;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kc = lane + 64 * r;
      const int xc = fwd ? x - (dlo + kc) : x - d_f + dlo + kc;
      if (kc < nd) acc[r] = popc64_acc(tmpl ^ ld_word(other, xc, lv.W), acc[r]);
    }
  }
}

__device__ __forceinline__ void match_block_generic(const MatchParamsDev& P, const FrameDev& fr,
                                                    const MatchWs& ws, const DebugDev& dbg,
                                                    const BlockCtx& c, int lane, void* lds) {
  uint32_t* costf = (uint32_t*)lds;
  uint32_t* costb = costf + 256;
  const LevelDev& lv = fr.lv[c.level];
  const PathDev& ph = P.path[c.level];
  const int nd = ph.nd, dlo = ph.dlo;
  const uint64_t mask = block_mask(ws, fr.box_off, fr.n_boxes, c.k, c.g, lane);
  const bool eligible = block_eligible(P, mask, c.g.nx * c.g.ny);
  if (!eligible) {
    write_block(ws, dbg, c, ph, mask, false, dlo, dlo, 0, (float)dlo, 0, lane);
    wave_sync();
    return;
  }
  uint32_t acc[4];
  generic_costs(lv, c.g, mask, dlo, nd, true, 0, lane, acc);
  uint32_t key = 0xFFFFFFFFu;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int kc = lane + 64 * r;
    if (kc < nd) {
      key = min(key, (acc[r] << 16) | (uint32_t)kc);
      costf[kc] = acc[r];
    }
  }
  key = wave_min_dpp(key);
  const int best = (int)(key & 0xFFFFu);
  const int d_f = dlo + best;
  wave_sync();
  const int ca = (int)costf[max(best - 1, 0)];
  const int cb = (int)costf[min(best + 1, nd - 1)];
  const float d_sub = subpixel(d_f, best, nd, ca, (int)(key >> 16), cb);
  generic_costs(lv, c.g, mask, dlo, nd, false, d_f, lane, acc);
  uint32_t bkey = 0xFFFFFFFFu;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int kc = lane + 64 * r;
    if (kc < nd) {
      bkey = min(bkey, (acc[r] << 16) | (uint32_t)kc);
      costb[kc] = acc[r];
    }
  }
  bkey = wave_min_dpp(bkey);
  const int d_b = dlo + (int)(bkey & 0xFFFFu);
  const int lr_ok = abs(d_b - d_f) <= P.lr_tol;
  if (c.b < dbg.cap_blocks && (dbg.cost_fwd || dbg.cost_bwd)) {
    wave_sync();
    for (int kc = lane; kc < nd && kc < dbg.cap_nd; kc += 64) {
      if (dbg.cost_fwd) dbg.cost_fwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costf[kc];
      if (dbg.cost_bwd) dbg.cost_bwd[(size_t)c.b * dbg.cap_nd + kc] = (uint16_t)costb[kc];
    }
  }
  write_block(ws, dbg, c, ph, mask, true, d_f, d_b, lr_ok, d_sub, lr_ok, lane);
  wave_sync();
}

// ---------------------------------------------------------------------------------
// TILED block with a vertical range (the census cost over (dx, dy), Sec. 4.3.2). The
// register-blocked row costs of match_block_tiled, repeated for every vertical offset.
// Consecutive offsets read strip rows moved by one. When all ROWS + ndy - 1 rows fit
// kDyFullLoads loads per lane (short strips) they are staged at once; otherwise the
// strip lives in an LDS ring of ROWS + 1 rows: step t reads rows t .. t + ROWS - 1 (lane row j from ring slot
// (t + j) mod (ROWS + 1)) while row t + ROWS, which step t + 1 needs, is loaded into the
// one slot step t does not read. Each row is loaded once per direction, its latency
// hidden behind the previous step. Rows and columns outside the level image read as
// zero. Every (d, e) cost is kept in LDS (uint16) for the parabola, which runs along d at
// the winning e; keys order ties by d, then e.
// LDS per wave: dy_wave_lds_bytes(ROWS, nd, ndy).
// ---------------------------------------------------------------------------------
// the CH chunks of strip row y (words x_first + 64 c + lane, zero outside the image or
// at and past sw)
template <int CH>
__device__ __forceinline__ void load_row_dy(uint64_t (&w)[CH], const uint64_t* __restrict__ img,
                                            int pitch, int W, int H, int x_first, int y, int sw,
                                            int lane) {
  const bool row_ok = y >= 0 && y < H;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int m = 64 * c + lane, x = x_first + m;
    const bool ok = row_ok && m < sw && x >= 0 && x < W;
    w[c] = img[ok ? (size_t)y * pitch + x : 0];
    w[c] = ok ? w[c] : 0ull;
  }
}

template <int CH>
__device__ __forceinline__ void store_row_dy(uint64_t* __restrict__ slot, const uint64_t (&w)[CH],
                                             int SWr, int lane) {
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (64 * c + lane < SWr) slot[64 * c + lane] = w[c];
}

// One direction's search over every (d, e): rows y_top + t + jj for steps t = 0 .. ndy-1,
// strip columns from x_first. Step t is vertical index e = (fwd ? t : ndy - 1 - t); strip
// position q is candidate index (fwd ? nd - 1 - q : q). Returns the lane's least key
// (cost << 16 | (d index * ndy + e)); costs go to cost[d index * ndy + e].
template <int ROWS, int NX, int CPL, int CH>
__device__ __forceinline__ uint32_t search_dy(const uint64_t (&t)[NX], uint64_t* __restrict__ S,
                                              int SWr, int passes, const uint64_t* __restrict__ img,
                                              int pitch, int W, int H, int x_first, int y_top,
                                              int ny, int sw, int nd, int ndy, bool fwd,
                                              uint32_t rowmask, uint32_t col_all, uint32_t col_any,
                                              uint16_t* __restrict__ cost, int lane) {
  constexpr int NR = ROWS + 1;
  constexpr int PC = (64 / ROWS) * CPL;
  static_assert(PC == kDyPass, "a pass covers kDyPass candidates");
  const int j = lane % ROWS, grp = lane / ROWS;
  // all ROWS + ndy - 1 rows at once when they fit (wave-uniform), else the ring
  const bool full = dy_full(ROWS, nd, ndy);
  if (full) {
    // word idx = lane + 64 k of the rows x SWr block, every load issued before a store
    const int n = (ROWS + ndy - 1) * SWr;
    uint64_t w[kDyFullLoads];
#pragma unroll
    for (int k = 0; k < kDyFullLoads; ++k) {
      const int idx = lane + 64 * k;
      const int r = idx / SWr, m = idx - r * SWr, x = x_first + m, y = y_top + r;
      const bool ok = idx < n && m < sw && x >= 0 && x < W && y >= 0 && y < H;
      w[k] = img[ok ? (size_t)y * pitch + x : 0];
      w[k] = ok ? w[k] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < kDyFullLoads; ++k)
      if (lane + 64 * k < n) S[lane + 64 * k] = w[k];
  } else {
    // rows 0 .. ROWS - 1, every load issued before the first store
    uint64_t w[ROWS][CH];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) load_row_dy<CH>(w[r], img, pitch, W, H, x_first, y_top + r, sw, lane);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) store_row_dy<CH>(S + r * SWr, w[r], SWr, lane);
  }
  wave_sync();
  uint32_t key = 0xFFFFFFFFu;
  uint32_t acc[CPL];
  for (int st = 0; st < ndy; ++st) {
    const bool more = !full && st + 1 < ndy;
    uint64_t pre[CH];
    if (more) load_row_dy<CH>(pre, img, pitch, W, H, x_first, y_top + st + ROWS, sw, lane);
    const int e = fwd ? st : ndy - 1 - st;
    const uint64_t* srow = S + (full ? st + j : (st + j) % NR) * SWr;
    for (int ps = 0; ps < passes; ++ps) {
      if (j < ny) row_costs<NX, CPL>(t, srow + ps * PC + grp * CPL, rowmask, col_all, col_any, acc);
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc)
        if (j >= ny) acc[cc] = 0;
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const uint32_t tot = row_sum<ROWS>(acc[cc]);
        const int q = ps * PC + grp * CPL + cc;
        if (q < nd) {
          const int id = (fwd ? nd - 1 - q : q) * ndy + e;
          key = min(key, (tot << 16) | (uint32_t)id);
          if (j == 0) cost[id] = (uint16_t)tot;
        }
      }
    }
    // the slot of row st - 1, which step st does not read
    if (more) {
      store_row_dy<CH>(S + ((st + ROWS) % NR) * SWr, pre, SWr, lane);
      wave_sync();
    }
  }
  wave_sync();   // every read of S and write of cost done before the caller goes on
  return key;
}

template <int ROWS, int NX>
__device__ __forceinline__ void match_block_dy(const MatchParamsDev& P, const FrameDev& fr,
                                               const MatchWs& ws, const DebugDev& dbg,
                                               const BlockCtx& c, int lane, void* lds) {
  constexpr int CPL = dy_cpl(ROWS);
  constexpr int CH = dy_chunks(ROWS);
  const LevelDev& lv = fr.lv[c.level];
  const PathDev& ph = P.path[c.level];
  const int nd = ph.nd, dlo = ph.dlo, dhi = dlo + nd - 1;
  const int ndy = ph.ndy, dylo = ph.dylo;
  const int passes = (nd + kDyPass - 1) / kDyPass;
  const int SWr = passes * kDyPass + NX - 1;   // strip row stride (words)
  const int sw = nd + NX - 1;                  // words a row's candidates read
  auto r16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
  uint64_t* S = (uint64_t*)lds;
  uint64_t* T = (uint64_t*)((char*)lds + r16(sizeof(uint64_t) * dy_lds_rows(ROWS, nd, ndy) * SWr));
  uint16_t* costf = (uint16_t*)((char*)T + r16(sizeof(uint64_t) * ROWS * NX));
  uint16_t* costb = (uint16_t*)((char*)costf + r16(sizeof(uint16_t) * (size_t)nd * ndy));
  const int j = lane % ROWS;
  const int nx = c.g.nx, ny = c.g.ny;
  const int X0 = c.g.cx, Y0 = c.g.cy;

  // forward template CL(X0 + i, Y0 + j): the block lies inside the level image
  for (int idx = lane; idx < ROWS * NX; idx += 64) {
    const int jj = idx / NX, i = idx % NX;
    T[idx] = jj < ny && i < nx ? lv.L[(size_t)(Y0 + jj) * lv.pitch + X0 + i] : 0ull;
  }
  const uint64_t mask = block_mask(ws, fr.box_off, fr.n_boxes, c.k, c.g, lane);
  const bool eligible = block_eligible(P, mask, nx * ny);
  wave_sync();
  if (!eligible) {
    write_block(ws, dbg, c, ph, mask, false, dlo, dlo, 0, (float)dlo, 0, lane);
    wave_sync();
    return;
  }
  const uint32_t rowmask = j < ny ? (uint32_t)((mask >> (j * nx)) & ((1u << nx) - 1u)) : 0u;
  uint32_t col_all = (1u << nx) - 1u, col_any = 0;
  for (int jj = 0; jj < ny; ++jj) {
    const uint32_t r = (uint32_t)((mask >> (jj * nx)) & ((1u << nx) - 1u));
    col_all &= r;
    col_any |= r;
  }
  uint64_t t[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) t[i] = T[j * NX + i];
  // forward: strip row of step e holds CR(X0 - dhi + m, Y0 + dylo + e + jj); entry q + i
  // holds CR(X0 + i - d) for d = dhi - q
  uint32_t key = search_dy<ROWS, NX, CPL, CH>(t, S, SWr, passes, lv.R, lv.pitch, lv.W, lv.H,
                                               X0 - dhi, Y0 + dylo, ny, sw, nd, ndy, true,
                                               rowmask, col_all, col_any, costf, lane);
  key = wave_min_u32(key, ROWS);
  const int best_id = (int)(key & 0xFFFFu);
  const int kf = best_id / ndy, ef = best_id - kf * ndy;
  const int d_f = dlo + kf, dy_f = dylo + ef;
  const int ca = (int)costf[max(kf - 1, 0) * ndy + ef];
  const int cb = (int)costf[min(kf + 1, nd - 1) * ndy + ef];
  const float d_sub = subpixel(d_f, kf, nd, ca, (int)(key >> 16), cb);
  // backward template CR(X0 - d_f + i, Y0 + dy_f + j), zero outside the image
  {
    const int y = Y0 + dy_f + j;
    const bool row_ok = j < ny && y >= 0 && y < lv.H;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int x = X0 - d_f + i;
      const bool ok = row_ok && i < nx && x >= 0 && x < lv.W;
      t[i] = lv.R[ok ? (size_t)y * lv.pitch + x : 0];
      t[i] = ok ? t[i] : 0ull;
    }
  }
  // backward: offset e reads CL(X0 - d_f + dlo + m, Y0 + dy_f - dylo - e + jj); the steps
  // run e from the last offset down, so that the rows move down by one per step
  uint32_t bkey = search_dy<ROWS, NX, CPL, CH>(t, S, SWr, passes, lv.L, lv.pitch, lv.W, lv.H,
                                                X0 - d_f + dlo, Y0 + dy_f - dylo - (ndy - 1), ny,
                                                sw, nd, ndy, false, rowmask, col_all, col_any,
                                                costb, lane);
  bkey = wave_min_u32(bkey, ROWS);
  const int bid = (int)(bkey & 0xFFFFu);
  const int kb = bid / ndy, eb = bid - kb * ndy;
  const int d_b = dlo + kb, dy_b = dylo + eb;
  const int lr_ok = abs(d_b - d_f) <= P.lr_tol;   // consistency on d only (Sec. 4.3.3)
  if (c.b < dbg.cap_blocks && (dbg.cost_fwd || dbg.cost_bwd)) {
    for (int q = lane; q < nd && q < dbg.cap_nd; q += 64) {
      if (dbg.cost_fwd) dbg.cost_fwd[(size_t)c.b * dbg.cap_nd + q] = costf[q * ndy + ef];
      if (dbg.cost_bwd) dbg.cost_bwd[(size_t)c.b * dbg.cap_nd + q] = costb[q * ndy + eb];
    }
  }
  write_block(ws, dbg, c, ph, mask, true, d_f, d_b, lr_ok, d_sub, lr_ok, lane, dy_f, dy_b);
  wave_sync();
}

// Work item of frame f at `level` from its record: wave w of the workgroup runs blocks
// r.first + w + 4 j of the box that exist.
__device__ __forceinline__ BoxPlan item_plan(const ItemRec& r, int f, int level) {
  BoxPlan pl = {};
  pl.status = -1;
  pl.level = level;
  pl.lx0 = r.lx0; pl.ly0 = r.ly0; pl.lw = r.lw; pl.lh = r.lh;
  pl.nbx = r.nbx; pl.bw = r.bw; pl.bh = r.bh; pl.ox = r.ox; pl.oy = r.oy;
  pl.off = r.off; pl.nblk = r.nblk; pl.frame = f;
  return pl;
}
template <class RunBlock>
__device__ __forceinline__ void run_item_rec(const MatchParamsDev& P, const FrameDev& fr, int f,
                                             int level, const ItemRec& r, int wave, RunBlock run) {
  const BoxPlan pl = item_plan(r, f, level);
  // the wave's blocks step by kItemWaves along the grid's rows: one division per item
  int local = r.first + wave;
  int v = local / pl.nbx, u = local - v * pl.nbx;
  for (int j = wave; j < P.item_blocks[level]; j += kItemWaves) {
    if (local < r.nblk) run(block_ctx(P, fr, f, r.k, pl, local, u, v, level));
    local += kItemWaves;
    u += kItemWaves;
    while (u >= pl.nbx) {
      u -= pl.nbx;
      ++v;
    }
  }
}

// Loop of a workgroup over the work items of one level of every frame (frames in
// order, each frame's items in box order), dealt XCD by XCD (xcd_deal). Item numbers
// come from the workgroup index, so the loop is uniform across the workgroup and needs
// no shared counter. body(f, q, at) gets the frame, the item number within the frame's
// level and the item's record within the frame's records (close items first, then far).
template <class Body>
__device__ __forceinline__ void level_items(const FramesDev& FR, const MatchWs& ws, int level,
                                            Body body) {
  const int lane = threadIdx.x & 63;
  const int n_close = lane < FR.n ? ws.fcount[lane * FC_N + FC_CLOSE_ITEMS] : 0;
  const int n_far = lane < FR.n ? ws.fcount[lane * FC_N + FC_FAR_ITEMS] : 0;
  const int cnt = level == 0 ? n_far : n_close;
  const int incl = wave_incl_scan(cnt, lane);
  const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
  const Deal dl = xcd_deal(total);
  for (int q = dl.first; q < dl.end; q += dl.step) {
    const uint64_t m = __ballot(lane < FR.n && incl > q);
    const int f = __ffsll((unsigned long long)m) - 1;
    const int excl = __builtin_amdgcn_readfirstlane(__shfl(incl - cnt, f, 64));
    const int skip = level == 0 ? __builtin_amdgcn_readlane(n_close, f) : 0;
    body(f, q - excl, q - excl + skip);
  }
}

// ---------------------------------------------------------------------------------
// aggregation: one workgroup (256 threads) per box
// ---------------------------------------------------------------------------------
struct AggLds {
  float vals[kAggMax];    // the box's valid values (boxes of at most kAggMax blocks)
  int32_t hist[1024];     // value histogram of the trimmed median; per-wave digit counts
                          // of the global radix sort ([kItemWaves][256])
  float list[2][64];      // values of the bins holding the two middle ranks
  int32_t scratch[272];   // radix bins [0, 256), then scalars
  int32_t n_valid, n_eligible, seg_start, seg_len;
  uint32_t vmin, vmax;    // bit patterns of the smallest and largest valid value
  int32_t bin[2], rank[2], count[2];
  uint32_t pick[2];
};

__device__ __forceinline__ float median_sorted(const float* v, int m) {
  if (m & 1) return v[(m - 1) / 2];
  return (v[m / 2 - 1] + v[m / 2]) * 0.5f;
}

// k-th smallest (0-based) of the n non-negative floats in vals (LDS or global memory):
// radix select on their bit patterns (monotone for non-negative floats), 8 bits per pass
__device__ __forceinline__ uint32_t radix_select(const float* vals, int n, int k, int32_t* sc) {
  const int tid = threadIdx.x;
  uint32_t prefix = 0, pmask = 0;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    sc[tid] = 0;   // 256 bins
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      const uint32_t u = __float_as_uint(vals[i]);
      if ((u & pmask) == prefix) atomicAdd(&sc[(u >> shift) & 255u], 1);
    }
    __syncthreads();
    if (tid < 64) {
      const int c0 = sc[4 * tid], c1 = sc[4 * tid + 1], c2 = sc[4 * tid + 2], c3 = sc[4 * tid + 3];
      const int sum = c0 + c1 + c2 + c3;
      const int incl = wave_incl_scan(sum, tid);
      const int excl = incl - sum;
      if (k >= excl && k < incl) {   // exactly one lane
        int d = 4 * tid, kk = k - excl;
        if (kk >= c0) { kk -= c0; ++d;
          if (kk >= c1) { kk -= c1; ++d;
            if (kk >= c2) { kk -= c2; ++d; } } }
        sc[256] = d;
        sc[257] = kk;
      }
    }
    __syncthreads();
    prefix |= (uint32_t)sc[256] << shift;
    pmask |= 255u << shift;
    k = sc[257];
    __syncthreads();
  }
  return prefix;
}

// Ascending sort of the n non-negative floats at a (global memory) by their bit
// patterns: four stable counting passes of 8 bits, least significant first, between a
// and tmp (n floats); the sorted values end in a. One workgroup of 256 threads. A pass
// counts the digits, scans them to the start of each digit's range, then scatters 256
// values at a time in index order: a value's place is its digit's start, plus the
// values of that digit in earlier waves of the round, plus those of lower lanes of its
// own wave (found with eight ballots, one per digit bit). cnt: kItemWaves x 256 ints,
// base: 256 ints of LDS.
__device__ __forceinline__ void radix_sort_global(float* a, float* tmp, int n, int32_t* cnt,
                                                  int32_t* base) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    const float* src = (pass & 1) ? tmp : a;
    float* dst = (pass & 1) ? a : tmp;
    base[tid] = 0;
    for (int w = 0; w < kItemWaves; ++w) cnt[w * 256 + tid] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += 256) atomicAdd(&base[(__float_as_uint(src[i]) >> shift) & 255u], 1);
    __syncthreads();
    // exclusive scan of the 256 digit counts (thread t holds digit t)
    {
      const int c = base[tid];
      const int incl = wave_incl_scan(c, lane);
      __syncthreads();
      if (lane == 63) cnt[wave] = incl;   // wave totals (cnt is all zero otherwise)
      __syncthreads();
      int excl = incl - c;
      for (int w = 0; w < wave; ++w) excl += cnt[w];
      __syncthreads();
      base[tid] = excl;
      if (tid < kItemWaves) cnt[tid] = 0;
      __syncthreads();
    }
    for (int c0 = 0; c0 < n; c0 += 256) {
      const int i = c0 + tid;
      const bool ok = i < n;
      const float v = ok ? src[i] : 0.0f;
      const uint32_t dg = (__float_as_uint(v) >> shift) & 255u;
      uint64_t same = __ballot(ok);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((dg >> b) & 1u);
        same &= ((dg >> b) & 1u) ? m : ~m;
      }
      const int before = (int)__popcll(same & below);
      if (ok && before == 0) cnt[wave * 256 + dg] = (int)__popcll(same);
      __syncthreads();
      if (ok) {
        int pos = base[dg] + before;
        for (int w = 0; w < wave; ++w) pos += cnt[w * 256 + dg];
        dst[pos] = v;
      }
      __syncthreads();
      int add = 0;
      for (int w = 0; w < kItemWaves; ++w) {
        add += cnt[w * 256 + tid];
        cnt[w * 256 + tid] = 0;
      }
      base[tid] += add;
      __syncthreads();
    }
  }
  // the last pass wrote into a; make its stores visible to the whole workgroup
  __threadfence_block();
  __syncthreads();
}

// Bin of v among 1024 equal-width bins over [vmin, vmin + 1024 / scale]: a monotone map,
// so every value of a lower bin is smaller than every value of a higher one.
__device__ __forceinline__ int value_bin(float v, float vmin, float scale) {
  return min((int)((v - vmin) * scale), 1023);
}

// Over the counts in sm.hist (1024 bins), the bins of ranks r1 and r2 (0-based; r2 only
// when want2) and the ranks within them, into sm.bin and sm.rank. All 256 threads; ends
// with a barrier.
__device__ __forceinline__ void find_rank_bins(AggLds& sm, int r1, int r2, bool want2) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // thread t owns bins 4t .. 4t + 3
  const int c0 = sm.hist[4 * tid], c1 = sm.hist[4 * tid + 1], c2 = sm.hist[4 * tid + 2],
            c3 = sm.hist[4 * tid + 3];
  const int sum = c0 + c1 + c2 + c3;
  const int incl = wave_incl_scan(sum, lane);
  if (lane == 63) sm.scratch[256 + wave] = incl;
  __syncthreads();
  int excl = incl - sum;
  for (int v = 0; v < wave; ++v) excl += sm.scratch[256 + v];
  for (int j = 0; j < (want2 ? 2 : 1); ++j) {
    const int kj = j ? r2 : r1;
    if (kj >= excl && kj < excl + sum) {   // exactly one thread
      int b = 4 * tid, kk = kj - excl;
      if (kk >= c0) { kk -= c0; ++b;
        if (kk >= c1) { kk -= c1; ++b;
          if (kk >= c2) { kk -= c2; ++b; } } }
      sm.bin[j] = b;
      sm.rank[j] = kk;
    }
  }
  __syncthreads();
}

// The values whose key (key(v) < 1024, or -1 for none) is kb1 or kb2 gathered into the
// two lists (list 1 only when the keys differ), and the values of ranks sm.rank[0] and
// sm.rank[1] within their key picked by one wave into sm.pick. Every key count is at most
// 64. All 256 threads; ends with a barrier.
template <typename Key>
__device__ __forceinline__ void pick_in_lists(AggLds& sm, const float* vals, int n, Key key,
                                              int kb1, int kb2, bool want2) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += 256) {
    const float v = vals[i];
    const int b = key(v);
    if (b == kb1) sm.list[0][atomicAdd(&sm.count[0], 1)] = v;
    else if (b == kb2) sm.list[1][atomicAdd(&sm.count[1], 1)] = v;
  }
  __syncthreads();
  if (wave == 0) {
    for (int j = 0; j < (want2 ? 2 : 1); ++j) {
      const int li = (j == 1 && kb2 != kb1) ? 1 : 0;
      const int c = sm.count[li];
      const float* lst = sm.list[li];
      const float x = lane < c ? lst[lane] : 0.0f;
      int less = 0, eq = 0;
      for (int i = 0; i < c; ++i) {
        const float y = lst[i];
        less += y < x;
        eq += y == x;
      }
      // lanes holding equal values agree, so any of them may store
      if (lane < c && sm.rank[j] >= less && sm.rank[j] < less + eq) sm.pick[j] = __float_as_uint(x);
    }
  }
  __syncthreads();
}

// The k-th and (k + 1)-th smallest (0-based) of the n non-negative floats in vals (LDS
// or global memory; the second only when want2), as bit patterns. The values are binned
// by value (value_bin); a scan of the bin counts finds the bins of the two ranks and
// their ranks within them; one wave then ranks the few values of each such bin against
// each other. When a bin holds more than 64 values (a box's values crowd a few bins when
// a few outliers stretch the range), the values of the one or two bins are binned again
// over each bin's own span, 512 sub-bins each, and the same steps run on the sub-bins.
// A radix selection over all values handles a sub-bin of more than 64 values or a range
// too narrow to scale. vmin, vmax: the smallest and largest value. Every step is a
// monotone map of the value, so the order statistics are exact.
__device__ __forceinline__ void select_middle(AggLds& sm, const float* vals, int n, int k,
                                              bool want2, float vmin, float vmax, uint32_t* u1,
                                              uint32_t* u2) {
  const int tid = threadIdx.x;
  if (vmin == vmax) {
    *u1 = *u2 = __float_as_uint(vmin);
    return;
  }
  const float scale = 1024.0f / (vmax - vmin);
  if (scale < 1e30f) {
    for (int i = tid; i < n; i += 256) atomicAdd(&sm.hist[value_bin(vals[i], vmin, scale)], 1);
    if (tid == 0) { sm.count[0] = 0; sm.count[1] = 0; }
    __syncthreads();
    find_rank_bins(sm, k, k + 1, want2);
    const int b1 = sm.bin[0], b2 = want2 ? sm.bin[1] : b1;
    const int n1 = sm.hist[b1], n2 = sm.hist[b2];
    if (n1 <= 64 && n2 <= 64) {
      pick_in_lists(sm, vals, n, [&](float v) { return value_bin(v, vmin, scale); }, b1, b2, want2);
      *u1 = sm.pick[0];
      *u2 = want2 ? sm.pick[1] : sm.pick[0];
      return;
    }
    // second level: bin b1's values into sub-bins 0..511 and, when the second rank lies
    // in a later bin b2, bin b2's into 512..1023; ranks counted over the two bins together
    const int r1 = sm.rank[0], r2 = want2 ? (b2 == b1 ? sm.rank[1] : n1 + sm.rank[1]) : r1;
    auto sub = [&](float v) {
      const int b = value_bin(v, vmin, scale);
      if (b != b1 && b != b2) return -1;
      const int q = min(max((int)(((v - vmin) * scale - (float)b) * 512.0f), 0), 511);
      return b == b1 ? q : 512 + q;
    };
    __syncthreads();   // every thread has read the first level's counts
    for (int i = tid; i < 1024; i += 256) sm.hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      const int q = sub(vals[i]);
      if (q >= 0) atomicAdd(&sm.hist[q], 1);
    }
    __syncthreads();
    find_rank_bins(sm, r1, r2, want2);
    const int s1 = sm.bin[0], s2 = want2 ? sm.bin[1] : s1;
    if (sm.hist[s1] <= 64 && sm.hist[s2] <= 64) {
      pick_in_lists(sm, vals, n, sub, s1, s2, want2);
      *u1 = sm.pick[0];
      *u2 = want2 ? sm.pick[1] : sm.pick[0];
      return;
    }
    __syncthreads();   // every thread has read the second level's counts
  }
  *u1 = radix_select(vals, n, k, sm.scratch);
  *u2 = want2 ? radix_select(vals, n, k + 1, sm.scratch) : *u1;
}

__device__ __forceinline__ void aggregate_box(const MatchParamsDev& P, const MatchWs& ws, int kg,
                                              ocsr_box_result* out, bool timed_out, AggLds& sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const BoxPlan pl = ws.plan[kg];
  ocsr_box_result r = {};
  if (pl.status != -1 || timed_out) {
    if (tid == 0) {
      r.reason = timed_out ? OCSR_REASON_INTERNAL_TIMEOUT : pl.status;
      out[kg] = r;
    }
    return;
  }
  const int base = pl.frame * P.cap_blocks + pl.off;
  // a box of at most kAggMax blocks gathers its valid values into LDS; a larger one
  // compacts them in place at the front of its own block values in global memory (a
  // value moves to an index no larger than its own, and every chunk is loaded before
  // any of it is stored)
  const bool in_lds = pl.nblk <= kAggMax;
  // the rest runs with vals in LDS or in global memory, each instance with its pointer's
  // memory space known to the compiler (LDS reads rather than generic ones, whose
  // latency is that of a memory access)
  auto rest = [&](float* vals) {
    if (tid == 0) {
      sm.n_valid = 0;
      sm.n_eligible = 0;
      sm.vmin = 0x7FFFFFFFu;
      sm.vmax = 0;
    }
    for (int i = tid; i < 1024; i += 256) sm.hist[i] = 0;
    __syncthreads();
    uint32_t vlo = 0x7FFFFFFFu, vhi = 0;   // bit patterns of non-negative floats
    // gather the valid values: one LDS atomic per wave, positions from the ballot. Flags
    // and values of up to kGather blocks per thread are loaded before any is used.
    constexpr int kGather = 4;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int b0 = 0; b0 < pl.nblk; b0 += 256 * kGather) {
      uint32_t fl[kGather];
      float v[kGather];
  #pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int i = b0 + 256 * u + tid;
        const int at = base + (i < pl.nblk ? i : 0);
        fl[u] = ws.blk_flag[at];
        v[u] = ws.blk_val[at];
        fl[u] = i < pl.nblk ? fl[u] : 0u;
      }
      if (!in_lds) __syncthreads();   // the chunk is loaded before it is overwritten
  #pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const uint64_t mv = __ballot((fl[u] & 2) != 0);
        const uint64_t me = __ballot((fl[u] & 1) != 0);
        int wbase = 0;
        if (lane == 0 && (mv | me)) {
          wbase = atomicAdd(&sm.n_valid, (int)__popcll(mv));
          atomicAdd(&sm.n_eligible, (int)__popcll(me));
        }
        wbase = __shfl(wbase, 0, 64);
        if (fl[u] & 2) {
          vals[wbase + __popcll(mv & below)] = v[u];
          vlo = min(vlo, __float_as_uint(v[u]));
          vhi = max(vhi, __float_as_uint(v[u]));
        }
      }
      if (!in_lds) __syncthreads();
    }
    vlo = wave_min_u32(vlo);
    vhi = (uint32_t)wave_max((int)vhi);
    if (lane == 0) {
      atomicMin(&sm.vmin, vlo);
      atomicMax(&sm.vmax, vhi);
    }
    if (!in_lds) __threadfence_block();   // compacted values visible to the workgroup
    __syncthreads();
    const int nv = sm.n_valid, ne = sm.n_eligible;
    r.n_blocks = pl.nblk;
    r.n_eligible = ne;
    r.n_valid = nv;
    if (ne == 0 || nv == 0) {
      if (tid == 0) {
        r.reason = ne == 0 ? OCSR_REASON_NO_ELIGIBLE_BLOCKS : OCSR_REASON_NO_VALID_BLOCKS;
        out[kg] = r;
      }
      return;
    }
    float d_box = 0.0f;
    bool ok = true;
    if (pl.level == 0 && pl.nblk == 1) {
      // Alg. 2: a FAR object matched as one block takes that block's result; CLOSE
      // objects always go through the robust aggregation
      d_box = vals[0];
      r.n_used = 1;
    } else if (P.agg_mode == OCSR_AGG_TRIMMED_MEDIAN) {
      // symmetric trim of floor(pct * n / 100) values at each end, then the median: the
      // one or two middle order statistics, found by selection
      const int t = P.trim_pct * nv / 100;
      const int m = nv - 2 * t;
      r.n_used = m > 0 ? m : 0;
      if (m <= 0 || m < P.n_min) {
        ok = false;
      } else {
        const int k1 = t + (m - 1) / 2;
        uint32_t u1, u2;
        select_middle(sm, vals, nv, k1, (m & 1) == 0, __uint_as_float(sm.vmin),
                      __uint_as_float(sm.vmax), &u1, &u2);
        d_box = (m & 1) ? __uint_as_float(u1) : (__uint_as_float(u1) + __uint_as_float(u2)) * 0.5f;
      }
    } else {
      if (in_lds) {
        // bitonic sort of the valid values, padded with +inf to a power of two
        int n2 = 1;
        while (n2 < nv) n2 <<= 1;
        for (int i = nv + tid; i < n2; i += 256) sm.vals[i] = __builtin_inff();
        __syncthreads();
        for (int kk = 2; kk <= n2; kk <<= 1) {
          for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < n2; i += 256) {
              const int ixj = i ^ j;
              if (ixj > i) {
                const float a = sm.vals[i], c = sm.vals[ixj];
                const bool up = (i & kk) == 0;
                if ((a > c) == up) { sm.vals[i] = c; sm.vals[ixj] = a; }
              }
            }
            __syncthreads();
          }
        }
      } else {
        // the values in global memory, ordered by a radix sort through the box's slots of
        // the sort buffer
        radix_sort_global(vals, ws.agg_tmp + base, nv, sm.hist, sm.scratch);
      }
      // longest run whose consecutive gaps stay below tau_d; the first run wins a tie
      if (tid < 64) {
        int best_start = 0, best_len = 1, start = 0;
        for (int b0 = 0; b0 < nv; b0 += 64) {
          const int q = b0 + tid;
          const bool brk = q > 0 && q < nv && !(vals[q] - vals[q - 1] < P.tau_d);
          uint64_t m = __ballot(brk);
          while (m) {
            const int pos = b0 + __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int len = pos - start;
            if (len > best_len) { best_len = len; best_start = start; }
            start = pos;
          }
        }
        const int len = nv - start;
        if (len > best_len) { best_len = len; best_start = start; }
        if (tid == 0) { sm.seg_start = best_start; sm.seg_len = best_len; }
      }
      __syncthreads();
      const int seg_start = sm.seg_start, seg_len = sm.seg_len;
      r.n_used = seg_len;
      if (seg_len < P.n_min) ok = false;
      else d_box = median_sorted(vals + seg_start, seg_len);
    }
    if (tid == 0) {
      if (!ok) {
        r.reason = OCSR_REASON_TOO_FEW_CONSISTENT;
      } else {
        r.disparity = d_box;
        if (!(d_box > P.d_eps)) {
          r.reason = OCSR_REASON_NONPOSITIVE_DISPARITY;
        } else {
          r.depth = P.fb / d_box;   // Eq. 1, IEEE fp32 division
          r.valid = 1;
          r.reason = OCSR_REASON_OK;
        }
      }
      out[kg] = r;
    }
  };
  if (in_lds) rest(sm.vals);
  else rest(ws.blk_val + base);
}

// ---------------------------------------------------------------------------------
// Matchers of one level's TILED blocks, for the generic pair kernel: the register-blocked
// kernel (ROWS block rows per wave, CPL candidates per lane, PASSES passes) and the
// row-half kernel (32 CPL candidates per wave).
// run_item: wave `wave`'s share of work item r (frame f, level `level`).
// frame_state: what a matcher reads per frame before an item's record arrives (issued
// first, so that its loads and the record's are in flight together).
struct NoFrameState {};
template <int ROWS, int NX, int CPL, int PASSES>
struct TiledMatcher {
  static constexpr size_t kLds = (Tiled<ROWS, NX, CPL, PASSES>::kLdsBytes + 15) & ~(size_t)15;
  using State = NoFrameState;
  static __device__ __forceinline__ State frame_state(const MatchWs&, const FrameDev&, int) { return {}; }
  static __device__ __forceinline__ void run_item(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg, int f,
                                                  int level, const ItemRec& r, int wave, int lane,
                                                  void* lds, const State& = State()) {
    run_item_rec(P, fr, f, level, r, wave, [&](const BlockCtx& c) {
      match_block_tiled<ROWS, NX, CPL, PASSES>(P, fr, ws, dbg, c, lane, lds);
    });
  }
};
// (its frame state: the frame's box rectangles in lanes, when they fit)
template <int CPL>
struct HalfMatcher {
  static constexpr size_t kLds = (Half<CPL>::kLdsBytes + 15) & ~(size_t)15;
  using State = OccLanes;
  static __device__ __forceinline__ State frame_state(const MatchWs& ws, const FrameDev& fr, int lane) {
    return frame_lanes(ws, fr.box_off, fr.n_boxes, lane);
  }
  static __device__ __forceinline__ void run_item(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg, int f,
                                                  int level, const ItemRec& r, int wave, int lane,
                                                  void* lds, const State& st) {
    OccLanes oc = st;
    box_candidates(oc, fr.n_boxes, r.k, lane);
    run_item_rec(P, fr, f, level, r, wave, [&](const BlockCtx& c) {
      match_block_half<CPL>(P, fr, ws, dbg, c, oc, lane, lds);
    });
  }
};
// any block of up to 64 points (GRID blocks included), lanes over candidates
struct GenericMatcher {
  static constexpr size_t kLds = kGenericLdsBytes;
  using State = NoFrameState;
  static __device__ __forceinline__ State frame_state(const MatchWs&, const FrameDev&, int) { return {}; }
  static __device__ __forceinline__ void run_item(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg, int f,
                                                  int level, const ItemRec& r, int wave, int lane,
                                                  void* lds, const State& = State()) {
    run_item_rec(P, fr, f, level, r, wave, [&](const BlockCtx& c) {
      match_block_generic(P, fr, ws, dbg, c, lane, lds);
    });
  }
};
// four blocks per wave: wave w takes blocks r.first + 4 w .. + 3 of a 16-block item
template <int CPL>
struct QuadMatcher {
  static constexpr size_t kLds = (Quad<CPL>::kLdsBytes + 15) & ~(size_t)15;
  using State = NoFrameState;
  static __device__ __forceinline__ State frame_state(const MatchWs&, const FrameDev&, int) { return {}; }
  static __device__ __forceinline__ void run_item(const MatchParamsDev& P, const FrameDev& fr,
                                                  const MatchWs& ws, const DebugDev& dbg, int f,
                                                  int level, const ItemRec& r, int wave, int lane,
                                                  void* lds, const State& = State()) {
    const int first = r.first + 4 * wave;
    if (first < r.nblk && first < r.first + P.item_blocks[level])
      match_blocks_quad<CPL>(P, fr, ws, dbg, f, level, r, first, lane, lds);
  }
};

// ---------------------------------------------------------------------------------
// work items
// ---------------------------------------------------------------------------------
// Work item q of the frame's level: wave w of the workgroup runs blocks
// item_blocks * (q - first item of the box) + w + 4 j of the item's box that exist.
template <class RunBlock>
__device__ __forceinline__ void run_item(const MatchParamsDev& P, const FrameDev& fr, int f,
                                         int n_total, const MatchWs& ws, int level, int q,
                                         int wave, int lane, RunBlock run) {
  const int k = find_box(ws.litem_end + (size_t)level * n_total + fr.box_off, fr.n_boxes, q, lane);
  const BoxPlan pl = ws.plan[fr.box_off + k];
  const int first = P.item_blocks[level] * (q - pl.ioff);
  for (int j = wave; j < P.item_blocks[level]; j += kItemWaves) {
    const int local = first + j;
    if (local < pl.nblk) run(block_ctx(P, fr, f, k, pl, local, level));
  }
}

}  // namespace dev
}  // namespace ocsr
