// Census transform of one 64 x 32 tile of level pixels by one workgroup of 256
// threads (Sec. 4.3.1: census equation and Alg. 1).
//
// The tile plus its halo is staged in LDS as vertical pixel pairs (two 8-bit samples
// in the two 16-bit halves of a word). Each lane owns one column and eight rows (four
// pairs) and keeps the pair words of its window in registers. One packed 16-bit
// subtract (centre pair - neighbour pair) decides a comparison for both pixels of a
// pair: a half is >= 0xFF01 exactly when the neighbour is brighter, so its bits 8..15
// all carry the comparison bit and one AND-OR drops both bits into place in a
// byte-per-code-byte accumulator. Byte permutes then assemble the two 64-bit codes:
// about one VALU instruction per comparison bit, with no lane-mask traffic.
//
// Bit order: Alg. 1 starts from the sentinel and, for i = -SX..SX (x, outer) and
// j = -SY..SY (y, inner), shifts left and appends [I(x+i, y+j) > I(x, y)]; the first
// comparison therefore ends at bit n-1 (n = (2SX+1)(2SY+1)) and the sentinel at bit n.
// Pixels whose window leaves the level image store 0.
#pragma once

#include "dev_common.hpp"

namespace ocsr {
namespace dev {

constexpr int kCensusRowsPerLane = 8;   // 4 waves x 8 rows = kCensusTileY

template <int SX, int SY>
struct CensusTile {
  static constexpr int LW = kCensusTileX + 2 * SX;
  static constexpr int PR = kCensusTileY + 2 * SY - 1;            // rows of pixel pairs
  static constexpr int WR = kCensusRowsPerLane - 1 + 2 * SY;      // pair rows per lane
  static constexpr int N = (2 * SX + 1) * (2 * SY + 1);           // comparisons
  static constexpr size_t kLdsBytes = sizeof(uint32_t) * (PR * LW + 64);   // + spare words
  static_assert(N + 1 <= 64, "window wider than a 64-bit code");
};

// One census tile: the uint8 source img (pitch bytes, W x H) at level scale s (level
// image Ws x Hs = W/s x H/s), the level position (X0, Y0) of the tile, and the
// descriptor image out (out_pitch words).
struct CensusJob {
  const uint8_t* img;
  int W, H, pitch, s, Ws, Hs;
  uint64_t* out;
  int out_pitch, X0, Y0;
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// P[r * LW + c] = I(c, r) | I(c, r + 1) << 16 over the tile and its halo (level
// samples, c and r counted from the halo's corner). A position outside the level image
// reads some valid byte of the image instead: only pixels whose window leaves the image
// see such values, and their words are stored as 0 regardless.
__device__ __forceinline__ int clamp_to(int v, int n) { return v < 0 ? 0 : (v < n ? v : n - 1); }

// Stages tile j in P through registers. For the first 64 columns wave w loads source rows
// w*RB .. w*RB + RB of the tile (one more than the pair rows it writes): the row address
// is wave-uniform, so each load is one scalar base plus the lane's unsigned column
// offset. The 2 SX halo columns to their right take one pair word per thread. All loads
// are issued before the first is waited for. census_load issues them into registers and
// census_put writes those to P, so that a caller can keep one tile's loads in flight
// while it works on another; census_stage does both. Called by all 256 threads of the
// workgroup.
template <int SX, int SY>
struct CensusRegs {
  using T = CensusTile<SX, SY>;
  static constexpr int RB = (T::PR + 1 + 3) / 4;
  static constexpr int NX = T::LW - 64, NH = (NX * T::PR + 255) / 256;
  static_assert(NX > 0 && NX <= 64, "one pass of 64 columns, then the halo columns");
  uint32_t px[RB + 1];
  uint32_t hlo[NH], hhi[NH];
};

template <int SX, int SY>
__device__ __forceinline__ void census_load(const CensusJob& j, CensusRegs<SX, SY>& g) {
  using G = CensusRegs<SX, SY>;
  constexpr int PR = G::T::PR, RB = G::RB, NX = G::NX, NH = G::NH;
  const uint8_t* img = uniform(j.img);
  const int pitch = uniform(j.pitch), s = uniform(j.s);
  const int X0 = uniform(j.X0), Y0 = uniform(j.Y0);
  const int Ws = uniform(j.Ws), Hs = uniform(j.Hs);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  // each row through a buffer resource over that row (scalar setup), the lane's clamped
  // column a byte offset fixed for the tile: no per-load address arithmetic
  const uint32_t coff = (uint32_t)(s * clamp_to(X0 - SX + lane, Ws));
  const int wbytes = uniform(j.W);
#pragma unroll
  for (int k = 0; k <= RB; ++k) {
    const int Yc = clamp_to(Y0 - SY + wave * RB + k, Hs);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(img + (size_t)(s * Yc) * pitch), (short)0, wbytes, 0x00020000);
    g.px[k] = __builtin_amdgcn_raw_buffer_load_b8(rs, coff, 0, 0);
  }
  // halo word t = pr NX + (pc - 64): its two source bytes through per-thread addresses
  // (threads past the halo load the last row's word again and store it to the spare
  // words)
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int t = (int)threadIdx.x + 256 * i;
    const int pr = min(t / NX, PR - 1);
    const int pc = 64 + t % NX;
    const size_t col = (size_t)(s * clamp_to(X0 - SX + pc, Ws));
    g.hlo[i] = img[(size_t)(s * clamp_to(Y0 - SY + pr, Hs)) * pitch + col];
    g.hhi[i] = img[(size_t)(s * clamp_to(Y0 - SY + pr + 1, Hs)) * pitch + col];
  }
}

template <int SX, int SY>
__device__ __forceinline__ void census_put(const CensusRegs<SX, SY>& g, uint32_t* P) {
  using G = CensusRegs<SX, SY>;
  constexpr int LW = G::T::LW, PR = G::T::PR, RB = G::RB, NX = G::NX, NH = G::NH;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int pr = wave * RB + k;   // wave-uniform: the test is a scalar branch
    if (pr < PR) P[pr * LW + lane] = g.px[k] | (g.px[k + 1] << 16);
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int t = (int)threadIdx.x + 256 * i;
    P[t < NX * PR ? (t / NX) * LW + 64 + t % NX : PR * LW + lane] = g.hlo[i] | (g.hhi[i] << 16);
  }
}

template <int SX, int SY>
__device__ __forceinline__ void census_stage(const CensusJob& j, uint32_t* P) {
  CensusRegs<SX, SY> g;
  census_load<SX, SY>(j, g);
  census_put<SX, SY>(g, P);
}

// The census words of tile j from P (staged by census_stage), after a barrier. Called
// by all 256 threads of the workgroup.
template <int SX, int SY>
__device__ __forceinline__ void census_compute(const CensusJob& j, int sentinel, const uint32_t* P) {
  using T = CensusTile<SX, SY>;
  constexpr int LW = T::LW, WR = T::WR, N = T::N;
  uint64_t* out = uniform(j.out);
  const int s = uniform(j.s), out_pitch = uniform(j.out_pitch);
  const int X0 = uniform(j.X0), Y0 = uniform(j.Y0);
  const int Ws = uniform(j.Ws), Hs = uniform(j.Hs);
  const int lane = threadIdx.x & 63;
  const int r0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kCensusRowsPerLane;
  uint64_t* orow = uniform(out + (size_t)(Y0 + r0) * out_pitch);   // the wave's first row
  // the lane's window words are read one window column at a time, so that only one
  // column (WR words) is held besides the accumulators
  const uint32_t* Pl = P + r0 * LW + lane;
  const int X = X0 + lane;
  const bool x_in = X < Ws;
  const bool x_def = X >= SX && X < Ws - SX;
  constexpr int NP = kCensusRowsPerLane / 2;
  static_assert(NP == 2 || NP == 4, "the accumulation barrier below names two or four pairs");
  // pair pp holds pixels A = (X, Y0 + r0 + 2pp) and B = (X, YA + 1) in its low / high half
  uint32_t acc[NP][8];
  u16x2 c2[NP];
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[pp][k] = 0;
    c2[pp] = __builtin_bit_cast(u16x2, Pl[(2 * pp + SY) * LW + SX]);
  }
#pragma unroll
  for (int i = 0; i < 2 * SX + 1; ++i) {
    uint32_t v[WR];
#pragma unroll
    for (int rr = 0; rr < WR; ++rr) v[rr] = Pl[rr * LW + i];
#pragma unroll
    for (int jj = 0; jj < 2 * SY + 1; ++jj) {
      // the centre against itself: its bit is 0, nothing to file
      if (i == SX && jj == SY) continue;
      const int pos = N - 1 - (i * (2 * SY + 1) + jj);   // Alg. 1 order, MSB first
      const int q = pos >> 3;
      uint32_t d[NP];
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) {
        // half = centre - neighbour: in 0..255 when the neighbour is not brighter, in
        // 0xFF01..0xFFFF when it is, so bits 8..15 of each half all equal the bit
        d[pp] = __builtin_bit_cast(uint32_t, c2[pp] - __builtin_bit_cast(u16x2, v[2 * pp + jj]));
      }
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) acc[pp][q] = (d[pp] & (0x01000100u << (pos & 7))) | acc[pp][q];
      // One v_and_or_b32 per comparison and pair. The empty asm keeps the compiler from
      // regrouping the ORs into v_or3_b32 trees (an extra v_and_b32 per bit); the four
      // pairs' subtracts are issued ahead of their AND-ORs, so no packed-result wait
      // state is needed.
      if constexpr (NP == 4)
        asm volatile("" : "+v"(acc[0][q]), "+v"(acc[1][q]), "+v"(acc[2][q]), "+v"(acc[3][q]));
      else
        asm volatile("" : "+v"(acc[0][q]), "+v"(acc[1][q]));
    }
  }
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    if (sentinel) acc[pp][N >> 3] |= 0x01000100u << (N & 7);
    // code byte k of A is byte 1 of acc[k], of B byte 3
    const uint32_t x01 = __builtin_amdgcn_perm(acc[pp][1], acc[pp][0], 0x07030501u);
    const uint32_t x23 = __builtin_amdgcn_perm(acc[pp][3], acc[pp][2], 0x07030501u);
    const uint32_t x45 = __builtin_amdgcn_perm(acc[pp][5], acc[pp][4], 0x07030501u);
    const uint32_t x67 = __builtin_amdgcn_perm(acc[pp][7], acc[pp][6], 0x07030501u);
    const uint64_t codeA = ((uint64_t)__builtin_amdgcn_perm(x67, x45, 0x05040100u) << 32) |
                           __builtin_amdgcn_perm(x23, x01, 0x05040100u);
    const uint64_t codeB = ((uint64_t)__builtin_amdgcn_perm(x67, x45, 0x07060302u) << 32) |
                           __builtin_amdgcn_perm(x23, x01, 0x07060302u);
    // rows are wave-uniform: the row address steps by the pitch (scalar adds), the
    // lane's column is an unsigned offset
    const int YA = Y0 + r0 + 2 * pp;
    const int YB = YA + 1;
    if (YA < Hs && x_in) {
      const bool def = x_def && YA >= SY && YA < Hs - SY;
      orow[(uint32_t)X] = def ? codeA : 0ull;
    }
    orow += out_pitch;
    if (YB < Hs && x_in) {
      const bool def = x_def && YB >= SY && YB < Hs - SY;
      orow[(uint32_t)X] = def ? codeB : 0ull;
    }
    orow += out_pitch;
  }
}


// One tile, staged through registers.
template <int SX, int SY>
__device__ __forceinline__ void census_tile(const uint8_t* __restrict__ img, int W, int H,
                                            int pitch, int s, uint64_t* __restrict__ out,
                                            int out_pitch, int X0, int Y0, int sentinel,
                                            uint32_t* P) {
  const CensusJob j{img, W, H, pitch, s, W / s, H / s, out, out_pitch, X0, Y0};
  census_stage<SX, SY>(j, P);
  __syncthreads();
  census_compute<SX, SY>(j, sentinel, P);
}

// Any window: one pixel per thread per row, straight from global memory (no LDS).
__device__ __forceinline__ void census_tile_generic(const uint8_t* __restrict__ img, int W, int H,
                                                    int pitch, int s, uint64_t* __restrict__ out,
                                                    int out_pitch, int X0, int Y0, int sx, int sy,
                                                    int sentinel) {
  const int Ws = W / s, Hs = H / s;
  const int X = X0 + (threadIdx.x & 63);
  for (int Y = Y0 + (int)(threadIdx.x >> 6); Y < Y0 + kCensusTileY; Y += 4) {
    if (X >= Ws || Y >= Hs) continue;
    uint64_t code = 0;
    if (X >= sx && X < Ws - sx && Y >= sy && Y < Hs - sy) {
      const uint8_t c = img[(size_t)(s * Y) * pitch + (size_t)(s * X)];
      code = sentinel ? 1ull : 0ull;
      for (int i = -sx; i <= sx; ++i)
        for (int j = -sy; j <= sy; ++j) {
          const uint8_t n = img[(size_t)(s * (Y + j)) * pitch + (size_t)(s * (X + i))];
          code = (code << 1) | (n > c ? 1ull : 0ull);
        }
    }
    out[(size_t)Y * out_pitch + X] = code;
  }
}

// Whether a box's search reads some pixel of the census tile [X0, X0 + 64) x
// [Y0, Y0 + 32) of one view at one level. A ranged box belongs to the level of its
// far/close type (Sec. 4.3.4); its blocks lie in the level rectangle [x0, x1) x [y0, y1)
// of its eligible pixels (the same clipping as the plan). With candidates dlo..dhi, the
// forward search reads the right view on [x0 - dhi, x1 - dlo); the template and the
// backward search read the left view on [x0 - (dhi - dlo), x1 + (dhi - dlo)); all on
// rows [y0, y1). The loop and the result are uniform over the wave.
__device__ __forceinline__ bool census_tile_needed(const MatchParamsDev& MP, const FrameDev& fr,
                                                   const ocsr_box* __restrict__ boxes, int level,
                                                   int view, int X0, int Y0) {
  const int lane = threadIdx.x & 63;
  const LevelDev& lv = fr.lv[level];
  const int s = lv.scale;
  const int dlo = MP.path[level].dlo, dhi = dlo + MP.path[level].nd - 1;
  const int ext_lo = view ? dhi : dhi - dlo;   // the read range starts this far left of x0
  const int ext_hi = view ? -dlo : dhi - dlo;  // and ends this far right of x1
  // rows: the right view is read at y + dy, the left view (backward) at y + dy_f - dy
  const int eylo = MP.path[level].dylo, eyhi = eylo + MP.path[level].ndy - 1;
  const int ey_lo = view ? -eylo : eyhi - eylo;  // rows start this far above y0
  const int ey_hi = view ? eyhi : eyhi - eylo;   // and end this far below y1
  for (int base = 0; base < fr.n_boxes; base += 64) {
    const int i = base + lane;
    bool hit = false;
    if (i < fr.n_boxes) {
      const ocsr_box b = boxes[fr.box_off + i];
      const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
      const int cx1 = min(b.x1, fr.W), cy1 = min(b.y1, fr.H);
      if ((b.flags & OCSR_BOX_RANGE) && cx0 < cx1 && cy0 < cy1 &&
          (max(cx1 - cx0, cy1 - cy0) < MP.tau_s ? 0 : 1) == level) {
        const int x0 = max(cdiv_nonneg(cx0, s), lv.sx), x1 = min(cdiv_nonneg(cx1, s), lv.W - lv.sx);
        const int y0 = max(cdiv_nonneg(cy0, s), lv.sy), y1 = min(cdiv_nonneg(cy1, s), lv.H - lv.sy);
        hit = x0 < x1 && y0 < y1 && y0 - ey_lo < Y0 + kCensusTileY && Y0 < y1 + ey_hi &&
              x0 - ext_lo < X0 + kCensusTileX && X0 < x1 + ext_hi;
      }
    }
    if (__ballot(hit)) return true;
  }
  return false;
}

// Census tile c of a whole-frame call: the tiles of frame f start at
// FR.f[f].tile_begin and run over view L then R at level 1, then L and R at level 0.
// Level 1 comes first: its tiles are few and mostly read by the close boxes, so they are
// dispatched ahead of the many, mostly skipped, tiles of level 0.
struct FrameTile {
  int f, level, view;
  CensusJob job;
};
// Frame-local tile t of frame f (the frame's tiles number fewer than 2^30; the row of a
// tile comes from the frame's reciprocal of its tiles per row, without a division).
__device__ __forceinline__ FrameTile frame_tile_local(const FrameDev& fr, int f, int t) {
  int level = 1, tiles = fr.tiles1, tiles_x = fr.tiles1_x;
  uint64_t recip = fr.tx_recip[1];
  if (t >= 2 * fr.tiles1) {
    t -= 2 * fr.tiles1;
    level = 0;
    tiles = fr.tiles0;
    tiles_x = fr.tiles0_x;
    recip = fr.tx_recip[0];
  }
  const int view = t >= tiles ? 1 : 0;
  t -= view ? tiles : 0;
  const int ty = (int)(((uint64_t)(uint32_t)t * recip) >> 40);
  const int tx = t - ty * tiles_x;
  const LevelDev& lv = fr.lv[level];
  FrameTile ft;
  ft.f = f;
  ft.level = level;
  ft.view = view;
  ft.job = CensusJob{view ? fr.imgR : fr.imgL, fr.W, fr.H, fr.pitch, lv.scale, lv.W, lv.H,
                     (uint64_t*)(view ? lv.R : lv.L), lv.pitch, tx * kCensusTileX, ty * kCensusTileY};
  return ft;
}
__device__ __forceinline__ FrameTile frame_tile(const FramesDev& FR, int c) {
  int f = 0;
  for (int k = 1; k < FR.n; ++k)
    if (c >= FR.f[k].tile_begin) f = k;
  return frame_tile_local(FR.f[f], f, c - FR.f[f].tile_begin);
}

// Makes tile j: window (SX, SY) > (-1, -1) through LDS, (-1, -1) the generic code with
// (sx, sy). All 256 threads of the workgroup.
template <int SX, int SY>
__device__ __forceinline__ void make_census_tile(const CensusJob& j, int sx, int sy, int sentinel,
                                                 uint32_t* P) {
  if constexpr (SX >= 0) {
    census_stage<SX, SY>(j, P);
    __syncthreads();
    census_compute<SX, SY>(j, sentinel, P);
  } else {
    census_tile_generic(j.img, j.W, j.H, j.pitch, j.s, j.out, j.out_pitch, j.X0, j.Y0, sx, sy, sentinel);
  }
}

// Makes census tile c of a whole-frame call. With `check` set and MP.full_census clear,
// a tile no box's search reads is skipped (every wave of the workgroup takes the same
// decision). Window (SX, SY) > (-1, -1) takes the LDS code; (-1, -1) the generic code
// with (sx, sy).
template <int SX, int SY>
__device__ __forceinline__ void frame_census_tile(const MatchParamsDev& MP, const FramesDev& FR,
                                                  const ocsr_box* __restrict__ boxes, int c,
                                                  int sx, int sy, int sentinel, uint32_t* P,
                                                  bool check = true, int* verdict = nullptr) {
  const FrameTile ft = frame_tile(FR, c);
  const CensusJob& j = ft.job;
  if (check && !MP.full_census) {
    const FrameDev& fr = FR.f[ft.f];
    bool needed;
    if (verdict) {
      // wave 0 tests the tile and shares the verdict through LDS (verdict must not alias P)
      if (threadIdx.x < 64) {
        const bool v = census_tile_needed(MP, fr, boxes, ft.level, ft.view, j.X0, j.Y0);
        if (threadIdx.x == 0) *verdict = v ? 1 : 0;
      }
      __syncthreads();
      needed = *verdict != 0;
    } else {
      needed = census_tile_needed(MP, fr, boxes, ft.level, ft.view, j.X0, j.Y0);
    }
    if (!needed) return;
  }
  make_census_tile<SX, SY>(j, sx, sy, sentinel, P);
}

// Sets, in bits, the tile bits of the frame's boxes (thread t0 of nt threads; atomic ORs,
// so threads may share a map). With fewer boxes than threads, tpb threads share a box and
// take every tpb-th of its tile rows: thread t0 takes boxes t0 / tpb, t0 / tpb + nt / tpb,
// ... and rows sub, sub + tpb, ... of each.
__device__ __forceinline__ void mark_frame_tiles(const MatchParamsDev& MP, const FrameDev& fr,
                                                 const ocsr_box* __restrict__ boxes,
                                                 uint32_t* bits, int t0, int nt) {
  const int tpb = max(1, min(8, nt / max(fr.n_boxes, 1)));
  const int sub = t0 % tpb, groups = nt / tpb;
  if (t0 >= groups * tpb) return;
  for (int i = t0 / tpb; i < fr.n_boxes; i += groups) {
    const ocsr_box b = boxes[fr.box_off + i];
    const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
    const int cx1 = min(b.x1, fr.W), cy1 = min(b.y1, fr.H);
    if (!(b.flags & OCSR_BOX_RANGE) || !(cx0 < cx1 && cy0 < cy1)) continue;
    const int level = max(cx1 - cx0, cy1 - cy0) < MP.tau_s ? 0 : 1;
    const LevelDev& lv = fr.lv[level];
    const int s = lv.scale;
    const int x0 = max(cdiv_nonneg(cx0, s), lv.sx), x1 = min(cdiv_nonneg(cx1, s), lv.W - lv.sx);
    const int y0 = max(cdiv_nonneg(cy0, s), lv.sy), y1 = min(cdiv_nonneg(cy1, s), lv.H - lv.sy);
    if (!(x0 < x1 && y0 < y1)) continue;
    const int dlo = MP.path[level].dlo, dhi = dlo + MP.path[level].nd - 1;
    const int eylo = MP.path[level].dylo, eyhi = eylo + MP.path[level].ndy - 1;
    const int tiles_x = level ? fr.tiles1_x : fr.tiles0_x;
    const int tiles = level ? fr.tiles1 : fr.tiles0;
    const int tiles_y = tiles / tiles_x;
    const int lbase = level ? 0 : 2 * fr.tiles1;
    for (int view = 0; view < 2; ++view) {
      const int a = max(x0 - (view ? dhi : dhi - dlo), 0);
      const int e = min(x1 + (view ? -dlo : dhi - dlo), tiles_x * kCensusTileX);
      if (a >= e) continue;
      const int ta = a / kCensusTileX, tb = (e - 1) / kCensusTileX;
      const int ya = max(y0 + (view ? eylo : eylo - eyhi), 0);
      const int yb = min(y1 + (view ? eyhi : eyhi - eylo), tiles_y * kCensusTileY);
      if (ya >= yb) continue;
      for (int ty = ya / kCensusTileY + sub; ty <= (yb - 1) / kCensusTileY; ty += tpb) {
        const int first = lbase + view * tiles + ty * tiles_x + ta;
        const int last = first + (tb - ta);
        for (int wd = first >> 5; wd <= (last >> 5); ++wd) {
          const int lo = max(first - 32 * wd, 0), hi = min(last - 32 * wd, 31);
          const uint32_t upto = hi == 31 ? 0xFFFFFFFFu : ((1u << (hi + 1)) - 1u);
          atomicOr(&bits[wd], upto & ~((1u << lo) - 1u));
        }
      }
    }
  }
}

// Word i of an empty tile map of n_tiles tiles, or of a full one with MP.full_census.
__device__ __forceinline__ uint32_t tile_map_init(const MatchParamsDev& MP, int n_tiles, int i) {
  const int rem = n_tiles - 32 * i;
  return !MP.full_census ? 0u : rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
}

// Writes the tiles set in the OR of n_maps maps (map m at bits + m * stride words) to
// fr.tile_list in increasing tile number and their number to the frame's FC_TILES
// counter. All 256 threads of the workgroup, after the maps are complete; sc: 8 ints.
__device__ __forceinline__ void compact_frame_tiles(const FrameDev& fr, int f, const MatchWs& ws,
                                                    const uint32_t* bits, int n_maps, int stride,
                                                    int* sc) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n_tiles = 2 * (fr.tiles0 + fr.tiles1);
  const int n_words = (n_tiles + 31) >> 5;
  auto word = [&](int i) {
    uint32_t m = 0;
    for (int k = 0; k < n_maps; ++k) m |= bits[k * stride + i];
    return m;
  };
  // thread t owns words [t wpt, (t + 1) wpt); ranks run in word order
  const int wpt = (n_words + 255) >> 8;
  const int w0 = tid * wpt;
  int cnt = 0;
  for (int k = 0; k < wpt; ++k)
    if (w0 + k < n_words) cnt += __popc(word(w0 + k));
  const int incl = wave_incl_scan(cnt, lane);
  if (lane == 63) sc[wave] = incl;
  __syncthreads();
  int r = incl - cnt;
  for (int v = 0; v < wave; ++v) r += sc[v];
  for (int k = 0; k < wpt; ++k) {
    uint32_t m = w0 + k < n_words ? word(w0 + k) : 0u;
    while (m) {
      const int bit = __ffs(m) - 1;
      m &= m - 1;
      fr.tile_list[r++] = 32 * (w0 + k) + bit;
    }
  }
  if (tid == 255) ws.fcount[f * FC_N + FC_TILES] = r;
}

// The plan step's list of the census tiles of frame f: every tile some ranged box's
// search reads (the ranges of census_tile_needed), or every tile with MP.full_census,
// in increasing frame-local tile number (the order frame_census_tile decodes: level 1,
// view L then R, then level 0), written to fr.tile_list; their number to the frame's
// FC_TILES counter. One workgroup of 256 threads; bits: kFrameTileWords words of LDS,
// sc: 8 ints. The frame's tiles must number at most 32 kFrameTileWords.
__device__ __forceinline__ void list_frame_tiles(const MatchParamsDev& MP, const FrameDev& fr, int f,
                                                 const ocsr_box* __restrict__ boxes,
                                                 const MatchWs& ws, uint32_t* bits, int* sc) {
  const int tid = threadIdx.x;
  const int n_tiles = 2 * (fr.tiles0 + fr.tiles1);
  const int n_words = (n_tiles + 31) >> 5;
  for (int i = tid; i < n_words; i += 256) bits[i] = tile_map_init(MP, n_tiles, i);
  __syncthreads();
  if (!MP.full_census) {
    mark_frame_tiles(MP, fr, boxes, bits, tid, 256);
    __syncthreads();
  }
  compact_frame_tiles(fr, f, ws, bits, 1, 0, sc);
}

}  // namespace dev
}  // namespace ocsr
