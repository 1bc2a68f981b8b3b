// Census transform on gfx950 (Sec. 4.3.1: census equation and Alg. 1).
//
// One workgroup of 256 threads (4 wave64) produces a 64 x 32 tile of level pixels.
// The level samples of the tile plus its halo are staged once in LDS; each lane then
// owns one column and eight consecutive rows, pulls the (2SX+1) x (8+2SY) window of
// values it needs into registers and builds eight codes with a compare and an
// add-with-carry per bit (c = c + c + [n > centre]), filling the high and low halves
// of the 64-bit word separately so that no 64-bit shift is issued.
//
// Bit order: Alg. 1 starts from the sentinel and, for i = -SX..SX (x, outer) and
// j = -SY..SY (y, inner), shifts left and appends [I(x+i, y+j) > I(x, y)]; the
// first comparison therefore ends at bit n-1 (n = (2SX+1)(2SY+1)) and the sentinel
// at bit n. Pixels whose window leaves the level image store 0.
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

constexpr int TX = kCensusTileX;
constexpr int TY = kCensusTileY;
constexpr int ROWS_PER_LANE = 8;   // 4 waves x 8 rows = TY

__device__ __forceinline__ int find_job(const CensusJobsDev& jobs, int tile) {
  int j = 0;
  for (int k = 1; k < jobs.n; ++k)
    if (tile >= jobs.job[k].tile_begin) j = k;
  return j;
}

template <int SX, int SY>
__global__ __launch_bounds__(256) void census_tiled(CensusJobsDev jobs, int sentinel) {
  constexpr int LW = TX + 2 * SX;
  constexpr int LH = TY + 2 * SY;
  constexpr int N = (2 * SX + 1) * (2 * SY + 1);   // comparisons (centre included)
  constexpr int NHI = N > 32 ? N - 32 : 0;         // comparisons landing in the high word
  static_assert(N + 1 <= 64, "window wider than a 64-bit code");
  __shared__ uint32_t tile[LH][LW];

  const int jid = find_job(jobs, blockIdx.x);
  const CensusJobDev& jb = jobs.job[jid];
  const int s = jb.scale;
  const int Ws = jb.W / s, Hs = jb.H / s;
  const int t = blockIdx.x - jb.tile_begin;
  const int X0 = (t % jb.tiles_x) * TX;
  const int Y0 = (t / jb.tiles_x) * TY;
  const uint8_t* __restrict__ img = jb.img;

  for (int idx = threadIdx.x; idx < LW * LH; idx += 256) {
    const int ly = idx / LW, lx = idx - ly * LW;
    const int X = X0 - SX + lx, Y = Y0 - SY + ly;
    uint32_t v = 0;
    if (X >= 0 && X < Ws && Y >= 0 && Y < Hs) v = img[(size_t)(s * Y) * jb.pitch + (size_t)(s * X)];
    tile[ly][lx] = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int r0 = (threadIdx.x >> 6) * ROWS_PER_LANE;
  uint32_t v[2 * SX + 1][ROWS_PER_LANE + 2 * SY];
#pragma unroll
  for (int i = 0; i < 2 * SX + 1; ++i)
#pragma unroll
    for (int j = 0; j < ROWS_PER_LANE + 2 * SY; ++j) v[i][j] = tile[r0 + j][lane + i];

  const int X = X0 + lane;
  const bool x_in = X < Ws;
  const bool x_def = X >= SX && X < Ws - SX;
  uint64_t* __restrict__ out = jb.out;
#pragma unroll
  for (int r = 0; r < ROWS_PER_LANE; ++r) {
    const int Y = Y0 + r0 + r;
    const uint32_t c = v[SX][r + SY];
    uint32_t hi = NHI > 0 ? (uint32_t)sentinel : 0u;
    uint32_t lo = NHI > 0 ? 0u : (uint32_t)sentinel;
#pragma unroll
    for (int i = 0; i < 2 * SX + 1; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * SY + 1; ++j) {
        const int term = i * (2 * SY + 1) + j;
        const uint32_t b = v[i][r + j] > c ? 1u : 0u;
        if (term < NHI) hi = hi + hi + b;
        else lo = lo + lo + b;
      }
    }
    if (x_in && Y < Hs) {
      const bool def = x_def && Y >= SY && Y < Hs - SY;
      const uint64_t code = def ? (((uint64_t)hi << 32) | lo) : 0ull;
      out[(size_t)Y * jb.out_pitch + X] = code;
    }
  }
}

// Any window: one pixel per thread, straight from global memory.
__global__ __launch_bounds__(256) void census_generic(CensusJobsDev jobs, int sx, int sy,
                                                      int sentinel) {
  const int jid = find_job(jobs, blockIdx.x);
  const CensusJobDev& jb = jobs.job[jid];
  const int s = jb.scale;
  const int Ws = jb.W / s, Hs = jb.H / s;
  const int t = blockIdx.x - jb.tile_begin;
  const int X = (t % jb.tiles_x) * TX + (threadIdx.x & 63);
  const int Y0 = (t / jb.tiles_x) * TY + (threadIdx.x >> 6);
  for (int Y = Y0; Y < (t / jb.tiles_x) * TY + TY; Y += 4) {
    if (X >= Ws || Y >= Hs) continue;
    uint64_t code = 0;
    if (X >= sx && X < Ws - sx && Y >= sy && Y < Hs - sy) {
      const uint8_t c = jb.img[(size_t)(s * Y) * jb.pitch + (size_t)(s * X)];
      code = sentinel ? 1ull : 0ull;
      for (int i = -sx; i <= sx; ++i)
        for (int j = -sy; j <= sy; ++j) {
          const uint8_t n = jb.img[(size_t)(s * (Y + j)) * jb.pitch + (size_t)(s * (X + i))];
          code = (code << 1) | (n > c ? 1ull : 0ull);
        }
    }
    jb.out[(size_t)Y * jb.out_pitch + X] = code;
  }
}

}  // namespace

hipError_t launch_census(const CensusJobsDev& jobs, int total_tiles, int sx, int sy,
                         int sentinel, hipStream_t stream) {
  if (total_tiles <= 0) return hipSuccess;
  dim3 grid(total_tiles), block(256);
  if (sx == 3 && sy == 4) {
    census_tiled<3, 4><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else if (sx == 2 && sy == 2) {
    census_tiled<2, 2><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else if (sx == 4 && sy == 3) {
    census_tiled<4, 3><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else {
    census_generic<<<grid, block, 0, stream>>>(jobs, sx, sy, sentinel);
  }
  return hipGetLastError();
}

}  // namespace ocsr
