// Dense counterpart of the object-centric path: every pixel, every disparity. Not part
// of the paper's method; it is the dense matcher the object-centric path is measured
// against (same census descriptors, same Hamming cost).
//
//   C(x, y, d)  = sum over the (2R+1)^2 window around (x, y), clipped to the image, of
//                 popcount(CL(x', y') ^ CR(x' - d, y'))   (CR is 0 outside the image)
//   d_L(x, y)   = smallest d in [dmin, dmax] minimising C(x, y, d)
//   d_R(xr, y)  = smallest d minimising C(xr + d, y, d) over d with xr + d inside
//   disp(x, y)  = d_L if x - d_L >= 0 and |d_L - d_R(x - d_L, y)| <= lr_tol, else -1
//
// One wave per strip of 64 - 2R output columns (lanes = 64 columns: the strip and an
// R-column halo on each side) and band of kBand output rows. The wave walks the band's rows once per chunk of 8
// disparities: per row it forms the 8 per-pixel costs (2 x v_xor_b32 + 2 x
// v_bcnt_u32_b32 each), packs them in pairs into 16-bit halves, updates the vertical
// window sums with the row that enters and the one that leaves (a ring of 2R+1 rows in
// registers), adds the horizontal neighbours with wave-wide DPP shifts, and keeps the
// running minimum of the key cost << 8 | (d - dmin) of each output row. Costs stay
// below 2^16 (at most 49 x 64 = 3136), so two of them share a 32-bit add without carry.
//
// The right view runs the same kernel with the roles of the images swapped: the
// term at right column x' is popcount(CL(x' + d, y') ^ CR(x', y')) when x' + d is
// inside the image and 0 otherwise, and C(xr + d, y, d) is the window sum of those
// terms around xr.
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

constexpr int kBand = 8;     // output rows per wave
constexpr int kChunk = 8;    // disparities per pass
template <int R>
constexpr int strip() { return 64 - 2 * R; }   // output columns per wave

struct DenseArgs {
  const uint64_t* CL;
  const uint64_t* CR;
  int32_t W, H, pitch;        // descriptor image size and row pitch (words)
  int32_t dlo, nd;            // disparities dlo .. dlo + nd - 1
  int16_t* out;               // [H][W] winning disparity (-1: no candidate)
  // several pairs in one launch (grid z): pair z reads CL + z * cl_zstride (words; the
  // right image is shared) and writes out + z * out_zstride
  int64_t cl_zstride, out_zstride;
};

__device__ __forceinline__ uint32_t popc64(uint64_t v) {
  return (uint32_t)__popc((uint32_t)v) + (uint32_t)__popc((uint32_t)(v >> 32));
}

__device__ __forceinline__ uint32_t shr1(uint32_t v) {   // lane i gets lane i - 1
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t shl1(uint32_t v) {   // lane i gets lane i + 1
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
}

// One pass over the band's rows for disparities d0 .. d0 + kChunk - 1 (c0 = d0 - dlo),
// updating key[] of the kBand output rows. MASKED: some lane of the wave reads a word
// outside the image for some d of the chunk, so every term is checked; otherwise
// every word and term of the pass is inside and no check is made.
// RIGHT = 0: the left view (term at column x' pairs CL(x') with CR(x' - d));
// RIGHT = 1: the right view (term at column x' pairs CL(x' + d) with CR(x')).
template <int R, int RIGHT, bool MASKED>
__device__ __forceinline__ void dense_pass(const DenseArgs& a, int x, int y0, int c0,
                                          uint32_t (&key)[kBand]) {
  constexpr int NW = 2 * R + 1;            // window rows
  constexpr int NR = kBand + 2 * R;        // rows walked
  constexpr int NP = kChunk / 2;           // packed cost pairs
  const int W = a.W, d0 = a.dlo + c0;
  // byte offsets within a row of the fixed word (x) and of the moving words (the
  // other image at x -/+ d); a word outside the image reads column 0 and is dropped
  const bool f_in = x >= 0 && x < W;
  const uint32_t f_off = 8u * (uint32_t)(f_in ? x : 0);
  uint32_t m_off[kChunk];
  bool m_in[kChunk];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    const int xm = RIGHT ? x + d0 + j : x - d0 - j;
    m_in[j] = xm >= 0 && xm < W;
    m_off[j] = 8u * (uint32_t)(m_in[j] ? xm : 0);
  }
  // an opaque row pitch keeps the row addresses from being hoisted out of the pass
  int pitch_bytes = a.pitch * 8;
  asm volatile("" : "+s"(pitch_bytes));
  const char* fixed_img = (const char*)(RIGHT ? a.CR : a.CL);
  const char* moving_img = (const char*)(RIGHT ? a.CL : a.CR);

  uint32_t ring[NW][NP], V[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    V[m] = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) ring[w][m] = 0;
  }
  // row i of the pass is image row y0 - R + i; rows outside the image read row 0 and
  // are dropped. Row i + 1 is loaded while row i is processed.
  auto load_row = [&](int i, uint64_t& f, uint64_t (&mv)[kChunk]) {
    const int yy = y0 - R + i;
    const size_t ro = (size_t)((yy >= 0 && yy < a.H) ? yy : 0) * (size_t)pitch_bytes;
    f = *(const uint64_t*)(fixed_img + ro + f_off);
#pragma unroll
    for (int j = 0; j < kChunk; ++j) mv[j] = *(const uint64_t*)(moving_img + ro + m_off[j]);
  };
  uint64_t cur_f, cur_m[kChunk];
  load_row(0, cur_f, cur_m);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    uint64_t nxt_f = 0, nxt_m[kChunk];
    if (i + 1 < NR) load_row(i + 1, nxt_f, nxt_m);
    const int yy = y0 - R + i;
    uint32_t t[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) t[m] = 0;
    if (yy >= 0 && yy < a.H) {
#pragma unroll
      for (int j = 0; j < kChunk; ++j) {
        uint32_t c;
        if (MASKED) {
          // the term counts where its left-image column is inside; the right-image
          // word outside the image is 0
          const uint64_t fw = f_in ? cur_f : 0ull;
          const uint64_t mw = m_in[j] ? cur_m[j] : 0ull;
          const bool term = RIGHT ? m_in[j] : f_in;
          c = term ? popc64(fw ^ mw) : 0u;
        } else {
          c = popc64(cur_f ^ cur_m[j]);
        }
        t[j / 2] |= c << (16 * (j & 1));
      }
    }
    // vertical window: add the entering row, drop the row 2R+1 rows back
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      V[m] = V[m] + t[m] - ring[i % NW][m];
      ring[i % NW][m] = t[m];
    }
    if (i >= 2 * R) {                      // V is the window of output row y0 + i - 2R
      const int o = i - 2 * R;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        uint32_t h = V[m], l = V[m], r = V[m];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          l = shr1(l);
          r = shl1(r);
          h += l + r;
        }
        // keys cost << 8 | (d - dlo) of the pair's two disparities; a right-view
        // candidate needs its left-image column x + d inside the image
        const uint32_t klo = ((h & 0xFFFFu) << 8) | (uint32_t)(c0 + 2 * m);
        const uint32_t khi = ((h >> 16) << 8) | (uint32_t)(c0 + 2 * m + 1);
        const bool in_lo = c0 + 2 * m < a.nd && (!RIGHT || !MASKED || m_in[2 * m]);
        const bool in_hi = c0 + 2 * m + 1 < a.nd && (!RIGHT || !MASKED || m_in[2 * m + 1]);
        key[o] = min(key[o], min(in_lo ? klo : 0xFFFFFFFFu, in_hi ? khi : 0xFFFFFFFFu));
      }
    }
    if (i + 1 < NR) {
      cur_f = nxt_f;
#pragma unroll
      for (int j = 0; j < kChunk; ++j) cur_m[j] = nxt_m[j];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int R, int RIGHT>
__global__ __launch_bounds__(256) void dense_kernel(DenseArgs a) {
  a.CL += (int64_t)blockIdx.z * a.cl_zstride;
  a.out += (int64_t)blockIdx.z * a.out_zstride;
  const int lane = threadIdx.x & 63;
  const int band = blockIdx.y * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int y0 = band * kBand;
  if (y0 >= a.H) return;                   // whole wave; the kernel has no barrier
  const int xw = blockIdx.x * strip<R>() - R;   // column of lane 0
  const int x = xw + lane;

  uint32_t key[kBand];
#pragma unroll
  for (int i = 0; i < kBand; ++i) key[i] = 0xFFFFFFFFu;
  for (int c0 = 0; c0 < a.nd; c0 += kChunk) {
    // every lane's words inside the image for the whole chunk?
    const int d0 = a.dlo + c0;
    const bool inside = RIGHT ? (xw >= 0 && xw + 63 + d0 + kChunk - 1 < a.W)
                              : (xw - d0 - (kChunk - 1) >= 0 && xw + 63 < a.W);
    if (inside) dense_pass<R, RIGHT, false>(a, x, y0, c0, key);
    else dense_pass<R, RIGHT, true>(a, x, y0, c0, key);
  }
  if (lane < R || lane >= R + strip<R>() || x >= a.W) return;
#pragma unroll
  for (int o = 0; o < kBand; ++o) {
    const int y = y0 + o;
    if (y < a.H)
      a.out[(size_t)y * a.W + x] = key[o] == 0xFFFFFFFFu ? (int16_t)-1
                                                        : (int16_t)(a.dlo + (int)(key[o] & 0xFFu));
  }
}

// The L/R check of one row segment of 256 pixels. With `partial` set, the workgroup also
// stores how many of its checked disparities are > d_min at
// partial[(z * H + y) * gridDim.x + blockIdx.x].
__global__ __launch_bounds__(256) void dense_check_kernel(const int16_t* __restrict__ dl,
                                                          const int16_t* __restrict__ dr, int W,
                                                          int H, int lr_tol, int16_t* disp,
                                                          int d_min, int32_t* partial) {
  __shared__ int part[4];
  const size_t plane = (size_t)blockIdx.z * W * H;   // pair z of a multi-pair launch
  dl += plane;
  dr += plane;
  disp += plane;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  int above = 0;
  if (x < W) {
    const int d = dl[(size_t)y * W + x];
    const int xr = x - d;
    int ok = 0;
    if (d >= 0 && xr >= 0) {
      const int db = dr[(size_t)y * W + xr];
      ok = db >= 0 && abs(d - db) <= lr_tol;
    }
    disp[(size_t)y * W + x] = ok ? (int16_t)d : (int16_t)-1;
    above = ok && d > d_min ? 1 : 0;
  }
  if (!partial) return;   // uniform over the launch
  for (int o = 32; o > 0; o >>= 1) above += __shfl_xor(above, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = above;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[((size_t)blockIdx.z * H + y) * gridDim.x + blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// counts[z] = the sum of map z's n partial counts: one workgroup per map, no atomics
__global__ __launch_bounds__(256) void count_above_kernel(const int32_t* __restrict__ partial, int n,
                                                          int32_t* counts) {
  __shared__ int part[4];
  const int32_t* p = partial + (size_t)blockIdx.x * n;
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 256) c += p[i];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

template <int R>
hipError_t launch_dense_r(const DenseArgs& left, const DenseArgs& right, hipStream_t s, int nz = 1) {
  const dim3 grid((left.W + strip<R>() - 1) / strip<R>(), (left.H + 4 * kBand - 1) / (4 * kBand), nz);
  dense_kernel<R, 0><<<grid, 256, 0, s>>>(left);
  dense_kernel<R, 1><<<grid, 256, 0, s>>>(right);
  return hipGetLastError();
}

}  // namespace

bool dense_radius_supported(int radius) { return radius >= 1 && radius <= 3; }

hipError_t launch_dense(const uint64_t* CL, const uint64_t* CR, int W, int H, int pitch, int dmin,
                        int dmax, int radius, int lr_tol, int16_t* disp, int16_t* d_left,
                        int16_t* d_right, hipStream_t stream, const LaunchTimer* timer) {
  const DenseArgs left = {CL, CR, W, H, pitch, dmin, dmax - dmin + 1, d_left, 0, 0};
  const DenseArgs right = {CL, CR, W, H, pitch, dmin, dmax - dmin + 1, d_right, 0, 0};
  if (timer) timer->before(timer->ctx, "dense", stream);
  hipError_t e = hipErrorNotSupported;
  if (radius == 1) e = launch_dense_r<1>(left, right, stream);
  if (radius == 2) e = launch_dense_r<2>(left, right, stream);
  if (radius == 3) e = launch_dense_r<3>(left, right, stream);
  if (timer) timer->after(timer->ctx, "dense", stream);
  if (e != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "dense_check", stream);
  dense_check_kernel<<<dim3((W + 255) / 256, H), 256, 0, stream>>>(d_left, d_right, W, H, lr_tol,
                                                                   disp, 0, nullptr);
  if (timer) timer->after(timer->ctx, "dense_check", stream);
  return hipGetLastError();
}

// Dense counterpart of nz pairs at once: pair z is (CL0 - z rows, CR), i.e. the left
// descriptors moved down by z more rows; then the pixels above d_min of each map.
hipError_t launch_dense_offsets(const uint64_t* CL0, const uint64_t* CR, int W, int H, int pitch,
                                int nz, int dmin, int dmax, int radius, int lr_tol, int d_min,
                                int16_t* disp, int16_t* d_left, int16_t* d_right, int32_t* partial,
                                int32_t* counts, hipStream_t stream, const LaunchTimer* timer) {
  const int64_t plane = (int64_t)W * H;
  const DenseArgs left = {CL0, CR, W, H, pitch, dmin, dmax - dmin + 1, d_left, -(int64_t)pitch, plane};
  const DenseArgs right = {CL0, CR, W, H, pitch, dmin, dmax - dmin + 1, d_right, -(int64_t)pitch, plane};
  if (timer) timer->before(timer->ctx, "rect_dense", stream);
  hipError_t e = hipErrorNotSupported;
  if (radius == 1) e = launch_dense_r<1>(left, right, stream, nz);
  if (radius == 2) e = launch_dense_r<2>(left, right, stream, nz);
  if (radius == 3) e = launch_dense_r<3>(left, right, stream, nz);
  if (timer) timer->after(timer->ctx, "rect_dense", stream);
  if (e != hipSuccess) return e;
  if (timer) timer->before(timer->ctx, "rect_count", stream);
  const int bx = (W + 255) / 256;
  dense_check_kernel<<<dim3(bx, H, nz), 256, 0, stream>>>(d_left, d_right, W, H, lr_tol, disp, d_min,
                                                          partial);
  count_above_kernel<<<nz, 256, 0, stream>>>(partial, H * bx, counts);
  if (timer) timer->after(timer->ctx, "rect_count", stream);
  return hipGetLastError();
}

}  // namespace ocsr
