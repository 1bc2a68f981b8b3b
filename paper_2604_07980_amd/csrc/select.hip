// Priority object selection under a per-frame budget (Sec. 4.3.5, last sentence): frontal
// candidates (clipped-box centre in a central crop) first, then by proximity (larger
// clipped bottom y, the occlusion rule's nearness cue), then by box index. A candidate's
// rank is the number of candidates of its frame with a smaller key; the first
// max_objects stay ranged. Workgroup (x, f) ranks boxes 256 x .. 256 x + 255 of frame f
// against every box of the frame, staged 256 keys at a time in LDS.
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

// ~0 for a box that is not a candidate (it ranks behind every candidate)
__device__ __forceinline__ uint64_t select_key(const ocsr_box& b, int idx, const SelectFrameDev& fr) {
  const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
  const int cx1 = min(b.x1, fr.W), cy1 = min(b.y1, fr.H);
  if (!(b.flags & OCSR_BOX_RANGE) || !(cx0 < cx1 && cy0 < cy1)) return ~0ull;
  const int u2 = cx0 + cx1 - 1, v2 = cy0 + cy1 - 1;   // twice the centre
  const bool frontal = 2 * fr.X0 <= u2 && u2 < 2 * fr.X1 && 2 * fr.Y0 <= v2 && v2 < 2 * fr.Y1;
  return ((uint64_t)(frontal ? 0 : 1) << 48) | ((uint64_t)(65535 - cy1) << 24) | (uint64_t)idx;
}

__global__ __launch_bounds__(256) void select_kernel(SelectDev S, const ocsr_box* __restrict__ in,
                                                     ocsr_box* __restrict__ out,
                                                     int32_t* __restrict__ rank) {
  __shared__ uint64_t keys[256];
  const SelectFrameDev& fr = S.f[blockIdx.y];
  const int n = fr.n_boxes;
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if ((int)blockIdx.x * 256 >= n) return;   // the whole workgroup leaves together
  ocsr_box b = {};
  uint64_t key = ~0ull;
  if (i < n) {
    b = in[fr.box_off + i];
    key = select_key(b, i, fr);
  }
  int r = 0;
  for (int base = 0; base < n; base += 256) {
    const int j = base + (int)threadIdx.x;
    keys[threadIdx.x] = j < n ? select_key(in[fr.box_off + j], j, fr) : ~0ull;
    __syncthreads();
    const int m = min(256, n - base);
    for (int k = 0; k < m; ++k) r += keys[k] < key ? 1 : 0;
    __syncthreads();
  }
  if (i < n) {
    const bool cand = key != ~0ull;
    if (cand && r >= S.max_objects) b.flags &= ~OCSR_BOX_RANGE;
    out[fr.box_off + i] = b;
    if (rank) rank[fr.box_off + i] = cand ? r : -1;
  }
}

}  // namespace

hipError_t launch_select(const SelectDev& S, const ocsr_box* in, ocsr_box* out, int32_t* rank,
                         int max_boxes, hipStream_t stream, const LaunchTimer* timer) {
  if (max_boxes <= 0) return hipSuccess;
  return timed_launch(timer, "select", select_kernel, dim3((max_boxes + 255) / 256, S.n), dim3(256),
                      0, stream, S, in, out, rank);
}

}  // namespace ocsr
