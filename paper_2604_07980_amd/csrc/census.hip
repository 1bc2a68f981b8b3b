// Census transform kernels (Sec. 4.3.1) for the census entry points: one workgroup per
// 64 x 32 tile of one job (an image at one level). The tile code is in dev_census.hpp.
#include "dev_census.hpp"

namespace ocsr {
namespace {

__device__ __forceinline__ int find_job(const CensusJobsDev& jobs, int tile) {
  int j = 0;
  for (int k = 1; k < jobs.n; ++k)
    if (tile >= jobs.job[k].tile_begin) j = k;
  return j;
}

template <int SX, int SY>
__global__ __launch_bounds__(256) void census_kernel(CensusJobsDev jobs, int sentinel) {
  __shared__ uint32_t P[dev::CensusTile<SX, SY>::kLdsBytes / sizeof(uint32_t)];
  const CensusJobDev& jb = jobs.job[find_job(jobs, blockIdx.x)];
  const int t = blockIdx.x - jb.tile_begin;
  dev::census_tile<SX, SY>(jb.img, jb.W, jb.H, jb.pitch, jb.scale, jb.out, jb.out_pitch,
                           (t % jb.tiles_x) * kCensusTileX, (t / jb.tiles_x) * kCensusTileY,
                           sentinel, P);
}

__global__ __launch_bounds__(256) void census_kernel_generic(CensusJobsDev jobs, int sx, int sy,
                                                             int sentinel) {
  const CensusJobDev& jb = jobs.job[find_job(jobs, blockIdx.x)];
  const int t = blockIdx.x - jb.tile_begin;
  dev::census_tile_generic(jb.img, jb.W, jb.H, jb.pitch, jb.scale, jb.out, jb.out_pitch,
                           (t % jb.tiles_x) * kCensusTileX, (t / jb.tiles_x) * kCensusTileY, sx,
                           sy, sentinel);
}

}  // namespace

hipError_t launch_census(const CensusJobsDev& jobs, int total_tiles, int sx, int sy,
                         int sentinel, hipStream_t stream) {
  if (total_tiles <= 0) return hipSuccess;
  dim3 grid(total_tiles), block(256);
  if (sx == 3 && sy == 4) {
    census_kernel<3, 4><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else if (sx == 2 && sy == 2) {
    census_kernel<2, 2><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else if (sx == 4 && sy == 3) {
    census_kernel<4, 3><<<grid, block, 0, stream>>>(jobs, sentinel);
  } else {
    census_kernel_generic<<<grid, block, 0, stream>>>(jobs, sx, sy, sentinel);
  }
  return hipGetLastError();
}

}  // namespace ocsr
