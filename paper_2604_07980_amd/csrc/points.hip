// Per-box 3D point and covariance (Sec. 4.3.6 Q-matrix equation; Sec. 4.3.7 depth variance
// and covariance rotation). One thread per box: the box's image point and aggregated
// disparity through the reprojection matrix, the rigid transform to the IMU frame, the
// depth variance propagated from the disparity variance, and the camera-frame diagonal
// covariance rotated into the IMU frame. All in fp32.
#include "ocsr_internal.hpp"

namespace ocsr {
namespace {

__global__ __launch_bounds__(256) void box_points_kernel(const ocsr_box* __restrict__ boxes,
                                                         const ocsr_box_result* __restrict__ res,
                                                         int n, PointParamsDev pp,
                                                         ocsr_box_point* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const ocsr_box b = boxes[i];
  const ocsr_box_result r = res[i];
  const int cx0 = max(b.x0, 0), cy0 = max(b.y0, 0);
  const int cx1 = min(b.x1, pp.width), cy1 = min(b.y1, pp.height);
  ocsr_box_point o = {};
  const float in[4] = {0.5f * (float)(cx0 + cx1 - 1), 0.5f * (float)(cy0 + cy1 - 1), r.disparity, 1.0f};
  float h[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    h[k] = pp.Q[4 * k] * in[0] + pp.Q[4 * k + 1] * in[1] + pp.Q[4 * k + 2] * in[2] + pp.Q[4 * k + 3] * in[3];
  if (r.valid && cx0 < cx1 && cy0 < cy1 && h[3] != 0.0f) {
#pragma unroll
    for (int k = 0; k < 3; ++k) o.p_cam[k] = h[k] / h[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      o.p_imu[k] = pp.R[3 * k] * o.p_cam[0] + pp.R[3 * k + 1] * o.p_cam[1] + pp.R[3 * k + 2] * o.p_cam[2] + pp.t[k];
    // (dZ/dd)^2 var_d = Z^4 var_d / (f b)^2, as (Z^2 / (f b))^2 var_d
    const float zz = o.p_cam[2] * o.p_cam[2] / pp.fb;
    o.var_z = zz * zz * pp.var_d;
    const float s[3] = {pp.var_x, pp.var_y, o.var_z};
    // R diag(s) R^T, upper triangle row by row
    int q = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = a; c < 3; ++c)
        o.cov_imu[q++] = pp.R[3 * a] * s[0] * pp.R[3 * c] + pp.R[3 * a + 1] * s[1] * pp.R[3 * c + 1] +
                         pp.R[3 * a + 2] * s[2] * pp.R[3 * c + 2];
    o.valid = 1;
  }
  out[i] = o;
}

}  // namespace

hipError_t launch_box_points(const ocsr_box* boxes, const ocsr_box_result* res, int n,
                             const PointParamsDev& pp, ocsr_box_point* out, hipStream_t stream,
                             const LaunchTimer* timer) {
  if (n <= 0) return hipSuccess;
  return timed_launch(timer, "points", box_points_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                      boxes, res, n, pp, out);
}

}  // namespace ocsr
