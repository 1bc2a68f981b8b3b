/*
 * CPU oracle for the object-centric census template-matching path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no source with
 * the HIP library: its own types, its own loops, no common headers.
 *
 * Every function follows the paper's statement of the method step by step
 * (Sec. 4.3 "Census-Based Template Matching" and Alg. 2), with the readings of
 * silent points stated next to the code that takes them.
 */
#ifndef OCSR_ORACLE_H
#define OCSR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MODE_TILED = 0, ORC_MODE_GRID = 1 };
enum { ORC_AGG_SEGMENT_MEDIAN = 0, ORC_AGG_TRIMMED_MEDIAN = 1 };
enum {
  ORC_OK = 0, ORC_NOT_RANGED = 1, ORC_CLIPPED_EMPTY = 2, ORC_NO_ELIGIBLE_BLOCKS = 3,
  ORC_NO_VALID_BLOCKS = 4, ORC_TOO_FEW_CONSISTENT = 5, ORC_NONPOSITIVE_DISPARITY = 6,
  ORC_CAPACITY_OVERFLOW = 7
};

typedef struct { int32_t mode, bw, bh, n_side, dmin, dmax; } orc_path;

typedef struct {
  int32_t sx, sy;            /* census half-window of both levels */
  int32_t close_scale;       /* s of the close level; the far level is s = 1 */
  int32_t tau_s;             /* FAR iff max clipped side < tau_s (px) */
  orc_path far_path, close_path;
  int32_t lr_tol;            /* accept |d_b - d_f| <= lr_tol (level px) */
  int32_t min_point_pct;     /* block eligible iff 100*points >= pct*nx*ny */
  int32_t agg_mode;
  float   tau_d;
  int32_t n_min, trim_pct;
  float   focal_px, baseline_m, d_eps;
  int32_t max_blocks_per_box; /* > 0: boxes tiling into more blocks report
                               * CAPACITY_OVERFLOW; 0: no limit (the method sets none) */
  int32_t cap_blocks;         /* total block capacity (prefix rule), <= 0: unlimited */
  int32_t dy_min, dy_max;     /* vertical offsets searched, full-res px; 0, 0: none */
} orc_params;

typedef struct {
  float   disparity, depth;
  int32_t valid, reason, n_blocks, n_eligible, n_valid, n_used;
} orc_box_result;

typedef struct {
  int32_t box, level_scale, u, v;
  int32_t px0, py0, nx, ny;        /* level position of point 0 and point grid size */
  uint64_t mask;
  int32_t eligible, d_f, d_b, lr_ok;
  float   d_sub;                   /* level px */
  int32_t valid;
  int32_t dlo, nd;                 /* level search range [dlo, dlo + nd) */
  int32_t dy_f, dy_b;              /* level vertical offsets of the two winners */
} orc_block;

/* Priority object selection under a budget (Sec. 4.3.5, last sentence). boxes: int32
 * [n][5] of one W x H frame. A candidate has flag bit 0 and a non-empty clipped box.
 * Candidates are sorted frontal first (clipped centre in the crop, given in permille of
 * W and H), then by larger clipped bottom y, then by index; the first max_objects keep
 * bit 0. flags_out: [n] new flags; rank: [n] position in that order, -1 if no candidate. */
void orc_select_boxes(const int32_t* boxes, int32_t n, int32_t W, int32_t H, int32_t max_objects,
                      const int32_t* crop_permille, int32_t* flags_out, int32_t* rank);

/* Auto-rectification offset (Sec. 5.1). For each delta in [delta_min, delta_max]: the
 * ROI pair with the left descriptors moved down by delta (left row roi_y0 + y - delta,
 * right row roi_y0 + y), the dense counterpart orc_dense on it, and the number of pixels
 * whose disparity is > d_min. counts: [n_offsets]; maps (nullable): [n_offsets][roi_h][roi_w].
 * Returns 0, or -1 when the moved ROI leaves the image. */
int32_t orc_rect_counts(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                        int32_t roi_x0, int32_t roi_y0, int32_t roi_w, int32_t roi_h,
                        int32_t delta_min, int32_t delta_max, int32_t dmin, int32_t dmax,
                        int32_t radius, int32_t lr_tol, int32_t d_min, int32_t* counts,
                        int16_t* maps, int32_t n_threads);

/* The offset estimate of each of T frames (counts: [T][n_offsets]) and its temporal
 * filter: the median of the last `window` estimates, approached from the previous
 * output by at most max_step per frame (Sec. 5.1, filter equations). */
void orc_rect_filter(const int32_t* counts, int32_t T, int32_t n_offsets, int32_t delta_min,
                     int32_t window, int32_t max_step, int32_t initial, int32_t* raw,
                     int32_t* filtered);

/* Census of one level: out is [H/s][W/s] row-major, pitch W/s. Returns 0, or -1
 * when the window does not fit in 64 bits or an argument is out of range. */
int32_t orc_census(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                   int32_t sx, int32_t sy, int32_t s, int32_t sentinel, uint64_t* out);

/* Per-box disparity and depth. L0/R0: level s = 1 descriptors [H][W];
 * L1/R1: level s = close_scale descriptors [H/s][W/s] (may be NULL when no box
 * is CLOSE). boxes: int32 [n][5] = x0, y0, x1, y1 (half-open, px), flags
 * (bit 0: produce a range). Debug arrays may be NULL; when given, blocks[] has
 * room for cap_dbg blocks and cost_f/cost_b for cap_dbg * cap_nd entries.
 * Returns the total number of blocks tiled (>= 0) or -1 on bad arguments. */
int32_t orc_match_boxes(const uint64_t* L0, const uint64_t* R0,
                        const uint64_t* L1, const uint64_t* R1,
                        int32_t W, int32_t H, const int32_t* boxes, int32_t n,
                        const orc_params* p, orc_box_result* out,
                        orc_block* blocks, uint16_t* cost_f, uint16_t* cost_b,
                        int32_t cap_dbg, int32_t cap_nd, int32_t n_threads);

/* Aggregation of one box and its depth. vals (n_valid values, sorted in place)
 * are the full-res disparities of its valid blocks; n_blocks the blocks it was
 * tiled into; far_object: 1 for a box of type FAR (a FAR box of one block takes
 * that block's result, Alg. 2); r->n_eligible must be set by the caller. */
void orc_aggregate(float* vals, int32_t n_valid, int32_t n_blocks, int32_t far_object,
                   const orc_params* p, orc_box_result* r);

/* Dense counterpart: per-pixel WTA over [dmin, dmax] of the (2r+1)^2 box sum
 * of Hamming costs (clipped window), with a left/right check. disp: int16 [H][W],
 * -1 where invalid. disp_r (nullable): right-view WTA. */
int32_t orc_dense(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                  int32_t dmin, int32_t dmax, int32_t radius, int32_t lr_tol,
                  int16_t* disp, int16_t* disp_r, int32_t n_threads);

/* Dense counterpart at n sampled pixels (xy: int32 [n][2]); out: int16 [n]. */
int32_t orc_dense_at(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                     int32_t dmin, int32_t dmax, int32_t radius, int32_t lr_tol,
                     const int32_t* xy, int32_t n, int16_t* out, int32_t n_threads);

/* Per-box 3D point and covariance (Sec. 4.3.6 Q-matrix equation; Sec. 4.3.7 depth
 * variance and covariance rotation), in fp64. The box's image point is the centre of
 * its box clipped to the W x H image in pixel-index coordinates, ((cx0 + cx1 - 1) / 2,
 * (cy0 + cy1 - 1) / 2); d is the box result's disparity. (X, Y, Z, W') = Q (u, v, d, 1),
 * p_cam = (X, Y, Z) / W', p_imu = R p_cam + t, var_z = Z^4 var_d / (f^2 b^2),
 * cov_imu = R diag(var_x, var_y, var_z) R^T (upper triangle xx, xy, xz, yy, yz, zz).
 * A box whose result is not valid, whose clipped box is empty or whose W' is 0 gets
 * valid = 0 and zeros. Q, R row-major. */
typedef struct {
  double p_cam[3], p_imu[3], cov_imu[6], var_z;
  int32_t valid;
} orc_point;

void orc_box_points(const int32_t* boxes, const orc_box_result* res, int32_t n, int32_t W,
                    int32_t H, const double* Q, const double* R, const double* t, double f,
                    double b, double var_d, double var_x, double var_y, orc_point* out);

#ifdef __cplusplus
}
#endif
#endif
