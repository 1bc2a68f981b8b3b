/*
 * ocsr.h -- C ABI of the object-centric census stereo ranging library (gfx950).
 *
 * The library computes, on one MI355X GPU, the object-centric template-matching
 * method of "Object-Centric Stereo Ranging for Autonomous Driving: From Dense
 * Disparity to Census-Based Template Matching", Sec. 4.3:
 *
 *   census(image) -> 64-bit descriptors                  (Sec. 4.3.1, census eq., Alg. 1)
 *   match_boxes(descL, descR, boxes, params) -> per box  (Sec. 4.3.2-4.3.6, Alg. 2)
 *       far/close split, occlusion-aware block sampling, forward Hamming block
 *       search with winner-take-all, parabola sub-pixel refinement, backward
 *       verification, robust aggregation, depth Z = f b / d (Eq. 1).
 *
 * Conventions shared by every entry point:
 *   - Pointers marked (dev) are device memory of the current HIP device, owned by
 *     the caller; pointers marked (host) are host memory read during the call only.
 *     The library never frees or keeps caller memory, and calls no hipMalloc on
 *     the matching path: scratch space is the caller's workspace (ws, ws_bytes).
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream). Outputs are valid once the caller synchronizes that stream.
 *   - Disparity d >= 0 is the left-to-right shift: the right-image match of left
 *     pixel (x, y) is (x - d, y + dy). The vertical offset dy is 0 unless the caller
 *     asks for a vertical range (ocsr_match_params.dy_min, dy_max) for pairs whose
 *     rectification has drifted.
 *   - Return value: OCSR_OK (0) or a negative status. Arguments are validated before
 *     anything is enqueued; on a negative status nothing was enqueued (except
 *     OCSR_E_HIP, reported when a launch fails). ocsr_last_error() then returns a
 *     message for the calling thread. No exception crosses the ABI; kernels never trap.
 *   - Data-dependent outcomes (a box too small, no consistent block, ...) are not
 *     errors: they are per-box reason codes (OCSR_REASON_*).
 */
#ifndef OCSR_H
#define OCSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCSR_ABI_VERSION 3

/* status codes */
#define OCSR_OK 0
#define OCSR_E_INVALID (-1)      /* bad argument, nothing enqueued */
#define OCSR_E_WORKSPACE (-2)    /* ws_bytes smaller than the matching *_workspace_bytes */
#define OCSR_E_CAPACITY (-3)     /* a size beyond a documented limit */
#define OCSR_E_HIP (-4)          /* a HIP runtime call failed */
#define OCSR_E_UNSUPPORTED (-5)  /* e.g. a census window of more than 64 bits */

/* per-box reason codes (ocsr_box_result.reason) */
#define OCSR_REASON_OK 0
#define OCSR_REASON_NOT_RANGED 1             /* flags bit 0 clear: the box only occludes */
#define OCSR_REASON_CLIPPED_EMPTY 2          /* no area inside the image */
#define OCSR_REASON_NO_ELIGIBLE_BLOCKS 3     /* no block with enough unoccluded points */
#define OCSR_REASON_NO_VALID_BLOCKS 4        /* every block failed the L/R check */
#define OCSR_REASON_TOO_FEW_CONSISTENT 5     /* aggregation kept fewer than n_min blocks */
#define OCSR_REASON_NONPOSITIVE_DISPARITY 6  /* disparity <= d_eps: no finite depth */
#define OCSR_REASON_CAPACITY_OVERFLOW 7      /* the box's blocks did not fit (see below) */
#define OCSR_REASON_INTERNAL_TIMEOUT 8       /* a bounded wait inside a fused launch expired:
                                                a library defect; the result is not valid */

#define OCSR_MODE_TILED 0   /* box cut into bw x bh blocks, every pixel a point */
#define OCSR_MODE_GRID 1    /* whole box one block, n_side x n_side grid of points */

#define OCSR_AGG_SEGMENT_MEDIAN 0  /* median of the longest run of gaps < tau_d (Sec. 4.3.4) */
#define OCSR_AGG_TRIMMED_MEDIAN 1  /* median after a symmetric trim of trim_pct percent */

#define OCSR_BOX_RANGE 1u   /* ocsr_box.flags: produce a range (else the box only occludes) */

/* Most frames one ocsr_range_batch call takes. */
#define OCSR_MAX_BATCH_FRAMES 16
/* Largest search range (level candidates) of one path. */
#define OCSR_MAX_CANDIDATES 256
/* Largest vertical offset (full-res px) and most (d, dy) candidates of a path with a
 * vertical range (ocsr_match_params.dy_min, dy_max). */
#define OCSR_MAX_DY 32
#define OCSR_MAX_DY_CANDIDATES 2048

typedef struct ocsr_ctx ocsr_ctx;

/* Library ABI version (OCSR_ABI_VERSION of the build). */
int32_t ocsr_abi_version(void);

/* Message of the calling thread's last non-zero status ("" if none). The pointer
 * stays valid until the thread's next library call. */
const char* ocsr_last_error(void);

/* Creates a context bound to HIP device `device` (it becomes current for the
 * calling thread). The context holds launch-shape tables and timing state only.
 * Returns OCSR_OK and *out, or a negative status. */
int32_t ocsr_ctx_create(int32_t device, ocsr_ctx** out);
void ocsr_ctx_destroy(ocsr_ctx* ctx);

/* ------------------------------------------------------------------------------ */
/* Census transform (Sec. 4.3.1, census equation; Alg. 1)                           */
/* ------------------------------------------------------------------------------ */
/* Window (2 sx + 1) wide and (2 sy + 1) tall, sx, sy >= 0. Level `scale` >= 1 samples
 * the source at (scale x, scale y): the output has floor(W/scale) x floor(H/scale)
 * words. Bit order is Alg. 1's: the word starts as the sentinel (1, or 0 when
 * sentinel == 0), then for i = -sx..sx (outer), j = -sy..sy (inner) it shifts left by
 * one and appends [I(x+i, y+j) > I(x, y)]. The centre term is included (always 0).
 * A pixel whose window leaves the level image stores 0. Requires
 * (2sx+1)(2sy+1) + (sentinel != 0) <= 64, else OCSR_E_UNSUPPORTED. */
typedef struct {
  int32_t sx, sy;
  int32_t scale;
  int32_t sentinel;
} ocsr_census_params;

/* img (dev): uint8 [H][pitch_bytes], W <= pitch_bytes. out (dev): uint64 rows of
 * out_pitch_elems >= W/scale words, H/scale rows. */
int32_t ocsr_census(ocsr_ctx* ctx, const uint8_t* img, int32_t width, int32_t height,
                    int32_t pitch_bytes, const ocsr_census_params* params, uint64_t* out,
                    int32_t out_pitch_elems, void* stream);

/* Several census transforms in one launch (e.g. both views at both levels of a
 * frame). jobs (host): n_jobs descriptions; every job uses params' window and
 * sentinel and its own scale. n_jobs <= OCSR_MAX_CENSUS_JOBS. */
#define OCSR_MAX_CENSUS_JOBS 64
typedef struct {
  const uint8_t* img;      /* dev, uint8 [height][pitch_bytes] */
  uint64_t* out;           /* dev, uint64 [height/scale][out_pitch_elems] */
  int32_t width, height, pitch_bytes, out_pitch_elems;
  int32_t scale;
  int32_t reserved;
} ocsr_census_job;
int32_t ocsr_census_many(ocsr_ctx* ctx, const ocsr_census_job* jobs, int32_t n_jobs,
                         int32_t sx, int32_t sy, int32_t sentinel, void* stream);

/* ------------------------------------------------------------------------------ */
/* Object-centric matching (Sec. 4.3.2-4.3.6, Alg. 2)                               */
/* ------------------------------------------------------------------------------ */
/* Descriptors of one level: both views, same geometry. W, H are the level size
 * (floor of the image size / scale); pitch_elems >= W. sx, sy: the census window the
 * descriptors were made with (the matcher only uses pixels whose census is defined). */
typedef struct {
  const uint64_t* L;       /* dev */
  const uint64_t* R;       /* dev */
  int32_t width, height, pitch_elems;
  int32_t scale;
  int32_t sx, sy;
} ocsr_level;

/* Detection box in full-resolution pixels, half-open [x0, x1) x [y0, y1). */
typedef struct {
  int32_t x0, y0, x1, y1;
  uint32_t flags;          /* OCSR_BOX_RANGE: produce a range; every box may occlude */
} ocsr_box;

/* One matching path (Sec. 4.3.4). Disparity range [dmin, dmax] in full-res px,
 * 0 <= dmin <= dmax; a path on level s searches level disparities
 * floor(dmin/s) .. floor(dmin/s) + ceil((dmax - dmin + 1)/s) - 1, at most
 * OCSR_MAX_CANDIDATES of them. TILED: 1 <= bw * bh <= 64. GRID: 1 <= n_side <= 8. */
typedef struct {
  int32_t mode;
  int32_t bw, bh;
  int32_t n_side;
  int32_t dmin, dmax;
} ocsr_path;

typedef struct {
  uint32_t struct_size;    /* sizeof(ocsr_match_params) */
  int32_t tau_s;           /* FAR iff max(clipped width, height) < tau_s (Sec. 4.3.4) */
  ocsr_path far_path;      /* FAR boxes: level 0 (scale 1) */
  ocsr_path close_path;    /* CLOSE boxes: level 1 (scale s, e.g. 2) */
  int32_t lr_tol;          /* a block passes the L/R check (Sec. 4.3.3) iff
                            * |d_b - d_f| <= lr_tol, counted in level px of the block's
                            * path (on a close level of scale s, lr_tol 1 allows s
                            * full-res px). The paper's strict |dx_v| < tau_v on integer
                            * residuals is lr_tol = tau_v - 1 (lr_tol 0 for tau_v 1). */
  int32_t min_point_pct;   /* block eligible iff points > 0 and 100 points >= pct nx ny */
  int32_t agg_mode;        /* OCSR_AGG_* */
  float tau_d;             /* segment gap threshold, full-res px */
  int32_t n_min;           /* fewest blocks an aggregate may rest on */
  int32_t trim_pct;        /* 0..49, TRIMMED_MEDIAN only */
  float focal_px;          /* f */
  float baseline_m;        /* b */
  float d_eps;             /* disparity <= d_eps: NONPOSITIVE_DISPARITY */
  /* Vertical offsets searched together with the disparity, full-res px (the census
   * cost of Sec. 4.3.2 over (dx, dy)); dy_min = dy_max = 0 searches dy = 0 only.
   * -OCSR_MAX_DY <= dy_min <= dy_max <= OCSR_MAX_DY. A path on level s searches the
   * level offsets floor(dy_min/s) .. ceil(dy_max/s) (its ndy values); the forward
   * winner is the least cost over (d, dy), ties to the smaller d, then the smaller dy.
   * The backward search starts at the forward match (x - d_f, y + dy_f) and visits
   * (d, dy) at (x - d_f + d, y + dy_f - dy); the L/R check compares d_b with d_f only.
   * Limits with a vertical range: nd * ndy <= OCSR_MAX_DY_CANDIDATES per path, and
   * the path's working set must fit a workgroup's LDS (an 8 x 8 path takes up to 21
   * level offsets with 96 candidates, 12 with 128, and at most 160 candidates); beyond
   * them the call returns OCSR_E_UNSUPPORTED. Rows outside
   * the level image read as all-zero descriptors, as columns do. */
  int32_t dy_min, dy_max;
} ocsr_match_params;

typedef struct {
  float disparity;         /* full-res px (0 unless aggregation succeeded) */
  float depth;             /* Z = f b / disparity, metres (0 unless valid) */
  int32_t valid;           /* 1 iff reason == OCSR_REASON_OK */
  int32_t reason;          /* OCSR_REASON_* */
  int32_t n_blocks;        /* blocks the box was tiled into */
  int32_t n_eligible;      /* blocks with enough unoccluded points */
  int32_t n_valid;         /* eligible blocks that passed the L/R check */
  int32_t n_used;          /* blocks the aggregate rests on */
} ocsr_box_result;

/* Per-block record of the debug output, blocks numbered box by box, then by block
 * row and column (a box's blocks are contiguous). */
typedef struct {
  int32_t box, level_scale, u, v;
  int32_t px0, py0, nx, ny;   /* level position of point 0; point grid nx x ny */
  uint64_t mask;              /* bit j*nx+i: point (i, j) unoccluded */
  int32_t eligible, d_f, d_b, lr_ok;
  float d_sub;                /* sub-pixel forward disparity, level px */
  int32_t valid;
  int32_t dlo, nd;            /* level search range [dlo, dlo + nd) */
  int32_t dy_f, dy_b;         /* level vertical offsets of the forward and backward winners */
} ocsr_block_record;

/* Optional debug outputs of ocsr_match_boxes (any pointer may be NULL). Blocks
 * numbered >= cap_blocks are not recorded; costs hold cap_nd entries per block. */
typedef struct {
  int32_t cap_blocks, cap_nd;
  int32_t* n_blocks;              /* dev, 1 int: blocks numbered (incl. overflowed boxes) */
  ocsr_block_record* blocks;      /* dev, [cap_blocks] */
  uint16_t* cost_fwd;             /* dev, [cap_blocks][cap_nd]: S_f(dlo + k) at dy_f */
  uint16_t* cost_bwd;             /* dev, [cap_blocks][cap_nd]: S_b(dlo + k) at dy_b */
} ocsr_debug;

/* Workspace of ocsr_match_boxes for up to n_boxes boxes and cap_blocks blocks in
 * total. Blocks are numbered by a prefix over the boxes in order; a box whose
 * range of numbers passes cap_blocks (and every box after it) is reported
 * CAPACITY_OVERFLOW. That is the only limit on a box's blocks: the aggregation of
 * Sec. 4.3.4 takes every valid block of a box, however many (boxes of more than 4096
 * blocks are aggregated from the workspace instead of on-chip memory). cap_blocks
 * <= 2^24. */
size_t ocsr_match_workspace_bytes(int32_t n_boxes, int32_t cap_blocks);

/* Matches every ranged box. lv0 (host struct, dev arrays): descriptors of level 0,
 * scale 1, used by the FAR path. lv1: the level used by the CLOSE path (its scale
 * is the close level's s); required -- a caller whose boxes are all FAR may pass
 * lv0 again. boxes (dev): [n_boxes]. out (dev): [n_boxes]. ws (dev): at least
 * ocsr_match_workspace_bytes(n_boxes, cap_blocks) bytes, 256-byte aligned; its
 * contents on entry do not matter. dbg: NULL for no debug output. */
int32_t ocsr_match_boxes(ocsr_ctx* ctx, const ocsr_level* lv0, const ocsr_level* lv1,
                         const ocsr_box* boxes, int32_t n_boxes,
                         const ocsr_match_params* params, int32_t cap_blocks,
                         void* ws, size_t ws_bytes, ocsr_box_result* out,
                         const ocsr_debug* dbg, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ocsr_match_boxes with its scratch in
 * a library-owned device array of OCSR_NOALLOC_SCRATCH_BYTES per device instead of a
 * caller workspace. The array is made when the library's code is loaded on a device and
 * held until the process ends; its device address is resolved once per device by
 * ocsr_ctx_create. The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine, and no timing events: the context's timing does not cover it).
 * Same arguments, results and errors as ocsr_match_boxes without ws and ws_bytes;
 * OCSR_E_CAPACITY when ocsr_match_workspace_bytes(n_boxes, cap_blocks) exceeds
 * OCSR_NOALLOC_SCRATCH_BYTES (cap_blocks above 670 656 with 64 boxes).
 * Every call on a device shares that device's array, which keeps the last call's
 * contents (the kernels write every counter they read, so no clearing is needed):
 * calls that overlap on one device (two host threads, or two streams without an order
 * between them) race and give undefined results. */
#define OCSR_NOALLOC_SCRATCH_BYTES (16u << 20)
int32_t ocsr_match_boxes_noalloc(ocsr_ctx* ctx, const ocsr_level* lv0, const ocsr_level* lv1,
                                 const ocsr_box* boxes, int32_t n_boxes,
                                 const ocsr_match_params* params, int32_t cap_blocks,
                                 ocsr_box_result* out, const ocsr_debug* dbg, void* stream);

/* ------------------------------------------------------------------------------ */
/* Per-box 3D point and covariance (Sec. 4.3.6 Q-matrix equation; Sec. 4.3.7 depth  */
/* variance and covariance rotation equations)                                      */
/* ------------------------------------------------------------------------------ */
/* Camera geometry of the point step. The box's image point (u, v) is the centre of
 * its box clipped to the width x height image, in pixel-index coordinates:
 * u = (cx0 + cx1 - 1) / 2, v = (cy0 + cy1 - 1) / 2. */
typedef struct {
  int32_t width, height;   /* full-resolution image size */
  double Q[16];            /* 4x4 reprojection matrix of the rectified pair, row-major */
  double R[9];             /* rotation of T_cam->imu, row-major */
  double t[3];             /* translation of T_cam->imu */
  double focal_px;         /* f of the depth variance */
  double baseline_m;       /* b of the depth variance */
  double var_d;            /* sigma_d^2: the configured disparity variance, px^2 */
  double var_x, var_y;     /* sigma_x^2, sigma_y^2: lateral variances in the camera frame */
} ocsr_point_params;

typedef struct {
  float p_cam[3];          /* (X, Y, Z) / W with (X, Y, Z, W) = Q (u, v, d, 1) */
  float p_imu[3];          /* R p_cam + t */
  float cov_imu[6];        /* R diag(var_x, var_y, var_z) R^T: xx, xy, xz, yy, yz, zz */
  float var_z;             /* Z^4 var_d / (f^2 b^2), Z = p_cam[2] */
  int32_t valid;           /* 1 iff the box result is valid, its clipped box is not
                            * empty and W != 0; otherwise every field is 0 */
  int32_t reserved[2];
} ocsr_box_point;

/* One 3D point per box from its aggregated disparity d = results[i].disparity
 * (full-resolution px). boxes, results (dev): [n_boxes], as given to or returned by a
 * ranging call. pp (host). out (dev): [n_boxes]. Computed in fp32 from the parameters
 * rounded to fp32. OCSR_E_INVALID for n_boxes < 0, null pointers with n_boxes > 0, a
 * non-positive image size, f or b, or a negative variance. */
int32_t ocsr_box_points(ocsr_ctx* ctx, const ocsr_box* boxes, const ocsr_box_result* results,
                        int32_t n_boxes, const ocsr_point_params* pp, ocsr_box_point* out,
                        void* stream);

/* ------------------------------------------------------------------------------ */
/* Whole frame: census of both views at both levels, then matching (Alg. 2)         */
/* ------------------------------------------------------------------------------ */
/* Census window and the close level's scale of a frame. */
typedef struct {
  int32_t sx, sy, sentinel;
  int32_t close_scale;     /* >= 1 */
} ocsr_frame_params;

size_t ocsr_frame_workspace_bytes(int32_t width, int32_t height,
                                  const ocsr_frame_params* fp, int32_t n_boxes,
                                  int32_t cap_blocks);

/* imgL, imgR (dev): uint8 [height][pitch_bytes]. Same outputs as ocsr_match_boxes.
 *
 * The workspace starts with the frame's four descriptor images, each 256-byte aligned
 * and row-contiguous at its level width: L and R at scale 1, then L and R at the close
 * scale (level size = floor(size / close_scale)). Per level, a ranged box of that level's
 * type (Sec. 4.3.4) lies on the level rectangle [x0, x1) x [y0, y1) of its eligible
 * pixels, and for candidates dlo..dhi its searches read the right view on
 * [x0 - dhi, x1 - dlo) and the left view on [x0 - (dhi - dlo), x1 + (dhi - dlo)), rows
 * [y0, y1); with level vertical offsets eylo..eyhi (a vertical range) the right view's
 * rows are [y0 + eylo, y1 + eyhi) and the left view's [y0 - (eyhi - eylo),
 * y1 + (eyhi - eylo)). By default (OCSR_OPTION_FULL_CENSUS 0) the call makes the descriptors of
 * every 64 x 32 tile (tiles start at multiples of 64 and 32) that meets such a range
 * of some box, and leaves the rest of the images undefined; with the option on, of
 * every tile. */
int32_t ocsr_range_frame(ocsr_ctx* ctx, const uint8_t* imgL, const uint8_t* imgR,
                         int32_t width, int32_t height, int32_t pitch_bytes,
                         const ocsr_frame_params* fp, const ocsr_box* boxes,
                         int32_t n_boxes, const ocsr_match_params* params,
                         int32_t cap_blocks, void* ws, size_t ws_bytes,
                         ocsr_box_result* out, void* stream);

/* ------------------------------------------------------------------------------ */
/* Batch of frames in one launch sequence (Alg. 2 over many frames)                 */
/* ------------------------------------------------------------------------------ */
/* One frame of a batch. Frames may differ in size; every frame uses the same census
 * window, close scale and matching parameters. Its boxes are
 * boxes[box_offset .. box_offset + n_boxes) of the batch's box array, and its results
 * land at the same positions of the output array. */
typedef struct {
  const uint8_t* imgL;     /* dev, uint8 [height][pitch_bytes] */
  const uint8_t* imgR;     /* dev, same geometry */
  int32_t width, height, pitch_bytes;
  int32_t box_offset, n_boxes;
  int32_t reserved;
} ocsr_frame;

/* Workspace of ocsr_range_batch: the four descriptor images of every frame, the plan
 * of every box and cap_blocks blocks per frame. frames (host): n_frames entries; only
 * their sizes and box counts are read (image pointers may be NULL). Returns 0 for an
 * invalid description. */
size_t ocsr_batch_workspace_bytes(const ocsr_frame* frames, int32_t n_frames,
                                  const ocsr_frame_params* fp, int32_t cap_blocks);

/* Ranges every box of up to OCSR_MAX_BATCH_FRAMES frames. Results are those of one
 * ocsr_range_frame call per frame, bit for bit. frames (host): n_frames entries; boxes
 * (dev) and out (dev): the total box count of the batch, frame by frame. */
int32_t ocsr_range_batch(ocsr_ctx* ctx, const ocsr_frame* frames, int32_t n_frames,
                         const ocsr_frame_params* fp, const ocsr_box* boxes,
                         const ocsr_match_params* params, int32_t cap_blocks, void* ws,
                         size_t ws_bytes, ocsr_box_result* out, void* stream);

/* ------------------------------------------------------------------------------ */
/* Priority object selection under a budget (Sec. 4.3.5, last sentence)           */
/* ------------------------------------------------------------------------------ */
/* When a frame has more candidate objects than the budget, those in a central crop
 * (frontal) take precedence and what is left of the budget goes to the others, nearest
 * first. A candidate is a box with OCSR_BOX_RANGE whose clipped area is not empty.
 * Candidates are ordered by the key (not frontal, larger clipped bottom y first, lower
 * box index first): a larger bottom y is nearer the camera, the cue the occlusion rule
 * uses. Frontal: the centre of the clipped box, ((cx0 + cx1 - 1)/2, (cy0 + cy1 - 1)/2),
 * lies in the crop [floor(W x0/1000), floor(W x1/1000)) x [floor(H y0/1000),
 * floor(H y1/1000)), given in permille of the frame size. */
typedef struct {
  int32_t max_objects;        /* budget per frame: candidates kept ranged, >= 0 */
  int32_t crop_permille[4];   /* x0, y0, x1, y1; 0 <= x0 <= x1 <= 1000, same for y */
} ocsr_select_params;

/* Most boxes of one frame ocsr_select_boxes takes. */
#define OCSR_MAX_SELECT_BOXES 16384

/* frames (host): n_frames descriptions; only width, height, box_offset and n_boxes are
 * read (images may be NULL). in (dev): the frames' boxes. out (dev): the same boxes,
 * each candidate whose rank is >= max_objects with OCSR_BOX_RANGE cleared (it still
 * occludes); every other field and box as in `in`. out must not overlap in. rank (dev,
 * nullable): int32 per box, the candidate's rank in its frame (0 first), -1 for boxes
 * that are not candidates. n_boxes per frame <= OCSR_MAX_SELECT_BOXES, else
 * OCSR_E_CAPACITY. */
int32_t ocsr_select_boxes(ocsr_ctx* ctx, const ocsr_frame* frames, int32_t n_frames,
                          const ocsr_box* in, const ocsr_select_params* params, ocsr_box* out,
                          int32_t* rank, void* stream);

/* ------------------------------------------------------------------------------ */
/* Dense counterpart                                                                */
/* ------------------------------------------------------------------------------ */
/* Not part of the paper's method: the dense matcher the object-centric path is
 * measured against, on the same descriptors and Hamming cost. For every pixel and
 * every d in [dmin, dmax]: C(x, y, d) = sum over the (2 radius + 1)^2 window around
 * (x, y), clipped to the image, of popcount(CL(x', y') ^ CR(x' - d, y')) (CR reads
 * outside the image are 0). d_L(x, y) is the smallest d minimising C(x, y, d);
 * d_R(xr, y) the smallest d minimising C(xr + d, y, d) over d with xr + d < width
 * (-1 if none). disp(x, y) = d_L where x - d_L >= 0, d_R(x - d_L, y) >= 0 and
 * |d_L - d_R(x - d_L, y)| <= lr_tol, else -1.
 *
 * lv (host struct, dev descriptors): one level's left/right descriptors (any scale).
 * 0 <= dmin <= dmax, dmax - dmin < OCSR_MAX_CANDIDATES; radius 1..3 (else
 * OCSR_E_UNSUPPORTED); lr_tol >= 0. disp (dev): int16 [height][width], row-contiguous;
 * disp_right (dev, nullable): receives d_R. ws: ocsr_dense_workspace_bytes() bytes. */
size_t ocsr_dense_workspace_bytes(int32_t width, int32_t height);
int32_t ocsr_dense_match(ocsr_ctx* ctx, const ocsr_level* lv, int32_t dmin, int32_t dmax,
                         int32_t radius, int32_t lr_tol, int16_t* disp, int16_t* disp_right,
                         void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------ */
/* Auto-rectification offset (Sec. 5.1)                                             */
/* ------------------------------------------------------------------------------ */
/* For every integer vertical offset delta in [delta_min, delta_max] the dense matcher
 * above runs on a region of interest whose left descriptors are moved down by delta:
 * the pair (CL(roi_x0 + x, roi_y0 + y - delta), CR(roi_x0 + x, roi_y0 + y)) for
 * 0 <= x < roi_w, 0 <= y < roi_h, its windows clipped to the ROI. counts[k] is the
 * number of ROI pixels whose checked disparity is > d_min at delta = delta_min + k: the
 * quantity the offset search maximises (Sec. 5.1, offset equation). The paper's
 * matcher there is block matching; this library's dense census matcher stands in for
 * it. The paper runs one stream per offset; here every offset is one slice of the same
 * launches. */
typedef struct {
  int32_t roi_x0, roi_y0, roi_w, roi_h;   /* level px; rows roi_y0 - delta must stay inside */
  int32_t delta_min, delta_max;           /* level px, delta_max - delta_min < OCSR_MAX_RECT_OFFSETS */
  int32_t dmin, dmax, radius, lr_tol;     /* the dense matcher's range, window, L/R tolerance */
  int32_t d_min;                          /* >= 0: pixels with disparity > d_min count */
} ocsr_rect_params;
#define OCSR_MAX_RECT_OFFSETS 64

/* Bytes of the workspace of ocsr_rect_offset_counts (0 if p is invalid). */
size_t ocsr_rect_workspace_bytes(const ocsr_rect_params* p);
/* lv (host struct, dev descriptors): one level; the ROI moved by every offset lies inside
 * it (else OCSR_E_INVALID). counts (dev): int32 [n_offsets]. disp (dev, nullable): int16
 * [n_offsets][roi_h][roi_w], the checked disparity maps (-1: invalid). */
int32_t ocsr_rect_offset_counts(ocsr_ctx* ctx, const ocsr_level* lv, const ocsr_rect_params* p,
                                int32_t* counts, int16_t* disp, void* ws, size_t ws_bytes,
                                void* stream);

/* The per-frame estimate and its temporal filter (Sec. 5.1, filter equations), on the
 * host. The estimate delta* is the offset of the largest count; ties go to the smallest
 * |delta|, then to the smaller delta. The filter keeps the last `window` estimates; its
 * output moves from the previous output towards their median (the lower middle value
 * of an even count) by at most max_step per frame. The first previous output is
 * `initial`. */
typedef struct ocsr_rect_filter ocsr_rect_filter;
int32_t ocsr_rect_filter_create(int32_t window, int32_t max_step, int32_t initial,
                                ocsr_rect_filter** out);
void ocsr_rect_filter_destroy(ocsr_rect_filter* f);
/* counts (host): n_offsets counts of one frame for offsets delta_min, delta_min + 1, ...
 * Writes the frame's estimate to *raw and the filtered offset to *filtered. */
int32_t ocsr_rect_filter_update(ocsr_rect_filter* f, const int32_t* counts, int32_t n_offsets,
                                int32_t delta_min, int32_t* raw, int32_t* filtered);

/* ------------------------------------------------------------------------------ */
/* Options and timing                                                               */
/* ------------------------------------------------------------------------------ */
/* OCSR_OPTION_FUSED: 0 (default) runs whole frames and batches as the multi-launch
 * sequence (census of every view and level of every frame, plan, one match launch per
 * level, aggregation); 1 runs them as one persistent launch of co-resident workgroups
 * (census, planning, matching and aggregation in three phases split by grid barriers)
 * when a fused kernel is built for the census window and path shapes, else falls back
 * to the multi-launch sequence. Both give identical results. */
#define OCSR_OPTION_FUSED 1
/* OCSR_OPTION_WAVES_PER_CU: cap on the workgroups per compute unit of the persistent
 * launch (0 = the library's default, 2; 1..32 = cap; never more than fit). */
#define OCSR_OPTION_WAVES_PER_CU 2
/* OCSR_OPTION_MATCH_WGS_PER_CU: workgroups per compute unit of the grid of each matching
 * launch (1..64, default 16). The launch deals its work items over this grid. */
#define OCSR_OPTION_MATCH_WGS_PER_CU 4
/* OCSR_OPTION_BLOCKS_PER_WAVE: blocks each wave of a matching workgroup takes per work
 * item (1..8, default 1); a work item holds 4 x this many blocks of one box. */
#define OCSR_OPTION_BLOCKS_PER_WAVE 5
/* OCSR_OPTION_GRAPH: 1 submits whole-frame and batch calls (ocsr_range_frame,
 * ocsr_range_batch) as HIP graphs: the first call with a given set of arguments
 * (every frame description, device pointer, size, parameter and option) captures its
 * launches and instantiates them, and later calls with the same arguments replay the
 * instantiated graph with a single submission. Up to 128 graphs are kept per context,
 * least recently used dropped first. The kernels read their inputs at replay time,
 * so new image or box contents at the same addresses are picked up; a change of any
 * address or size captures a new graph. Results are identical to 0 (default). */
#define OCSR_OPTION_GRAPH 3
/* OCSR_OPTION_FULL_CENSUS: whole-frame and batch calls make the descriptors of a view
 * and level only on the 64 x 32 level-pixel tiles that some ranged box's search reads
 * (0, default), or on every tile (1). Box results are identical either way; the
 * option only decides which workspace descriptors are defined after the call (see
 * ocsr_range_frame). */
#define OCSR_OPTION_FULL_CENSUS 6
/* OCSR_OPTION_CENSUS_TILE_LIST: 1 (default) lets whole-frame and batch calls with at
 * least 8 tiles of 64 x 32 level pixels per resident workgroup slot of the GPU (and at
 * most 131072 tiles in any frame) make the census with persistent workgroups, one per
 * slot, that each list the tiles to make from the boxes and take an equal share of
 * them; other calls, and every call with 0, launch one workgroup per tile, which makes
 * its tile or leaves. Results and the tiles made are the same either way. */
#define OCSR_OPTION_CENSUS_TILE_LIST 7
/* OCSR_OPTION_LEVEL_LAUNCHES: how the blocks of the two levels are matched. 0 (default):
 * one launch for both levels in calls of one frame when a kernel for the pair of chosen
 * variants is built, one launch per level otherwise; 1: always one launch per level;
 * 2: one launch for both levels whenever such a kernel is built. Results are identical
 * either way. */
#define OCSR_OPTION_LEVEL_LAUNCHES 8
int32_t ocsr_ctx_set_option(ocsr_ctx* ctx, int32_t option, int32_t value);

/* ------------------------------------------------------------------------------ */
/* Matching kernel variants (for tuners)                                            */
/* ------------------------------------------------------------------------------ */
/* A TILED path's blocks run in one of three kernel families, named by (rows, cpl,
 * passes):
 *   rows = 1: four blocks of up to 4 x 4 points per wave, 16 lanes per block, each lane
 *             `cpl` consecutive candidates over all of its block's points (16 * cpl
 *             candidates, passes = 1);
 *   rows = 2: one block of up to 8 x 8 points per wave, lanes over 32 candidate groups
 *             of `cpl` consecutive candidates and the block's two halves of 4 rows
 *             (32 * cpl candidates, passes = 1);
 *   rows = 4 or 8: a register-blocked kernel with `rows` block rows per wave (blocks up
 *             to 4 x 4 or 8 x 8), `cpl` consecutive candidates per lane and `passes`
 *             passes over the candidates, covering (64 / rows) * cpl * passes candidates.
 * Any variant that covers a path gives identical results; they differ in speed only. By
 * default the first covering variant in the library's order of preference is used:
 * rows = 1 for blocks up to 4 x 4 and 32 or 64 candidates, rows = 2 for blocks up to
 * 8 x 8 and up to 128 candidates, else the register-blocked kernels.
 *
 * ocsr_variant_candidates: writes up to `cap` (rows, cpl, passes) triples (host arrays)
 * that cover bw x bh blocks and n_candidates level candidates; returns how many exist
 * (may exceed cap), or a negative status. */
int32_t ocsr_variant_candidates(int32_t bw, int32_t bh, int32_t n_candidates, int32_t* rows,
                                int32_t* cpl, int32_t* passes, int32_t cap);
/* Chooses the variant for paths of bw x bh blocks and n_candidates level candidates in
 * this context ((rows, cpl, passes) == (0, 0, 0) restores the default; (0, 4, 1) is the
 * generic kernel). OCSR_E_INVALID if the variant does not cover such a path. */
int32_t ocsr_ctx_set_variant(ocsr_ctx* ctx, int32_t bw, int32_t bh, int32_t n_candidates,
                             int32_t rows, int32_t cpl, int32_t passes);

/* Graph submissions of the context so far: replays of a cached graph (*hits) and
 * captures (*builds). Either pointer may be NULL. */
int32_t ocsr_ctx_graph_stats(ocsr_ctx* ctx, int64_t* hits, int64_t* builds);

/* When enabled, each kernel launch of the context is bracketed by HIP events on
 * its stream; ocsr_ctx_kernel_time() then reports, per kernel name, the number of
 * launches and their summed duration (ms) since the last reset. Reading
 * synchronizes on the recorded events. Kernel names: census (with the plan in
 * whole-frame calls), plan (descriptor-level calls), match (both levels in one launch),
 * match_close and match_far (one launch per level, when no kernel for the pair of
 * variants is built), aggregate, reset and fused (the persistent launch), graph (one
 * replay of a whole-frame or batch call with OCSR_OPTION_GRAPH on), dense and
 * dense_check (the dense counterpart), points (ocsr_box_points), select
 * (ocsr_select_boxes), rect_dense and rect_count (ocsr_rect_offset_counts). */
int32_t ocsr_ctx_set_timing(ocsr_ctx* ctx, int32_t enable);
int32_t ocsr_ctx_kernel_time(ocsr_ctx* ctx, const char* kernel, int64_t* launches,
                             double* total_ms);
int32_t ocsr_ctx_reset_timing(ocsr_ctx* ctx);

/* ------------------------------------------------------------------------------ */
/* Measurement                                                                      */
/* ------------------------------------------------------------------------------ */
/* Measures the int32 vector-ALU rate of the context's device, the peak the census and
 * matching kernels are priced against: every lane of 16 workgroups of 256 threads per
 * compute unit runs 8 independent chains of the matching cost arithmetic
 * (b = acc ^ b, acc = popcount(b) + acc: one v_xor_b32 and one v_bcnt_u32_b32 per step)
 * for `iters` steps, on the null stream, after three untimed launches. Synchronizes.
 * *ops_per_s: lane operations per second of the timed launch; *ms (nullable): its
 * duration. OCSR_E_INVALID for a null ctx or ops_per_s or iters outside 1..2^20. */
int32_t ocsr_measure_int_rate(ocsr_ctx* ctx, int32_t iters, double* ops_per_s, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* OCSR_H */
