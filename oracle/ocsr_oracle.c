/*
 * CPU oracle for the object-centric census template-matching path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the library. Plain scalar loops in
 * the order the paper states the method; OpenMP only splits independent
 * outer iterations (rows, boxes). Built with -ffp-contract=off so that every
 * fp32 operation below is one IEEE operation.
 *
 * Paper map:
 *   census ............ Sec. 4.3.1, census equation and Alg. 1
 *   block cost ........ Sec. 4.3.2, census cost equation, over (dx, dy) offsets
 *   sub-pixel ......... Sec. 4.3.2, parabola equation
 *   forward-backward .. Sec. 4.3.3
 *   far / close ....... Sec. 4.3.4, type equation, Alg. 2
 *   aggregation ....... Sec. 4.3.4, four aggregation steps
 *   occluders ......... Sec. 4.3.5
 *   depth ............. Eq. 1 (Z = f b / d), and d_full = s d_down (Sec. 4.1)
 *   3D point .......... Sec. 4.3.6, Q-matrix equation, then T_cam->imu
 *   covariance ........ Sec. 4.3.7, depth-variance and rotation equations
 *   object budget ..... Sec. 4.3.5, last sentence (frontal first, then proximity)
 *   rectification ..... Sec. 5.1, offset equation and filter equations
 */
#include "ocsr_oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

static int ceil_div_nonneg(int a, int s) { return (a + s - 1) / s; }
static int floor_div(int a, int s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }
static int ceil_div(int a, int s) { return -floor_div(-a, s); }
static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------------ */
/* Census (Sec. 4.3.1). Bit order follows Alg. 1: start from the sentinel, then   */
/* for i = -Sx..Sx (x, outer), j = -Sy..Sy (y, inner) shift left and append       */
/* [I(x+i, y+j) > I(x, y)]. Level s samples the source at (s x, s y): the census  */
/* image is smaller and its coordinates are scaled (Sec. 4.3.1, last paragraph).  */
/* A pixel whose window leaves the level image is undefined and stores 0.         */
/* ------------------------------------------------------------------------------ */
int32_t orc_census(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                   int32_t sx, int32_t sy, int32_t s, int32_t sentinel, uint64_t* out) {
  if (!img || !out || W <= 0 || H <= 0 || s <= 0 || sx < 0 || sy < 0 || pitch < W) return -1;
  int nbits = (2 * sx + 1) * (2 * sy + 1) + (sentinel ? 1 : 0);
  if (nbits > 64) return -1;
  int Ws = W / s, Hs = H / s;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Hs; ++y) {
    for (int x = 0; x < Ws; ++x) {
      uint64_t code = 0;
      int defined = (x >= sx) && (x < Ws - sx) && (y >= sy) && (y < Hs - sy);
      if (defined) {
        uint8_t center = img[(size_t)(s * y) * pitch + (size_t)(s * x)];
        code = sentinel ? 1u : 0u;
        for (int i = -sx; i <= sx; ++i) {
          for (int j = -sy; j <= sy; ++j) {
            uint8_t nb = img[(size_t)(s * (y + j)) * pitch + (size_t)(s * (x + i))];
            code = (code << 1) | (uint64_t)(nb > center ? 1 : 0);
          }
        }
      }
      out[(size_t)y * Ws + x] = code;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Sparse matching                                                                 */
/* ------------------------------------------------------------------------------ */
typedef struct {
  const uint64_t *L, *R;
  int W, H;      /* level size */
  int s;
} level_t;

/* descriptor read; outside the level image reads as 0 */
static uint64_t rd(const level_t* lv, const uint64_t* img, int x, int y) {
  if (x < 0 || y < 0 || x >= lv->W || y >= lv->H) return 0;
  return img[(size_t)y * lv->W + x];
}

typedef struct {
  int cx0, cy0, cx1, cy1;   /* clipped full-res box */
  int empty;
} clip_t;

static int boxes_overlap(const clip_t* a, const clip_t* b) {
  return !a->empty && !b->empty && a->cx0 < b->cx1 && b->cx0 < a->cx1 &&
         a->cy0 < b->cy1 && b->cy0 < a->cy1;
}

/* S(P, dx, dy) of the census-cost equation with dx = -d, over the masked points.
 * dir = +1: forward, template CL at p, search CR at (p.x - d, p.y + e).
 * dir = -1: backward, template CR at the forward match q = (p.x - d_f, p.y + e_f),
 *           search CL at (q.x + d, q.y - e), so that (d, e) = (d_f, e_f) returns to p. */
static int block_cost(const level_t* lv, const int* xs, const int* ys, int nx, int ny,
                      uint64_t mask, int dir, int d, int e, int d_f, int e_f) {
  int sum = 0;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      int k = j * nx + i;
      if (!((mask >> k) & 1u)) continue;
      uint64_t a, b;
      if (dir > 0) {
        a = rd(lv, lv->L, xs[i], ys[j]);
        b = rd(lv, lv->R, xs[i] - d, ys[j] + e);
      } else {
        a = rd(lv, lv->R, xs[i] - d_f, ys[j] + e_f);
        b = rd(lv, lv->L, xs[i] - d_f + d, ys[j] + e_f - e);
      }
      sum += popcount64(a ^ b);
    }
  }
  return sum;
}

static int cmp_float(const void* a, const void* b) {
  float x = *(const float*)a, y = *(const float*)b;
  return (x > y) - (x < y);
}

/* median of v[0..m-1] (sorted): odd m -> middle; even m -> mean of the two middle */
static float median_sorted(const float* v, int m) {
  if (m & 1) return v[(m - 1) / 2];
  return (v[m / 2 - 1] + v[m / 2]) * 0.5f;
}

/* Per-box aggregation (Sec. 4.3.4) and depth (Eq. 1). vals: the full-res
 * disparities of the valid blocks (sorted in place). n_blocks: blocks the box was
 * tiled into; far_object: the box is of type FAR; r->n_eligible must be set by the
 * caller. */
void orc_aggregate(float* vals, int32_t n_valid, int32_t n_blocks, int32_t far_object,
                   const orc_params* p, orc_box_result* r) {
  r->n_valid = n_valid;
  r->n_blocks = n_blocks;
  r->disparity = 0.0f; r->depth = 0.0f; r->valid = 0; r->n_used = 0;
  if (r->n_eligible == 0) { r->reason = ORC_NO_ELIGIBLE_BLOCKS; return; }
  if (n_valid == 0) { r->reason = ORC_NO_VALID_BLOCKS; return; }
  float d_box;
  if (far_object && n_blocks == 1) {
    /* Alg. 2: a FAR object matched as a single block takes that block's result;
     * CLOSE objects always go through the robust aggregation below */
    d_box = vals[0];
    r->n_used = 1;
  } else {
    qsort(vals, (size_t)n_valid, sizeof(float), cmp_float);  /* step 1: sort */
    if (p->agg_mode == ORC_AGG_SEGMENT_MEDIAN) {
      /* step 2: longest run whose consecutive differences stay below tau_d;
       * the first such run wins a tie */
      int best_start = 0, best_len = 1, start = 0;
      for (int k = 1; k <= n_valid; ++k) {
        if (k == n_valid || !(vals[k] - vals[k - 1] < p->tau_d)) {
          int len = k - start;
          if (len > best_len) { best_len = len; best_start = start; }
          start = k;
        }
      }
      r->n_used = best_len;
      /* step 3: at least N_min blocks */
      if (best_len < p->n_min) { r->reason = ORC_TOO_FEW_CONSISTENT; return; }
      d_box = median_sorted(vals + best_start, best_len);  /* step 4 */
    } else {
      /* symmetric trim of floor(pct * n / 100) values at each end, then the median */
      int t = p->trim_pct * n_valid / 100;
      int m = n_valid - 2 * t;
      r->n_used = m > 0 ? m : 0;
      if (m <= 0 || m < p->n_min) { r->reason = ORC_TOO_FEW_CONSISTENT; return; }
      d_box = median_sorted(vals + t, m);
    }
  }
  r->disparity = d_box;
  if (!(d_box > p->d_eps)) { r->reason = ORC_NONPOSITIVE_DISPARITY; return; }
  float fb = p->focal_px * p->baseline_m;  /* Z = f b / d */
  r->depth = fb / d_box;
  r->valid = 1;
  r->reason = ORC_OK;
}

typedef struct {
  int level;            /* 0 far (s = 1), 1 close */
  const orc_path* path;
  int s;
  int lx0, ly0, lw, lh; /* level box */
  int nbx, nby, bw, bh, ox, oy;
  int dlo, nd;
  int dylo, ndy;        /* level vertical offsets [dylo, dylo + ndy) */
  int n_blocks;
} plan_t;

static void plan_box(const orc_params* p, const clip_t* c, const level_t* lv0,
                     const level_t* lv1, plan_t* pl) {
  memset(pl, 0, sizeof(*pl));
  int side = imax(c->cx1 - c->cx0, c->cy1 - c->cy0);
  int far = side < p->tau_s;                       /* type equation, Sec. 4.3.4 */
  const level_t* lv = far ? lv0 : lv1;
  pl->level = far ? 0 : 1;
  pl->path = far ? &p->far_path : &p->close_path;
  pl->s = lv->s;
  int s = lv->s;
  /* level search range: the full-res range divided by s (Sec. 4.3.4, close path) */
  int dmin = pl->path->dmin, dmax = pl->path->dmax;
  pl->dlo = floor_div(dmin, s);
  pl->nd = ceil_div_nonneg(dmax - dmin + 1, s);
  /* level vertical range: the smallest level range whose full-res offsets s*e cover
   * [dy_min, dy_max] (a 2D offset search, Sec. 4.3.2); 0, 0 gives the single e = 0 */
  pl->dylo = floor_div(p->dy_min, s);
  pl->ndy = ceil_div(p->dy_max, s) - pl->dylo + 1;
  /* level pixels whose full-res position s*x lies in the box and whose census is defined */
  int x0 = imax(ceil_div(c->cx0, s), p->sx), x1 = imin(ceil_div(c->cx1, s), lv->W - p->sx);
  int y0 = imax(ceil_div(c->cy0, s), p->sy), y1 = imin(ceil_div(c->cy1, s), lv->H - p->sy);
  pl->lx0 = x0; pl->ly0 = y0; pl->lw = x1 - x0; pl->lh = y1 - y0;
  if (pl->lw <= 0 || pl->lh <= 0) { pl->lw = pl->lh = 0; pl->n_blocks = 0; return; }
  if (pl->path->mode == ORC_MODE_TILED) {
    pl->bw = imin(pl->path->bw, pl->lw);
    pl->bh = imin(pl->path->bh, pl->lh);
    pl->nbx = imax(1, pl->lw / pl->path->bw);
    pl->nby = imax(1, pl->lh / pl->path->bh);
    pl->ox = pl->lx0 + (pl->lw - pl->nbx * pl->bw) / 2;
    pl->oy = pl->ly0 + (pl->lh - pl->nby * pl->bh) / 2;
  } else {
    pl->nbx = pl->nby = 1;
    pl->bw = imin(pl->path->n_side, pl->lw);
    pl->bh = imin(pl->path->n_side, pl->lh);
  }
  pl->n_blocks = pl->nbx * pl->nby;
}

/* point columns / rows of block (u, v) */
static void block_points(const plan_t* pl, int u, int v, int* xs, int* ys, int* nx, int* ny) {
  if (pl->path->mode == ORC_MODE_TILED) {
    *nx = pl->bw; *ny = pl->bh;
    for (int i = 0; i < pl->bw; ++i) xs[i] = pl->ox + u * pl->bw + i;
    for (int j = 0; j < pl->bh; ++j) ys[j] = pl->oy + v * pl->bh + j;
  } else {
    /* regular grid over the whole box, one sample at the centre of each cell */
    *nx = pl->bw; *ny = pl->bh;
    for (int i = 0; i < pl->bw; ++i) xs[i] = pl->lx0 + (2 * i + 1) * pl->lw / (2 * pl->bw);
    for (int j = 0; j < pl->bh; ++j) ys[j] = pl->ly0 + (2 * j + 1) * pl->lh / (2 * pl->bh);
  }
}

int32_t orc_match_boxes(const uint64_t* L0, const uint64_t* R0,
                        const uint64_t* L1, const uint64_t* R1,
                        int32_t W, int32_t H, const int32_t* boxes, int32_t n,
                        const orc_params* p, orc_box_result* out,
                        orc_block* blocks, uint16_t* cost_f, uint16_t* cost_b,
                        int32_t cap_dbg, int32_t cap_nd, int32_t n_threads) {
  if (!L0 || !R0 || !p || !out || n < 0 || (n > 0 && !boxes) || W <= 0 || H <= 0) return -1;
  if (p->close_scale <= 0 || p->sx < 0 || p->sy < 0) return -1;
  if (p->dy_min > p->dy_max) return -1;
  {
    const orc_path* ps[2] = {&p->far_path, &p->close_path};
    for (int k = 0; k < 2; ++k) {
      const orc_path* q = ps[k];
      if (q->dmin < 0 || q->dmax < q->dmin) return -1;
      if (q->mode == ORC_MODE_TILED && (q->bw <= 0 || q->bh <= 0 || q->bw * q->bh > 64)) return -1;
      if (q->mode == ORC_MODE_GRID && (q->n_side <= 0 || q->n_side > 8)) return -1;
      if (q->mode != ORC_MODE_TILED && q->mode != ORC_MODE_GRID) return -1;
    }
  }
  level_t lv0 = {L0, R0, W, H, 1};
  level_t lv1 = {L1, R1, W / p->close_scale, H / p->close_scale, p->close_scale};
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif

  clip_t* clip = (clip_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(clip_t));
  plan_t* plan = (plan_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(plan_t));
  int* off = (int*)calloc((size_t)n + 1, sizeof(int));
  int* status = (int*)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
  for (int i = 0; i < n; ++i) {
    const int32_t* b = boxes + 5 * i;
    clip_t* c = &clip[i];
    c->cx0 = imax(b[0], 0); c->cy0 = imax(b[1], 0);
    c->cx1 = imin(b[2], W); c->cy1 = imin(b[3], H);
    c->empty = !(c->cx0 < c->cx1 && c->cy0 < c->cy1);
  }
  /* per-box status before matching, and the block prefix */
  long total = 0;
  for (int i = 0; i < n; ++i) {
    memset(&out[i], 0, sizeof(out[i]));
    off[i] = (int)total;
    if (!(boxes[5 * i + 4] & 1)) { status[i] = ORC_NOT_RANGED; continue; }
    if (clip[i].empty) { status[i] = ORC_CLIPPED_EMPTY; continue; }
    plan_box(p, &clip[i], &lv0, &lv1, &plan[i]);
    if (plan[i].level == 1 && (!L1 || !R1)) { free(clip); free(plan); free(off); free(status); return -1; }
    if (plan[i].n_blocks == 0) { status[i] = ORC_NO_ELIGIBLE_BLOCKS; continue; }
    /* the method sets no limit on a box's blocks; a caller may impose one */
    if (p->max_blocks_per_box > 0 && plan[i].n_blocks > p->max_blocks_per_box) {
      status[i] = ORC_CAPACITY_OVERFLOW;
      plan[i].n_blocks = 0;
      continue;
    }
    /* capacity rule: blocks are numbered by an unconditional prefix over the
     * boxes; a box whose range passes the capacity is not matched */
    if (p->cap_blocks > 0 && total + plan[i].n_blocks > p->cap_blocks) {
      status[i] = ORC_CAPACITY_OVERFLOW;
      total += plan[i].n_blocks;
      plan[i].n_blocks = 0;
      continue;
    }
    status[i] = -1; /* to be matched */
    total += plan[i].n_blocks;
  }
  off[n] = (int)total;

#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n; ++i) {
    orc_box_result* r = &out[i];
    if (status[i] >= 0) { r->reason = status[i]; continue; }
    const plan_t* pl = &plan[i];
    const level_t* lv = pl->level ? &lv1 : &lv0;
    int s = pl->s;
    r->n_blocks = pl->n_blocks;
    float* vals = (float*)malloc(sizeof(float) * (size_t)pl->n_blocks);
    int* fcost = (int*)malloc(sizeof(int) * (size_t)pl->nd);
    int* bcost = (int*)malloc(sizeof(int) * (size_t)pl->nd);
    int* fall = (int*)malloc(sizeof(int) * (size_t)pl->nd * (size_t)pl->ndy);  /* S at (k, e) */
    int n_valid = 0, n_elig = 0;
    for (int v = 0; v < pl->nby; ++v) {
      for (int u = 0; u < pl->nbx; ++u) {
        int bidx = off[i] + v * pl->nbx + u;
        int xs[64], ys[64], nx, ny;
        block_points(pl, u, v, xs, ys, &nx, &ny);
        /* occlusion-aware sampling (Sec. 4.3.5): drop points inside any box that
         * overlaps this one and has a larger bottom y */
        uint64_t mask = 0;
        for (int j = 0; j < ny; ++j) {
          for (int ii = 0; ii < nx; ++ii) {
            int fx = s * xs[ii], fy = s * ys[j];
            int hidden = 0;
            for (int o = 0; o < n && !hidden; ++o) {
              if (o == i) continue;
              if (!boxes_overlap(&clip[i], &clip[o])) continue;
              if (!(clip[o].cy1 > clip[i].cy1)) continue;
              if (fx >= clip[o].cx0 && fx < clip[o].cx1 && fy >= clip[o].cy0 && fy < clip[o].cy1)
                hidden = 1;
            }
            if (!hidden) mask |= (uint64_t)1 << (j * nx + ii);
          }
        }
        int npts = popcount64(mask);
        int eligible = npts > 0 && 100 * npts >= p->min_point_pct * nx * ny;
        int d_f = pl->dlo, d_b = pl->dlo, e_f = 0, e_b = 0, lr_ok = 0, valid = 0;
        float d_sub = (float)pl->dlo;
        if (eligible) {
          ++n_elig;
          /* forward: exhaustive search over (d, e), winner-take-all; ties go to the
           * smallest d, then the smallest e */
          int best = -1, ebest = 0, bestc = 0;
          for (int k = 0; k < pl->nd; ++k) {
            for (int ei = 0; ei < pl->ndy; ++ei) {
              int c = block_cost(lv, xs, ys, nx, ny, mask, +1, pl->dlo + k, pl->dylo + ei, 0, 0);
              fall[k * pl->ndy + ei] = c;
              if (best < 0 || c < bestc) { best = k; ebest = ei; bestc = c; }
            }
          }
          d_f = pl->dlo + best;
          e_f = pl->dylo + ebest;
          /* costs along d at the winning e (parabola and debug output) */
          for (int k = 0; k < pl->nd; ++k) fcost[k] = fall[k * pl->ndy + ebest];
          /* parabola through the forward costs at d_f - 1, d_f, d_f + 1 */
          if (best > 0 && best < pl->nd - 1) {
            int a = fcost[best - 1], c = fcost[best], b = fcost[best + 1];
            int num = a - b;
            int den = 2 * (a + b - 2 * c);
            float offs = (float)num / (float)den;
            d_sub = (float)d_f + offs;
          } else {
            d_sub = (float)d_f;
          }
          /* backward: templates at the matched right positions, search the left */
          int bbest = -1, bebest = 0, bbestc = 0;
          for (int k = 0; k < pl->nd; ++k) {
            for (int ei = 0; ei < pl->ndy; ++ei) {
              int c = block_cost(lv, xs, ys, nx, ny, mask, -1, pl->dlo + k, pl->dylo + ei, d_f, e_f);
              fall[k * pl->ndy + ei] = c;
              if (bbest < 0 || c < bbestc) { bbest = k; bebest = ei; bbestc = c; }
            }
          }
          d_b = pl->dlo + bbest;
          e_b = pl->dylo + bebest;
          for (int k = 0; k < pl->nd; ++k) bcost[k] = fall[k * pl->ndy + bebest];
          /* consistency on the horizontal offset only (Sec. 4.3.3) */
          lr_ok = abs(d_b - d_f) <= p->lr_tol;
          valid = lr_ok;
          if (valid) vals[n_valid++] = (float)s * d_sub;
          if (cost_f && bidx < cap_dbg)
            for (int k = 0; k < pl->nd && k < cap_nd; ++k) cost_f[(size_t)bidx * cap_nd + k] = (uint16_t)fcost[k];
          if (cost_b && bidx < cap_dbg)
            for (int k = 0; k < pl->nd && k < cap_nd; ++k) cost_b[(size_t)bidx * cap_nd + k] = (uint16_t)bcost[k];
        }
        if (blocks && bidx < cap_dbg) {
          orc_block* bk = &blocks[bidx];
          bk->box = i; bk->level_scale = s; bk->u = u; bk->v = v;
          bk->px0 = xs[0]; bk->py0 = ys[0]; bk->nx = nx; bk->ny = ny;
          bk->mask = mask; bk->eligible = eligible; bk->d_f = d_f; bk->d_b = d_b;
          bk->lr_ok = lr_ok; bk->d_sub = d_sub; bk->valid = valid;
          bk->dlo = pl->dlo; bk->nd = pl->nd;
          bk->dy_f = e_f; bk->dy_b = e_b;
        }
      }
    }
    r->n_eligible = n_elig;
    orc_aggregate(vals, n_valid, pl->n_blocks, pl->level == 0, p, r);
    free(vals); free(fcost); free(bcost); free(fall);
  }
  free(clip); free(plan); free(off); free(status);
  return (int32_t)total;
}

/* ------------------------------------------------------------------------------ */
/* Dense counterpart: every pixel, every disparity, (2r+1)^2 clipped box sum.      */
/* ------------------------------------------------------------------------------ */
static uint64_t rdd(const uint64_t* img, int W, int H, int x, int y) {
  if (x < 0 || y < 0 || x >= W || y >= H) return 0;
  return img[(size_t)y * W + x];
}

/* C(x, y, d): box sum of popcount(CL(x', y') ^ CR(x' - d, y')) over the window
 * clipped to the image */
static int dense_cost(const uint64_t* CL, const uint64_t* CR, int W, int H,
                      int x, int y, int d, int r) {
  int sum = 0;
  for (int v = -r; v <= r; ++v) {
    int yy = y + v;
    if (yy < 0 || yy >= H) continue;
    for (int u = -r; u <= r; ++u) {
      int xx = x + u;
      if (xx < 0 || xx >= W) continue;
      sum += popcount64(rdd(CL, W, H, xx, yy) ^ rdd(CR, W, H, xx - d, yy));
    }
  }
  return sum;
}

static int dense_left_wta(const uint64_t* CL, const uint64_t* CR, int W, int H,
                          int x, int y, int dmin, int dmax, int r) {
  int best = -1, bestc = 0;
  for (int d = dmin; d <= dmax; ++d) {
    int c = dense_cost(CL, CR, W, H, x, y, d, r);
    if (best < 0 || c < bestc) { best = d; bestc = c; }
  }
  return best;
}

/* right view: match of right pixel xr is left pixel xr + d */
static int dense_right_wta(const uint64_t* CL, const uint64_t* CR, int W, int H,
                           int xr, int y, int dmin, int dmax, int r) {
  int best = -1, bestc = 0;
  for (int d = dmin; d <= dmax; ++d) {
    int xl = xr + d;
    if (xl < 0 || xl >= W) continue;
    int c = dense_cost(CL, CR, W, H, xl, y, d, r);
    if (best < 0 || c < bestc) { best = d; bestc = c; }
  }
  return best;
}

int32_t orc_dense(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                  int32_t dmin, int32_t dmax, int32_t radius, int32_t lr_tol,
                  int16_t* disp, int16_t* disp_r, int32_t n_threads) {
  if (!CL || !CR || !disp || W <= 0 || H <= 0 || dmin < 0 || dmax < dmin || radius < 0) return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  int16_t* dl = (int16_t*)malloc(sizeof(int16_t) * (size_t)W * H);
  int16_t* dr = (int16_t*)malloc(sizeof(int16_t) * (size_t)W * H);
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      dl[(size_t)y * W + x] = (int16_t)dense_left_wta(CL, CR, W, H, x, y, dmin, dmax, radius);
      dr[(size_t)y * W + x] = (int16_t)dense_right_wta(CL, CR, W, H, x, y, dmin, dmax, radius);
    }
  }
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      int d = dl[(size_t)y * W + x];
      int xr = x - d;
      int ok = xr >= 0 && dr[(size_t)y * W + xr] >= 0 && abs(d - dr[(size_t)y * W + xr]) <= lr_tol;
      disp[(size_t)y * W + x] = (int16_t)(ok ? d : -1);
      if (disp_r) disp_r[(size_t)y * W + x] = dr[(size_t)y * W + x];
    }
  }
  free(dl); free(dr);
  return 0;
}

int32_t orc_dense_at(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                     int32_t dmin, int32_t dmax, int32_t radius, int32_t lr_tol,
                     const int32_t* xy, int32_t n, int16_t* out, int32_t n_threads) {
  if (!CL || !CR || !xy || !out || W <= 0 || H <= 0 || dmin < 0 || dmax < dmin || radius < 0) return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < n; ++k) {
    int x = xy[2 * k], y = xy[2 * k + 1];
    int d = dense_left_wta(CL, CR, W, H, x, y, dmin, dmax, radius);
    int xr = x - d;
    int ok = 0;
    if (xr >= 0) {
      int db = dense_right_wta(CL, CR, W, H, xr, y, dmin, dmax, radius);
      ok = db >= 0 && abs(d - db) <= lr_tol;
    }
    out[k] = (int16_t)(ok ? d : -1);
  }
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Per-box 3D point (Sec. 4.3.6) and covariance (Sec. 4.3.7), fp64.               */
/* ------------------------------------------------------------------------------ */
void orc_box_points(const int32_t* boxes, const orc_box_result* res, int32_t n, int32_t W,
                    int32_t H, const double* Q, const double* R, const double* t, double f,
                    double b, double var_d, double var_x, double var_y, orc_point* out) {
  for (int i = 0; i < n; ++i) {
    orc_point o;
    memset(&o, 0, sizeof(o));
    const int32_t* bx = boxes + 5 * i;
    const int cx0 = imax(bx[0], 0), cy0 = imax(bx[1], 0);
    const int cx1 = imin(bx[2], W), cy1 = imin(bx[3], H);
    if (res[i].valid && cx0 < cx1 && cy0 < cy1) {
      /* the box's image point: mean of its clipped pixel indices */
      const double uvd1[4] = {0.5 * (cx0 + cx1 - 1), 0.5 * (cy0 + cy1 - 1), (double)res[i].disparity, 1.0};
      double h[4];
      for (int r = 0; r < 4; ++r) {
        h[r] = 0.0;
        for (int c = 0; c < 4; ++c) h[r] += Q[4 * r + c] * uvd1[c];
      }
      if (h[3] != 0.0) {
        for (int k = 0; k < 3; ++k) o.p_cam[k] = h[k] / h[3];
        /* T_cam->imu: rotate, then translate */
        for (int r = 0; r < 3; ++r) {
          o.p_imu[r] = t[r];
          for (int c = 0; c < 3; ++c) o.p_imu[r] += R[3 * r + c] * o.p_cam[c];
        }
        /* sigma_Z^2 = (dZ/dd)^2 sigma_d^2 = Z^4 sigma_d^2 / (f^2 b^2) */
        const double Z = o.p_cam[2];
        o.var_z = Z * Z * Z * Z * var_d / (f * f * b * b);
        /* R diag(sigma_x^2, sigma_y^2, sigma_Z^2) R^T */
        const double dg[3] = {var_x, var_y, o.var_z};
        int q = 0;
        for (int r = 0; r < 3; ++r)
          for (int c = r; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[3 * r + k] * dg[k] * R[3 * c + k];
            o.cov_imu[q++] = acc;
          }
        o.valid = 1;
      }
    }
    out[i] = o;
  }
}

/* ------------------------------------------------------------------------------ */
/* Priority object selection (Sec. 4.3.5, last sentence): sort the candidates and   */
/* keep the first max_objects.                                                      */
/* ------------------------------------------------------------------------------ */
typedef struct {
  int frontal;   /* 1: clipped centre inside the central crop */
  int bottom;    /* clipped bottom y: larger is nearer */
  int index;
} sel_t;

static int cmp_sel(const void* a, const void* b) {
  const sel_t* p = (const sel_t*)a;
  const sel_t* q = (const sel_t*)b;
  if (p->frontal != q->frontal) return q->frontal - p->frontal;   /* frontal first */
  if (p->bottom != q->bottom) return q->bottom - p->bottom;       /* nearer first */
  return p->index - q->index;
}

void orc_select_boxes(const int32_t* boxes, int32_t n, int32_t W, int32_t H, int32_t max_objects,
                      const int32_t* crop_permille, int32_t* flags_out, int32_t* rank) {
  /* the crop in px: floor of the permille fractions of the frame size */
  long cx0 = (long)W * crop_permille[0] / 1000, cy0 = (long)H * crop_permille[1] / 1000;
  long cx1 = (long)W * crop_permille[2] / 1000, cy1 = (long)H * crop_permille[3] / 1000;
  sel_t* c = (sel_t*)malloc(sizeof(sel_t) * (size_t)(n > 0 ? n : 1));
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const int32_t* b = boxes + 5 * i;
    flags_out[i] = b[4];
    rank[i] = -1;
    int x0 = imax(b[0], 0), y0 = imax(b[1], 0), x1 = imin(b[2], W), y1 = imin(b[3], H);
    if (!(b[4] & 1) || !(x0 < x1 && y0 < y1)) continue;
    /* centre of the clipped box in pixel-index coordinates */
    double u = (x0 + x1 - 1) / 2.0, v = (y0 + y1 - 1) / 2.0;
    c[m].frontal = u >= cx0 && u < cx1 && v >= cy0 && v < cy1;
    c[m].bottom = y1;
    c[m].index = i;
    ++m;
  }
  qsort(c, (size_t)m, sizeof(sel_t), cmp_sel);
  for (int k = 0; k < m; ++k) {
    rank[c[k].index] = k;
    if (k >= max_objects) flags_out[c[k].index] &= ~1;
  }
  free(c);
}

/* ------------------------------------------------------------------------------ */
/* Auto-rectification offset (Sec. 5.1): move the left image's rows by delta, run  */
/* the dense matcher over the ROI, count the disparities above d_min; then argmax   */
/* over delta and the temporal median filter with a clamped step.                   */
/* ------------------------------------------------------------------------------ */
int32_t orc_rect_counts(const uint64_t* CL, const uint64_t* CR, int32_t W, int32_t H,
                        int32_t roi_x0, int32_t roi_y0, int32_t roi_w, int32_t roi_h,
                        int32_t delta_min, int32_t delta_max, int32_t dmin, int32_t dmax,
                        int32_t radius, int32_t lr_tol, int32_t d_min, int32_t* counts,
                        int16_t* maps, int32_t n_threads) {
  if (roi_w <= 0 || roi_h <= 0 || delta_min > delta_max || roi_x0 < 0 || roi_x0 + roi_w > W ||
      roi_y0 - delta_max < 0 || roi_y0 + roi_h - delta_min > H || roi_y0 < 0 || roi_y0 + roi_h > H)
    return -1;
  size_t px = (size_t)roi_w * roi_h;
  uint64_t* sl = (uint64_t*)malloc(px * sizeof(uint64_t));
  uint64_t* sr = (uint64_t*)malloc(px * sizeof(uint64_t));
  int16_t* d = (int16_t*)malloc(px * sizeof(int16_t));
  /* the right ROI does not move */
  for (int y = 0; y < roi_h; ++y)
    for (int x = 0; x < roi_w; ++x) sr[(size_t)y * roi_w + x] = CR[(size_t)(roi_y0 + y) * W + roi_x0 + x];
  for (int delta = delta_min; delta <= delta_max; ++delta) {
    int k = delta - delta_min;
    /* the left image moved down by delta: row y of the moved image is row y - delta */
    for (int y = 0; y < roi_h; ++y)
      for (int x = 0; x < roi_w; ++x)
        sl[(size_t)y * roi_w + x] = CL[(size_t)(roi_y0 + y - delta) * W + roi_x0 + x];
    if (orc_dense(sl, sr, roi_w, roi_h, dmin, dmax, radius, lr_tol, d, NULL, n_threads) != 0) {
      free(sl); free(sr); free(d);
      return -1;
    }
    int c = 0;
    for (size_t i = 0; i < px; ++i) c += d[i] > d_min;
    counts[k] = c;
    if (maps) memcpy(maps + (size_t)k * px, d, px * sizeof(int16_t));
  }
  free(sl); free(sr); free(d);
  return 0;
}

static int cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

void orc_rect_filter(const int32_t* counts, int32_t T, int32_t n_offsets, int32_t delta_min,
                     int32_t window, int32_t max_step, int32_t initial, int32_t* raw,
                     int32_t* filtered) {
  int prev = initial;
  int* win = (int*)malloc(sizeof(int) * (size_t)(window > 0 ? window : 1));
  for (int t = 0; t < T; ++t) {
    const int32_t* c = counts + (size_t)t * n_offsets;
    /* delta* = argmax of the count; among equal counts the offset nearest 0, then the
     * lower one */
    int best = delta_min;
    for (int k = 1; k < n_offsets; ++k) {
      int dk = delta_min + k, cb = c[best - delta_min];
      if (c[k] > cb || (c[k] == cb && (abs(dk) < abs(best) || (abs(dk) == abs(best) && dk < best))))
        best = dk;
    }
    raw[t] = best;
    /* median of raw[t - window + 1 .. t] (those that exist), lower middle if even */
    int m = 0;
    for (int u = t - window + 1; u <= t; ++u)
      if (u >= 0) win[m++] = raw[u];
    qsort(win, (size_t)m, sizeof(int), cmp_int);
    int med = win[(m - 1) / 2];
    /* clamped change from the previous output */
    int step = med - prev;
    if (step > max_step) step = max_step;
    if (step < -max_step) step = -max_step;
    prev += step;
    filtered[t] = prev;
  }
  free(win);
}
