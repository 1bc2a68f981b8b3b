/*
 * Runs every entry point of the oracle on small synthetic inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure, like the rest of
 * oracle/): out-of-bounds reads or writes, overflows and other undefined behaviour in
 * the oracle abort the run. Inputs: a blurred-noise-like texture from a fixed linear
 * congruential sequence, the right view shifted by a known disparity, boxes of every
 * kind (far, close, clipped, empty, not ranged, overlapping, one-pixel), both matching
 * modes, both aggregations, a vertical range, the dense matcher, the rectification
 * counts and filter, the object selection and the 3D points.
 *
 *   gcc -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all -fopenmp \
 *       ocsr_oracle.c sanitize_driver.c -lm -o sanitize_driver && ./sanitize_driver
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ocsr_oracle.h"

static uint32_t g_state = 12345u;
static uint32_t lcg(void) {
  g_state = g_state * 1664525u + 1013904223u;
  return g_state >> 8;
}

/* texture: a smoothed random field, right view = left moved left by `shift` px */
static void make_pair(int W, int H, int shift, uint8_t* L, uint8_t* R) {
  int* raw = (int*)malloc(sizeof(int) * (size_t)(W + 8) * (size_t)(H + 8));
  for (int i = 0; i < (W + 8) * (H + 8); ++i) raw[i] = (int)(lcg() & 255u);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int acc = 0;
      for (int dy = 0; dy < 3; ++dy)
        for (int dx = 0; dx < 3; ++dx) acc += raw[(y + dy) * (W + 8) + x + dx];
      L[y * W + x] = (uint8_t)(acc / 9);
    }
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int xs = x + shift;
      R[y * W + x] = xs < W ? L[y * W + xs] : (uint8_t)(lcg() & 255u);
    }
  free(raw);
}

static orc_params base_params(void) {
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.sx = 3; p.sy = 4; p.close_scale = 2; p.tau_s = 24;
  p.far_path.mode = ORC_MODE_TILED; p.far_path.bw = 4; p.far_path.bh = 4; p.far_path.n_side = 8;
  p.far_path.dmin = 0; p.far_path.dmax = 15;
  p.close_path.mode = ORC_MODE_TILED; p.close_path.bw = 8; p.close_path.bh = 8;
  p.close_path.n_side = 8; p.close_path.dmin = 0; p.close_path.dmax = 31;
  p.lr_tol = 1; p.min_point_pct = 50; p.agg_mode = ORC_AGG_TRIMMED_MEDIAN; p.tau_d = 1.0f;
  p.n_min = 3; p.trim_pct = 20; p.focal_px = 2000.0f; p.baseline_m = 0.3f; p.d_eps = 0.0f;
  return p;
}

int main(void) {
  const int W = 96, H = 72, S = 2;
  uint8_t* L = (uint8_t*)malloc((size_t)W * H);
  uint8_t* R = (uint8_t*)malloc((size_t)W * H);
  make_pair(W, H, 6, L, R);
  uint64_t* L0 = (uint64_t*)malloc(sizeof(uint64_t) * W * H);
  uint64_t* R0 = (uint64_t*)malloc(sizeof(uint64_t) * W * H);
  uint64_t* L1 = (uint64_t*)malloc(sizeof(uint64_t) * (W / S) * (H / S));
  uint64_t* R1 = (uint64_t*)malloc(sizeof(uint64_t) * (W / S) * (H / S));
  /* census at several windows and levels, both sentinel settings */
  const int wins[4][2] = {{3, 4}, {2, 2}, {4, 3}, {0, 0}};
  for (int k = 0; k < 4; ++k)
    for (int sen = 0; sen < 2; ++sen)
      for (int s = 1; s <= 3; ++s) {
        uint64_t* out = (uint64_t*)malloc(sizeof(uint64_t) * (W / s) * (H / s));
        if (orc_census(L, W, H, W, wins[k][0], wins[k][1], s, sen, out) != 0) return 1;
        free(out);
      }
  if (orc_census(L, W, H, W, 3, 4, 1, 1, L0) || orc_census(R, W, H, W, 3, 4, 1, 1, R0) ||
      orc_census(L, W, H, W, 3, 4, S, 1, L1) || orc_census(R, W, H, W, 3, 4, S, 1, R1))
    return 1;
  /* boxes: far, close, clipped, empty, not ranged, overlapping, one pixel */
  const int32_t boxes[] = {10, 10, 30, 28, 1,  40, 8, 90, 60, 1,  -20, -20, 12, 12, 1,
                           50, 50, 50, 70, 1,  20, 40, 60, 70, 0,  35, 30, 70, 66, 1,
                           5, 60, 6, 61, 1,   80, 0, 200, 100, 1};
  const int n = 8;
  orc_box_result res[8];
  orc_block* blk = (orc_block*)malloc(sizeof(orc_block) * 4096);
  uint16_t* cf = (uint16_t*)malloc(sizeof(uint16_t) * 4096 * 64);
  uint16_t* cb = (uint16_t*)malloc(sizeof(uint16_t) * 4096 * 64);
  for (int v = 0; v < 6; ++v) {
    orc_params p = base_params();
    if (v == 1) p.agg_mode = ORC_AGG_SEGMENT_MEDIAN;
    if (v == 2) { p.far_path.mode = ORC_MODE_GRID; p.close_path.mode = ORC_MODE_GRID; p.close_path.n_side = 5; }
    if (v == 3) { p.dy_min = -2; p.dy_max = 3; }
    if (v == 4) p.cap_blocks = 40;
    if (v == 5) { p.max_blocks_per_box = 6; p.lr_tol = 0; p.min_point_pct = 100; }
    const int32_t total = orc_match_boxes(L0, R0, L1, R1, W, H, boxes, n, &p, res, blk, cf, cb,
                                          4096, 64, 2);
    if (total < 0 || total > 4096) return 2;
  }
  /* aggregation alone: empty, one value, runs */
  {
    orc_params p = base_params();
    float vals[7] = {10.0f, 10.2f, 10.4f, 30.0f, 30.1f, 3.0f, 0.0f};
    orc_box_result r;
    for (int m = 0; m <= 7; ++m)
      for (int far = 0; far < 2; ++far) {
        memset(&r, 0, sizeof(r));
        r.n_eligible = m;
        float tmp[7];
        memcpy(tmp, vals, sizeof(vals));
        orc_aggregate(m ? tmp : NULL, m, m > 0 ? m : 1, far, &p, &r);
      }
  }
  /* dense, the single-pixel form, the rectification counts and filter */
  int16_t* disp = (int16_t*)malloc(sizeof(int16_t) * W * H);
  int16_t* dispr = (int16_t*)malloc(sizeof(int16_t) * W * H);
  if (orc_dense(L0, R0, W, H, 0, 31, 2, 1, disp, dispr, 2) != 0) return 3;
  const int32_t xy[6] = {0, 0, W - 1, H - 1, 40, 30};
  int16_t at[3];
  if (orc_dense_at(L0, R0, W, H, 0, 31, 2, 1, xy, 3, at, 1) != 0) return 4;
  int32_t counts[5];
  int16_t* maps = (int16_t*)malloc(sizeof(int16_t) * 5 * 40 * 20);
  if (orc_rect_counts(L0, R0, W, H, 10, 20, 40, 20, -2, 2, 0, 15, 2, 1, 1, counts, maps, 2) != 0)
    return 5;
  int32_t seq[5 * 6], raw[6], filt[6];
  for (int i = 0; i < 30; ++i) seq[i] = (int32_t)(lcg() % 100u);
  orc_rect_filter(seq, 6, 5, -2, 3, 1, 0, raw, filt);
  /* selection and points */
  const int32_t crop[4] = {333, 0, 667, 1000};
  int32_t flags[8], rank[8];
  orc_select_boxes(boxes, n, W, H, 3, crop, flags, rank);
  const double Q[16] = {1, 0, 0, -47.5, 0, 1, 0, -35.5, 0, 0, 0, 2000, 0, 0, 1 / 0.3, 0};
  const double Rm[9] = {0, 0, 1, -1, 0, 0, 0, -1, 0}, t[3] = {1.2, 0.0, 1.5};
  orc_point pts[8];
  orc_box_points(boxes, res, n, W, H, Q, Rm, t, 2000.0, 0.3, 0.25, 0.01, 0.01, pts);
  free(L); free(R); free(L0); free(R0); free(L1); free(R1); free(blk); free(cf); free(cb);
  free(disp); free(dispr); free(maps);
  printf("sanitize_driver: ok\n");
  return 0;
}
