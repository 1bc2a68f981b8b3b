// Exercises the host side of libocsr that runs without a GPU -- argument validation,
// workspace sizing, the kernel-variant table and the rectification-offset filter -- for
// a build whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer. With
// no device, context creation fails cleanly and every call with a null context returns
// OCSR_E_INVALID before touching the device.
#include <cstdio>
#include <cstring>
#include <vector>

#include "ocsr.h"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "host_abi_driver: check failed: %s\n", #c); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

int main() {
  CHECK(ocsr_abi_version() == OCSR_ABI_VERSION);
  CHECK(std::strlen(ocsr_last_error()) == 0);
  ocsr_ctx* ctx = nullptr;
  const int32_t rc = ocsr_ctx_create(0, &ctx);
  CHECK(rc == OCSR_OK || rc < 0);
  if (rc == OCSR_OK) ocsr_ctx_destroy(ctx);
  CHECK(ocsr_ctx_create(-1, &ctx) < 0);
  CHECK(std::strlen(ocsr_last_error()) > 0);
  // workspace sizes, valid and invalid
  CHECK(ocsr_match_workspace_bytes(64, 1 << 16) > 0);
  CHECK(ocsr_match_workspace_bytes(0, 1) > 0);
  ocsr_frame_params fp{3, 4, 1, 2};
  CHECK(ocsr_frame_workspace_bytes(1920, 1080, &fp, 64, 1 << 16) > 0);
  std::vector<ocsr_frame> frames(3);
  for (int k = 0; k < 3; ++k) {
    std::memset(&frames[k], 0, sizeof(ocsr_frame));
    frames[k].width = 320 + 64 * k;
    frames[k].height = 240;
    frames[k].pitch_bytes = frames[k].width;
    frames[k].box_offset = 10 * k;
    frames[k].n_boxes = 10;
  }
  CHECK(ocsr_batch_workspace_bytes(frames.data(), 3, &fp, 1 << 12) > 0);
  frames[1].box_offset = 3;   // overlapping box ranges: invalid
  CHECK(ocsr_batch_workspace_bytes(frames.data(), 3, &fp, 1 << 12) == 0);
  CHECK(ocsr_batch_workspace_bytes(frames.data(), 0, &fp, 1 << 12) == 0);
  CHECK(ocsr_dense_workspace_bytes(1920, 1080) > 0);
  ocsr_rect_params rp{0, 300, 960, 128, -4, 4, 0, 63, 2, 1, 2};
  CHECK(ocsr_rect_workspace_bytes(&rp) > 0);
  rp.delta_max = rp.delta_min + OCSR_MAX_RECT_OFFSETS;   // too many offsets
  CHECK(ocsr_rect_workspace_bytes(&rp) == 0);
  // kernel variants, with a capacity smaller than the count
  int32_t rows[4], cpl[4], passes[4];
  const int32_t n = ocsr_variant_candidates(8, 8, 96, rows, cpl, passes, 4);
  CHECK(n >= 4);
  CHECK(ocsr_variant_candidates(8, 8, 96, rows, cpl, passes, 0) == n);
  CHECK(ocsr_variant_candidates(9, 8, 32, rows, cpl, passes, 4) == 0);
  CHECK(ocsr_variant_candidates(8, 8, 257, rows, cpl, passes, 4) == 0);
  // calls with a null context fail before anything is enqueued
  ocsr_match_params mp;
  std::memset(&mp, 0, sizeof(mp));
  mp.struct_size = sizeof(mp);
  CHECK(ocsr_match_boxes(nullptr, nullptr, nullptr, nullptr, 1, &mp, 16, nullptr, 0, nullptr,
                         nullptr, nullptr) == OCSR_E_INVALID);
  CHECK(ocsr_match_boxes_noalloc(nullptr, nullptr, nullptr, nullptr, 1, &mp, 16, nullptr, nullptr,
                                 nullptr) == OCSR_E_INVALID);
  CHECK(ocsr_range_batch(nullptr, frames.data(), 3, &fp, nullptr, &mp, 16, nullptr, 0, nullptr,
                         nullptr) < 0);
  CHECK(ocsr_census(nullptr, nullptr, 10, 10, 10, nullptr, nullptr, 10, nullptr) < 0);
  // the rectification filter: window, clamped step, ties
  ocsr_rect_filter* f = nullptr;
  CHECK(ocsr_rect_filter_create(0, 1, 0, &f) < 0);
  CHECK(ocsr_rect_filter_create(5, 1, 0, &f) == OCSR_OK && f != nullptr);
  int32_t counts[9];
  for (int t = 0; t < 200; ++t) {
    for (int k = 0; k < 9; ++k) counts[k] = (t * 7 + k * 13) % 50;
    int32_t raw = 0, filt = 0;
    CHECK(ocsr_rect_filter_update(f, counts, 9, -4, &raw, &filt) == OCSR_OK);
    CHECK(raw >= -4 && raw <= 4);
  }
  CHECK(ocsr_rect_filter_update(f, counts, 0, -4, nullptr, nullptr) < 0);
  ocsr_rect_filter_destroy(f);
  std::printf("host_abi_driver: ok\n");
  return 0;
}
