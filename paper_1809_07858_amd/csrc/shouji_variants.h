// Parameters of the variant kernels (window width, MAGNET).  Kept apart
// from shouji_internal.h, which the plain, batched and two-length kernels
// share.
#pragma once

#include <stdint.h>

namespace shouji {

// Window-width variant (bit-sliced, 2048 pairs per wavefront).
struct WindowParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    int32_t max_len;
    int32_t E;
    int32_t Ee;
    int32_t W;
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t n;
};

// MAGNET filter (one pair per lane, LDS stack of pending subproblems).
constexpr int kMagnetBlock = 256;
constexpr int kMagnetStageWords = 16;  // most words per sequence staged in LDS (max_len <= 256)
struct MagnetParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    int32_t max_len;
    int32_t E;       // min(E, max_len): the same results as E for every pair
    int32_t Ee;      // diagonals examined: min(E, max_len - 1)
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t n;
};

}  // namespace shouji
