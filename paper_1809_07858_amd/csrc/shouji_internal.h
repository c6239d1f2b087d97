// Internal constants and launch parameters shared by the kernels and the C ABI.
#pragma once
#include <stdint.h>

namespace shouji {

constexpr int kWave = 64;                     // CDNA wavefront width
constexpr int kPairLanes = 32;                // lanes per pair group (one lane half)
constexpr int kPairsPerLane = 32;             // one pair per bit of a 32-bit plane
constexpr int kPairsPerWave = kPairLanes * kPairsPerLane;  // both halves hold the same pairs
constexpr int kRingStride = kPairLanes;       // ring entries per position
constexpr int kBlock = 8;                     // windows per block
constexpr int kCols = kBlock + 3;             // text columns one block reads
constexpr int kMirror = kCols - 1;            // ring slots duplicated past its end
constexpr int kLenBits = 11;                  // lengths 0..1024
constexpr int kHalf = 16;                     // bases per packed word
constexpr int kWavesPerGroup = 4;             // wavefronts per workgroup
constexpr size_t kLdsPerCU = 160 * 1024;      // gfx950

struct PlainParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    int32_t max_len;
    int32_t E;       // threshold of the decision
    int32_t Ee;      // diagonals on each side actually built: min(E, max_len-1)
    int32_t R;       // pattern ring slots
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t n;
    int32_t lds_wave_bytes;  // LDS bytes owned by one wavefront
    int32_t ring_only;       // no length array: LDS holds the pattern ring only
    int32_t qh;              // quarter layout: pattern word offset of the passes
};

// Two-length form: reads and references of different lengths, with a
// counting mode (global, local, glocal at the start or at the end).
struct LocalParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *read_lengths;
    const int32_t *ref_lengths;
    int32_t max_len;
    int32_t E;
    int32_t Ee;
    int32_t R;
    int32_t mode;
    int32_t len_bits;         // bit planes stored per length: bits of max_len
    int32_t waves_per_group;
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t n;
    int32_t lds_wave_bytes;
};

// One group of up to 1024 pairs [base, min(base+1024, n)) for filter_group.
struct GroupJob {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;   // or null: every pair has max_len bases (read lengths in the two-length form)
    const int32_t *ref_lengths;  // two-length form only: reference (text) lengths
    int32_t mode;             // two-length form only: counting mode
    int32_t len_bits;         // two-length form only: bit planes per length
    int32_t max_len;
    int32_t Ee;               // diagonals built on each side
    int32_t E;                // decision threshold when Edec is null
    const int32_t *Edec;      // per-pair decision thresholds, or null
    const int64_t *perm;      // output index of each pair, or null (identity)
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t base;
    int64_t n;
};

struct TilesParams {
    const uint32_t *breads;   // binned words, word-major with leading dimension ld
    const uint32_t *brefs;
    int64_t ld;
    const int32_t *blens;
    const int32_t *bE;
    const int64_t *bperm;
    const int4 *tiles;        // start, count, Ee, unused
    const int32_t *ntiles;    // device count of valid tiles
    int32_t max_len;
    int32_t R;
    int32_t lds_wave_bytes;
    int32_t waves_per_group;
    int32_t qh;               // quarter layout: pattern word offset of the passes
    uint8_t *out_accept;
    int16_t *out_popcount;
};

// Pattern ring slots.  Iteration j reads pattern positions [16j-Ee, 16j+18+Ee]
// (both lane halves).  After its searches the word that iteration j+1 first
// needs, word j+1+H0 with H0 = (18+Ee)/16, is written; it must not overwrite
// positions from 16j+16-Ee on.
inline int ring_slots(int Ee) {
    const int H0 = (kBlock + kCols - 1 + Ee) / kHalf;
    const int a = 2 * Ee + kBlock + kCols;
    const int b = kHalf * (H0 + 1) + Ee;
    return a > b ? a : b;
}
// The same rounded up to a multiple of 8: each half of a word (8 positions
// starting at a multiple of 8) then lands in 8 consecutive slots and is
// written in paired LDS stores without a wrap test.  A launch takes it when
// its CUs still hold as many wavefronts (the kernel handles either size).
inline int ring_slots_aligned(int Ee) { return (ring_slots(Ee) + 7) / 8 * 8; }
// LDS of one wavefront with a ring of R slots: the ring (+ mirror); the
// per-position masks of the iteration's positions lo .. lo+kBlock+kCols+Ee-1;
// the bit planes of the 32 lengths per lane (+ valid plane).  Lanes l and
// l+32 hold the same pairs, so masks and length planes are stored once per
// pair lane.
__host__ __device__ inline int mask_slots(int Ee) { return kBlock + kCols + Ee; }
// two-length form: pattern-position masks cover lo - Ee .. lo + 18 + Ee
__host__ __device__ inline int pattern_mask_slots(int Ee) { return kBlock + kCols + 2 * Ee; }
// LDS of one wavefront of a plain launch without lengths: the ring only.
inline size_t ring_lds_wave_bytes(int R) { return (size_t)(R + kMirror) * kRingStride * 8; }
inline size_t plain_lds_wave_bytes(int Ee, int R) {
    return (size_t)(R + kMirror) * kRingStride * 8 + (size_t)mask_slots(Ee) * kPairLanes * 4 +
           (size_t)(kLenBits + 1) * kPairLanes * 4;
}

// LDS of one wavefront in the two-length form: ring, text masks of the 19
// text columns, pattern masks, and len_bits bit planes of both lengths.
inline size_t local_lds_wave_bytes(int Ee, int len_bits, int R) {
    return (size_t)(R + kMirror) * kRingStride * 8 + (size_t)(kBlock + kCols) * kPairLanes * 4 +
           (size_t)pattern_mask_slots(Ee) * kPairLanes * 4 + (size_t)(2 * len_bits) * kPairLanes * 4;
}

// Quarter layout (four lane groups of 16 lanes, 512 pairs per wavefront,
// iterations of 32 windows) for large thresholds.  Pass k writes pattern words
// 2k+h and 2k+h+1, h = floor((34+Ee)/16) - 3; the ring must keep iteration j's
// positions [32j-Ee, 32j+34+Ee] while pass j+2 writes words 2j+4+h, 2j+5+h.
constexpr int kQuarterLanes = 16;
constexpr int kQuarterPairs = 512;
inline int quarter_h(int Ee) { return (34 + Ee) / 16 - 3; }
inline int quarter_ring_slots(int Ee) {
    const int a = 64 + 16 * quarter_h(Ee) + Ee, b = 2 * Ee + 35;
    return a > b ? a : b;
}
inline int quarter_ring_slots_aligned(int Ee) { return (quarter_ring_slots(Ee) + 7) / 8 * 8; }
inline size_t quarter_lds_wave_bytes(int Ee, int R, bool ring_only) {
    size_t b = (size_t)(R + kMirror) * kQuarterLanes * 8;
    if (!ring_only)
        b += (size_t)(3 * kBlock + kCols + Ee) * kQuarterLanes * 4 + (size_t)(kLenBits + 1) * kQuarterLanes * 4;
    return b;
}

__global__ void shouji_plain_kernel(PlainParams prm);
__global__ void shouji_plain_q_kernel(PlainParams prm);
__global__ void shouji_plain_ring_q_kernel(PlainParams prm);
__global__ void shouji_tiles_q_kernel(TilesParams prm);
__global__ void shouji_plain_ring_kernel(PlainParams prm);
__global__ void shouji_local_kernel(LocalParams prm);
__global__ void shouji_tiles_kernel(TilesParams prm);

// Thread-local error text behind shouji_last_error (printf-style format).
int set_error(int code, const char *fmt, ...);
int clear_error();

}  // namespace shouji
