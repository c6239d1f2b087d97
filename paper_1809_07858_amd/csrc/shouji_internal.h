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
inline size_t plain_lds_wave_bytes(int Ee) {
    return (size_t)(ring_slots(Ee) + kMirror) * kRingStride * 8 + (size_t)(kCols + Ee) * kWave * 4;
}

__global__ void shouji_plain_kernel(PlainParams prm);

}  // namespace shouji
