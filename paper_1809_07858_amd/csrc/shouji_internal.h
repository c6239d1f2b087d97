// Internal constants and launch parameters shared by the kernels and the C ABI.
#pragma once
#include <stdint.h>

namespace shouji {

constexpr int kWave = 64;                     // CDNA wavefront width
constexpr int kPairsPerLane = 32;             // one pair per bit of a 32-bit plane
constexpr int kPairsPerWave = kWave * kPairsPerLane;
constexpr int kBlock = 8;                     // windows per block
constexpr int kCols = kBlock + 3;             // text columns one block reads
constexpr int kMirror = kCols - 1;            // ring slots duplicated past its end
constexpr int kLenBits = 11;                  // lengths 0..1024

struct PlainParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    int32_t max_len;
    int32_t E;       // threshold of the decision
    int32_t Ee;      // diagonals on each side actually built: min(E, max_len-1)
    int32_t R;       // pattern ring slots per lane
    uint8_t *out_accept;
    int16_t *out_popcount;
    int64_t n;
};

// Ring slots needed: a block reads pattern positions [i0-Ee, i0+10+Ee] and a
// half-chunk of 16 positions is written just before it is first needed.
inline int ring_slots(int Ee) { return 2 * Ee + 26; }
inline size_t plain_lds_bytes(int Ee) {
    return (size_t)(ring_slots(Ee) + kMirror) * kWave * 8 + (size_t)(kCols + Ee) * kWave * 4;
}

__global__ void shouji_plain_kernel(PlainParams prm);

}  // namespace shouji
