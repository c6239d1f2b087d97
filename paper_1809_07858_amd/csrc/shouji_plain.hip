// Shouji pre-alignment filter for MI355X (gfx950): the plain form.
//
// Method: Alser et al., Shouji, Sec. 2.2 (Steps 1-3), Eq. 1, Supplementary
// Algorithm 1 (with Algorithm 2 as the zero counter).  Everything is exact
// integer bit work; no MFMA, no floating point.
//
// Data layout in registers ("pair-sliced" bit planes).  A lane owns 32 pairs
// (pairs base + 64k + lane, k = 0..31) and every 32-bit register holds one
// bit of one quantity for those 32 pairs: bit k belongs to pair k.  A
// wavefront therefore filters 2048 pairs, and one VALU instruction evaluates
// one gate of the filter's circuit for 2048 pairs at once.  The window loop
// (the only serial dependence of the method) becomes the instruction stream.
//
// Per lane:
//  * sequences arrive as 2-bit packed words, 16 bases per dword, word-major,
//    so a wavefront load reads one word of 64 consecutive pairs (256 B);
//  * a 32x32 bit transpose turns the 32 dwords of one 16-base half-chunk into
//    32 planes: plane 2u = low code bit of base u, plane 2u+1 = high bit;
//  * pattern planes go to a per-lane ring in LDS (the diagonals need pattern
//    positions up to E away from the text column); text planes stay in VGPRs;
//  * windows are processed in blocks of 8.  For each candidate diagonal (in
//    the order lower 1, upper 1, ..., lower E, upper E, main) the 11 cells of
//    the block's columns are built (XOR of code planes, OR of the two bits:
//    Eq. 1), counted with 2-bit pair sums, and each window's segment is
//    compared with the running winner by the key (ones, first bit) -- fewer
//    ones first, then a leading zero -- keeping the earliest on full ties;
//  * then the Shouji bit-vector update runs as a bit-sliced 8-state machine
//    whose state is S[i..i+2] (S[i+3] is still 1 when window i runs): write iff
//    ones(Z) <= ones(S[i..i+2]), which is "more zeros" for the 4-bit window;
//    S[i] is final after window i and is added to a carry-save ones counter;
//  * the counter planes are transposed back to one count per pair.
//
// Cells outside the m x m map (pattern or text index outside [0, m)) are
// mismatches, in the interior blocks no such cell exists and no mask is
// applied; the boundary blocks OR in per-pair masks kept in LDS.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shouji_internal.h"

namespace shouji {

// 32x32 bit transpose in registers: after the call a[b] bit k == old a[k] bit b.
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
#define SHOUJI_TSTAGE(S, M)                                          \
    _Pragma("unroll") for (int i = 0; i < 32; i++) {                 \
        if ((i & (S)) == 0) {                                        \
            const uint32_t t = ((a[i] >> (S)) ^ a[i + (S)]) & (M);   \
            a[i + (S)] ^= t;                                         \
            a[i] ^= t << (S);                                        \
        }                                                            \
    }
    SHOUJI_TSTAGE(16, 0x0000FFFFu)
    SHOUJI_TSTAGE(8, 0x00FF00FFu)
    SHOUJI_TSTAGE(4, 0x0F0F0F0Fu)
    SHOUJI_TSTAGE(2, 0x33333333u)
    SHOUJI_TSTAGE(1, 0x55555555u)
#undef SHOUJI_TSTAGE
}

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return (a & b) | (c & (a | b));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return v;
}

// Running winner of the window search for the 8 windows of a block, one
// register per plane and window: key planes (ones = K3 K2 K1, first bit K0)
// and the segment's remaining bits Z1..Z3 (Z0 == K0).
struct Winner {
    uint32_t K0[kBlock], K1[kBlock], K2[kBlock], K3[kBlock];
    uint32_t Z1[kBlock], Z2[kBlock], Z3[kBlock];
};

// One candidate diagonal over one block: build 11 cells, count each window's
// segment, and fold it into the running winner.
template <bool FIRST, bool MASKED>
__device__ __forceinline__ void candidate(Winner &W, const uint2 *__restrict__ ring,
                                          const uint32_t *__restrict__ nv, int lane, int i0,
                                          int d, int R, const uint32_t (&tl)[kCols],
                                          const uint32_t (&th)[kCols]) {
    int slot0 = (i0 - d) % R;
    if (slot0 < 0) slot0 += R;
    const uint2 *rp = ring + slot0 * kWave + lane;
    uint32_t cell[kCols];
#pragma unroll
    for (int t = 0; t < kCols; t++) {
        const uint2 pv = rp[t * kWave];
        cell[t] = (pv.x ^ tl[t]) | (pv.y ^ th[t]);
    }
    if (MASKED) {
        if (d < 0) {
            // pattern index j - d > j: the pattern side runs out first
            const uint32_t *np = nv + (-d) * kWave + lane;
#pragma unroll
            for (int t = 0; t < kCols; t++) cell[t] |= np[t * kWave];
        } else {
            const uint32_t *np = nv + lane;
#pragma unroll
            for (int t = 0; t < kCols; t++) {
                cell[t] |= np[t * kWave];
                if (i0 + t - d < 0) cell[t] = ~0u;  // before the pattern's start
            }
        }
    }
    // 2-bit sums of neighbouring cells: x = exactly one is 1, a = both are 1
    uint32_t x[kCols - 1], a[kCols - 1];
#pragma unroll
    for (int t = 0; t < kCols - 1; t++) {
        x[t] = cell[t] ^ cell[t + 1];
        a[t] = cell[t] & cell[t + 1];
    }
#pragma unroll
    for (int w = 0; w < kBlock; w++) {
        // ones of cells w..w+3 = pair sum (w) + pair sum (w+2): 3-bit r2 r1 r0
        const uint32_t r0 = x[w] ^ x[w + 2];
        const uint32_t u = x[w] & x[w + 2];
        const uint32_t r1 = a[w] ^ a[w + 2] ^ u;
        const uint32_t r2 = a[w] & a[w + 2];
        const uint32_t k0 = cell[w];
        if (FIRST) {
            W.K0[w] = k0; W.K1[w] = r0; W.K2[w] = r1; W.K3[w] = r2;
            W.Z1[w] = cell[w + 1]; W.Z2[w] = cell[w + 2]; W.Z3[w] = cell[w + 3];
        } else {
            // lt = (r2 r1 r0 k0) < (K3 K2 K1 K0), borrow chain from the low bit
            const uint32_t b0 = ~k0 & W.K0[w];
            const uint32_t b1 = maj3(~r0, W.K1[w], b0);
            const uint32_t b2 = maj3(~r1, W.K2[w], b1);
            const uint32_t lt = maj3(~r2, W.K3[w], b2);
            W.K0[w] = (lt & k0) | (~lt & W.K0[w]);
            W.K1[w] = (lt & r0) | (~lt & W.K1[w]);
            W.K2[w] = (lt & r1) | (~lt & W.K2[w]);
            W.K3[w] = (lt & r2) | (~lt & W.K3[w]);
            W.Z1[w] = (lt & cell[w + 1]) | (~lt & W.Z1[w]);
            W.Z2[w] = (lt & cell[w + 2]) | (~lt & W.Z2[w]);
            W.Z3[w] = (lt & cell[w + 3]) | (~lt & W.Z3[w]);
        }
    }
}

struct FsmState {
    uint32_t s0, s1, s2;                 // S[i], S[i+1], S[i+2] before window i
    uint32_t ones, twos, fours, e[8];    // carry-save ones counter of final S bits
};

template <bool MASKED>
__device__ __forceinline__ void run_block(FsmState &F, const uint2 *__restrict__ ring,
                                          const uint32_t *__restrict__ nv, int lane, int i0,
                                          int Ee, int R, const uint32_t (&tl)[kCols],
                                          const uint32_t (&th)[kCols]) {
    Winner W;
    // evaluation order: L1, U1, L2, U2, ..., LE, UE, M
    if (Ee == 0) {
        candidate<true, MASKED>(W, ring, nv, lane, i0, 0, R, tl, th);
    } else {
        candidate<true, MASKED>(W, ring, nv, lane, i0, -1, R, tl, th);
        for (int c = 1; c <= 2 * Ee; c++) {
            // c odd: upper diagonal (c+1)/2; c even: lower diagonal c/2+1; last: main
            const int d = (c == 2 * Ee) ? 0 : ((c & 1) ? (c + 1) / 2 : -(c / 2 + 1));
            candidate<false, MASKED>(W, ring, nv, lane, i0, d, R, tl, th);
        }
    }
    // Shouji bit-vector update, window by window
    uint32_t o[kBlock];
#pragma unroll
    for (int w = 0; w < kBlock; w++) {
        const uint32_t q0 = F.s0 ^ F.s1 ^ F.s2;     // ones(S[i..i+2]) = q1 q0
        const uint32_t q1 = maj3(F.s0, F.s1, F.s2);
        // (q1 q0) < (K2 K1) ?
        const uint32_t c0 = ~q0 & W.K1[w];
        const uint32_t c1 = maj3(~q1, W.K2[w], c0);
        // write iff ones(Z) <= ones(S[i..i+2]):  K3 == 0 and not (q < K2 K1)
        const uint32_t wr = ~(W.K3[w] | c1);
        o[w] = (wr & W.K0[w]) | (~wr & F.s0);
        const uint32_t n1 = (wr & W.Z1[w]) | (~wr & F.s1);
        const uint32_t n2 = (wr & W.Z2[w]) | (~wr & F.s2);
        const uint32_t n3 = ~wr | W.Z3[w];
        F.s0 = n1; F.s1 = n2; F.s2 = n3;
    }
    // Harley-Seal carry-save accumulation of the 8 final bits
    uint32_t t1, t2, f1, f2, g;
#define SHOUJI_CSA(h, l, a_, b_, c_)                 \
    {                                                \
        const uint32_t u_ = (a_) ^ (b_);             \
        h = ((a_) & (b_)) | (u_ & (c_));             \
        l = u_ ^ (c_);                               \
    }
    SHOUJI_CSA(t1, F.ones, F.ones, o[0], o[1])
    SHOUJI_CSA(t2, F.ones, F.ones, o[2], o[3])
    SHOUJI_CSA(f1, F.twos, F.twos, t1, t2)
    SHOUJI_CSA(t1, F.ones, F.ones, o[4], o[5])
    SHOUJI_CSA(t2, F.ones, F.ones, o[6], o[7])
    SHOUJI_CSA(f2, F.twos, F.twos, t1, t2)
    SHOUJI_CSA(g, F.fours, F.fours, f1, f2)
#undef SHOUJI_CSA
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint32_t cy = F.e[b] & g;
        F.e[b] ^= g;
        g = cy;
    }
}

__device__ __forceinline__ void load_half(const uint32_t *__restrict__ seq, int64_t ld,
                                          int64_t base, int64_t n, int lane, int h,
                                          uint32_t (&raw)[32]) {
    const uint32_t *row = seq + (int64_t)h * ld;
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int64_t p = base + (int64_t)k * kWave + lane;
        raw[k] = p < n ? row[p] : 0u;
    }
}

__global__ __launch_bounds__(kWave) void shouji_plain_kernel(PlainParams prm) {
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x;
    const int R = prm.R;
    const int Ee = prm.Ee;
    uint2 *ring = reinterpret_cast<uint2 *>(lds);
    uint32_t *nv = lds + (R + kMirror) * kWave * 2;
    const int64_t base = (int64_t)blockIdx.x * kPairsPerWave;
    const int64_t n = prm.n;

    // ---- lengths: effective length per pair (0 for padding and invalid pairs)
    uint32_t lenw[32];
    int lmin = 0x7fffffff, lmax = -1;
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int64_t p = base + (int64_t)k * kWave + lane;
        int m = -1;
        if (p < n) m = prm.lengths ? prm.lengths[p] : prm.max_len;
        const bool ok = (m >= 0 && m <= prm.max_len);
        lenw[k] = ok ? (uint32_t)m : 0u;
        if (ok) { lmin = min(lmin, m); lmax = max(lmax, m); }
    }
    lmin = wave_min(lmin);
    lmax = wave_max(lmax);
    const int m_max = lmax < 0 ? 0 : lmax;
    const int m_min = lmax < 0 ? 0 : lmin;
    const bool uniform = (m_min == m_max);
    transpose32(lenw);                 // lenw[b] = bit b of the 32 lengths
    uint32_t Lb[kLenBits];
#pragma unroll
    for (int b = 0; b < kLenBits; b++) Lb[b] = lenw[b];

    FsmState F;
    F.s0 = F.s1 = F.s2 = ~0u;
    F.ones = F.twos = F.fours = 0u;
#pragma unroll
    for (int b = 0; b < 8; b++) F.e[b] = 0u;

    const int nblocks = (m_max + kBlock - 1) / kBlock;
    uint32_t Tc[32], Tn[32];
    if (nblocks > 0) {
        load_half(prm.refs, prm.ld, base, n, lane, 0, Tc);
        transpose32(Tc);
    }
    int p_loaded = 0;  // pattern half-chunks already in the ring

    auto ensure_pattern = [&](int upto) {
        upto = min(upto, m_max - 1);
        while (p_loaded * 16 <= upto) {
            uint32_t raw[32];
            load_half(prm.reads, prm.ld, base, n, lane, p_loaded, raw);
            transpose32(raw);
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int q = p_loaded * 16 + u;
                const int slot = q % R;
                const uint2 v = make_uint2(raw[2 * u], raw[2 * u + 1]);
                ring[slot * kWave + lane] = v;
                if (slot < kMirror) ring[(slot + R) * kWave + lane] = v;
            }
            p_loaded++;
        }
    };
    // Per-pair "position is past the end" masks for columns i0 .. i0+10+Ee
    auto fill_masks = [&](int i0) {
        for (int s = 0; s <= kCols - 1 + Ee; s++) {
            const int xpos = i0 + s;
            uint32_t inv;
            if (uniform) {
                inv = xpos >= m_max ? ~0u : 0u;
            } else {
                uint32_t g = 0u;  // g = (length > xpos), bit-sliced over the 32 pairs
#pragma unroll
                for (int b = 0; b < kLenBits; b++) {
                    const uint32_t sx = ((xpos >> b) & 1) ? ~0u : 0u;
                    g = (sx & (Lb[b] & g)) | (~sx & (Lb[b] | g));
                }
                inv = ~g;
            }
            nv[s * kWave + lane] = inv;
        }
    };
    auto block = [&](int i0, const uint32_t (&tl)[kCols], const uint32_t (&th)[kCols]) {
        const bool masked = (i0 < Ee) || (i0 + kCols - 1 + Ee >= m_min);
        if (masked) {
            fill_masks(i0);
            run_block<true>(F, ring, nv, lane, i0, Ee, R, tl, th);
        } else {
            run_block<false>(F, ring, nv, lane, i0, Ee, R, tl, th);
        }
    };

    for (int b = 0; b < nblocks; b += 2) {
        const int i0 = b * kBlock;  // = 16 * half index
        const int h = b >> 1;
        ensure_pattern(i0 + kCols - 1 + Ee);
        {
            uint32_t tl[kCols], th[kCols];
#pragma unroll
            for (int t = 0; t < kCols; t++) { tl[t] = Tc[2 * t]; th[t] = Tc[2 * t + 1]; }
            block(i0, tl, th);
        }
        if (b + 1 < nblocks) {
            if ((h + 1) * 16 < m_max) {
                load_half(prm.refs, prm.ld, base, n, lane, h + 1, Tn);
                transpose32(Tn);
            } else {
#pragma unroll
                for (int k = 0; k < 32; k++) Tn[k] = 0u;
            }
            ensure_pattern(i0 + kBlock + kCols - 1 + Ee);
            uint32_t tl[kCols], th[kCols];
#pragma unroll
            for (int t = 0; t < kCols; t++) {
                const int u = kBlock + t;  // position within the half-chunk pair
                tl[t] = u < 16 ? Tc[2 * u] : Tn[2 * (u - 16)];
                th[t] = u < 16 ? Tc[2 * u + 1] : Tn[2 * (u - 16) + 1];
            }
            block(i0 + kBlock, tl, th);
#pragma unroll
            for (int k = 0; k < 32; k++) Tc[k] = Tn[k];
        }
    }

    // ---- counts back to one value per pair
    uint32_t cnt[32];
    cnt[0] = F.ones; cnt[1] = F.twos; cnt[2] = F.fours;
#pragma unroll
    for (int b = 0; b < 8; b++) cnt[3 + b] = F.e[b];
#pragma unroll
    for (int b = 11; b < 32; b++) cnt[b] = 0u;
    transpose32(cnt);  // cnt[k] = ones of S over windows [0, 8*nblocks) for pair k
    const int nwin = nblocks * kBlock;
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int64_t p = base + (int64_t)k * kWave + lane;
        if (p >= n) continue;
        const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
        uint8_t acc;
        int16_t pc;
        if (m < 0 || m > prm.max_len) {
            acc = 0xFF;
            pc = -1;
        } else {
            // S stays 1 on [m, nwin): those ones are not part of the pair
            const int ones = (int)cnt[k] - (nwin - m);
            acc = ones <= prm.E ? 1 : 0;
            pc = (int16_t)ones;
        }
        prm.out_accept[p] = acc;
        if (prm.out_popcount) prm.out_popcount[p] = pc;
    }
}

}  // namespace shouji
