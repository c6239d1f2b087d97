// Bit-sliced building blocks shared by the kernels that hold one bit of one
// quantity for 32 pairs in each 32-bit register: three-input gates
// (v_bitop3_b32), the 32x32 bit transpose between packed words and bit
// planes, wave-wide min / max, and the load of one packed word for 32 pairs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shouji_internal.h"

namespace shouji {

// Truth table of a 3-input boolean function for v_bitop3_b32: bit
// (a<<2 | b<<1 | c) of the immediate is f(a, b, c) for src0 = a, src1 = b,
// src2 = c.
template <class F>
constexpr unsigned truth_table(F f) {
    unsigned t = 0;
    for (int i = 0; i < 8; i++)
        if (f((i >> 2) & 1, (i >> 1) & 1, i & 1)) t |= 1u << i;
    return t;
}
constexpr unsigned kTTCell = truth_table([](int a, int b, int c) { return a | (b ^ c); });
constexpr unsigned kTTXor3 = truth_table([](int a, int b, int c) { return a ^ b ^ c; });
constexpr unsigned kTTMaj = truth_table([](int a, int b, int c) { return a + b + c >= 2; });
constexpr unsigned kTTMajNotA = truth_table([](int a, int b, int c) { return (1 - a) + b + c >= 2; });
constexpr unsigned kTTAndNotA = truth_table([](int a, int b, int) { return !a && b; });
constexpr unsigned kTTNor = truth_table([](int a, int b, int) { return !(a | b); });
constexpr unsigned kTTOrNotA = truth_table([](int a, int b, int) { return !a || b; });
constexpr unsigned kTTMux = truth_table([](int a, int b, int c) { return a ? b : c; });
constexpr unsigned kTTOr3 = truth_table([](int a, int b, int c) { return a | b | c; });
constexpr unsigned kTTAnd3 = truth_table([](int a, int b, int c) { return a & b & c; });
constexpr unsigned kTTAndXnor = truth_table([](int a, int b, int c) { return a & (b == c); });

template <unsigned TT>
__device__ __forceinline__ uint32_t gate(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
// select: m ? a : b, bit by bit
__device__ __forceinline__ uint32_t mux(uint32_t m, uint32_t a, uint32_t b) {
    return gate<kTTMux>(m, a, b);
}

// 32x32 bit transpose in registers: after the call a[b] bit k == old a[k] bit b.
// Stages 16 and 8 move whole bytes (one v_perm_b32 per word); stages 4, 2, 1
// are a shift and a bit-field select per word.  The masks and shift counts of
// those stages are held in VGPRs (made opaque to the compiler): on gfx950 the
// SIMD runs two wavefronts' VALU instructions side by side only when every
// operand is a VGPR, while one with a scalar or literal operand takes it alone
// (about 1.6x the cost at two wavefronts per SIMD).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const uint32_t lo = __builtin_amdgcn_perm(a[i + 16], a[i], 0x05040100u);
        const uint32_t hi = __builtin_amdgcn_perm(a[i + 16], a[i], 0x07060302u);
        a[i] = lo;
        a[i + 16] = hi;
    }
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if ((i & 8) == 0) {
            const uint32_t lo = __builtin_amdgcn_perm(a[i + 8], a[i], 0x06020400u);
            const uint32_t hi = __builtin_amdgcn_perm(a[i + 8], a[i], 0x07030501u);
            a[i] = lo;
            a[i + 8] = hi;
        }
    }
    uint32_t m4 = 0x0F0F0F0Fu, m2 = 0x33333333u, m1 = 0x55555555u, s4 = 4u, s2 = 2u, s1 = 1u;
    asm volatile("" : "+v"(m4), "+v"(m2), "+v"(m1), "+v"(s4), "+v"(s2), "+v"(s1));
#define SHOUJI_TSTAGE(S, M, SV)                                      \
    _Pragma("unroll") for (int i = 0; i < 32; i++) {                 \
        if ((i & (S)) == 0) {                                        \
            const uint32_t lo = mux((M), a[i], a[i + (S)] << (SV));  \
            const uint32_t hi = mux((M), a[i] >> (SV), a[i + (S)]);  \
            a[i] = lo;                                               \
            a[i + (S)] = hi;                                         \
        }                                                            \
    }
    SHOUJI_TSTAGE(4, m4, s4)
    SHOUJI_TSTAGE(2, m2, s2)
    SHOUJI_TSTAGE(1, m1, s1)
#undef SHOUJI_TSTAGE
}

// Parity of this wavefront's slot on its SIMD (field WAVE_ID of the HW_ID
// hardware register).  Two wavefronts that share a SIMD from the start of a
// launch sit in consecutive slots.
__device__ __forceinline__ int wave_slot_parity() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 4) & 1;   // hwreg(HW_ID, offset 0, 4 bits)
}
// Issue priority of this wavefront, 1 or 0 (s_setprio takes an immediate).
__device__ __forceinline__ void wave_priority(int hi) {
    if (hi)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// Wave-wide maximum / minimum (all 64 lanes active), returned uniform: DPP
// lane swaps within each row of 16 lanes (quad permutes, then the half-row
// and row mirrors), then the four rows' values read into scalar registers.
// No LDS traffic and no LDS latency.
template <bool MAX>
__device__ __forceinline__ int wave_reduce(int v) {
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ int wave_max(int v) { return wave_reduce<true>(v); }
__device__ __forceinline__ int wave_min(int v) { return wave_reduce<false>(v); }

// One 16-base word of 32 pairs (pair = base + PL*k + pl for bit k) from row
// `row` (= seq + w*ld + base).  `full`: all 32 * PL pairs of the wavefront
// exist.  Otherwise only row[0 .. left-1] exist: a missing pair reads the last one
// (its bits are never written out), so no load is predicated; the bound is
// made opaque so that the per-pair indices are not hoisted out of the
// caller's loop and kept live in registers.
template <int PL = kPairLanes>
__device__ __forceinline__ void load_word(const uint32_t *__restrict__ row, bool full, int left, int pl,
                                          uint32_t (&raw)[32]) {
    const uint32_t *q = row + pl;
    if (full) {
#pragma unroll
        for (int k = 0; k < 32; k++) raw[k] = q[k * PL];
    } else {
        int last = left - 1 - pl;            // q[last] is the wavefront's last pair
        asm volatile("" : "+v"(last));
#pragma unroll
        for (int k = 0; k < 32; k++) raw[k] = q[min(k * PL, last)];
    }
}

}  // namespace shouji
