// Shouji pre-alignment filter for MI355X (gfx950): the plain form.
//
// Method: Alser et al., Shouji, Sec. 2.2 (Steps 1-3), Eq. 1, Supplementary
// Algorithm 1 (with Algorithm 2 as the zero counter).  Everything is exact
// integer bit work; no MFMA, no floating point.
//
// Data layout in registers ("pair-sliced" bit planes).  Every 32-bit
// register holds one bit of one quantity for 32 pairs: bit k belongs to pair
// base + 32k + (lane & 31).  Lanes l and l+32 hold the same 32 pairs, so a
// wavefront filters 1024 pairs; its low lane half searches the even blocks of
// 8 windows and its high half the odd ones, and one VALU instruction
// evaluates one gate of the filter's circuit for two blocks of 32 x 32 pairs.
// The window loop (the only serial dependence of the method) becomes the
// instruction stream.
//
// Per wavefront:
//  * sequences arrive as 2-bit packed words, 16 bases per dword, word-major,
//    so a load of one word for 32 lanes reads 32 consecutive pairs (128 B);
//  * a 32x32 bit transpose turns the 32 dwords of one 16-base word into 32
//    planes: plane 2u = low code bit of base u, plane 2u+1 = high bit.  One
//    transpose pass handles a pattern word on the low half and a text word
//    on the high half;
//  * pattern planes go to a ring in LDS shared by both halves (the diagonals
//    need pattern positions up to E away from the text column); text planes
//    stay in VGPRs and reach the low half by lane swaps;
//  * windows are processed in blocks of 8.  For each candidate diagonal (in
//    Algorithm 1's order d = +1, -1, ..., +E, -E, main) the 11 cells of
//    the block's columns are built (XOR of code planes, OR of the two bits:
//    Eq. 1), and each window's segment is compared with the running winner
//    by the key (ones, first bit) -- fewer ones first, then a leading zero --
//    kept as a 3-bit rank, keeping the earliest on full ties;
//  * then the Shouji bit-vector update runs as a bit-sliced 8-state machine
//    whose state is S[i..i+2] (S[i+3] is still 1 when window i runs): write iff
//    ones(Z) <= ones(S[i..i+2]), which is "more zeros" for the 4-bit window.
//    It is serial: the low half updates block 2j, hands the 3-plane state to
//    the high half for block 2j+1, and gets it back.  S[i] is final after
//    window i; both halves add their final bits to carry-save counters;
//  * the two halves' counters are added and transposed back to one count per
//    pair.
//
// Cells outside the m x m map (pattern or text index outside [0, m)) are
// mismatches, in the interior blocks no such cell exists and no mask is
// applied; the boundary blocks OR in per-pair masks kept in LDS, or, when
// every pair has the same length (a call without a length array), masks
// computed from the positions, so that LDS holds the pattern ring only.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "shouji_bitslice.h"
#include "shouji_internal.h"

namespace shouji {

// A window's key -- ones of its 4-bit segment (0..4), then its first bit --
// takes 8 values, so it is kept as a 3-bit rank R2 R1 R0 in key order:
// (0,0) (1,0) (1,1) (2,0) (2,1) (3,0) (3,1) (4,1) -> 0..7.  With c0 the first
// cell and o' the ones of the other three: rank bit 2 = c0 ? o' >= 1 : o' == 3,
// bit 0 = c0 ? o' == 3 : o' >= 1, bit 1 = c0 ? o' != 1 : o' == 2; the first
// bit is 1 for ranks 2, 4, 6, 7, o' is odd for ranks 1, 4, 5, 7 (so the last
// bit is Z3 = (o' mod 2) ^ Z1 ^ Z2), and ones <= q iff rank <= 2q.
constexpr unsigned kTTOrIfAndElse = truth_table([](int a, int b, int c) { return a ? (b | c) : (b & c); });
constexpr unsigned kTTAndIfOrElse = truth_table([](int a, int b, int c) { return a ? (b & c) : (b | c); });
constexpr unsigned kTTOrIfXorElse = truth_table([](int a, int b, int c) { return a ? (b | c) : (b ^ c); });
constexpr unsigned kTTXnorIfAndElse = truth_table([](int a, int b, int c) { return a ? (b == c) : (b & c); });
constexpr unsigned kTTRankFirst = truth_table([](int a, int b, int c) {
    const int r = a << 2 | b << 1 | c;
    return r == 2 || r == 4 || r == 6 || r == 7;
});
constexpr unsigned kTTRankOddRest = truth_table([](int a, int b, int c) {
    const int r = a << 2 | b << 1 | c;
    return r == 1 || r == 4 || r == 5 || r == 7;
});
constexpr unsigned kTTOr = truth_table([](int a, int b, int) { return a | b; });

// The rank gates, checked on every 4-cell segment at compile time: the rank
// orders the keys (fewer ones first, then a leading zero), the first bit and
// the last bit follow from it (the latter with the two middle bits), and
// "ones <= q iff rank <= 2q" holds for every state count q in 0..3.
constexpr int tt_eval(unsigned tt, int a, int b, int c) { return (int)((tt >> (a << 2 | b << 1 | c)) & 1u); }
constexpr int rank_of(int c0, int c1, int c2, int c3) {
    const int r2 = tt_eval(kTTOrIfAndElse, c0, c1, tt_eval(kTTOrIfAndElse, c0, c2, c3));
    const int r0 = tt_eval(kTTAndIfOrElse, c0, c1, tt_eval(kTTAndIfOrElse, c0, c2, c3));
    const int r1 = c1 ? tt_eval(kTTOrIfXorElse, c0, c2, c3) : tt_eval(kTTXnorIfAndElse, c0, c2, c3);
    return r2 << 2 | r1 << 1 | r0;
}
constexpr bool rank_gates_hold() {
    for (int x = 0; x < 16; x++) {
        const int c0 = x & 1, c1 = (x >> 1) & 1, c2 = (x >> 2) & 1, c3 = (x >> 3) & 1;
        const int ones = c0 + c1 + c2 + c3;
        const int r = rank_of(c0, c1, c2, c3);
        if (r != (ones == 0 ? 0 : 2 * ones - 1 + c0 - (ones == 4 ? 1 : 0))) return false;
        if (tt_eval(kTTRankFirst, r >> 2, (r >> 1) & 1, r & 1) != c0) return false;
        if ((tt_eval(kTTRankOddRest, r >> 2, (r >> 1) & 1, r & 1) ^ c1 ^ c2) != c3) return false;
        for (int q = 0; q < 4; q++)
            if ((ones <= q) != (r <= 2 * q)) return false;
    }
    return true;
}
static_assert(rank_gates_hold(), "rank gates disagree with the key order");

// Running winner of the window search for the NB windows of a block (8, or
// 4 in a short last iteration), one register per plane and window: the key's
// rank planes R2 R1 R0 and the segment's bits Z1, Z2 (Z0 and Z3 follow from
// the rank and them).
template <int NB>
struct Winner {
    uint32_t R0[NB], R1[NB], R2[NB];
    uint32_t Z1[NB], Z2[NB];
};

// One candidate diagonal d over one block of NB windows: build NB+3 cells,
// rank each window's key, and fold it into the running winner.  `rp`
// points at this lane's ring entry for pattern position i0 - d; consecutive
// positions are kRingStride entries apart (all entries are loaded before the
// first use).  `masked` (uniform): some cell may lie outside the map.  With
// one length per pair, nv[s] masks position i0+s; with two (TWO), nv[s]
// masks text position i0+s and nvp[s] pattern position i0-Ee+s.  REGM: every
// pair has length reg_mlen, and the masks are computed from the positions
// instead of read from nv.
template <bool FIRST, int NB, bool TWO, bool REGM, int PL = kPairLanes>
__device__ __forceinline__ void candidate(Winner<NB> &W, const uint2 (&pv)[NB + 3],
                                          const uint32_t *__restrict__ nv, const uint32_t *__restrict__ nvp,
                                          int Ee, int i0, int d, bool masked,
                                          const uint32_t (&tl)[NB + 3], const uint32_t (&th)[NB + 3],
                                          int reg_mlen) {
    constexpr int C = NB + 3;
    uint32_t cell[C];
#pragma unroll
    for (int t = 0; t < C; t++) {
        // Eq. 1: mismatch iff either code bit differs
        cell[t] = gate<kTTCell>(pv[t].x ^ tl[t], pv[t].y, th[t]);
    }
    if (masked && TWO && REGM) {
        // text column i0+t past the reference (per-pair masks), pattern
        // position i0+t-d outside the read (every read has length reg_mlen)
#pragma unroll
        for (int t = 0; t < C; t++) {
            cell[t] |= nv[t * PL];
            if (i0 + t - d < 0 || i0 + t - d >= reg_mlen) cell[t] = ~0u;
        }
    } else if (masked && TWO) {
        // text column i0+t past the reference, pattern position i0+t-d
        // outside the read
        const uint32_t *np = nvp + (Ee - d) * PL;
#pragma unroll
        for (int t = 0; t < C; t++) cell[t] |= nv[t * PL] | np[t * PL];
    } else if (REGM && masked) {
        // d < 0: the pattern index i0+t-d runs out first; d >= 0: the text
        // column i0+t, and pattern indices below 0
        const int first = d < 0 ? i0 - d : i0;
#pragma unroll
        for (int t = 0; t < C; t++) {
            if (first + t >= reg_mlen || i0 + t - d < 0) cell[t] = ~0u;
        }
    } else if (masked) {
        if (d < 0) {
            // pattern index j - d > j: the pattern side runs out first
            const uint32_t *np = nv + (-d) * PL;
#pragma unroll
            for (int t = 0; t < C; t++) cell[t] |= np[t * PL];
        } else {
            const uint32_t *np = nv;
#pragma unroll
            for (int t = 0; t < C; t++) {
                cell[t] |= np[t * PL];
                if (i0 + t - d < 0) cell[t] = ~0u;  // before the pattern's start
            }
        }
    }
#pragma unroll
    for (int w = 0; w < NB; w++) {
        // rank of the key of cells w..w+3 (7 gates)
        const uint32_t c0 = cell[w], c1 = cell[w + 1], c2 = cell[w + 2], c3 = cell[w + 3];
        const uint32_t r2 = gate<kTTOrIfAndElse>(c0, c1, gate<kTTOrIfAndElse>(c0, c2, c3));
        const uint32_t r0 = gate<kTTAndIfOrElse>(c0, c1, gate<kTTAndIfOrElse>(c0, c2, c3));
        const uint32_t r1 = mux(c1, gate<kTTOrIfXorElse>(c0, c2, c3), gate<kTTXnorIfAndElse>(c0, c2, c3));
        if (FIRST) {
            W.R0[w] = r0; W.R1[w] = r1; W.R2[w] = r2;
            W.Z1[w] = c1; W.Z2[w] = c2;
        } else {
            // lt = (r2 r1 r0) < (R2 R1 R0): borrow chain from the low bit
            const uint32_t b0 = gate<kTTAndNotA>(r0, W.R0[w], W.R0[w]);
            const uint32_t b1 = gate<kTTMajNotA>(r1, W.R1[w], b0);
            const uint32_t lt = gate<kTTMajNotA>(r2, W.R2[w], b1);
            W.R0[w] = mux(lt, r0, W.R0[w]);
            W.R1[w] = mux(lt, r1, W.R1[w]);
            W.R2[w] = mux(lt, r2, W.R2[w]);
            W.Z1[w] = mux(lt, c1, W.Z1[w]);
            W.Z2[w] = mux(lt, c2, W.Z2[w]);
        }
    }
}

// Issue pacing of the two wavefronts that share a SIMD, for the quarter
// layout's long iterations.  At equal priority the SIMD favours the older
// one, which then finishes its window loop ahead and leaves the other to run
// alone at a lower issue rate.  Each posts the index of the iteration it
// starts in a table held per SIMD (hardware ids XCC_ID and HW_ID: SE, SH, CU,
// SIMD) and slot parity and reads the other's post one iteration later; the
// one behind takes priority, the one ahead gives it up, level ones take
// turns by iteration and slot parity.  Only scheduling reads the table: a
// stale post, or one from another kernel on the same SIMD, changes the
// speed, never a result.  (The two-half layout takes turns only: with its
// shorter iterations the post and its read cost more than they balance,
// E = 2 taking 15% longer.)
__device__ uint32_t g_simd_pace[8 * 8 * 2 * 16 * 4 * 2];

struct SimdPace {
    uint32_t *mine, *other;
    int par;
    uint32_t seen;  // the other's post, loaded at the previous step
    __device__ __forceinline__ void begin() {
        const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);          // HW_ID, all 32 bits
        const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u;    // XCC_ID
        const unsigned simd = (hw >> 4) & 3u, cu = (hw >> 8) & 15u, sh = (hw >> 12) & 1u, se = (hw >> 13) & 7u;
        const unsigned slot = (((xcc * 8u + se) * 2u + sh) * 16u + cu) * 4u + simd;
        par = (int)(hw & 1u);   // WAVE_ID bit 0: two wavefronts that share a SIMD from the start sit in slots 0 and 1
        mine = g_simd_pace + 2 * slot + par;
        other = g_simd_pace + 2 * slot + (par ^ 1);
        __hip_atomic_store(mine, 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // not in the loop yet
    }
    // before iteration j of the window loop
    __device__ __forceinline__ void step(int j) {
        if (j == 0) {
            wave_priority(par);
        } else {
            const int o = (int)__builtin_amdgcn_readfirstlane(seen);   // the other's iteration one step ago
            if (o > j - 1)
                wave_priority(1);
            else if (o < j - 1)
                wave_priority(0);
            else
                wave_priority((j & 1) ^ par);
        }
        __hip_atomic_store(mine, (uint32_t)j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        seen = __hip_atomic_load(other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

struct FsmState {
    uint32_t s0, s1, s2;                 // S[i], S[i+1], S[i+2] before window i
    uint32_t ones, twos, fours, e[8];    // carry-save ones counter of final S bits
};

// A candidate whose cells can leave the map in this iteration takes the
// masked path: lo = first window of the iteration, hi_col = last text column
// the iteration reads, m_min = shortest length in the group.
__device__ __forceinline__ bool needs_mask(int d, int lo, int hi_col, int m_min) {
    return (d > lo) || (hi_col >= m_min) || (hi_col - d >= m_min);
}

// The C ring entries (pattern planes of C consecutive positions) of one
// candidate, starting at ring slot `slot`.
template <int C, int PL = kRingStride>
__device__ __forceinline__ void ring_load(const uint2 *__restrict__ rb, int slot, uint2 (&pv)[C]) {
    const uint2 *rp = rb + slot * PL;
#pragma unroll
    for (int t = 0; t < C; t++) pv[t] = rp[t * PL];
}

// Window search of one block of NB windows at i0 (sb = ring slot of i0): the
// winner of every window over all 2E+1 diagonals.
template <int NB, bool TWO, bool MASKS = true, bool REGM = false, int PL = kPairLanes>
__device__ __forceinline__ void block_winners(Winner<NB> &W, const uint2 *__restrict__ ring,
                                              const uint32_t *__restrict__ nv,
                                              const uint32_t *__restrict__ nvp, int pl, int i0,
                                              int sb, int Ee, int R, int lo, int hi_col, int m_min,
                                              const uint32_t (&tl)[NB + 3],
                                              const uint32_t (&th)[NB + 3], int reg_mlen = -1) {
    // evaluation order (Algorithm 1): d = +1, -1, +2, -2, ..., +E, -E, then
    // the main diagonal (d > 0: text index exceeds pattern index by d, the
    // diagonal Algorithm 1 calls lower j, drawn as upper in Fig. 6); diagonal
    // d reads the pattern from position i0 - d, i.e. ring slot sb - d (mod R).
    // The ring entries of the next candidate are loaded while the current one
    // is evaluated (two register buffers, A and B, used in turn).
    constexpr int C = NB + 3;
    const uint2 *rb = ring + pl;
    uint2 A[C], B[C];
    // MASKS = false: the caller knows that no cell of the block leaves the map
    auto mk = [&](int d) { return MASKS && needs_mask(d, lo, hi_col, m_min); };
    if (Ee == 0) {
        ring_load<C, PL>(rb, sb, A);
        candidate<true, NB, TWO, REGM, PL>(W, A, nv, nvp, Ee, i0, 0, mk(0), tl, th, reg_mlen);
        return;
    }
    int sP = sb == 0 ? R - 1 : sb - 1;   // slot of d = +k
    int sN = sb + 1 == R ? 0 : sb + 1;   // slot of d = -k
    ring_load<C, PL>(rb, sP, A);
    ring_load<C, PL>(rb, sN, B);
    candidate<true, NB, TWO, REGM, PL>(W, A, nv, nvp, Ee, i0, 1, mk(1), tl, th, reg_mlen);
    // A <- the next d > 0 (or the main diagonal when E = 1)
    sP = sP == 0 ? R - 1 : sP - 1;
    ring_load<C, PL>(rb, Ee >= 2 ? sP : sb, A);
    candidate<false, NB, TWO, REGM, PL>(W, B, nv, nvp, Ee, i0, -1, mk(-1), tl, th, reg_mlen);
    for (int k = 2; k <= Ee; k++) {
        // A holds d = +k; B <- d = -k
        sN = sN + 1 == R ? 0 : sN + 1;
        ring_load<C, PL>(rb, sN, B);
        candidate<false, NB, TWO, REGM, PL>(W, A, nv, nvp, Ee, i0, k, mk(k), tl, th, reg_mlen);
        // A <- d = +(k+1), or the main diagonal after the last k
        sP = sP == 0 ? R - 1 : sP - 1;
        ring_load<C, PL>(rb, k < Ee ? sP : sb, A);
        candidate<false, NB, TWO, REGM, PL>(W, B, nv, nvp, Ee, i0, -k, mk(-k), tl, th, reg_mlen);
    }
    candidate<false, NB, TWO, REGM, PL>(W, A, nv, nvp, Ee, i0, 0, mk(0), tl, th, reg_mlen);
}

// Where the zeros of the final bit-vector lie, for the local and glocal
// counts (Sec. 2.2.3: the ones before the first and after the last zero are
// not counted).  Each lane half tracks the blocks it updates.
struct Ends {
    uint32_t seen;                 // a final bit of this half's blocks was 0
    uint32_t first[kLenBits];      // position of the first such zero (bit planes)
    uint32_t last[kLenBits];       // position of the last such zero
};

// Fold the NB final bits o[] of positions start..start+NB-1 (start a
// multiple of NB, uniform) into the tracker.
template <int NB>
__device__ __forceinline__ void track_ends(Ends &X, const uint32_t (&o)[NB], int start) {
    constexpr int LB = NB == 8 ? 3 : (NB == 4 ? 2 : 1);   // index bits within the block
    uint32_t any, f[LB], l[LB];
    if constexpr (NB == 8) {
        const uint32_t all_lo = gate<kTTAnd3>(o[0], o[1], o[2]) & o[3];   // no zero in 0..3
        const uint32_t all_hi = gate<kTTAnd3>(o[4], o[5], o[6]) & o[7];   // no zero in 4..7
        any = ~(all_lo & all_hi);
        // first zero: the quad, then the pair, then the bit
        f[2] = all_lo;
        uint32_t q[4];
#pragma unroll
        for (int j = 0; j < 4; j++) q[j] = mux(all_lo, o[4 + j], o[j]);
        f[1] = q[0] & q[1];
        f[0] = mux(f[1], q[2], q[0]);
        // last zero: the quad, then the pair, then the bit
        l[2] = ~all_hi;
        uint32_t r[4];
#pragma unroll
        for (int j = 0; j < 4; j++) r[j] = mux(all_hi, o[j], o[4 + j]);
        l[1] = ~(r[2] & r[3]);
        l[0] = ~mux(l[1], r[3], r[1]);
    } else if constexpr (NB == 4) {
        const uint32_t all = gate<kTTAnd3>(o[0], o[1], o[2]) & o[3];
        any = ~all;
        f[1] = o[0] & o[1];
        f[0] = mux(f[1], o[2], o[0]);
        l[1] = ~(o[2] & o[3]);
        l[0] = ~mux(l[1], o[3], o[1]);
    } else {
        static_assert(NB == 2, "blocks of 8, 4 or 2 windows");
        any = ~(o[0] & o[1]);
        f[0] = o[0];
        l[0] = ~o[1];
    }
    const uint32_t nf = any & ~X.seen;    // this block holds the first zero
#pragma unroll
    for (int b = 0; b < kLenBits; b++) {
        const uint32_t sb = ((start >> b) & 1) ? ~0u : 0u;
        X.first[b] = mux(nf, b < LB ? f[b < LB ? b : 0] : sb, X.first[b]);
        X.last[b] = mux(any, b < LB ? l[b < LB ? b : 0] : sb, X.last[b]);
    }
    X.seen |= any;
}

// Shouji bit-vector update over the NB windows of a block: the serial part
// (one lane half at a time).  o[w] receives the bit S[start+w] that became
// final at window start+w.
template <int NB>
__device__ __forceinline__ void block_fsm(FsmState &F, const Winner<NB> &W, uint32_t (&o)[NB]) {
#pragma unroll
    for (int w = 0; w < NB; w++) {
        const uint32_t q0 = gate<kTTXor3>(F.s0, F.s1, F.s2);  // ones(S[i..i+2]) = q1 q0
        const uint32_t q1 = gate<kTTMaj>(F.s0, F.s1, F.s2);
        // write iff ones(Z) <= ones(S[i..i+2]) iff rank <= (q1 q0 0):
        // keep = (q1 q0 0) < (R2 R1 R0), a borrow chain whose low step is R0
        const uint32_t b1 = gate<kTTMajNotA>(q0, W.R1[w], W.R0[w]);
        const uint32_t keep = gate<kTTMajNotA>(q1, W.R2[w], b1);
        const uint32_t z0 = gate<kTTRankFirst>(W.R2[w], W.R1[w], W.R0[w]);
        const uint32_t z3 = gate<kTTXor3>(gate<kTTRankOddRest>(W.R2[w], W.R1[w], W.R0[w]), W.Z1[w], W.Z2[w]);
        o[w] = mux(keep, F.s0, z0);
        const uint32_t n1 = mux(keep, F.s1, W.Z1[w]);
        const uint32_t n2 = mux(keep, F.s2, W.Z2[w]);
        const uint32_t n3 = gate<kTTOr>(keep, z3, z3);
        F.s0 = n1; F.s1 = n2; F.s2 = n3;
    }
}

// Carry-save accumulation of the NB final bits o[] of a block (and, with
// TWO, the positions of their zeros; the block starts at position `start`).
// Independent per lane half, so both halves run it together.
template <int NB, bool TWO>
__device__ __forceinline__ void block_count(FsmState &F, const uint32_t (&o)[NB], Ends &X, int start, int ebits) {
    uint32_t t1, t2, f1, f2, g;
#define SHOUJI_CSA(h, l, a_, b_, c_)                       \
    {                                                      \
        const uint32_t aa_ = (a_), bb_ = (b_), cc_ = (c_); \
        h = gate<kTTMaj>(aa_, bb_, cc_);                   \
        l = gate<kTTXor3>(aa_, bb_, cc_);                  \
    }
    SHOUJI_CSA(t1, F.ones, F.ones, o[0], o[1])
    if constexpr (NB == 2) {
        f1 = F.twos & t1;                 // weight 4
        F.twos ^= t1;
    } else {
        SHOUJI_CSA(t2, F.ones, F.ones, o[2], o[3])
        SHOUJI_CSA(f1, F.twos, F.twos, t1, t2)
    }
    if constexpr (NB == 8) {
        SHOUJI_CSA(t1, F.ones, F.ones, o[4], o[5])
        SHOUJI_CSA(t2, F.ones, F.ones, o[6], o[7])
        SHOUJI_CSA(f2, F.twos, F.twos, t1, t2)
        SHOUJI_CSA(g, F.fours, F.fours, f1, f2)
    } else if constexpr (NB == 4) {
        g = F.fours & f1;
        F.fours ^= f1;
    } else {
        static_assert(NB == 2, "blocks of 8, 4 or 2 windows");
        g = F.fours & f1;
        F.fours ^= f1;
    }
#undef SHOUJI_CSA
    // the eights counter: one pulse per block at most, so (uniform) ebits
    // bits hold every count of this half
#pragma unroll
    for (int b = 0; b < 8; b++) {
        if (b < ebits) {
            const uint32_t cy = F.e[b] & g;
            F.e[b] ^= g;
            g = cy;
        }
    }
    if constexpr (TWO) track_ends<NB>(X, o, start);
}

// Every value of one lane half (0: lanes 0-31, 1: lanes 32-63) to all lanes.
__device__ __forceinline__ uint32_t from_half0(uint32_t v) {
    return __builtin_amdgcn_permlane32_swap(v, v, false, false)[0];
}
__device__ __forceinline__ uint32_t from_half1(uint32_t v) {
    return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
}

// A wavefront filters 1024 pairs.  Lanes l and l+32 hold the same 32 pairs
// (bit k of a plane = pair base + 32k + (l & 31)); the low lane half searches
// the even blocks of 8 windows, the high half the odd ones (the searches are
// independent).  The bit-vector update is serial: it runs on the low half for
// block 2j, the 3-plane state S[i..i+2] moves to the high half with one lane
// swap per plane, the high half updates block 2j+1 and hands the state back.
// Both halves read one pattern ring in LDS.
//
// TWO: reads and references of different lengths (J.lengths = read lengths,
// J.ref_lengths = reference lengths) and a counting mode (J.mode); the map
// has the reference's columns, cells outside the read are mismatches, and
// the ones before the first / after the last zero of the bit-vector can be
// left out of the count (Sec. 2.2.3).
template <bool TWO, bool RO = false>
__device__ __forceinline__ void filter_group(const GroupJob &J, uint32_t *lds, int R, int lane) {
    // The younger of the two wavefronts on a SIMD (odd slot) takes issue
    // priority through the prologue, so that both reach the window loop at
    // about the same time (the older one's loads were issued first).
    wave_priority(wave_slot_parity());
    const int half = lane >> 5;
    const int pl = lane & (kPairLanes - 1);
    const int Ee = J.Ee;
    uint2 *ring = reinterpret_cast<uint2 *>(lds);
    // masks of (text) positions lo + s at nv[s * 32 + pl]; this half's block
    // starts at s = 8 * half.  TWO: pattern-position masks of lo - Ee + s at
    // nvp[s * 32 + pl], then the bit planes of the reference and read lengths.
    uint32_t *nv = lds + (R + kMirror) * kRingStride * 2;
    uint32_t *nvh = nv + kBlock * half * kPairLanes + pl;
    // (TWO needs text masks of the 19 text columns only, and J.len_bits bit
    // planes per length)
    uint32_t *nvp = nv + (TWO ? kBlock + kCols : mask_slots(Ee)) * kPairLanes;
    uint32_t *nvph = nvp + kBlock * half * kPairLanes + pl;
    uint32_t *lbv = (TWO ? nvp + pattern_mask_slots(Ee) * kPairLanes : nvp) + pl;   // length bit planes
    const int nlb = TWO ? J.len_bits : kLenBits;                                  // planes per length
    uint32_t *lbvp = lbv + nlb * kPairLanes;                                      // TWO: read lengths
    const int64_t base = J.base;
    const int64_t n = J.n;
    const bool full = base + kPairsPerWave <= n;
    // the low half reads pattern words, the high half text words (a select of
    // the two addresses, not an indexed pair, so that it stays in registers)
    const uint32_t *seq = reinterpret_cast<const uint32_t *>(
        half ? reinterpret_cast<uintptr_t>(J.refs) : reinterpret_cast<uintptr_t>(J.reads));

    // ---- lengths: effective length per pair (0 for padding and invalid
    // pairs) and the valid-pair plane (bit k: pair k has a length in range)
    // (TWO: lenw = reference lengths, lenr = read lengths)
    uint32_t lenw[32], lenr[TWO ? 32 : 1];
    uint32_t valid = 0u;
    int lmin = 0x7fffffff, lmax = -1, rmin = 0x7fffffff, rmax = -1;
    // pairs of this wavefront: lane pair q = 32k + pl exists iff q < left
    const int left = (int)min(n - base, (int64_t)kPairsPerWave);
    // Loads are never predicated (a missing pair reads the last one and is
    // then replaced by -1), and each length is materialised at once, so that
    // no per-pair lane mask stays live into the window loop.  All loads are
    // issued first: text / pattern word 0 (which does not depend on the
    // lengths), then the lengths.
    const int nwords = (J.max_len + kHalf - 1) / kHalf;
    uint32_t raw0[32];
    if (nwords > 0) {
        load_word(seq + base, full, left, pl, raw0);
    } else {
#pragma unroll
        for (int k = 0; k < 32; k++) raw0[k] = 0u;
    }
    // RO kernels are launched without a length array (every pair has
    // max_len bases), the others always with one: the choice is made at
    // compile time, so the length is not a per-lane select that keeps
    // max_len in a vector register
    const int32_t *lp = RO ? nullptr : J.lengths + base;
    const int32_t *tp = TWO ? J.ref_lengths + base : nullptr;
    int mv[32], mtv[TWO ? 32 : 1];
    if (full) {
#pragma unroll
        for (int k = 0; k < 32; k++) {
            mv[k] = RO ? J.max_len : lp[k * kPairLanes + pl];
            if constexpr (TWO) mtv[k] = tp[k * kPairLanes + pl];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 32; k++) {
            const int qi = min(k * kPairLanes + pl, left - 1);
            mv[k] = RO ? J.max_len : lp[qi];
            if constexpr (TWO) mtv[k] = tp[qi];
        }
    }
    // word 0 transposed while the lengths are still arriving (its loads are
    // issued first and complete first)
    transpose32(raw0);
    // Fast path (one length per pair, a full wavefront, every length in
    // range -- the usual case): the lengths are the planes' source as they
    // are, every pair is valid, and min / max come from the raw values.
    bool fast = false;
    if constexpr (!TWO) {
        int a = 0x7fffffff, b = -1;
#pragma unroll
        for (int k = 0; k < 32; k++) {
            a = min(a, mv[k]);
            b = max(b, mv[k]);
        }
        a = __builtin_amdgcn_readfirstlane(wave_min(a));
        b = __builtin_amdgcn_readfirstlane(wave_max(b));
        if (full && a >= 0 && b <= J.max_len) {
            fast = true;
#pragma unroll
            for (int k = 0; k < 32; k++) lenw[k] = (uint32_t)mv[k];
            valid = ~0u;
            lmin = a;
            lmax = b;
        }
    }
    if (!fast) {
#pragma unroll
        for (int k = 0; k < 32; k++) {
            const int q = k * kPairLanes + pl;
            const uint32_t inm = (full || q < left) ? ~0u : 0u;
            const int m = (int)(((uint32_t)mv[k] & inm) | ~inm);   // -1 for a missing pair
            if constexpr (TWO) {
                const int mt = (int)(((uint32_t)mtv[k] & inm) | ~inm);
                const bool ok = m >= 0 && m <= J.max_len && mt >= 0 && mt <= J.max_len;
                lenw[k] = ok ? (uint32_t)mt : 0u;
                lenr[k] = ok ? (uint32_t)m : 0u;
                valid |= ok ? (1u << k) : 0u;
                if (ok) {
                    lmin = min(lmin, mt); lmax = max(lmax, mt);
                    rmin = min(rmin, m); rmax = max(rmax, m);
                }
                asm volatile("" : "+v"(lenw[k]), "+v"(lenr[k]), "+v"(valid), "+v"(lmin), "+v"(lmax), "+v"(rmin),
                             "+v"(rmax));
            } else {
                // all-ones iff 0 <= m <= max_len
                const uint32_t okm = (uint32_t)m <= (uint32_t)J.max_len ? ~0u : 0u;
                lenw[k] = (uint32_t)m & okm;
                valid |= okm & (1u << k);
                lmin = min(lmin, (int)(((uint32_t)m & okm) | (~okm & 0x7fffffffu)));
                lmax = max(lmax, (int)(((uint32_t)m & okm) | ~okm));
                asm volatile("" : "+v"(lenw[k]), "+v"(valid), "+v"(lmin), "+v"(lmax));
            }
        }
        // wave-uniform after the reductions: keep them in scalar registers so
        // that every decision taken from them is a scalar branch
        lmin = __builtin_amdgcn_readfirstlane(wave_min(lmin));
        lmax = __builtin_amdgcn_readfirstlane(wave_max(lmax));
        if constexpr (TWO) {
            rmin = __builtin_amdgcn_readfirstlane(wave_min(rmin));
            rmax = __builtin_amdgcn_readfirstlane(wave_max(rmax));
        }
    }
    // m_max: windows (the reference's positions); m_min: shortest of both
    // sequences (below it no cell needs a mask); m_words: positions to load
    const int m_max = lmax < 0 ? 0 : lmax;
    const int m_min = lmax < 0 ? 0 : (TWO ? min(lmin, rmin) : lmin);
    const int m_words = lmax < 0 ? 0 : (TWO ? max(lmax, rmax) : lmax);
    const bool uniform = !TWO && (m_min == m_max);
    // TWO: every valid read has one length (rmax): the pattern-side masks
    // follow from the positions, only the reference side needs its table
    const bool read_uniform = TWO && lmax >= 0 && rmin == rmax;
    // RO: the wavefront's LDS holds the ring only (every pair has max_len
    // bases, so the lengths are uniform): masks from the positions, as for
    // any group whose valid pairs all have one length
    static_assert(!(TWO && RO), "the two-length form keeps its masks in LDS");
    if (!uniform) {
        // bit planes of the lengths, kept in LDS (read by the boundary masks
        // and the output only); with one length for all valid pairs none are
        // needed
        transpose32(lenw);             // lenw[b] = bit b of the 32 lengths
#pragma unroll
        for (int b = 0; b < kLenBits; b++)
            if (b < nlb) lbv[b * kPairLanes] = lenw[b];
        if constexpr (TWO) {
            transpose32(lenr);
#pragma unroll
            for (int b = 0; b < kLenBits; b++)
                if (b < nlb) lbvp[b * kPairLanes] = lenr[b];
        }
    }
    // The rest is compiled twice: UNI (a compile-time fact) when every valid
    // pair of the group has one length, so that a group of one length runs
    // the code of the kernel without a length array (the masks from the
    // positions, no mask table or length planes kept live).
    auto rest = [&](auto uni_tag) __attribute__((always_inline)) {
        constexpr bool UNI = decltype(uni_tag)::value;
        Ends X;
        if constexpr (TWO) {
            X.seen = 0u;
#pragma unroll
            for (int b = 0; b < kLenBits; b++) X.first[b] = X.last[b] = 0u;
        }

        FsmState F;
        F.s0 = F.s1 = F.s2 = ~0u;
        F.ones = F.twos = F.fours = 0u;
#pragma unroll
        for (int b = 0; b < 8; b++) F.e[b] = 0u;

        const int nblocks = (m_max + kBlock - 1) / kBlock;
        const int niter = (nblocks + 1) / 2;
        const int ebits = 32 - __builtin_clz((unsigned)niter | 1u);   // bits of niter (each half: <= niter blocks)
        const int nhalves = (m_words + kHalf - 1) / kHalf;  // words holding positions < m_words
        const int H0 = (kBlock + kCols - 1 + Ee) / kHalf; // last pattern word iteration 0 reads

        // Masks "position x is past the pair's end" (x < 0 counts as past) for
        // positions x0 .. x0+count-1, stored at dst[s * 32], from the length bit
        // planes at planes[b * 32] (nlb of them, higher bits zero), bit-sliced
        // over the 32 pairs.  The first non-negative position takes a full
        // compare (length <= x); each next one adds the pairs whose length
        // equals it, one gate per length bit.
        auto fill_range = [&](int x0, int count, const uint32_t *planes, uint32_t *dst) {
            // x0 opaque: its bit tests are not strength-reduced into values
            // carried through the window loop
            asm volatile("" : "+v"(x0));
            uint32_t lb[kLenBits];
#pragma unroll
            for (int b = 0; b < kLenBits; b++) lb[b] = b < nlb ? planes[b * kPairLanes] : 0u;
            uint32_t msk = ~0u;
            for (int s = 0; s < count; s++) {
                const int x = x0 + s;
                if (x == max(x0, 0)) {
                    uint32_t g = 0u;  // g = (length > x)
#pragma unroll
                    for (int b = 0; b < kLenBits; b++) {
                        const uint32_t sx = ((x >> b) & 1) ? ~0u : 0u;
                        g = mux(sx, lb[b] & g, lb[b] | g);
                    }
                    msk = ~g;
                } else if (x > 0) {
                    uint32_t e = ~0u;  // e = (length == x)
#pragma unroll
                    for (int b = 0; b < kLenBits; b++) {
                        const uint32_t sx = ((x >> b) & 1) ? ~0u : 0u;
                        e = gate<kTTAndXnor>(e, lb[b], sx);
                    }
                    msk |= e;
                }
                dst[s * kPairLanes] = x < 0 ? ~0u : msk;
            }
        };
        // per-lane masks of positions i0 .. i0+count-1, stored at dst[s * 32]
        // (groups of mixed lengths; a group of one length takes its masks from
        // the positions)
        auto fill_masks = [&](int i0, uint32_t *dst, int count) { fill_range(i0, count, lbv, dst); };
        // TWO: text masks of i0 .. i0+C-1 and pattern masks of i0-Ee .. i0+C-1+Ee
        // (a negative pattern position is outside the read)
        auto fill_masks2 = [&](int i0, uint32_t *dst, uint32_t *dstp, int C) {
            fill_range(i0, C, lbv, dst);
            fill_range(i0 - Ee, C + 2 * Ee, lbvp, dstp);
        };

        // One transpose pass: the low lane half turns pattern word pw into ring
        // entries (positions 16pw..16pw+15), the high half turns text word tw into
        // planes left in raw (plane 2u = low code bit of position 16tw+u).  A word
        // outside [0, limit) is replaced by a valid one: its positions lie beyond
        // every pair's length, where the masks override every cell, and a pattern
        // word outside the range is not written to the ring.
        auto pass_load = [&](int pw, int tw, int limit, uint32_t (&raw)[32]) {
            const int w = min(max(half ? tw : pw, 0), limit - 1);
            const uint32_t *row = seq + (int64_t)w * J.ld + base;
            load_word(row, full, left, pl, raw);
        };
        // The ring entries of pattern word pw (low half): slot by slot with the
        // wrap test when R is the minimal size, or as two runs of 8 consecutive
        // slots when R is a multiple of 8.
        auto ring_write = [&](int pw, int limit, uint32_t (&raw)[32]) {
            if (half == 0 && pw < limit && (R & 7) != 0) {
                int slot = (pw * kHalf) % R;
#pragma unroll
                for (int u = 0; u < kHalf; u++) {
                    const uint2 v = make_uint2(raw[2 * u], raw[2 * u + 1]);
                    ring[slot * kRingStride + pl] = v;
                    if (slot < kMirror) ring[(slot + R) * kRingStride + pl] = v;
                    slot = slot + 1 == R ? 0 : slot + 1;
                }
            } else if (half == 0 && pw < limit) {
                // R is a multiple of 8: each half word goes to 8 consecutive
                // slots (paired writes), the slots below kMirror also past R
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int s0 = (pw * kHalf + 8 * h) % R;
                    uint2 *dst = ring + s0 * kRingStride + pl;
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        dst[u * kRingStride] = make_uint2(raw[2 * (8 * h + u)], raw[2 * (8 * h + u) + 1]);
                    if (s0 < kMirror) {
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            if (s0 + u < kMirror)
                                dst[(R + u) * kRingStride] = make_uint2(raw[2 * (8 * h + u)], raw[2 * (8 * h + u) + 1]);
                    }
                }
            }
        };
        auto pass_finish = [&](int pw, int limit, uint32_t (&raw)[32]) {
            transpose32(raw);
            ring_write(pw, limit, raw);
        };
        auto pass = [&](int pw, int tw, uint32_t (&raw)[32]) {
            pass_load(pw, tw, nhalves, raw);
            pass_finish(pw, nhalves, raw);
        };

        // Text planes of a block: the 11 positions (low, high plane) of this lane's
        // block.  The low half's block 2j reads positions 0..10 of text word j, the
        // high half's block 2j+1 positions 8..15 of word j and 0..2 of word j+1.
        // The high half transposes every text word once and the low half receives
        // what it needs by lane swaps.  Two arrays alternate between iterations:
        // one holds the current block's planes; the other is started from the
        // newest word (start_text) and completed one pass later (finish_text).
        //
        // start_text, from text word w in the high half's raw: low half <- its
        // positions 0..10 (from the high half), high half <- its positions 8..15.
        auto start_text = [&](uint32_t (&T)[2 * kCols], const uint32_t (&raw)[32]) {
#pragma unroll
            for (int t = 0; t < 2 * kBlock; t++)  // low lanes: raw[t] of the high half; high lanes: own raw[16+t]
                T[t] = __builtin_amdgcn_permlane32_swap(raw[t], raw[2 * kBlock + t], false, false)[1];
            // low lanes: raw[t] of the high half (the partner raw[t+6] is a
            // position the block does not read, free to be overwritten)
#pragma unroll
            for (int t = 2 * kBlock; t < 2 * kCols; t++)
                T[t] = __builtin_amdgcn_permlane32_swap(raw[t], raw[t + 6], false, false)[1];
        };
        // finish_text, from text word w+1 in the high half's raw: high half <- its
        // positions 0..2 (the low half's planes are complete already).
        auto finish_text = [&](uint32_t (&T)[2 * kCols], const uint32_t (&raw)[32]) {
#pragma unroll
            for (int t = 2 * kBlock; t < 2 * kCols; t++) T[t] = half ? raw[t - 2 * kBlock] : T[t];
        };

        uint32_t TA[2 * kCols], TB[2 * kCols];
        if (nblocks > 0) {
            // pattern words 0..H0 into the ring; text words 0 and 1
            uint32_t raw1[32];
            ring_write(0, nhalves, raw0);
            start_text(TA, raw0);
            if (nhalves > 1) {       // else word 1 holds no position of any pair
                pass(1, 1, raw1);
                finish_text(TA, raw1);
                start_text(TB, raw1);
            }
            for (int hp = 2; hp <= H0; hp++) pass(hp, -1, raw1);
        }

        // Iteration j: blocks 2j (low half) and 2j+1 (high half) with text planes
        // Tc; afterwards Tn (started from word j+1) is completed for iteration j+1
        // and Tc is restarted from word j+2 for iteration j+2.
        // Every iteration but a short last one has two full blocks (its 16
        // windows start below m_max - 8).
        auto iteration = [&](int j, uint32_t (&Tc)[2 * kCols], uint32_t (&Tn)[2 * kCols]) {
            const int lo = kHalf * j;                       // first window of the iteration
            const int i0 = lo + kBlock * half;              // this lane's block
            const int hi_col = lo + kBlock + kCols - 1;     // last text column read
            Winner<kBlock> W;
            {
                uint32_t tl[kCols], th[kCols];
#pragma unroll
                for (int t = 0; t < kCols; t++) { tl[t] = Tc[2 * t]; th[t] = Tc[2 * t + 1]; }
                const int sb = i0 % R;
                if ((Ee > lo) || (hi_col + Ee >= m_min)) {
                    if constexpr (TWO) {
                        if (read_uniform) {
                            // one read length: pattern masks from the positions
                            fill_range(i0, kCols, lbv, nvh);
                            block_winners<kBlock, TWO, true, true>(W, ring, nvh, nvph, pl, i0, sb, Ee, R, lo, hi_col,
                                                                   m_min, tl, th, rmax);
                        } else {
                            fill_masks2(i0, nvh, nvph, kCols);
                            block_winners<kBlock, TWO, true, false>(W, ring, nvh, nvph, pl, i0, sb, Ee, R, lo, hi_col,
                                                                    m_min, tl, th);
                        }
                    } else if (UNI) {
                        // one length for every valid pair: the masks follow from
                        // the positions, as without a length array
                        block_winners<kBlock, false, true, true>(W, ring, nvh, nvph, pl, i0, sb, Ee, R, lo, hi_col,
                                                                 m_min, tl, th, m_max);
                    } else {
                        fill_masks(i0, nvh, kCols + Ee);
                        block_winners<kBlock, false, true, false>(W, ring, nvh, nvph, pl, i0, sb, Ee, R, lo, hi_col,
                                                                  m_min, tl, th);
                    }
                } else {
                    // interior: every pattern index i0+t-d lies in [0, m_min) and every
                    // text column below m_min, so no candidate needs a mask
                    block_winners<kBlock, TWO, false, UNI>(W, ring, nvh, nvph, pl, i0, sb, Ee, R, lo, hi_col, m_min,
                                                          tl, th);
                }
            }
            // the next pass (after all reads of iteration j): the pattern word
            // iteration j+1 first needs, and text word j+2 (a pass whose two words
            // both lie past every pair's end is skipped: their planes are never
            // unmasked).  Its loads are issued here, before the serial update and
            // the count, which cover their latency; the ring write comes after.
            const bool do_pass = j + 1 < niter && (j + 1 + H0 < nhalves || j + 2 < nhalves);
            uint32_t raw[32];
            if (do_pass) pass_load(j + 1 + H0, j + 2, nhalves, raw);
            // serial bit-vector update: block 2j on the low half, 2j+1 on the
            // high; then both halves count their final bits at once
            uint32_t o[kBlock];
            if (half == 0) block_fsm<kBlock>(F, W, o);
            F.s0 = from_half0(F.s0); F.s1 = from_half0(F.s1); F.s2 = from_half0(F.s2);
            if (half == 1) block_fsm<kBlock>(F, W, o);
            F.s0 = from_half1(F.s0); F.s1 = from_half1(F.s1); F.s2 = from_half1(F.s2);
            block_count<kBlock, TWO>(F, o, X, lo + kBlock * half, ebits);
            if (do_pass) {
                pass_finish(j + 1 + H0, nhalves, raw);
                finish_text(Tn, raw);
                start_text(Tc, raw);
            }
        };
        // A last iteration with at most 8 windows left runs blocks of NB = 4
        // windows (at most 4 left: NB = 2): the low half's at lo, the high half's
        // at lo+NB (if any window is left there).  Its text planes: the low half's
        // positions 0..NB+2 of word j are its own, the high half's positions
        // NB..2NB+2 are the low half's.
        auto short_iteration = [&](auto nb, int j, const uint32_t (&Tc)[2 * kCols], bool activeB) {
            constexpr int NB = decltype(nb)::value, C = NB + 3;
            const int lo = kHalf * j;
            const int i0 = lo + NB * half;
            uint32_t tl[C], th[C];
#pragma unroll
            for (int t = 0; t < C; t++) {
                tl[t] = __builtin_amdgcn_permlane32_swap(Tc[2 * t], Tc[2 * t + 2 * NB], false, false)[0];
                th[t] = __builtin_amdgcn_permlane32_swap(Tc[2 * t + 1], Tc[2 * t + 1 + 2 * NB], false, false)[0];
            }
            uint32_t *nvs = nv + NB * half * kPairLanes + pl;
            uint32_t *nvps = nvp + NB * half * kPairLanes + pl;
            Winner<NB> W;
            if constexpr (TWO) {
                if (read_uniform) {
                    fill_range(i0, C, lbv, nvs);
                    block_winners<NB, TWO, true, true>(W, ring, nvs, nvps, pl, i0, i0 % R, Ee, R, lo, lo + NB + C - 1,
                                                       m_min, tl, th, rmax);
                } else {
                    fill_masks2(i0, nvs, nvps, C);
                    block_winners<NB, TWO, true, false>(W, ring, nvs, nvps, pl, i0, i0 % R, Ee, R, lo, lo + NB + C - 1,
                                                        m_min, tl, th);
                }
            } else if (UNI) {
                block_winners<NB, false, true, true>(W, ring, nvs, nvps, pl, i0, i0 % R, Ee, R, lo, lo + NB + C - 1,
                                                     m_min, tl, th, m_max);
            } else {
                fill_masks(i0, nvs, C + Ee);
                block_winners<NB, false, true, false>(W, ring, nvs, nvps, pl, i0, i0 % R, Ee, R, lo, lo + NB + C - 1,
                                                      m_min, tl, th);
            }
            uint32_t o[NB];
            if (half == 0) block_fsm<NB>(F, W, o);
            F.s0 = from_half0(F.s0); F.s1 = from_half0(F.s1); F.s2 = from_half0(F.s2);
            if (half == 1 && activeB) block_fsm<NB>(F, W, o);
            if (half == 0 || activeB) block_count<NB, TWO>(F, o, X, lo + NB * half, ebits);
        };
        const int rem = m_max - kHalf * (niter - 1);        // windows of the last iteration
        const bool short_last = niter > 0 && rem <= kBlock;
        const int nlong = niter - (short_last ? 1 : 0);
        int j = 0;
        // The two wavefronts of a SIMD take issue priority in turn, one
        // iteration each (by slot parity).  At equal priority the SIMD
        // favours the older one, which then ends about an iteration ahead and
        // leaves the other to finish alone at a lower issue rate.
        const int par = wave_slot_parity();
        for (; j + 1 < nlong; j += 2) {
            wave_priority(par);
            iteration(j, TA, TB);
            wave_priority(par ^ 1);
            iteration(j + 1, TB, TA);
        }
        if (j < nlong) iteration(j, TA, TB);
        if (short_last) {
            uint32_t Tl[2 * kCols];
#pragma unroll
            for (int t = 0; t < 2 * kCols; t++) Tl[t] = (nlong & 1) ? TB[t] : TA[t];
            if (rem > 4)
                short_iteration(std::integral_constant<int, 4>(), nlong, Tl, true);
            else
                short_iteration(std::integral_constant<int, 2>(), nlong, Tl, rem > 2);
        }
        // windows whose final S bit went into the counter
        const int nwin = !short_last ? kHalf * niter
                                     : kHalf * nlong + (rem > 4 ? kBlock : (rem > 2 ? kBlock / 2 : kBlock / 4));

        // ---- add the two halves' ones counters (each half then holds the
        // total), then each half writes 16 of the 32 pairs of its lanes
        // the same register of the other lane half (one lane swap, no LDS)
        auto other_half = [half](uint32_t v) {
            const auto sw = __builtin_amdgcn_permlane32_swap(v, v, false, false);
            return half ? (uint32_t)sw[0] : (uint32_t)sw[1];
        };
        uint32_t cnt[32];
        cnt[0] = F.ones; cnt[1] = F.twos; cnt[2] = F.fours;
#pragma unroll
        for (int b = 0; b < 8; b++) cnt[3 + b] = F.e[b];
        {
            uint32_t cy = 0u;
#pragma unroll
            for (int b = 0; b < 11; b++) {
                const uint32_t o = other_half(cnt[b]);
                const uint32_t s_ = gate<kTTXor3>(cnt[b], o, cy);
                cy = gate<kTTMaj>(cnt[b], o, cy);
                cnt[b] = s_;
            }
        }
        // TWO: the zeros' first and last positions over both halves' blocks
        uint32_t pos[TWO ? 32 : 1];
        if constexpr (TWO) {
            uint32_t fh[kLenBits], lh[kLenBits];
            const uint32_t seen_h = other_half(X.seen);
#pragma unroll
            for (int b = 0; b < kLenBits; b++) { fh[b] = other_half(X.first[b]); lh[b] = other_half(X.last[b]); }
            // fh < first and last < lh: borrow chains from the low bit
            uint32_t flt = gate<kTTAndNotA>(fh[0], X.first[0], X.first[0]);
            uint32_t lgt = gate<kTTAndNotA>(X.last[0], lh[0], lh[0]);
#pragma unroll
            for (int b = 1; b < kLenBits; b++) {
                flt = gate<kTTMajNotA>(fh[b], X.first[b], flt);
                lgt = gate<kTTMajNotA>(X.last[b], lh[b], lgt);
            }
            // take the other half's position if it has a zero and this one has
            // none or a later first (earlier last) zero
            const uint32_t tf = seen_h & (~X.seen | flt);
            const uint32_t tl_ = seen_h & (~X.seen | lgt);
#pragma unroll
            for (int b = 0; b < 32; b++) pos[b] = 0u;
#pragma unroll
            for (int b = 0; b < kLenBits; b++) {
                pos[b] = mux(tf, fh[b], X.first[b]);
                pos[16 + b] = mux(tl_, lh[b], X.last[b]);
            }
            X.seen |= seen_h;
        }
        // rows 16.. carry each pair's length (unless all valid pairs have
        // length m_max) and valid bit through the transpose
#pragma unroll
        for (int b = 11; b < 32; b++)
            cnt[b] = (b >= 16 && b < 16 + nlb && !UNI) ? lbv[(b - 16) * kPairLanes] : 0u;
        cnt[16 + kLenBits] = valid;
        if constexpr (TWO) {
            cnt[17 + kLenBits] = X.seen;
            transpose32(pos);  // pos[k]: first zero | last zero << 16
        }
        transpose32(cnt);  // cnt[k]: ones of S over windows [0, nwin) | length << 16 | valid << 27 (| seen << 28)
        // both halves hold the same rows: the low half writes pairs k < 16, the
        // high half pairs k >= 16 (a lane swap brings row 16+k to register k)
#pragma unroll
        for (int k = 0; k < 16; k++) {
            cnt[k] = __builtin_amdgcn_permlane32_swap(cnt[k], cnt[16 + k], false, false)[0];
            if constexpr (TWO) pos[k] = __builtin_amdgcn_permlane32_swap(pos[k], pos[16 + k], false, false)[0];
        }
        // the pair-count bound again, opaque to the compiler here, so that the
        // stores' range checks are not computed (and kept live) before the loop
        int left_out = __builtin_amdgcn_readfirstlane(left);
        asm volatile("" : "+s"(left_out));
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const int kk = k + 16 * half;
            const int64_t p = base + (int64_t)kk * kPairLanes + pl;
            if (!full && kk * kPairLanes + pl >= left_out) continue;
            const uint32_t w = cnt[k];
            const int m = UNI ? m_max : (int)((w >> 16) & ((1u << kLenBits) - 1));
            uint8_t acc;
            int16_t pc;
            if (!((w >> (16 + kLenBits)) & 1u)) {
                acc = 0xFF;
                pc = -1;
            } else {
                // S stays 1 on [m, nwin): those ones are not part of the pair
                int ones = (int)(w & 0xFFFFu) - (nwin - m);
                if constexpr (TWO) {
                    if ((w >> (17 + kLenBits)) & 1u) {
                        // ones before the first zero, after the last zero
                        const int first = (int)(pos[k] & ((1u << kLenBits) - 1));
                        const int last = (int)((pos[k] >> 16) & ((1u << kLenBits) - 1));
                        if (J.mode == 1 || J.mode == 2) ones -= first;
                        if (J.mode == 1 || J.mode == 3) ones -= m - 1 - last;
                    }
                }
                const int E = J.Edec ? J.Edec[p] : J.E;
                acc = ones <= E ? 1 : 0;
                pc = (int16_t)ones;
            }
            const int64_t o = J.perm ? J.perm[p] : p;
            J.out_accept[o] = acc;
            if (J.out_popcount) J.out_popcount[o] = pc;
        }

    };
    if constexpr (TWO) {
        rest(std::false_type());
    } else if constexpr (RO) {
        rest(std::true_type());
    } else {
        if (uniform)
            rest(std::true_type());
        else
            rest(std::false_type());
    }
}

// ------------------------------------------------------------ quarter layout
// For large thresholds the pattern ring of the layout above (32 pair lanes,
// 2E+19 positions and a word of look-ahead) fills LDS so that a CU holds one
// wavefront per SIMD.  Here a wavefront filters 512 pairs in four lane groups
// of 16 lanes (g = lane >> 4; bit k of a plane is pair base + 16k + (lane &
// 15)), all holding the same pairs: an iteration covers 32 windows and group g
// searches block q(g) of 8 of them, q = 0, 1, 2, 3 for g = 0, 1, 3, 2, so that
// the bit-vector update's 3-plane state moves from block to block with one
// lane swap per plane (0 -> 1 and 3 -> 2 within a 32-lane half, 1 -> 3 and
// 2 -> 0 across the halves).  The ring holds 16 pair lanes per position, so a
// wavefront needs about half the LDS at the same threshold, and two per SIMD
// fit up to E = 31.  The search, the update, the count and the cell masking
// are the functions above with a lane stride of 16.
//
// Passes: pass k transposes text word 2k (group 0) and 2k+1 (group 3) and
// pattern words 2k+h and 2k+h+1 (groups 1 and 2; h = floor((34+E)/16) - 3,
// so that pass k+1 completes the pattern words iteration k reads).  Text
// planes of iteration k: group 0 takes word 2k's positions 0..10, group 3 word
// 2k+1's; group 1 word 2k's positions 8..15 (from group 0) and 2k+1's 0..2
// (from group 3); group 2 word 2k+1's 8..15 (from group 3) and word 2k+2's
// 0..2 (from group 0 of pass k+1).
constexpr int kQLanes = 16;
constexpr int kQPairs = kQLanes * kPairsPerLane;   // 512 pairs per wavefront
constexpr int kQWin = 4 * kBlock;                   // windows per iteration

template <bool RO>
__device__ __forceinline__ void filter_group4(const GroupJob &J, uint32_t *lds, int R, int h, int lane) {
    SimdPace pace;
    pace.begin();
    const int g = lane >> 4;
    const int q = g == 0 ? 0 : (g == 1 ? 1 : (g == 3 ? 2 : 3));   // block of the iteration
    const int pl = lane & (kQLanes - 1);
    const int Ee = J.Ee;
    uint2 *ring = reinterpret_cast<uint2 *>(lds);
    // masks of positions lo + s at nv[s * 16 + pl] (s < 35 + Ee), then the
    // bit planes of the 32 lengths per pair lane
    uint32_t *nv = lds + (R + kMirror) * kQLanes * 2;
    uint32_t *nvg = nv + kBlock * q * kQLanes + pl;
    uint32_t *lbv = nv + (3 * kBlock + kCols + Ee) * kQLanes + pl;
    const int64_t base = J.base;
    const int64_t n = J.n;
    const bool full = base + kQPairs <= n;
    // groups 0 and 3 read text words, groups 1 and 2 pattern words
    const bool text_group = g == 0 || g == 3;
    const uint32_t *seq = reinterpret_cast<const uint32_t *>(
        text_group ? reinterpret_cast<uintptr_t>(J.refs) : reinterpret_cast<uintptr_t>(J.reads));
    const int left = (int)min(n - base, (int64_t)kQPairs);

    // ---- lengths (as in filter_group, one length per pair)
    uint32_t lenw[32];
    uint32_t valid = 0u;
    int lmin = 0x7fffffff, lmax = -1;
    const int32_t *lp = RO ? nullptr : J.lengths + base;   // as in filter_group
    int mv[32];
    if (full) {
#pragma unroll
        for (int k = 0; k < 32; k++) mv[k] = RO ? J.max_len : lp[k * kQLanes + pl];
    } else {
#pragma unroll
        for (int k = 0; k < 32; k++) {
            const int qi = min(k * kQLanes + pl, left - 1);
            mv[k] = RO ? J.max_len : lp[qi];
        }
    }
    bool fast = false;
    {
        int a = 0x7fffffff, b = -1;
#pragma unroll
        for (int k = 0; k < 32; k++) {
            a = min(a, mv[k]);
            b = max(b, mv[k]);
        }
        a = __builtin_amdgcn_readfirstlane(wave_min(a));
        b = __builtin_amdgcn_readfirstlane(wave_max(b));
        if (full && a >= 0 && b <= J.max_len) {
            fast = true;
#pragma unroll
            for (int k = 0; k < 32; k++) lenw[k] = (uint32_t)mv[k];
            valid = ~0u;
            lmin = a;
            lmax = b;
        }
    }
    if (!fast) {
#pragma unroll
        for (int k = 0; k < 32; k++) {
            const int qq = k * kQLanes + pl;
            const uint32_t inm = (full || qq < left) ? ~0u : 0u;
            const int m = (int)(((uint32_t)mv[k] & inm) | ~inm);   // -1 for a missing pair
            const uint32_t okm = (uint32_t)m <= (uint32_t)J.max_len ? ~0u : 0u;
            lenw[k] = (uint32_t)m & okm;
            valid |= okm & (1u << k);
            lmin = min(lmin, (int)(((uint32_t)m & okm) | (~okm & 0x7fffffffu)));
            lmax = max(lmax, (int)(((uint32_t)m & okm) | ~okm));
            asm volatile("" : "+v"(lenw[k]), "+v"(valid), "+v"(lmin), "+v"(lmax));
        }
        lmin = __builtin_amdgcn_readfirstlane(wave_min(lmin));
        lmax = __builtin_amdgcn_readfirstlane(wave_max(lmax));
    }
    const int m_max = lmax < 0 ? 0 : lmax;
    const int m_min = lmax < 0 ? 0 : lmin;
    const bool uniform = m_min == m_max;
    if (!uniform) {
        transpose32(lenw);             // lenw[b] = bit b of the 32 lengths
#pragma unroll
        for (int b = 0; b < kLenBits; b++) lbv[b * kQLanes] = lenw[b];
    }

    // The rest is compiled twice, as in filter_group: UNI when every valid
    // pair of the group has one length.
    auto rest = [&](auto uni_tag) __attribute__((always_inline)) {
        constexpr bool UNI = decltype(uni_tag)::value;
        FsmState F;
        F.s0 = F.s1 = F.s2 = ~0u;
        F.ones = F.twos = F.fours = 0u;
#pragma unroll
        for (int b = 0; b < 8; b++) F.e[b] = 0u;
        Ends X;   // unused (global counting)

        const int niter = (m_max + kQWin - 1) / kQWin;
        const int ebits = 32 - __builtin_clz((unsigned)niter | 1u);   // bits of niter (one block per group and iteration)
        const int nhalves = (m_max + kHalf - 1) / kHalf;   // words holding positions < m_max

        // masks "position x is past the pair's end" for positions x0 .. x0+count-1
        // (as in filter_group; groups of mixed lengths only, a group of one
        // length takes its masks from the positions)
        auto fill_masks = [&](int i0, uint32_t *dst, int count) {
            int x0 = i0;
            asm volatile("" : "+v"(x0));
            uint32_t lb[kLenBits];
#pragma unroll
            for (int b = 0; b < kLenBits; b++) lb[b] = lbv[b * kQLanes];
            uint32_t msk = ~0u;
            for (int s = 0; s < count; s++) {
                const int x = x0 + s;
                if (s == 0) {
                    uint32_t gt = 0u;  // gt = (length > x)
#pragma unroll
                    for (int b = 0; b < kLenBits; b++) {
                        const uint32_t sx = ((x >> b) & 1) ? ~0u : 0u;
                        gt = mux(sx, lb[b] & gt, lb[b] | gt);
                    }
                    msk = ~gt;
                } else {
                    uint32_t e = ~0u;  // e = (length == x)
#pragma unroll
                    for (int b = 0; b < kLenBits; b++) {
                        const uint32_t sx = ((x >> b) & 1) ? ~0u : 0u;
                        e = gate<kTTAndXnor>(e, lb[b], sx);
                    }
                    msk |= e;
                }
                dst[s * kQLanes] = msk;
            }
        };

        // One pass: load (word indices clamped into [0, limit); a word outside it
        // is loaded from a valid index, its planes lie beyond every pair's length
        // or are never used), then transpose and write the pattern words.
        auto pass_load = [&](int k, uint32_t (&raw)[32]) {
            const int w = g == 0 ? 2 * k : (g == 3 ? 2 * k + 1 : (g == 1 ? 2 * k + h : 2 * k + h + 1));
            const int wc = min(max(w, 0), nhalves - 1);
            load_word<kQLanes>(seq + (int64_t)wc * J.ld + base, full, left, pl, raw);
        };
        auto pass_finish = [&](int k, uint32_t (&raw)[32]) {
            transpose32(raw);
            if (!text_group) {
                const int pw = g == 1 ? 2 * k + h : 2 * k + h + 1;
                if (pw >= 0 && pw < nhalves) {
                    if ((R & 7) != 0) {
                        int slot = (pw * kHalf) % R;
#pragma unroll
                        for (int u = 0; u < kHalf; u++) {
                            const uint2 v = make_uint2(raw[2 * u], raw[2 * u + 1]);
                            ring[slot * kQLanes + pl] = v;
                            if (slot < kMirror) ring[(slot + R) * kQLanes + pl] = v;
                            slot = slot + 1 == R ? 0 : slot + 1;
                        }
                    } else {
#pragma unroll
                        for (int hh = 0; hh < 2; hh++) {
                            const int s0 = (pw * kHalf + 8 * hh) % R;
                            uint2 *dst = ring + s0 * kQLanes + pl;
#pragma unroll
                            for (int u = 0; u < 8; u++)
                                dst[u * kQLanes] = make_uint2(raw[2 * (8 * hh + u)], raw[2 * (8 * hh + u) + 1]);
                            if (s0 < kMirror) {
#pragma unroll
                                for (int u = 0; u < 8; u++)
                                    if (s0 + u < kMirror)
                                        dst[(R + u) * kQLanes] =
                                            make_uint2(raw[2 * (8 * hh + u)], raw[2 * (8 * hh + u) + 1]);
                            }
                        }
                    }
                }
            }
        };
        // Text planes of an iteration's block (11 positions, low and high plane):
        // start_text from pass k (all but group 2's positions 8..10), finish_text
        // from pass k+1 (group 2's positions 8..10 = word 2k+2's 0..2, from group 0).
        auto start_text = [&](uint32_t (&T)[2 * kCols], const uint32_t (&raw)[32]) {
#pragma unroll
            for (int t = 0; t < 2 * kBlock; t++) {
                // groups 1 / 2: positions 8..15 of group 0's / group 3's word
                const auto sw = __builtin_amdgcn_permlane16_swap(raw[2 * kBlock + t], raw[2 * kBlock + t], false, false);
                T[t] = text_group ? raw[t] : (g == 1 ? (uint32_t)sw[0] : (uint32_t)sw[1]);
            }
#pragma unroll
            for (int t = 2 * kBlock; t < 2 * kCols; t++) {
                // group 1: positions 0..2 of group 3's word
                const auto sw = __builtin_amdgcn_permlane32_swap(raw[t - 2 * kBlock], raw[t - 2 * kBlock], false, false);
                T[t] = text_group ? raw[t] : (uint32_t)sw[1];
            }
        };
        auto finish_text = [&](uint32_t (&T)[2 * kCols], const uint32_t (&raw)[32]) {
#pragma unroll
            for (int t = 2 * kBlock; t < 2 * kCols; t++) {
                // group 2: positions 0..2 of group 0's word (the next text word)
                const auto sw = __builtin_amdgcn_permlane32_swap(raw[t - 2 * kBlock], raw[t - 2 * kBlock], false, false);
                T[t] = g == 2 ? (uint32_t)sw[0] : T[t];
            }
        };

        uint32_t TA[2 * kCols], TB[2 * kCols];
        if (niter > 0) {
            // pattern-only passes for words 0 .. h-1 (h > 0 only for E >= 30)
            for (int k = -((h + 1) / 2); k < 0; k++) {
                uint32_t raw[32];
                pass_load(k, raw);
                pass_finish(k, raw);
            }
            uint32_t raw[32];
            pass_load(0, raw);
            pass_finish(0, raw);
            start_text(TA, raw);
            pass_load(1, raw);
            pass_finish(1, raw);
            finish_text(TA, raw);
            start_text(TB, raw);
        }

        auto iteration = [&](int j, uint32_t (&Tc)[2 * kCols], uint32_t (&Tn)[2 * kCols]) {
            const int lo = kQWin * j;
            const int i0 = lo + kBlock * q;
            const int hi_col = lo + 3 * kBlock + kCols - 1;   // last text column of the iteration
            Winner<kBlock> W;
            {
                uint32_t tl[kCols], th[kCols];
#pragma unroll
                for (int t = 0; t < kCols; t++) { tl[t] = Tc[2 * t]; th[t] = Tc[2 * t + 1]; }
                const int sb = i0 % R;
                if ((Ee > lo) || (hi_col + Ee >= m_min)) {
                    if (UNI) {
                        block_winners<kBlock, false, true, true, kQLanes>(W, ring, nvg, nvg, pl, i0, sb, Ee, R, lo,
                                                                          hi_col, m_min, tl, th, m_max);
                    } else {
                        fill_masks(i0, nvg, kCols + Ee);
                        block_winners<kBlock, false, true, false, kQLanes>(W, ring, nvg, nvg, pl, i0, sb, Ee, R, lo,
                                                                           hi_col, m_min, tl, th);
                    }
                } else {
                    block_winners<kBlock, false, false, UNI, kQLanes>(W, ring, nvg, nvg, pl, i0, sb, Ee, R, lo, hi_col,
                                                                     m_min, tl, th);
                }
            }
            // the next pass's loads before the serial update (their latency is
            // covered by it)
            const bool do_pass = j + 2 <= niter;
            uint32_t raw[32];
            if (do_pass) pass_load(j + 2, raw);
            // serial update: blocks in the order of groups 0, 1, 3, 2
            uint32_t o[kBlock];
            if (g == 0) block_fsm<kBlock>(F, W, o);
            {   // 0 -> 1
                auto a = __builtin_amdgcn_permlane16_swap(F.s0, F.s0, false, false);
                auto b = __builtin_amdgcn_permlane16_swap(F.s1, F.s1, false, false);
                auto c = __builtin_amdgcn_permlane16_swap(F.s2, F.s2, false, false);
                F.s0 = a[0]; F.s1 = b[0]; F.s2 = c[0];
            }
            if (g == 1) block_fsm<kBlock>(F, W, o);
            {   // 1 -> 3
                auto a = __builtin_amdgcn_permlane32_swap(F.s0, F.s0, false, false);
                auto b = __builtin_amdgcn_permlane32_swap(F.s1, F.s1, false, false);
                auto c = __builtin_amdgcn_permlane32_swap(F.s2, F.s2, false, false);
                F.s0 = a[0]; F.s1 = b[0]; F.s2 = c[0];
            }
            if (g == 3) block_fsm<kBlock>(F, W, o);
            {   // 3 -> 2
                auto a = __builtin_amdgcn_permlane16_swap(F.s0, F.s0, false, false);
                auto b = __builtin_amdgcn_permlane16_swap(F.s1, F.s1, false, false);
                auto c = __builtin_amdgcn_permlane16_swap(F.s2, F.s2, false, false);
                F.s0 = a[1]; F.s1 = b[1]; F.s2 = c[1];
            }
            if (g == 2) block_fsm<kBlock>(F, W, o);
            {   // 2 -> 0
                auto a = __builtin_amdgcn_permlane32_swap(F.s0, F.s0, false, false);
                auto b = __builtin_amdgcn_permlane32_swap(F.s1, F.s1, false, false);
                auto c = __builtin_amdgcn_permlane32_swap(F.s2, F.s2, false, false);
                F.s0 = a[1]; F.s1 = b[1]; F.s2 = c[1];
            }
            block_count<kBlock, false>(F, o, X, i0, ebits);
            if (do_pass) {
                pass_finish(j + 2, raw);
                finish_text(Tn, raw);
                start_text(Tc, raw);
            }
        };
        int j = 0;
        for (; j + 1 < niter; j += 2) {
            pace.step(j);
            iteration(j, TA, TB);
            pace.step(j + 1);
            iteration(j + 1, TB, TA);
        }
        if (j < niter) iteration(j, TA, TB);
        const int nwin = kQWin * niter;

        // ---- sum the four groups' counters (each group then holds the total)
        uint32_t cnt[32];
        cnt[0] = F.ones; cnt[1] = F.twos; cnt[2] = F.fours;
#pragma unroll
        for (int b = 0; b < 8; b++) cnt[3 + b] = F.e[b];
        {
            uint32_t cy = 0u;
#pragma unroll
            for (int b = 0; b < 11; b++) {   // + the partner group in the same 32-lane half
                const auto sw = __builtin_amdgcn_permlane16_swap(cnt[b], cnt[b], false, false);
                const uint32_t o = (g & 1) ? (uint32_t)sw[0] : (uint32_t)sw[1];
                const uint32_t s_ = gate<kTTXor3>(cnt[b], o, cy);
                cy = gate<kTTMaj>(cnt[b], o, cy);
                cnt[b] = s_;
            }
            cy = 0u;
#pragma unroll
            for (int b = 0; b < 11; b++) {   // + the other half
                const auto sw = __builtin_amdgcn_permlane32_swap(cnt[b], cnt[b], false, false);
                const uint32_t o = (g >= 2) ? (uint32_t)sw[0] : (uint32_t)sw[1];
                const uint32_t s_ = gate<kTTXor3>(cnt[b], o, cy);
                cy = gate<kTTMaj>(cnt[b], o, cy);
                cnt[b] = s_;
            }
        }
#pragma unroll
        for (int b = 11; b < 32; b++)
            cnt[b] = (b >= 16 && b < 16 + kLenBits && !UNI) ? lbv[(b - 16) * kQLanes] : 0u;
        cnt[16 + kLenBits] = valid;
        transpose32(cnt);  // cnt[k]: ones of S over windows [0, nwin) | length << 16 | valid << 27
        // group g writes pairs k = 8g .. 8g+7 of its lanes
        int left_out = __builtin_amdgcn_readfirstlane(left);
        asm volatile("" : "+s"(left_out));
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t w = g == 0 ? cnt[i] : (g == 1 ? cnt[8 + i] : (g == 2 ? cnt[16 + i] : cnt[24 + i]));
            const int kk = 8 * g + i;
            const int64_t p = base + (int64_t)kk * kQLanes + pl;
            if (!full && kk * kQLanes + pl >= left_out) continue;
            const int m = UNI ? m_max : (int)((w >> 16) & ((1u << kLenBits) - 1));
            uint8_t acc;
            int16_t pc;
            if (!((w >> (16 + kLenBits)) & 1u)) {
                acc = 0xFF;
                pc = -1;
            } else {
                const int ones = (int)(w & 0xFFFFu) - (nwin - m);   // S stays 1 on [m, nwin)
                const int E = J.Edec ? J.Edec[p] : J.E;
                acc = ones <= E ? 1 : 0;
                pc = (int16_t)ones;
            }
            const int64_t o = J.perm ? J.perm[p] : p;
            J.out_accept[o] = acc;
            if (J.out_popcount) J.out_popcount[o] = pc;
        }
    };
    if constexpr (RO) {
        rest(std::true_type());
    } else {
        if (uniform)
            rest(std::true_type());
        else
            rest(std::false_type());
    }
}

template <bool RO>
__device__ __forceinline__ void plain_wave(const PlainParams &prm, uint32_t *lds_all) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    GroupJob J;
    J.reads = prm.reads;
    J.refs = prm.refs;
    J.ld = prm.ld;
    J.lengths = prm.lengths;
    J.max_len = prm.max_len;
    J.Ee = prm.Ee;
    J.E = prm.E;
    J.Edec = nullptr;
    J.perm = nullptr;
    J.out_accept = prm.out_accept;
    J.out_popcount = prm.out_popcount;
    J.ref_lengths = nullptr;
    J.len_bits = kLenBits;
    J.mode = 0;
    J.base = ((int64_t)blockIdx.x * kWavesPerGroup + wave) * kPairsPerWave;
    J.n = prm.n;
    if (J.base >= J.n) return;
    filter_group<false, RO>(J, lds_all + (size_t)wave * (prm.lds_wave_bytes / 4), prm.R, lane);
}

__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_plain_kernel(PlainParams prm) {
    extern __shared__ uint32_t lds_all[];
    plain_wave<false>(prm, lds_all);
}

// The same without a length array (every pair has max_len bases): the
// boundary masks follow from the positions and the wavefront's LDS holds the
// pattern ring only.
__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_plain_ring_kernel(PlainParams prm) {
    extern __shared__ uint32_t lds_all[];
    plain_wave<true>(prm, lds_all);
}

// Two-length form: reads and references of different lengths, local /
// glocal / global counting.  Workgroups of waves_per_group wavefronts.
__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_local_kernel(LocalParams prm) {
    extern __shared__ uint32_t lds_all[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    GroupJob J;
    J.reads = prm.reads;
    J.refs = prm.refs;
    J.ld = prm.ld;
    J.lengths = prm.read_lengths;
    J.ref_lengths = prm.ref_lengths;
    J.mode = prm.mode;
    J.len_bits = prm.len_bits;
    J.max_len = prm.max_len;
    J.Ee = prm.Ee;
    J.E = prm.E;
    J.Edec = nullptr;
    J.perm = nullptr;
    J.out_accept = prm.out_accept;
    J.out_popcount = prm.out_popcount;
    J.base = ((int64_t)blockIdx.x * prm.waves_per_group + wave) * kPairsPerWave;
    J.n = prm.n;
    if (wave >= prm.waves_per_group || J.base >= J.n) return;
    filter_group<true>(J, lds_all + (size_t)wave * (prm.lds_wave_bytes / 4), prm.R, lane);
}

// Batched form: one wavefront per tile of at most 1024 pairs of one bin of
// the binned workspace (equal E, lengths within one bucket).  Tiles are
// listed in decreasing cost, so the hardware's in-order dispatch hands the
// longest work out first.
__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_tiles_kernel(TilesParams prm) {
    extern __shared__ uint32_t lds_all[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t t = (int64_t)blockIdx.x * prm.waves_per_group + wave;
    if (wave >= prm.waves_per_group || t >= *prm.ntiles) return;
    const int4 tile = prm.tiles[t];                      // start, count, Ee, -
    GroupJob J;
    J.reads = prm.breads;
    J.refs = prm.brefs;
    J.ld = prm.ld;
    J.lengths = prm.blens;
    J.ref_lengths = nullptr;
    J.len_bits = kLenBits;
    J.mode = 0;
    J.max_len = prm.max_len;
    J.Ee = tile.z;
    J.E = 0;
    J.Edec = prm.bE;
    J.perm = prm.bperm;
    J.out_accept = prm.out_accept;
    J.out_popcount = prm.out_popcount;
    J.base = tile.x;
    J.n = (int64_t)tile.x + tile.y;
    filter_group<false>(J, lds_all + (size_t)wave * (prm.lds_wave_bytes / 4), prm.R, lane);
}

// Quarter layout (large E): wavefronts of 512 pairs.
template <bool RO>
__device__ __forceinline__ void plain_wave4(const PlainParams &prm, uint32_t *lds_all) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    GroupJob J;
    J.reads = prm.reads;
    J.refs = prm.refs;
    J.ld = prm.ld;
    J.lengths = prm.lengths;
    J.max_len = prm.max_len;
    J.Ee = prm.Ee;
    J.E = prm.E;
    J.Edec = nullptr;
    J.perm = nullptr;
    J.out_accept = prm.out_accept;
    J.out_popcount = prm.out_popcount;
    J.ref_lengths = nullptr;
    J.len_bits = kLenBits;
    J.mode = 0;
    J.base = ((int64_t)blockIdx.x * kWavesPerGroup + wave) * kQPairs;
    J.n = prm.n;
    if (J.base >= J.n) return;
    filter_group4<RO>(J, lds_all + (size_t)wave * (prm.lds_wave_bytes / 4), prm.R, prm.qh, lane);
}

__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_plain_q_kernel(PlainParams prm) {
    extern __shared__ uint32_t lds_all[];
    plain_wave4<false>(prm, lds_all);
}

__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_plain_ring_q_kernel(PlainParams prm) {
    extern __shared__ uint32_t lds_all[];
    plain_wave4<true>(prm, lds_all);
}

// Batched tiles of the large-E class in the quarter layout: two wavefronts
// per tile of at most 1024 pairs (512 each).
__global__ __launch_bounds__(kWave * kWavesPerGroup, 2) void shouji_tiles_q_kernel(TilesParams prm) {
    extern __shared__ uint32_t lds_all[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t t2 = (int64_t)blockIdx.x * prm.waves_per_group + wave;
    const int64_t t = t2 >> 1;
    if (wave >= prm.waves_per_group || t >= *prm.ntiles) return;
    const int4 tile = prm.tiles[t];                      // start, count, Ee, -
    GroupJob J;
    J.reads = prm.breads;
    J.refs = prm.brefs;
    J.ld = prm.ld;
    J.lengths = prm.blens;
    J.ref_lengths = nullptr;
    J.len_bits = kLenBits;
    J.mode = 0;
    J.max_len = prm.max_len;
    J.Ee = tile.z;
    J.E = 0;
    J.Edec = prm.bE;
    J.perm = prm.bperm;
    J.out_accept = prm.out_accept;
    J.out_popcount = prm.out_popcount;
    J.base = (int64_t)tile.x + (t2 & 1) * kQPairs;
    J.n = (int64_t)tile.x + tile.y;
    if (J.base >= J.n) return;
    filter_group4<false>(J, lds_all + (size_t)wave * (prm.lds_wave_bytes / 4), prm.R, prm.qh, lane);
}

}  // namespace shouji
