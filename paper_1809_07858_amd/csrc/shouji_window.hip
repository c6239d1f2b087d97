// Window-width variant of the Shouji filter: W-column windows instead of 4
// (Suppl. Sec. 6.1 and Fig. 4 compare the false accept rates of window
// widths; 4 is the paper's choice).  Same steps as the plain form -- the
// 2E+1 diagonals of the neighbourhood map (Eq. 1), per window the diagonal
// segment with the most zeros (ties: a leading zero, then Algorithm 1's
// order d = +1, -1, ..., +E, -E, main), copied into S[i..i+W-1] when it has
// strictly more zeros, accept iff ones(S[0..m)) <= E -- with W a compile-time
// parameter (1..16) chosen at launch.
//
// Bit-sliced like the plain form: every 32-bit register holds one bit of one
// quantity for 32 pairs.  Here every lane has pairs of its own (bit k of lane
// l belongs to pair base + 64k + l), so a wavefront filters 2048 pairs and no
// state moves between lanes.  Per wavefront:
//  * packed words (16 bases, word-major) are loaded for 32 pairs at a time
//    and turned into bit planes by a 32x32 transpose; pattern planes go to a
//    ring in LDS, text planes to a second, smaller ring.  The next word is
//    loaded one step ahead (while a block is searched) and stored when the
//    first block that reads it starts;
//  * windows run in blocks of 4.  For each candidate diagonal the block's
//    W+3 cells are built (Eq. 1: either code bit differs), each window's W
//    cells are counted by a carry-save adder tree, and the segment replaces
//    the block's running winner when its key (ones, then the first bit) is
//    strictly smaller;
//  * the bit-vector update keeps S[i..i+W-2] as W-1 planes (S[i+W-1] is
//    still 1 when window i runs): write iff ones(Z) <= ones(S[i..i+W-2]);
//    S[i] is then final and is added to a bit-sliced counter;
//  * the counters are transposed back to one count per pair.
// Cells outside the map are mismatches: positions before the pattern start
// and, in a wavefront whose pairs all have one length, positions at or past
// it follow from the position alone; with mixed lengths a candidate near the
// end ORs in per-pair masks compared out of the length bit planes.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/shouji.h"
#include "shouji_bitslice.h"
#include "shouji_internal.h"
#include "shouji_launch.h"
#include "shouji_variants.h"

namespace shouji {

constexpr int kWinLanes = 64;                     // every lane holds its own 32 pairs
constexpr int kWinPairsPerWave = kWinLanes * 32;  // 2048
constexpr int kWinBlock = 4;                      // windows per block

__host__ __device__ constexpr int win_cols(int W) { return kWinBlock + W - 1; }
// Pattern ring: positions i0-E .. i0+C-1+E of a block, plus the rest of the
// last word loaded (15 positions).  Text ring: columns i0 .. i0+C-1, plus the
// rest of the last word, at most two words (a block's columns never reach a
// third word, and the word stored for a block is never the one two words
// back that an earlier block still read, as C <= 20).
__host__ __device__ constexpr int win_pattern_slots(int W, int Ee) { return win_cols(W) + 2 * Ee + kHalf - 1; }
__host__ __device__ constexpr int win_text_slots(int W) {
    return win_cols(W) + kHalf - 1 < 2 * kHalf ? win_cols(W) + kHalf - 1 : 2 * kHalf;
}
// The pattern ring's first C-1 slots are also kept past its end (a mirror),
// so that a candidate's C slots are one run from any start, where the mirror
// leaves four wavefronts per CU at E = 5 (W <= 10); wider windows read a
// wrapping run in two parts.
__host__ __device__ constexpr int win_mirror_slots(int W) { return W <= 10 ? win_cols(W) - 1 : 0; }
inline size_t win_lds_bytes(int W, int Ee) {
    return (size_t)(win_pattern_slots(W, Ee) + win_mirror_slots(W) + win_text_slots(W)) * kWinLanes * 8;
}
// bits of a count 0..v
__host__ __device__ constexpr int count_bits(int v) { return v <= 1 ? 1 : 1 + count_bits(v >> 1); }

// a + b + c = 2h + l, bit by bit
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t u = a ^ b;
    h = (a & b) | (u & c);
    l = u ^ c;
}

// Ones of the N planes x[0..N-1] (N <= 16) as bit planes o[0..4] of the
// count: column by column (weights 1, 2, 4, ...), three planes of a column
// are replaced by their sum while at least three remain, a last pair by a
// half adder, the carries going to the next column.  The plane counts are
// compile-time constants once the loops are unrolled.
template <int N>
__device__ __forceinline__ void count_planes(const uint32_t *x, uint32_t (&o)[5]) {
    static_assert(N >= 0 && N <= 16, "at most 16 planes");
    uint32_t col[5][16];
    int cnt[5] = {N, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < N; i++) col[0][i] = x[i];
#pragma unroll
    for (int w = 0; w < 5; w++) {
#pragma unroll
        for (int it = 0; it < 8; it++) {
            if (cnt[w] >= 3) {
                uint32_t h, l;
                csa(h, l, col[w][cnt[w] - 3], col[w][cnt[w] - 2], col[w][cnt[w] - 1]);
                col[w][cnt[w] - 3] = l;
                cnt[w] -= 2;
                if (w + 1 < 5) col[w + 1 < 5 ? w + 1 : 0][cnt[w + 1 < 5 ? w + 1 : 0]++] = h;
            }
        }
        if (cnt[w] == 2) {
            const uint32_t a = col[w][0], b = col[w][1];
            col[w][0] = a ^ b;
            cnt[w] = 1;
            if (w + 1 < 5) col[w + 1 < 5 ? w + 1 : 0][cnt[w + 1 < 5 ? w + 1 : 0]++] = a & b;
        }
        o[w] = cnt[w] ? col[w][0] : 0u;
    }
}

// core + a + b + c as bit planes out[0..4]: the three planes by one full
// adder into a 2-bit sum, then a ripple add into the core count's planes.
__device__ __forceinline__ void add_three(const uint32_t (&core)[5], uint32_t a, uint32_t b, uint32_t c,
                                          uint32_t (&out)[5]) {
    uint32_t s1, s0;
    csa(s1, s0, a, b, c);
    out[0] = core[0] ^ s0;
    uint32_t cy = core[0] & s0;
    uint32_t h;
    csa(h, out[1], core[1], s1, cy);
    cy = h;
#pragma unroll
    for (int k = 2; k < 5; k++) {
        out[k] = core[k] ^ cy;
        cy = core[k] & cy;
    }
}

// C consecutive ring slots from slot s (wave-uniform) of a ring of R slots.
template <int C>
__device__ __forceinline__ void win_ring_read(const uint2 *ring, int R, int s, int lane, uint2 (&v)[C]) {
    if (s + C <= R) {
        const uint2 *p = ring + s * kWinLanes + lane;
#pragma unroll
        for (int t = 0; t < C; t++) v[t] = p[t * kWinLanes];
    } else {
#pragma unroll
        for (int t = 0; t < C; t++) {
            const int x = s + t >= R ? s + t - R : s + t;
            v[t] = ring[x * kWinLanes + lane];
        }
    }
}

template <int W>
__global__ __launch_bounds__(kWinLanes, 1) void window_bs_kernel(WindowParams prm) {
    constexpr int NB = kWinBlock;
    constexpr int C = win_cols(W);
    constexpr int KB = count_bits(W);          // bits of a segment's ones count
    extern __shared__ __align__(16) uint32_t lds_win[];
    const int lane = threadIdx.x;
    const int Ee = prm.Ee;
    const int Rp = win_pattern_slots(W, Ee), Rt = win_text_slots(W);
    constexpr int MIR = win_mirror_slots(W);
    uint2 *pring = reinterpret_cast<uint2 *>(lds_win);
    uint2 *tring = pring + (Rp + MIR) * kWinLanes;
    static_assert(win_cols(W) <= 20, "a block's text columns span at most two words");

    const int64_t base = (int64_t)blockIdx.x * kWinPairsPerWave;
    const int left = (int)min(prm.n - base, (int64_t)kWinPairsPerWave);
    const bool full = left == kWinPairsPerWave;

    // ---- lengths: per pair (a missing pair reads the wavefront's last one),
    // the valid-pair plane, and the shortest / longest valid length
    uint32_t lenw[32];
    uint32_t valid = 0u;
    int lmin = 0x7fffffff, lmax = -1;
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int q = k * kWinLanes + lane;
        const int m = prm.lengths ? prm.lengths[base + min(q, left - 1)] : prm.max_len;
        const bool ok = q < left && m >= 0 && m <= prm.max_len;
        lenw[k] = ok ? (uint32_t)m : 0u;
        valid |= ok ? (1u << k) : 0u;
        if (ok) {
            lmin = min(lmin, m);
            lmax = max(lmax, m);
        }
    }
    lmin = __builtin_amdgcn_readfirstlane(wave_min(lmin));
    lmax = __builtin_amdgcn_readfirstlane(wave_max(lmax));
    const int m_max = lmax < 0 ? 0 : lmax;
    const int m_min = lmax < 0 ? 0 : lmin;
    const bool uniform = m_min == m_max;       // masks from the positions alone
    transpose32(lenw);                         // lenw[b] = bit b of the lengths
    // diagonals this wavefront needs: beyond m_max - 1 every cell is outside
    // the map, and such all-ones segments never win
    const int Ew = min(Ee, max(m_max - 1, 0));
    // per pair: position x (uniform) is at or past the pair's end, from the
    // length bit planes (mixed lengths only, near the end)
    auto past_end = [&](int x) {
        uint32_t g = 0u;                       // g = (length > x), from the low bit up
#pragma unroll
        for (int b = 0; b < kLenBits; b++) {
            const uint32_t sx = ((x >> b) & 1) ? ~0u : 0u;
            g = (sx & lenw[b] & g) | (~sx & (lenw[b] | g));
        }
        return ~g;
    };

    // ---- word loads: pattern word pw is first read by the block at
    // 16pw - (C-1+Ew), text word tw by the block at 16tw - (C-1); words are
    // loaded in that order, one ahead, and stored when first needed
    const int nw = (m_max + kHalf - 1) / kHalf;
    int np = 0, nt = 0;                        // next pattern / text word to load
    auto next_kind = [&]() -> int {            // 0 pattern, 1 text, -1 none left
        if (np >= nw && nt >= nw) return -1;
        if (nt >= nw) return 0;
        if (np >= nw) return 1;
        return kHalf * np - (C - 1 + Ew) <= kHalf * nt - (C - 1) ? 0 : 1;
    };
    auto need = [&](int kind, int w) { return kHalf * w - (C - 1) - (kind ? 0 : Ew); };
    uint32_t raw[32];
    int pk = next_kind(), pw = 0;
    auto issue = [&]() {
        if (pk < 0) return;
        pw = pk ? nt++ : np++;
        const uint32_t *seq = pk ? prm.refs : prm.reads;
        load_word<kWinLanes>(seq + (int64_t)pw * prm.ld + base, full, left, lane, raw);
    };
    issue();
    auto store = [&]() {
        uint2 *ring = pk ? tring : pring;
        const int R = pk ? Rt : Rp;
        int slot = (kHalf * pw) % R;
        transpose32(raw);                      // raw[2u], raw[2u+1]: code bits of position 16pw+u
#pragma unroll
        for (int u = 0; u < kHalf; u++) {
            const uint2 v = make_uint2(raw[2 * u], raw[2 * u + 1]);
            ring[slot * kWinLanes + lane] = v;
            if (MIR > 0 && pk == 0 && slot < MIR) ring[(slot + R) * kWinLanes + lane] = v;
            slot = slot + 1 == R ? 0 : slot + 1;
        }
    };

    uint32_t s[W > 1 ? W - 1 : 1];             // S[i..i+W-2] before window i
#pragma unroll
    for (int t = 0; t < W - 1; t++) s[t] = ~0u;
    uint32_t tot[kLenBits];                    // ones of the final bits, bit planes
#pragma unroll
    for (int b = 0; b < kLenBits; b++) tot[b] = 0u;

    int sb = 0, st = 0;                        // ring slots of position i0
    for (int i0 = 0; i0 < m_max; i0 += NB) {
        while (pk >= 0 && need(pk, pw) <= i0) {
            store();
            pk = next_kind();
            issue();
        }
        // some position the block reads reaches the shortest length
        const bool near_end = i0 + C - 1 + Ew >= m_min;
        uint32_t tl[C], th[C];
        {
            uint2 tv[C];
            win_ring_read<C>(tring, Rt, st, lane, tv);
#pragma unroll
            for (int t = 0; t < C; t++) { tl[t] = tv[t].x; th[t] = tv[t].y; }
        }
        // running winner of each window: count planes and the segment
        uint32_t wc[NB][KB], wz[NB][W];
        const bool any_mask = i0 < Ew || near_end;
        // one candidate diagonal d, with pv the pattern planes of positions
        // i0-d .. i0-d+C-1
        auto candidate = [&](auto first_tag, int d, const uint2 (&pv)[C]) {
            constexpr bool FIRST = decltype(first_tag)::value;
            uint32_t c[C];
#pragma unroll
            for (int t = 0; t < C; t++) c[t] = (pv[t].x ^ tl[t]) | (pv[t].y ^ th[t]);   // Eq. 1
            const bool masked = any_mask && (d > i0 || i0 + C - 1 >= m_min || i0 + C - 1 - d >= m_min);
            if (masked) {
                if (uniform) {
#pragma unroll
                    for (int t = 0; t < C; t++) {
                        const int xt = i0 + t, xp = i0 + t - d;
                        if (xt >= m_max || xp >= m_max || xp < 0) c[t] = ~0u;
                    }
                } else {
                    if (near_end) {
                        // d >= 0: the text column runs out first; d < 0: the
                        // pattern position i0+t-d
                        const int x0 = i0 + (d < 0 ? -d : 0);
#pragma unroll
                        for (int t = 0; t < C; t++) c[t] |= past_end(x0 + t);
                    }
#pragma unroll
                    for (int t = 0; t < C; t++)
                        if (i0 + t - d < 0) c[t] = ~0u;
                }
            }
            // the NB windows share cells NB-1 .. W-1: their ones are counted
            // once, each window then adds its NB-1 other cells
            constexpr bool kShared = W >= 6;
            static_assert(NB == 4, "each window has three cells outside the shared part");
            uint32_t core[5];
            if constexpr (kShared) count_planes<kShared ? W - (NB - 1) : 0>(c + (NB - 1), core);
#pragma unroll
            for (int w = 0; w < NB; w++) {
                uint32_t k[5];
                if constexpr (kShared) {
                    // cells w .. NB-2 before the shared part, W .. W+w-1 after it
                    uint32_t e[NB - 1];
#pragma unroll
                    for (int j = 0; j < NB - 1; j++) e[j] = j < NB - 1 - w ? c[w + j] : c[W + j - (NB - 1 - w)];
                    add_three(core, e[0], e[1], e[2], k);
                } else {
                    count_planes<W>(c + w, k);
                }
                if constexpr (FIRST) {
#pragma unroll
                    for (int b = 0; b < KB; b++) wc[w][b] = k[b];
#pragma unroll
                    for (int t = 0; t < W; t++) wz[w][t] = c[w + t];
                } else {
                    // lt = (count, first bit) < the winner's: borrow chain
                    uint32_t lt = ~c[w] & wz[w][0];
#pragma unroll
                    for (int b = 0; b < KB; b++) {
                        const uint32_t na = ~k[b], bb = wc[w][b];
                        lt = (na & bb) | (lt & (na | bb));
                    }
#pragma unroll
                    for (int b = 0; b < KB; b++) wc[w][b] = (lt & k[b]) | (~lt & wc[w][b]);
#pragma unroll
                    for (int t = 0; t < W; t++) wz[w][t] = (lt & c[w + t]) | (~lt & wz[w][t]);
                }
            }
        };
        using First = std::integral_constant<bool, true>;
        using Later = std::integral_constant<bool, false>;
        // pattern planes of a candidate: C ring slots from slot ps
        uint2 pv[C];
        auto rd = [&](int ps) {
            if constexpr (MIR > 0) {
                const uint2 *p = pring + ps * kWinLanes + lane;
#pragma unroll
                for (int t = 0; t < C; t++) pv[t] = p[t * kWinLanes];
            } else {
                win_ring_read<C>(pring, Rp, ps, lane, pv);
            }
        };
        if (Ew == 0) {
            rd(sb);
            candidate(First{}, 0, pv);
        } else {
            int sP = sb == 0 ? Rp - 1 : sb - 1;     // slot of position i0 - k
            int sN = sb + 1 == Rp ? 0 : sb + 1;     // slot of position i0 + k
            rd(sP);
            candidate(First{}, 1, pv);
            rd(sN);
            candidate(Later{}, -1, pv);
            for (int k = 2; k <= Ew; k++) {
                sP = sP == 0 ? Rp - 1 : sP - 1;
                sN = sN + 1 == Rp ? 0 : sN + 1;
                rd(sP);
                candidate(Later{}, k, pv);
                rd(sN);
                candidate(Later{}, -k, pv);
            }
            rd(sb);
            candidate(Later{}, 0, pv);
        }

        // ---- the bit-vector update, window by window
        uint32_t o[NB];
#pragma unroll
        for (int w = 0; w < NB; w++) {
            uint32_t os[5];
            count_planes<W - 1>(s, os);
            // gt = ones(Z) > ones(S[i..i+W-2]): borrow chain of os - ones(Z)
            uint32_t gt = 0u;
#pragma unroll
            for (int b = 0; b < KB; b++) {
                const uint32_t na = ~os[b], bb = wc[w][b];
                gt = (na & bb) | (gt & (na | bb));
            }
            const uint32_t wr = ~gt;
            const uint32_t s0 = W > 1 ? s[0] : ~0u;
            o[w] = (wr & wz[w][0]) | (~wr & s0);
#pragma unroll
            for (int t = 0; t < W - 1; t++) {
                const uint32_t nxt = t + 1 < W - 1 ? s[t + 1 < W - 1 ? t + 1 : 0] : ~0u;
                s[t] = (wr & wz[w][t + 1]) | (~wr & nxt);
            }
        }
        // final bits of positions at or past a pair's end are not counted
        if (uniform) {
#pragma unroll
            for (int w = 0; w < NB; w++)
                if (i0 + w >= m_max) o[w] = 0u;
        } else if (i0 + NB - 1 >= m_min) {
#pragma unroll
            for (int w = 0; w < NB; w++) o[w] &= ~past_end(i0 + w);
        }
        uint32_t q[5];
        count_planes<NB>(o, q);
        uint32_t cy = 0u;
#pragma unroll
        for (int b = 0; b < kLenBits; b++) {
            const uint32_t a = b < 3 ? q[b < 3 ? b : 0] : 0u;
            const uint32_t x = tot[b] ^ a;
            const uint32_t nc = (tot[b] & a) | (x & cy);
            tot[b] = x ^ cy;
            cy = nc;
        }
        sb += NB; if (sb >= Rp) sb -= Rp;
        st += NB; if (st >= Rt) st -= Rt;
    }

    // ---- counts back to one value per pair
    uint32_t cnt[32];
#pragma unroll
    for (int b = 0; b < 32; b++) cnt[b] = b < kLenBits ? tot[b < kLenBits ? b : 0] : 0u;
    transpose32(cnt);
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int qi = k * kWinLanes + lane;
        if (qi < left) {
            const bool ok = (valid >> k) & 1u;
            const int ones = (int)cnt[k];
            prm.out_accept[base + qi] = ok ? (ones <= prm.E ? 1 : 0) : 0xFF;
            if (prm.out_popcount) prm.out_popcount[base + qi] = ok ? (int16_t)ones : (int16_t)-1;
        }
    }
}

template <int W>
static int launch_window(const WindowParams &prm, unsigned grid, hipStream_t st) {
    static LdsLimit limit;
    const size_t bytes = win_lds_bytes(W, prm.Ee);
    if (int rc = raise_lds_limit(reinterpret_cast<const void *>(&window_bs_kernel<W>), limit, bytes)) return rc;
    hipLaunchKernelGGL(window_bs_kernel<W>, dim3(grid), dim3(kWinLanes), bytes, st, prm);
    return SHOUJI_OK;
}

}  // namespace shouji

extern "C" int shouji_filter_window(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                                    int32_t E, int32_t W, uint8_t *out_accept, int16_t *out_popcount,
                                    int64_t n_pairs, int32_t max_len, int64_t ld, void *stream) {
    using shouji::set_error;
    if (n_pairs < 0) return set_error(SHOUJI_ERR_ARG, "shouji_filter_window: n_pairs < 0");
    if (E < 0) return set_error(SHOUJI_ERR_ARG, "shouji_filter_window: E < 0 (%d)", E);
    if (W < 1 || W > SHOUJI_MAX_WINDOW)
        return set_error(SHOUJI_ERR_RANGE, "shouji_filter_window: W %d outside [1, %d]", W, SHOUJI_MAX_WINDOW);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_filter_window: max_len %d outside [0, %d]", max_len,
                         SHOUJI_MAX_LEN);
    const int32_t Ee = max_len > 0 ? (E < max_len - 1 ? E : max_len - 1) : 0;
    if (Ee > SHOUJI_MAX_E)
        return set_error(SHOUJI_ERR_RANGE, "shouji_filter_window: E %d (clamped %d) above %d", E, Ee, SHOUJI_MAX_E);
    if (n_pairs == 0) return shouji::clear_error();
    if (!reads || !refs || !out_accept)
        return set_error(SHOUJI_ERR_NULL, "shouji_filter_window: reads, refs and out_accept are required");
    if (ld < n_pairs)
        return set_error(SHOUJI_ERR_ARG, "shouji_filter_window: ld %lld < n_pairs %lld", (long long)ld,
                         (long long)n_pairs);
    const int64_t groups = (n_pairs + shouji::kWinPairsPerWave - 1) / shouji::kWinPairsPerWave;
    if (groups > 0x7fffffff) return set_error(SHOUJI_ERR_ARG, "shouji_filter_window: n_pairs too large");
    shouji::WindowParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.lengths = lengths;
    prm.max_len = max_len;
    prm.E = E;
    prm.Ee = Ee;
    prm.W = W;
    prm.out_accept = out_accept;
    prm.out_popcount = out_popcount;
    prm.n = n_pairs;
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)groups;
    int rc = SHOUJI_OK;
    switch (W) {
#define SHOUJI_WIN_CASE(w) \
    case w: rc = shouji::launch_window<w>(prm, grid, st); break;
        SHOUJI_WIN_CASE(1) SHOUJI_WIN_CASE(2) SHOUJI_WIN_CASE(3) SHOUJI_WIN_CASE(4)
        SHOUJI_WIN_CASE(5) SHOUJI_WIN_CASE(6) SHOUJI_WIN_CASE(7) SHOUJI_WIN_CASE(8)
        SHOUJI_WIN_CASE(9) SHOUJI_WIN_CASE(10) SHOUJI_WIN_CASE(11) SHOUJI_WIN_CASE(12)
        SHOUJI_WIN_CASE(13) SHOUJI_WIN_CASE(14) SHOUJI_WIN_CASE(15) SHOUJI_WIN_CASE(16)
#undef SHOUJI_WIN_CASE
    }
    if (rc != SHOUJI_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "shouji_filter_window: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
