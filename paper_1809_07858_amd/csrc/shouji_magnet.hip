// MAGNET pre-alignment filter (Suppl. Sec. 7.1, Algorithms 3 and 4): the
// variant of the Shouji paper that shares its neighbourhood map (Eq. 1) and
// replaces the window search by a divide-and-conquer extraction of the
// longest runs of matches.
//
// Per pair: the 2E+1 diagonals are indexed by text position.  Starting from
// the whole range, a subproblem [lo, hi] takes the longest run of zeros over
// all diagonals (per diagonal the leftmost of equally long runs; across
// diagonals the order d = -1, +1, -2, +2, ..., -E, +E, then the main
// diagonal, a later one replacing the kept run only when strictly longer),
// counts it as zeros of the MAGNET bit-vector, and splits into the parts
// right of it and left of it, each shortened by one encapsulating position;
// the right part is solved first.  At most E+1 runs are taken; a part with no
// zero on any diagonal takes none; the first subproblem stops the pair at
// once when its run is shorter than ceil((m-E)/(E+1)).  Accept iff the
// vector has at most E ones.  Runs taken lie in disjoint parts, so only
// their total length is kept.
//
// One pair per lane: the recursion is a stack of pending parts in LDS (the
// right part pushed last, so that its whole subtree is solved before the
// left part), E+1 entries per lane: every run taken pops one part and pushes
// at most two, and nothing is pushed after the (E+1)-th run, so at most E+1
// parts are ever pending; sized per launch, it leaves LDS for more
// wavefronts at small E.  For max_len <= 256, where the LDS it takes leaves a
// CU enough of its workgroups, each lane first copies its pair's words (both
// sequences', or the read's alone) into a column of LDS of its own (no
// barrier: no lane reads another's column), so the many re-reads of the same
// words by the run searches of every diagonal and part wait on LDS, not on
// the caches; the words not copied are read from global memory.  A diagonal's run search walks 16 text positions per step: the
// reference word, the read's two words around the diagonal's offset joined
// with v_alignbit, one XOR and a fold give the 16 match bits, and the
// longest run of matches in the word is found with doubling masks and a
// binary descent on its length (no loop over the mismatches).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shouji.h"
#include "shouji_internal.h"
#include "shouji_variants.h"

namespace shouji {

namespace {

// even-bit mask of the 2-bit fields 0..n-1 (n in [0, 16])
__device__ __forceinline__ uint32_t field_mask(int n) {
    return n >= 16 ? 0x55555555u : (0x55555555u & ((1u << (2 * n)) - 1u));
}

}  // namespace

template <int STAGED>
__global__ __launch_bounds__(kMagnetBlock) void magnet_kernel(MagnetParams prm) {
    // (E+1) stack entries per lane, then (STAGED) the lane's read words and
    // reference words, ceil(max_len/16) entries each
    extern __shared__ uint32_t stack[];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kMagnetBlock + tid;
    if (p >= prm.n) return;
    const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
    if (m < 0 || m > prm.max_len) {
        prm.out_accept[p] = 0xFF;
        if (prm.out_popcount) prm.out_popcount[p] = -1;
        return;
    }
    const int E = prm.E;
    const int Ee = prm.Ee;
    const uint32_t *P = prm.reads + p;
    const uint32_t *T = prm.refs + p;
    const int64_t ld = prm.ld;
    const int nw = (m + 15) >> 4;                       // words holding the pair's bases
    uint32_t *sP = stack + (prm.E + 1) * kMagnetBlock + tid;
    uint32_t *sT = sP + ((prm.max_len + 15) >> 4) * kMagnetBlock;
    if (STAGED) {
        for (int k = 0; k < nw; k++) {
            sP[k * kMagnetBlock] = P[(int64_t)k * ld];
            if (STAGED == 2) sT[k * kMagnetBlock] = T[(int64_t)k * ld];
        }
    }
    auto read_word = [&](int k) -> uint32_t { return STAGED ? sP[k * kMagnetBlock] : P[(int64_t)k * ld]; };
    auto ref_word = [&](int k) -> uint32_t { return STAGED == 2 ? sT[k * kMagnetBlock] : T[(int64_t)k * ld]; };
    const int thr = m > E ? (m - E + (E + 1) - 1) / (E + 1) : 0;   // ceil((m-E)/(E+1))

    // longest run of zeros of diagonal d inside text positions [lo, hi]
    // (leftmost of equal ones), one 16-position word at a time.  x marks the
    // word's matches inside the range (2-bit fields, even bits); a run that
    // reaches the word's end is carried into the next word.  In a word: the
    // carried run ends at the first mismatch; the runs strictly between the
    // first and the last mismatch are searched with doubling masks (r_k: a
    // run of at least k starts here) and a binary descent on the length; the
    // matches after the last mismatch are carried on.  The result is exact
    // when it is at least `need`; the walk stops as soon as no run of the
    // rest of the range can reach `need` or exceed the longest found.
    auto longest = [&](int d, int lo, int hi, int &start, int need) -> int {
        const int a = lo > d ? lo : d;                       // pattern index j-d >= 0
        const int b = hi < m - 1 + d ? hi : m - 1 + d;       // pattern index j-d < m
        int best = 0;
        start = 0;
        if (a > b) return 0;
        int carry = 0, cs = (a >> 4) * 16;                  // run reaching the word's start
        // read position 16w - d of field 0 of text word w lies in read word
        // w + dq at bit 2 * ((-d) mod 16), the same for every w; a word's upper
        // read word is the next word's lower one.  Fields in [a, b] have read
        // positions in [0, m), so a word index outside the read's words only
        // feeds fields that are masked: it is clamped to a valid word.
        const int dq = (-d) >> 4;                            // floor division
        const int ob = ((-d) & 15) * 2;
        auto rword = [&](int q) -> uint32_t { return read_word(min(max(q, 0), nw - 1)); };
        uint32_t lo_w = rword((a >> 4) + dq);
        // fields inside [a, b]: only the first and the last word are cut
        const int wa = a >> 4, wb = b >> 4;
        const uint32_t m_first = ~field_mask(a - 16 * wa), m_last = field_mask(b - 16 * wb + 1);
        for (int w = wa; w <= wb; w++) {
            const int rest = b - (a > 16 * w ? a : 16 * w) + 1;   // positions left in the range
            if (carry + rest <= (best > need - 1 ? best : need - 1)) break;
            const uint32_t tw = ref_word(w);
            const uint32_t hi_w = rword(w + dq + 1);
            const uint32_t pv = __builtin_amdgcn_alignbit(hi_w, lo_w, ob);
            lo_w = hi_w;
            const uint32_t xr = tw ^ pv;
            uint32_t in_range = 0x55555555u;
            if (w == wa) in_range &= m_first;
            if (w == wb) in_range &= m_last;
            const uint32_t x = ~(xr | (xr >> 1)) & in_range;  // matches
            if (x == 0x55555555u) {                          // 16 matches: the run goes on
                carry += 16;
                continue;
            }
            const uint32_t mis = ~x & 0x55555555u;           // mismatches (and positions out of range)
            const int lead = __builtin_ctz(mis) >> 1;
            if (carry + lead > best) {
                best = carry + lead;
                start = cs;
            }
            const int trail = 15 - ((31 - __builtin_clz(mis)) >> 1);
            // matches strictly between the first and the last mismatch
            // (lead <= 15, trail <= 15: the shifts stay below 32)
            const uint32_t xi = x & (0x55555555u << (2 * lead)) & (0x55555555u >> (2 * trail));
            if (xi) {
                const uint32_t r2 = xi & (xi >> 2), r4 = r2 & (r2 >> 4), r8 = r4 & (r4 >> 8);
                int L = 1;
                uint32_t cur = xi;
                uint32_t cand = cur & (r8 >> (2 * L));
                if (cand) { cur = cand; L += 8; }
                cand = cur & (r4 >> (2 * L));
                if (cand) { cur = cand; L += 4; }
                cand = L < 15 ? cur & (r2 >> (2 * L)) : 0u;
                if (cand) { cur = cand; L += 2; }
                cand = L < 16 ? cur & (xi >> (2 * L)) : 0u;
                if (cand) { cur = cand; L += 1; }
                if (L > best) {
                    best = L;
                    start = 16 * w + (__builtin_ctz(cur) >> 1);
                }
            }
            carry = trail;
            cs = 16 * w + 16 - trail;
        }
        if (carry > best) {
            best = carry;
            start = cs;
        }
        return best;
    };

    uint32_t *stk = stack + tid;                              // entry k at stk[k * kMagnetBlock]
    int sp = 0;
    if (m > 0) {
        stk[0] = (uint32_t)(m - 1) << 16;                    // [0, m-1]
        sp = 1;
    }
    int zeros = 0, taken = 0;
    bool first = true;
    while (sp > 0) {
        sp--;
        const uint32_t e = stk[sp * kMagnetBlock];
        const int lo = (int)(e & 0xFFFFu), hi = (int)(e >> 16);
        // The main diagonal comes last in the order but is searched first:
        // its run bounds what every other diagonal must reach.  A side
        // diagonal precedes it, so it takes over from the main run on a tie,
        // and from an earlier side run only when strictly longer.  A run of
        // length 0 takes nothing, and in the first call a run shorter than
        // thr stops the pair whichever diagonal holds it, so neither needs
        // an exact length.
        int s = 0;
        int len = longest(0, lo, hi, s, first ? thr : 1);
        bool main_kept = true;
        for (int r = 0; r < 2 * Ee; r++) {
            const int d = (r & 1) ? (r >> 1) + 1 : -((r >> 1) + 1);
            int need = main_kept ? len : len + 1;
            if (need < 1) need = 1;
            if (first && need < thr) need = thr;
            int st;
            const int l = longest(d, lo, hi, st, need);
            if (l >= need) {
                len = l;
                s = st;
                main_kept = false;
            }
        }
        if (first && len < thr) {                            // early termination: all ones
            zeros = 0;
            break;
        }
        first = false;
        if (len == 0) continue;                              // no zero in this part
        zeros += len;
        if (++taken == E + 1) break;                         // E+1 runs taken
        // left part [lo, s-2], then right part [s+len+1, hi] on top
        if (lo <= s - 2 && sp <= E) stk[(sp++) * kMagnetBlock] = (uint32_t)lo | ((uint32_t)(s - 2) << 16);
        if (s + len + 1 <= hi && sp <= E)
            stk[(sp++) * kMagnetBlock] = (uint32_t)(s + len + 1) | ((uint32_t)hi << 16);
    }
    const int ones = m - zeros;
    prm.out_accept[p] = ones <= E ? 1 : 0;
    if (prm.out_popcount) prm.out_popcount[p] = (int16_t)ones;
}

}  // namespace shouji

extern "C" int shouji_filter_magnet(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths, int32_t E,
                                    uint8_t *out_accept, int16_t *out_popcount, int64_t n_pairs, int32_t max_len,
                                    int64_t ld, void *stream) {
    using shouji::set_error;
    if (n_pairs < 0) return set_error(SHOUJI_ERR_ARG, "shouji_filter_magnet: n_pairs < 0");
    if (E < 0) return set_error(SHOUJI_ERR_ARG, "shouji_filter_magnet: E < 0 (%d)", E);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_filter_magnet: max_len %d outside [0, %d]", max_len,
                         SHOUJI_MAX_LEN);
    const int32_t Ee = max_len > 0 ? (E < max_len - 1 ? E : max_len - 1) : 0;
    if (Ee > SHOUJI_MAX_E)
        return set_error(SHOUJI_ERR_RANGE, "shouji_filter_magnet: E %d (clamped %d) above %d", E, Ee, SHOUJI_MAX_E);
    if (n_pairs == 0) return shouji::clear_error();
    if (!reads || !refs || !out_accept)
        return set_error(SHOUJI_ERR_NULL, "shouji_filter_magnet: reads, refs and out_accept are required");
    if (ld < n_pairs)
        return set_error(SHOUJI_ERR_ARG, "shouji_filter_magnet: ld %lld < n_pairs %lld", (long long)ld,
                         (long long)n_pairs);
    if ((n_pairs + shouji::kMagnetBlock - 1) / shouji::kMagnetBlock > 0x7fffffff)
        return set_error(SHOUJI_ERR_ARG, "shouji_filter_magnet: n_pairs too large");
    shouji::MagnetParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.lengths = lengths;
    prm.max_len = max_len;
    prm.E = E < max_len ? E : max_len;   // E >= m behaves as E = m: no early stop, every run, accepted
    prm.Ee = Ee;
    prm.out_accept = out_accept;
    prm.out_popcount = out_popcount;
    prm.n = n_pairs;
    const unsigned grid = (unsigned)((n_pairs + shouji::kMagnetBlock - 1) / shouji::kMagnetBlock);
    // a pair holds at most E+1 pending parts (each run taken pops one and
    // pushes at most two; after E+1 runs nothing is pushed)
    const size_t lds = (size_t)(prm.E + 1) * shouji::kMagnetBlock * 4;
    // staged: at most 32 stack entries (E <= 31 once max_len > 32) and 2 x 16
    // words per lane, 64 KiB per workgroup.  Staging both sequences pays while
    // a CU still holds at least half the workgroups it holds without it
    // (measured: 8-9% faster at m=100, E=2..10 and 4% at m=250, E=5; at m=250,
    // E=15 and 25, 3 and 2 workgroups instead of 8 and 6, 4% and 28% slower).
    // Else the read's words alone, when that keeps more than half (m=250,
    // E=15: 5 of 8, 5% faster; E=25: 3 of 6, 2% slower, so not there).
    const size_t staged = (size_t)2 * ((max_len + 15) / 16) * shouji::kMagnetBlock * 4;
    auto groups_per_cu = [](size_t bytes) {
        const size_t k = shouji::kLdsPerCU / bytes;
        const size_t cap = 32 / (shouji::kMagnetBlock / shouji::kWave);   // 8 wavefronts per SIMD
        return k < cap ? k : cap;
    };
    const bool fits = (max_len + 15) / 16 <= shouji::kMagnetStageWords && lds + staged <= 65536;
    if (fits && 2 * groups_per_cu(lds + staged) >= groups_per_cu(lds))
        hipLaunchKernelGGL(shouji::magnet_kernel<2>, dim3(grid), dim3(shouji::kMagnetBlock), lds + staged,
                           (hipStream_t)stream, prm);
    else if (fits && 2 * groups_per_cu(lds + staged / 2) > groups_per_cu(lds))
        hipLaunchKernelGGL(shouji::magnet_kernel<1>, dim3(grid), dim3(shouji::kMagnetBlock), lds + staged / 2,
                           (hipStream_t)stream, prm);
    else
        hipLaunchKernelGGL(shouji::magnet_kernel<0>, dim3(grid), dim3(shouji::kMagnetBlock), lds,
                           (hipStream_t)stream, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "shouji_filter_magnet: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
