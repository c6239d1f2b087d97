// Verification of filtered pairs: banded edit distance of the pairs the
// filter accepted.
//
// The filter's purpose (Sec. 1, Sec. 3.3, Table 3) is to spare the aligner
// the pairs it rejects; this is that aligner's threshold test on the GPU.
// For each pair to verify, the unit-cost global edit distance D[m][m] of read
// P and reference T is computed on a diagonal band |i - j| <= K, K = E
// (Ukkonen): a path leaving the band has more than K indels, so the band
// decides "distance <= E" exactly, and gives the distance when it is <= E.
//
// The band is computed column by column (one reference base per step) with
// the bit-vector recurrence of Myers (J. ACM 46(3), 1999) in the block form
// Hyyro describes for a boundary difference entering at the top: the band's
// W rows are W bits of two vectors, Pv and Mv, flagging the vertical
// differences D[i][j] - D[i-1][j] of +1 and -1, and one step turns the
// column j-1 vectors into column j with a handful of logic operations and
// one addition.  The band is kept on the diagonal by shifting it down one row
// after every step (its top row leaves, a new bottom row enters with
// difference +1, the value of a vertical step), and the value of the cell
// just above the band is carried in a scalar.  Cells outside the band are
// given values of real paths (a horizontal step in from above the band, a
// vertical step down below it), so every cell holds a value between the true
// distance and the band-restricted one, which keeps the test exact; rows
// above row 0 are virtual rows with D[i][j] = j - i that never match.
//
// Layout: pairs to verify are first collected into a list (an atomic counter
// in the caller's workspace; results go to each pair's own index), so that a
// wavefront holds only pairs that need work.  One pair per lane, a band of
// 32 rows (E <= 15) or 64 rows (E <= 31).  Columns go in chunks of 16 (one
// packed reference word): the reference word and the pattern words around
// the band are turned once per chunk into bit planes (low code bit, high code
// bit, position inside the read), so that a column takes its pattern planes
// with one funnel shift each and its reference base with one bit-field
// extract per plane.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace shouji {

// Verifier of filtered pairs (banded edit distance, one pair per lane).
struct VerifyParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    int32_t max_len;
    int32_t E;
    const uint16_t *list;             // per segment of pairs, the indices to verify within it
    const int32_t *seg_count;         // entries of each segment's list
    int64_t nseg;                     // segments
    int16_t *out;
};

// out: -2 for pairs the filter did not accept, -3 for invalid lengths.  A
// workgroup handles one segment of kCollectPairs pairs: it writes the indices
// (within the segment) of the pairs to verify to the segment's own slice of
// the list and their number to seg_count, so that no workgroup waits on
// another (a shared counter, taken with one atomic per workgroup, cost more
// than the rest of the pass) and nothing needs clearing between calls.
constexpr int kCollectBlock = 256;
constexpr int kCollectPer = 16;
constexpr int kCollectPairs = kCollectBlock * kCollectPer;
static_assert(kCollectPairs <= 65536 && kCollectPairs % 256 == 0,
              "indices within a segment are 16-bit; a verify workgroup lies in one segment");

__global__ __launch_bounds__(kCollectBlock) void verify_collect_kernel(
        const uint8_t *__restrict__ accept, const int32_t *__restrict__ lengths, int32_t max_len, int64_t n,
        int16_t *__restrict__ out, uint16_t *__restrict__ list, int32_t *__restrict__ seg_count) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kCollectPairs + tid;
    // every load of the lane first (none depends on another), then the tests
    int32_t mv[kCollectPer];
    uint32_t av[kCollectPer];
#pragma unroll
    for (int i = 0; i < kCollectPer; i++) {
        const int64_t p = base + (int64_t)i * kCollectBlock;
        const bool in = p < n;
        mv[i] = in && lengths ? lengths[p] : max_len;
        av[i] = in && accept ? accept[p] : 1u;
    }
    uint32_t want = 0u;                        // bit i: pair base + i * kCollectBlock is verified
#pragma unroll
    for (int i = 0; i < kCollectPer; i++) {
        const int64_t p = base + (int64_t)i * kCollectBlock;
        if (p >= n) continue;
        if (mv[i] < 0 || mv[i] > max_len)
            out[p] = -3;
        else if (av[i] != 1u)
            out[p] = -2;
        else
            want |= 1u << i;
    }
    // the list in pair order (pair tid + i * kCollectBlock is cell (i, wave)
    // of the workgroup, cells ordered i first), so that a verify wavefront
    // reads the words of neighbouring pairs: per cell the wanted pairs of
    // lower lanes, then an exclusive scan over the 64 cells
    constexpr int NW = kCollectBlock / 64;
    static_assert(kCollectPer * NW == 64, "one lane per cell in the scan");
    __shared__ int cell[kCollectPer * NW];
    const uint64_t lower = (1ull << lane) - 1ull;
    int below[kCollectPer];
#pragma unroll
    for (int i = 0; i < kCollectPer; i++) {
        const uint64_t b = __ballot((want >> i) & 1u);
        below[i] = __popcll(b & lower);
        if (lane == 0) cell[i * NW + wave] = __popcll(b);
    }
    __syncthreads();
    if (wave == 0) {
        const int v = cell[lane];
        int incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        cell[lane] = incl - v;
        if (lane == 63) seg_count[blockIdx.x] = incl;
    }
    __syncthreads();
    uint16_t *seg = list + (int64_t)blockIdx.x * kCollectPairs;
#pragma unroll
    for (int i = 0; i < kCollectPer; i++)
        if (want & (1u << i)) seg[cell[i * NW + wave] + below[i]] = (uint16_t)(tid + i * kCollectBlock);
}

// The 16 low code bits (or, for w >> 1, high code bits) of a packed word of
// 16 bases, as bits 0..15.
__device__ __forceinline__ uint32_t code_plane(uint32_t w) {
    uint32_t x = w & 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// Truth table of a three-input function for v_bitop3_b32 (bit a<<2|b<<1|c
// of the immediate is f(a, b, c)) and the gate itself.
template <class F>
constexpr unsigned vtt(F f) {
    unsigned t = 0;
    for (int i = 0; i < 8; i++)
        if (f((i >> 2) & 1, (i >> 1) & 1, i & 1)) t |= 1u << i;
    return t;
}
constexpr unsigned kTTNotOrXor = vtt([](int a, int b, int c) { return !(a | (b ^ c)); });
constexpr unsigned kTTXorOr = vtt([](int a, int b, int c) { return (a ^ b) | c; });
constexpr unsigned kTTOrNor = vtt([](int a, int b, int c) { return a | !(b | c); });
template <unsigned TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

// All ones when bit u of a code plane is set, else zero, as a band vector
// (the bit-field extract's result is unsigned: it is made signed before it
// is widened, so that a 64-bit mask is all ones in both halves).
template <typename V>
__device__ __forceinline__ V base_mask(uint32_t plane, int u) {
    return (V)(int64_t)(int32_t)__builtin_amdgcn_sbfe(plane, u, 1);
}

// Banded distance of one pair per lane, band half-width K = E.  V: the band
// vector (uint32_t: 32 rows, K <= 15; uint64_t: 64 rows, K <= 31).  Per column
// j (reference base T[j-1]) band bit b is row i = j-1-K+b before the step, and
// A = D[j-K-1][j] (the cell above the band) after it.  The pattern planes of a
// chunk c (columns 16c+1 .. 16c+16) come from a window of NF 16-bit fields,
// field q = pattern word c-BW+q, from which column 16c+1+u takes the bits at
// offset u + 16 BW - 1 - K (P[j-2-K+b] at bit b).
template <typename V, int BW>
__global__ __launch_bounds__(256) void verify_myers_kernel(VerifyParams prm) {
    constexpr int W = 8 * (int)sizeof(V);
    constexpr int NF = 4 * BW;                 // 16-bit fields of the window
    constexpr int NWW = NF / 2;                // 32-bit words of the window
    const int K = prm.E;
    // workgroup g takes entries 256 (g / nseg) .. +255 of segment g % nseg's
    // list: consecutive workgroups, which the dispatcher deals round the XCDs,
    // take different segments, and the workgroups past a segment's count
    // (which return at once) come last
    const int64_t s = (int64_t)blockIdx.x % prm.nseg;
    const int k = (int)((int64_t)blockIdx.x / prm.nseg) * 256 + (int)threadIdx.x;
    if (k >= prm.seg_count[s]) return;
    const int64_t p = s * kCollectPairs + prm.list[s * kCollectPairs + k];
    const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
    if (m == 0) {                              // empty pair: distance 0, no word to read
        prm.out[p] = 0;
        return;
    }
    const int64_t ld = prm.ld;
    const int nw = (prm.max_len + 15) / 16;    // >= 1 here
    const uint32_t *P = prm.reads + p;
    const uint32_t *T = prm.refs + p;

    // pattern word wd as planes; positions outside [0, m) are not in the read
    auto fetch = [&](int wd) -> uint32_t {
        return (wd >= 0 && wd < nw && 16 * wd < m) ? P[(int64_t)wd * ld] : 0u;
    };
    auto planes_of = [&](int wd, uint32_t w, uint32_t &lo, uint32_t &hi, uint32_t &in) {
        lo = code_plane(w);
        hi = code_plane(w >> 1);
        const int n = (wd >= 0 && wd < nw) ? min(16, m - 16 * wd) : 0;
        in = n > 0 ? (1u << n) - 1u : 0u;
    };
    auto field = [&](int wd, uint32_t &lo, uint32_t &hi, uint32_t &in) { planes_of(wd, fetch(wd), lo, hi, in); };
    uint32_t wlo[NWW], whi[NWW], win[NWW];
#pragma unroll
    for (int i = 0; i < NWW; i++) {
        uint32_t l0, h0, i0, l1, h1, i1;
        field(2 * i - BW, l0, h0, i0);
        field(2 * i + 1 - BW, l1, h1, i1);
        wlo[i] = l0 | (l1 << 16);
        whi[i] = h0 | (h1 << 16);
        win[i] = i0 | (i1 << 16);
    }
    // column 0: rows -K .. W-1-K; D[i][0] = |i| (vertical difference -1 on
    // rows <= 0, +1 below); A = D[-K-1][0] = K+1
    V Pv = 0, Mv = 0;
#pragma unroll
    for (int b = 0; b < W; b++) {
        if (b <= K) Mv |= (V)1 << b; else Pv |= (V)1 << b;
    }
    int A = K + 1;
    // Operands of the column step held in VGPRs (opaque to the compiler): the
    // SIMD runs two wavefronts' VALU instructions side by side only when every
    // operand is a VGPR.  obase: window offset of column 16c+1; ou[u] = obase+u,
    // the offset of column 16c+1+u, which is also where bit u of the chunk's
    // reference code planes sits once they are shifted left by obase.
    uint32_t obase = (uint32_t)(16 * BW - 1 - K), one = 1u;
    asm volatile("" : "+v"(obase), "+v"(one));
    const V vone = (V)one;
    uint32_t ou[16];
#pragma unroll
    for (int u = 0; u < 16; u++) {
        ou[u] = obase + (uint32_t)u;
        asm volatile("" : "+v"(ou[u]));
    }

    // the planes of the band at window offset o (0 <= o <= 30)
    auto planes = [&](const uint32_t (&w)[NWW], uint32_t o) -> V {
        if constexpr (W == 32) {
            return __builtin_amdgcn_alignbit(w[1], w[0], o);
        } else {
            const uint32_t lo = __builtin_amdgcn_alignbit(w[1], w[0], o);
            const uint32_t hi = __builtin_amdgcn_alignbit(w[2], w[1], o);
            return (V)lo | ((V)hi << 32);
        }
    };
    // one column: reference code planes tl, th (all ones or zero), window
    // offset o; IN: the band may hold rows above row 1 (pattern positions
    // below 0), which must not match.  Positions at or past m need no mask:
    // rows below row m never reach D[m][m].
    // The step folds the band's shift into the recurrence: with the +1 that
    // enters above the top row, the new bottom row's +1 and the old top row's
    // difference follow from Xv alone (the top bit of Pv stays 1 and that of Mv
    // stays 0 through every step).  Returns Xv, whose bit 0 gives the change
    // of A = D[j-1-K][j]: A_new = A + 1 - (bit 0 of Xv).
    auto column = [&](V tl, V th, uint32_t o, auto in_tag) -> V {
        constexpr bool IN = decltype(in_tag)::value;
        const V Plo = planes(wlo, o), Phi = planes(whi, o);
        if constexpr (W == 32 && !IN) {
            // the same step with every three-input function as one gate
            // (16 instructions per column with the extracts, the window
            // offsets and the bit-0 collection)
            const uint32_t Eq = bop3<kTTNotOrXor>(Plo ^ tl, Phi, th);   // P[i-1] == T[j-1]
            const uint32_t Xv = Eq | Mv;
            const uint32_t Xh = bop3<kTTXorOr>((Eq & Pv) + Pv, Pv, Eq);
            const uint32_t Ph = bop3<kTTOrNor>(Mv, Xh, Pv);
            const uint32_t xs = Xv >> vone;
            Pv = bop3<kTTOrNor>(Pv & Xh, xs, Ph);
            Mv = Ph & xs;
            return Xv;
        } else {
            // match bits: P[i-1] == T[j-1]
            V Eq = ~((Plo ^ tl) | (Phi ^ th));
            if constexpr (IN) Eq &= planes(win, o);
            const V Xv = Eq | Mv;
            const V Xh = (((Eq & Pv) + Pv) ^ Pv) | Eq;
            const V Ph = Mv | ~(Xh | Pv);
            const V Mh = Pv & Xh;
            const V xs = Xv >> vone;
            Pv = Mh | ~(xs | Ph);
            Mv = Ph & xs;
            return Xv;
        }
    };
    auto popc = [](V x) { return (int)__builtin_popcountll((unsigned long long)x); };

    const int nchunks = (m + 15) / 16;
    bool dead = false;
    // the words of the next chunk are loaded one chunk ahead
    uint32_t tw_next = T[0], pw_next = fetch(NF - BW);
    for (int c = 0; c < nchunks; c++) {
        const uint32_t tw = tw_next, pw = pw_next;
        if (c + 1 < nchunks) {
            tw_next = T[(int64_t)(c + 1) * ld];
            pw_next = fetch(c + 1 - BW + NF - 1);
        }
        if (c > 0) {
            // slide the window by one field; the new top field is word c-BW+NF-1
            uint32_t l, h, in;
            planes_of(c - BW + NF - 1, pw, l, h, in);
#pragma unroll
            for (int i = 0; i < NWW - 1; i++) {
                wlo[i] = __builtin_amdgcn_alignbit(wlo[i + 1], wlo[i], 16);
                whi[i] = __builtin_amdgcn_alignbit(whi[i + 1], whi[i], 16);
                win[i] = __builtin_amdgcn_alignbit(win[i + 1], win[i], 16);
            }
            wlo[NWW - 1] = (wlo[NWW - 1] >> 16) | (l << 16);
            whi[NWW - 1] = (whi[NWW - 1] >> 16) | (h << 16);
            win[NWW - 1] = (win[NWW - 1] >> 16) | (in << 16);
        }
        const uint32_t tlo = code_plane(tw), thi = code_plane(tw >> 1);
        // rows above row 1 only in the first chunks (16c <= K)
        auto chunk = [&](auto in_tag) {
            if (16 * c + 16 <= m) {
                // bit 0 of each column's Xv enters at bit 31 of xb; after the
                // 16 columns bits 16..31 hold them all
                const uint32_t tls = tlo << obase, ths = thi << obase;
                uint32_t xb = 0u;
#pragma unroll
                for (int u = 0; u < 16; u++) {
                    const V tl = (V)(int64_t)(int32_t)__builtin_amdgcn_sbfe(tls, ou[u], one);
                    const V th = (V)(int64_t)(int32_t)__builtin_amdgcn_sbfe(ths, ou[u], one);
                    const V Xv = column(tl, th, ou[u], in_tag);
                    xb = __builtin_amdgcn_alignbit((uint32_t)Xv, xb, one);
                }
                A += 16 - __popc(xb >> 16);
            } else {
                uint32_t o = obase;
                for (int u = 0; u < m - 16 * c; u++) {
                    const V Xv = column(base_mask<V>(tlo, u), base_mask<V>(thi, u), o, in_tag);
                    A += (int)one - (int)((uint32_t)Xv & one);
                    o += one;
                }
            }
        };
        if (16 * c <= K)
            chunk(std::integral_constant<bool, true>());
        else
            chunk(std::integral_constant<bool, false>());
        // every band cell is at least A minus the band's -1 differences: above
        // E, no path within E passes this column
        if (c + 1 < nchunks && A - popc(Mv) > prm.E) {
            dead = true;
            break;
        }
    }
    int res = -1;
    if (!dead) {
        // D[m][m]: rows m-K .. m are band bits 0 .. K
        const V low = (V)(((V)2 << K) - (V)1);
        const int d = A + popc(Pv & low) - popc(Mv & low);
        res = d <= prm.E ? d : -1;
    }
    prm.out[p] = (int16_t)res;
}

}  // namespace shouji

extern "C" int64_t shouji_verify_workspace_bytes(int64_t n_pairs) {
    if (n_pairs < 0) return shouji::set_error(SHOUJI_ERR_ARG, "shouji_verify_workspace_bytes: n_pairs < 0");
    shouji::clear_error();
    const int64_t nseg = (n_pairs + shouji::kCollectPairs - 1) / shouji::kCollectPairs;
    return (nseg * 4 + 255) / 256 * 256 + nseg * shouji::kCollectPairs * (int64_t)sizeof(uint16_t);
}

extern "C" int shouji_verify(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths, int32_t E,
                             const uint8_t *filter_accept, int16_t *out_distance, int64_t n_pairs,
                             int32_t max_len, int64_t ld, void *workspace, int64_t workspace_bytes,
                             void *stream) {
    using shouji::set_error;
    if (n_pairs < 0) return set_error(SHOUJI_ERR_ARG, "shouji_verify: n_pairs < 0");
    if (E < 0) return set_error(SHOUJI_ERR_ARG, "shouji_verify: E < 0 (%d)", E);
    if (E > SHOUJI_MAX_E) return set_error(SHOUJI_ERR_RANGE, "shouji_verify: E %d above %d", E, SHOUJI_MAX_E);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_verify: max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    if (n_pairs == 0) return shouji::clear_error();
    if (!reads || !refs || !out_distance || !workspace)
        return set_error(SHOUJI_ERR_NULL, "shouji_verify: reads, refs, out_distance and workspace are required");
    if (ld < n_pairs) return set_error(SHOUJI_ERR_ARG, "shouji_verify: ld %lld < n_pairs %lld", (long long)ld,
                                       (long long)n_pairs);
    if (workspace_bytes < shouji_verify_workspace_bytes(n_pairs))
        return set_error(SHOUJI_ERR_ARG, "shouji_verify: workspace of %lld bytes, %lld needed",
                         (long long)workspace_bytes, (long long)shouji_verify_workspace_bytes(n_pairs));
    if ((n_pairs + shouji::kCollectPairs - 1) / shouji::kCollectPairs * (shouji::kCollectPairs / 256) > 0x7fffffff)
        return set_error(SHOUJI_ERR_ARG, "shouji_verify: n_pairs too large");
    hipStream_t st = (hipStream_t)stream;
    // workspace: per segment of kCollectPairs pairs, its count (int32), then
    // its list of indices within the segment (uint16)
    const int64_t nseg = (n_pairs + shouji::kCollectPairs - 1) / shouji::kCollectPairs;
    auto *seg_count = reinterpret_cast<int32_t *>(workspace);
    auto *list = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(workspace) + (nseg * 4 + 255) / 256 * 256);
    const unsigned grid = (unsigned)(nseg * (shouji::kCollectPairs / 256));
    hipLaunchKernelGGL(shouji::verify_collect_kernel, dim3((unsigned)nseg), dim3(shouji::kCollectBlock), 0, st,
                       filter_accept, lengths, max_len, n_pairs, out_distance, list, seg_count);
    shouji::VerifyParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.lengths = lengths;
    prm.max_len = max_len;
    prm.E = E;
    prm.list = list;
    prm.seg_count = seg_count;
    prm.nseg = nseg;
    prm.out = out_distance;
    // the band vector that holds rows j-E .. j+E+1 (2E+2 rows): 32 or 64 bits
    if (E <= 15)
        hipLaunchKernelGGL((shouji::verify_myers_kernel<uint32_t, 1>), dim3(grid), dim3(256), 0, st, prm);
    else
        hipLaunchKernelGGL((shouji::verify_myers_kernel<uint64_t, 2>), dim3(grid), dim3(256), 0, st, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(SHOUJI_ERR_DEVICE, "shouji_verify: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
