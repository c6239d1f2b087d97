// Window-width variant of the Shouji filter: W-column windows instead of 4
// (Suppl. Sec. 6.1 and Fig. 4 compare the false accept rates of window
// widths; 4 is the paper's choice).  Same steps as the plain form -- the
// 2E+1 diagonals of the neighbourhood map (Eq. 1), per window the diagonal
// segment with the most zeros (ties: a leading zero, then Algorithm 1's
// order d = +1, -1, ..., +E, -E, main), copied into S[i..i+W-1] when it has
// strictly more zeros, accept iff ones(S[0..m)) <= E -- with W a run-time
// parameter (1..16).  A study variant, not a tuned path.
//
// One pair per lane.  Each diagonal keeps the W cells of the current window
// as the low W bits of one register; a new column enters every diagonal at
// once: the read window P[c-K .. c+K] is a shift register of 2-bit codes,
// and one XOR with the reference base T[c] broadcast to every field plus a
// fold gives the mismatch bit of every diagonal.  The search is then a
// popcount and a compare per diagonal.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shouji.h"
#include "shouji_internal.h"
#include "shouji_variants.h"

namespace shouji {

template <int K>
__global__ __launch_bounds__(256) void window_kernel(WindowParams prm) {
    constexpr int NF = 2 * K + 1;              // diagonals (and read-window fields)
    constexpr int WW = (2 * NF + 31) / 32;     // words of the 2-bit read window
    constexpr int TOPW = (2 * (NF - 1)) / 32;
    constexpr int TOPB = (2 * (NF - 1)) % 32;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= prm.n) return;
    const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
    if (m < 0 || m > prm.max_len) {
        prm.out_accept[p] = 0xFF;
        if (prm.out_popcount) prm.out_popcount[p] = -1;
        return;
    }
    const int W = prm.W, E = prm.E;
    const uint32_t *P = prm.reads + p;
    const uint32_t *T = prm.refs + p;
    const int64_t ld = prm.ld;

    // read window: field f holds P[c - K + f] for the column c being
    // inserted; vmask has bit 2f set when that position lies in [0, m)
    uint32_t pw[WW], vm[WW];
#pragma unroll
    for (int w = 0; w < WW; w++) pw[w] = vm[w] = 0u;
    uint32_t pword = 0u;
    int ppos = 0;                              // next read position to push
    auto push = [&]() {
        uint32_t code = 0u, valid = 0u;
        if (ppos < m) {
            if ((ppos & 15) == 0) pword = P[(int64_t)(ppos >> 4) * ld];
            code = (pword >> ((ppos & 15) * 2)) & 3u;
            valid = 1u;
        }
        ppos++;
#pragma unroll
        for (int w = 0; w < WW; w++) {
            pw[w] = w + 1 < WW ? __builtin_amdgcn_alignbit(pw[w + 1], pw[w], 2) : pw[w] >> 2;
            vm[w] = w + 1 < WW ? __builtin_amdgcn_alignbit(vm[w + 1], vm[w], 2) : vm[w] >> 2;
        }
        pw[TOPW] |= code << TOPB;
        vm[TOPW] |= valid << TOPB;
    };
    for (int s = 0; s <= K; s++) push();       // fields K..2K <- P[0..K]

    // fields of diagonals beyond E (when the compiled K exceeds E): all ones
    uint32_t beyond[WW];
#pragma unroll
    for (int w = 0; w < WW; w++) {
        uint32_t b = 0u;
        for (int f = 0; f < 16; f++) {
            const int field = w * 16 + f;
            if (field < NF && (field - K > E || K - field > E)) b |= 1u << (2 * f);
        }
        beyond[w] = b;
    }

    // diagonal registers in evaluation order: rank 2(k-1) is d = +k, rank
    // 2(k-1)+1 is d = -k, rank 2K the main diagonal; diagonal d reads field
    // K - d of the read window
    uint32_t reg[NF];
#pragma unroll
    for (int r = 0; r < NF; r++) reg[r] = 0u;
    uint32_t tword = 0u;
    int col = 0;                               // next text column to insert
    auto insert = [&]() {
        uint32_t ne[WW];
        if (col < m) {
            if ((col & 15) == 0) tword = T[(int64_t)(col >> 4) * ld];
            const uint32_t tc = (tword >> ((col & 15) * 2)) & 3u;
            const uint32_t cb = tc * 0x55555555u;
#pragma unroll
            for (int w = 0; w < WW; w++) {
                const uint32_t x = pw[w] ^ cb;
                ne[w] = ((x | (x >> 1)) & 0x55555555u) | (~vm[w] & 0x55555555u) | beyond[w];
            }
        } else {
#pragma unroll
            for (int w = 0; w < WW; w++) ne[w] = 0x55555555u;   // past the reference: all ones
        }
        col++;
        push();                                // the window for the next column
#pragma unroll
        for (int r = 0; r < NF; r++) {
            const int d = r == NF - 1 ? 0 : ((r & 1) ? -(r / 2 + 1) : (r / 2 + 1));
            const int f = K - d;
            const uint32_t cell = (ne[(2 * f) >> 5] >> ((2 * f) & 31)) & 1u;
            reg[r] = (reg[r] >> 1) | (cell << (W - 1));
        }
    };
    for (int s = 0; s < W; s++) insert();     // columns 0..W-1

    uint32_t sreg = (W >= 32 ? ~0u : ((1u << W) - 1u));   // S[i..i+W-1], all ones
    const uint32_t top = 1u << (W - 1);
    int ones = 0;
    for (int i = 0; i < m; i++) {
        // the winner: fewest ones, then a leading zero, then the earliest
        uint32_t best = reg[0];
        uint32_t bkey = (__builtin_popcount(reg[0]) << 1) | (reg[0] & 1u);
#pragma unroll
        for (int r = 1; r < NF; r++) {
            const uint32_t key = (__builtin_popcount(reg[r]) << 1) | (reg[r] & 1u);
            const bool lt = key < bkey;
            bkey = lt ? key : bkey;
            best = lt ? reg[r] : best;
        }
        // copy it into S[i..i+W-1] when it has strictly more zeros
        if (__builtin_popcount(best) < __builtin_popcount(sreg)) sreg = best;
        ones += (int)(sreg & 1u);              // S[i] is final
        sreg = (sreg >> 1) | top;              // S[i+W] enters as 1
        insert();                              // column i+W
    }
    prm.out_accept[p] = ones <= E ? 1 : 0;
    if (prm.out_popcount) prm.out_popcount[p] = (int16_t)ones;
}

template __global__ void window_kernel<2>(WindowParams);
template __global__ void window_kernel<4>(WindowParams);
template __global__ void window_kernel<6>(WindowParams);
template __global__ void window_kernel<8>(WindowParams);
template __global__ void window_kernel<12>(WindowParams);
template __global__ void window_kernel<16>(WindowParams);
template __global__ void window_kernel<24>(WindowParams);
template __global__ void window_kernel<31>(WindowParams);

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
    if ((n_pairs + 255) / 256 > 0x7fffffff) return set_error(SHOUJI_ERR_ARG, "shouji_filter_window: n_pairs too large");
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
    const unsigned grid = (unsigned)((n_pairs + 255) / 256);
    // the narrowest compiled band of diagonals that holds the clamped E
    if (Ee <= 2)
        hipLaunchKernelGGL(shouji::window_kernel<2>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 4)
        hipLaunchKernelGGL(shouji::window_kernel<4>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 6)
        hipLaunchKernelGGL(shouji::window_kernel<6>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 8)
        hipLaunchKernelGGL(shouji::window_kernel<8>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 12)
        hipLaunchKernelGGL(shouji::window_kernel<12>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 16)
        hipLaunchKernelGGL(shouji::window_kernel<16>, dim3(grid), dim3(256), 0, st, prm);
    else if (Ee <= 24)
        hipLaunchKernelGGL(shouji::window_kernel<24>, dim3(grid), dim3(256), 0, st, prm);
    else
        hipLaunchKernelGGL(shouji::window_kernel<31>, dim3(grid), dim3(256), 0, st, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "shouji_filter_window: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
