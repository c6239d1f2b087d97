// Verification of filtered pairs: banded edit distance of the pairs the
// filter accepted.
//
// The filter's purpose (Sec. 1, Sec. 3.3, Table 3) is to spare the aligner
// the pairs it rejects; this is that aligner's threshold test on the GPU.
// For each pair to verify, the unit-cost global edit distance between read
// and reference is computed with the textbook recurrence restricted to the
// band |i - j| <= K around the main diagonal (Ukkonen), K >= E chosen from a
// few compiled band widths: a path leaving the band has more than K >= E
// indels, so the band decides "distance <= E" exactly, and the distance
// itself when it is <= E.
//
// Layout: one pair per lane.  Pairs to verify are first collected into a
// list (an atomic counter in the caller's workspace; the order does not
// matter, results go to each pair's own index), so that a wavefront holds
// only pairs that need work.  Per lane the band's cells of one row live in
// registers, and the reference window T[i-K-1 .. i+K-1] is a shift register
// of 2-bit codes, from which one XOR and a fold give the match bits of all
// cells of the row.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace shouji {

namespace {
constexpr int32_t kBandInf = 0x3FFF;   // cells outside the map / band
}

// out: -2 for pairs the filter did not accept, -3 for invalid lengths;
// pairs to verify are appended to list (count in *count).  A workgroup
// handles kCollectPairs pairs and reserves its slice of the list with one
// atomic (one per 64 lanes serialises on the counter's address).
constexpr int kCollectBlock = 256;
constexpr int kCollectPer = 16;
constexpr int kCollectPairs = kCollectBlock * kCollectPer;

__global__ __launch_bounds__(kCollectBlock) void verify_collect_kernel(
        const uint8_t *__restrict__ accept, const int32_t *__restrict__ lengths, int32_t max_len, int64_t n,
        int16_t *__restrict__ out, int64_t *__restrict__ list, unsigned long long *__restrict__ count) {
    __shared__ int wave_total[kCollectBlock / 64];
    __shared__ unsigned long long block_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kCollectPairs + tid;
    uint32_t want = 0u;                        // bit i: pair base + i * kCollectBlock is verified
#pragma unroll
    for (int i = 0; i < kCollectPer; i++) {
        const int64_t p = base + (int64_t)i * kCollectBlock;
        if (p >= n) break;
        const int32_t m = lengths ? lengths[p] : max_len;
        if (m < 0 || m > max_len)
            out[p] = -3;
        else if (accept && accept[p] != 1)
            out[p] = -2;
        else
            want |= 1u << i;
    }
    // exclusive prefix of the per-lane counts over the workgroup
    const int c = __popc(want);
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wave_total[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kCollectBlock / 64; w++) {
        before += w < wave ? wave_total[w] : 0;
        total += wave_total[w];
    }
    if (tid == 0) block_base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
    __syncthreads();
    int64_t slot = (int64_t)block_base + before + incl - c;
    for (int i = 0; i < kCollectPer; i++)
        if (want & (1u << i)) list[slot++] = base + (int64_t)i * kCollectBlock;
}

__global__ void zero_counter_kernel(unsigned long long *count) { *count = 0ull; }

template <int K>
__global__ __launch_bounds__(256) void verify_band_kernel(VerifyParams prm) {
    constexpr int NB = 2 * K + 1;              // band cells of a row
    constexpr int WW = (2 * NB + 31) / 32;     // words of the 2-bit reference window
    constexpr int TOPW = (2 * (NB - 1)) / 32;  // word and bit of the window's top field
    constexpr int TOPB = (2 * (NB - 1)) % 32;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)*prm.count) return;
    const int64_t p = prm.list[t];
    const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
    const uint32_t *P = prm.reads + p;
    const uint32_t *T = prm.refs + p;
    const int64_t ld = prm.ld;

    // row 0: D[0][j] = j on the band (cell b <-> column j = i - K + b); Q = D + 1
    int32_t Q[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) Q[b] = b >= K ? b - K + 1 : kBandInf;

    // reference window: field b holds T[i - K + b - 1] while row i is computed
    uint32_t win[WW];
#pragma unroll
    for (int w = 0; w < WW; w++) win[w] = 0u;
    uint32_t tword = 0u;
    int q = 0;                                 // next reference position to push
    auto push = [&]() {
        uint32_t c = 0u;
        if (q < m) {
            if ((q & 15) == 0) tword = T[(int64_t)(q >> 4) * ld];
            c = (tword >> ((q & 15) * 2)) & 3u;
        }
        q++;
#pragma unroll
        for (int w = 0; w < WW; w++)
            win[w] = w + 1 < WW ? __builtin_amdgcn_alignbit(win[w + 1], win[w], 2) : win[w] >> 2;
        win[TOPW] |= c << TOPB;
    };
    for (int s = 0; s <= K; s++) push();       // fields K..2K <- T[0..K]

    uint32_t pword = 0u;
    int result = -1;
    bool done = false;
    for (int i = 1; i <= m; i++) {
        if (((i - 1) & 15) == 0) pword = P[(int64_t)((i - 1) >> 4) * ld];
        const uint32_t c = (pword >> (((i - 1) & 15) * 2)) & 3u;
        const uint32_t cb = c * 0x55555555u;   // c in every 2-bit field
        uint32_t eq[WW];
#pragma unroll
        for (int w = 0; w < WW; w++) {
            const uint32_t x = win[w] ^ cb;
            eq[w] = ~(x | (x >> 1)) & 0x55555555u;
        }
        // D[i][j] = min(D[i-1][j-1] + [P[i-1] != T[j-1]], D[i-1][j] + 1, D[i][j-1] + 1)
        int32_t left = kBandInf + 1;           // D[i][j-1] + 1
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int32_t eqb = (int32_t)((eq[(2 * b) >> 5] >> ((2 * b) & 31)) & 1u);
            const int32_t up = b + 1 < NB ? Q[b + 1] : kBandInf + 1;   // D[i-1][j] + 1
            const int32_t v = min(min(Q[b] - eqb, up), left);
            Q[b] = v + 1;
            left = v + 1;
        }
        push();
        // no path through row i stays within E: the distance exceeds E
        if ((i & 15) == 0 || i == m) {
            int32_t mn = Q[0];
#pragma unroll
            for (int b = 1; b < NB; b++) mn = min(mn, Q[b]);
            if (mn - 1 > prm.E) {
                done = true;
                break;
            }
        }
    }
    if (!done) {
        const int32_t d = Q[K] - 1;            // D[m][m]
        result = d <= prm.E ? d : -1;
    }
    prm.out[p] = (int16_t)result;
}

template __global__ void verify_band_kernel<2>(VerifyParams);
template __global__ void verify_band_kernel<4>(VerifyParams);
template __global__ void verify_band_kernel<6>(VerifyParams);
template __global__ void verify_band_kernel<8>(VerifyParams);
template __global__ void verify_band_kernel<12>(VerifyParams);
template __global__ void verify_band_kernel<16>(VerifyParams);
template __global__ void verify_band_kernel<24>(VerifyParams);
template __global__ void verify_band_kernel<31>(VerifyParams);

}  // namespace shouji

extern "C" int64_t shouji_verify_workspace_bytes(int64_t n_pairs) {
    if (n_pairs < 0) return shouji::set_error(SHOUJI_ERR_ARG, "shouji_verify_workspace_bytes: n_pairs < 0");
    shouji::clear_error();
    return 256 + n_pairs * (int64_t)sizeof(int64_t);
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
    if ((n_pairs + 255) / 256 > 0x7fffffff) return set_error(SHOUJI_ERR_ARG, "shouji_verify: n_pairs too large");
    hipStream_t st = (hipStream_t)stream;
    auto *count = reinterpret_cast<unsigned long long *>(workspace);
    auto *list = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(workspace) + 256);
    const unsigned grid = (unsigned)((n_pairs + 255) / 256);
    const unsigned cgrid = (unsigned)((n_pairs + shouji::kCollectPairs - 1) / shouji::kCollectPairs);
    hipLaunchKernelGGL(shouji::zero_counter_kernel, dim3(1), dim3(1), 0, st, count);
    hipLaunchKernelGGL(shouji::verify_collect_kernel, dim3(cgrid), dim3(shouji::kCollectBlock), 0, st,
                       filter_accept, lengths, max_len, n_pairs, out_distance, list, count);
    shouji::VerifyParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.lengths = lengths;
    prm.max_len = max_len;
    prm.E = E;
    prm.list = list;
    prm.count = count;
    prm.out = out_distance;
    // the narrowest compiled band that holds E
    if (E <= 2)
        hipLaunchKernelGGL(shouji::verify_band_kernel<2>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 4)
        hipLaunchKernelGGL(shouji::verify_band_kernel<4>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 6)
        hipLaunchKernelGGL(shouji::verify_band_kernel<6>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 8)
        hipLaunchKernelGGL(shouji::verify_band_kernel<8>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 12)
        hipLaunchKernelGGL(shouji::verify_band_kernel<12>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 16)
        hipLaunchKernelGGL(shouji::verify_band_kernel<16>, dim3(grid), dim3(256), 0, st, prm);
    else if (E <= 24)
        hipLaunchKernelGGL(shouji::verify_band_kernel<24>, dim3(grid), dim3(256), 0, st, prm);
    else
        hipLaunchKernelGGL(shouji::verify_band_kernel<31>, dim3(grid), dim3(256), 0, st, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(SHOUJI_ERR_DEVICE, "shouji_verify: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
