// Relayout of sequences packed 32 bases per 64-bit word, pair by pair, into
// the word-major layout of 16-base 32-bit words that the filters read.
//
// The method stores each base in 2 bits (Sec. 2.3: the bases the filter
// streams per second at its link rate are four per byte).  A caller that keeps
// a pair's words together, 64 bits at a time, has base j of a sequence in bits
// 2(j mod 32)..2(j mod 32)+1 of its word j / 32; the filters read row r of a
// sequence (bases 16r..16r+15, base j in bits 2(j mod 16)..) at r * ld + p for
// pair p, so that one wavefront load reads one row of consecutive pairs.  A
// 64-bit word w is exactly rows 2w (its low half) and 2w+1 (its high half).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace shouji {

// One pair per thread: its first nw64 words, read in order (a pair's words
// are contiguous, so the lines a wavefront touches are used whole over the
// loop), each written as two rows; consecutive threads write consecutive
// addresses of a row.  A row at or past nrows (the odd half of the last word
// when max_len needs an odd number of rows) is not written.
__global__ __launch_bounds__(256) void relayout_pair_major_kernel(const uint64_t *__restrict__ src, int64_t wps,
                                                                  int64_t n, int nrows, uint32_t *__restrict__ dst,
                                                                  int64_t ld) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint64_t *s = src + p * wps;
    const int nw64 = (nrows + 1) / 2;
    for (int w = 0; w < nw64; w++) {
        const uint64_t v = s[w];
        dst[(int64_t)(2 * w) * ld + p] = (uint32_t)v;
        if (2 * w + 1 < nrows) dst[(int64_t)(2 * w + 1) * ld + p] = (uint32_t)(v >> 32);
    }
}

}  // namespace shouji

extern "C" int shouji_relayout_pair_major(const uint64_t *src, int64_t words_per_seq, int64_t n_pairs,
                                          int32_t max_len, uint32_t *dst, int64_t ld, void *stream) {
    using shouji::set_error;
    if (n_pairs < 0) return set_error(SHOUJI_ERR_ARG, "shouji_relayout_pair_major: n_pairs < 0 (%lld)",
                                      (long long)n_pairs);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_relayout_pair_major: max_len %d outside [0, %d]", max_len,
                         SHOUJI_MAX_LEN);
    const int nrows = (max_len + SHOUJI_BASES_PER_WORD - 1) / SHOUJI_BASES_PER_WORD;
    const int64_t need = (max_len + 31) / 32;
    if (words_per_seq < need)
        return set_error(SHOUJI_ERR_ARG, "shouji_relayout_pair_major: words_per_seq %lld < %lld for max_len %d",
                         (long long)words_per_seq, (long long)need, max_len);
    if (n_pairs == 0 || nrows == 0) return shouji::clear_error();
    if (!src || !dst) return set_error(SHOUJI_ERR_NULL, "shouji_relayout_pair_major: src and dst are required");
    if (ld < n_pairs)
        return set_error(SHOUJI_ERR_ARG, "shouji_relayout_pair_major: ld %lld < n_pairs %lld", (long long)ld,
                         (long long)n_pairs);
    const int64_t grid = (n_pairs + 255) / 256;
    if (grid > 0x7fffffff) return set_error(SHOUJI_ERR_ARG, "shouji_relayout_pair_major: n_pairs too large");
    hipLaunchKernelGGL(shouji::relayout_pair_major_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       src, words_per_seq, n_pairs, nrows, dst, ld);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "shouji_relayout_pair_major: launch failed: %s", hipGetErrorString(e));
    return shouji::clear_error();
}
