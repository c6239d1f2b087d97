// Batched form of the Shouji filter: pairs of mixed lengths with one edit
// threshold per pair in one pass.
//
// The filter's cost per pair is proportional to (windows) x (2E+1 diagonals),
// and a wavefront filters 1024 pairs in lock step, so pairs are first grouped
// into bins of equal E and similar length (a length bucket of `bw` bases):
//   1. bin_count_kernel    histogram of (length bucket, E) keys
//   2. bin_plan_kernel     offsets of the bins in a binned workspace, and a
//                          list of tiles (<= 1024 pairs of one bin) per E class,
//                          in decreasing cost order
//   3. bin_scatter_kernel  copies every pair (words, length, E, original index)
//                          to its slot in the binned workspace; pairs with an
//                          invalid length or E get their sentinels here
//   4. shouji_tiles_kernel the plain filter on each tile (shouji_plain.hip),
//                          writing results back to the original pair index
// Within a bin every pair is filtered exactly as alone: E is equal, and cells
// beyond a pair's own length are masked to mismatches (the neighbourhood map
// of Eq. 1 ends there), which is what the single-pair method computes.
// Every kernel here is enqueued on the caller's stream and allocates nothing,
// so the whole pipeline can be captured in a graph (counters are cleared with
// a fill kernel, not a memset).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shouji_binning.h"
#include "shouji_internal.h"

namespace shouji {

__device__ __forceinline__ bool pair_key(int m, int e, int max_len, int bw, int &bin, int &Ee) {
    if (m < 0 || m > max_len || e < 0) return false;
    Ee = e < m - 1 ? e : (m > 0 ? m - 1 : 0);
    if (Ee > kMaxE) return false;
    bin = ((m + bw - 1) / bw) * kBinE + Ee;
    return true;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Histogram of the pair keys.  Each wavefront counts into its own LDS copy
// (copy w % ncopies) so that lanes of different wavefronts do not contend,
// and each thread loads four pairs before it counts them.  Workgroups are
// few and large: the closing global adds of all workgroups land on the few
// cache lines of counts[], and their number is what bounds this kernel.
__global__ __launch_bounds__(kCountThreads) void bin_count_kernel(const int32_t *__restrict__ lengths,
                                                        const int32_t *__restrict__ Ep, int64_t n,
                                                        int max_len, int bw, int nbins, int ncopies,
                                                        int32_t *__restrict__ counts) {
    extern __shared__ int32_t hist[];
    for (int b = threadIdx.x; b < nbins * ncopies; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    int32_t *mine = hist + (int)((threadIdx.x / kWave) % ncopies) * nbins;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += 4 * stride) {
        int m[4], e[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int64_t q = p + k * stride;
            m[k] = q < n ? (lengths ? lengths[q] : max_len) : -1;
            e[k] = q < n ? Ep[q] : -1;
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int bin, Ee;
            if (pair_key(m[k], e[k], max_len, bw, bin, Ee)) atomicAdd(&mine[bin], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        int32_t c = 0;
        for (int k = 0; k < ncopies; k++) c += hist[k * nbins + b];
        if (c) atomicAdd(&counts[b], c);
    }
}

// One workgroup of kPlanThreads threads.
//  offsets[b]  first slot of bin b in the binned workspace (bins in index order)
//  cursors[b]  = offsets[b], advanced by the scatter
//  tiles[c]    tile list of E class c (Ee <= class_bound[c]), longest first
//  ntiles[c]   number of tiles of class c
__global__ __launch_bounds__(kPlanThreads) void bin_plan_kernel(
    const int32_t *__restrict__ counts, int nbins, int nbucket_len, PlanOut out) {
    __shared__ int64_t part[kPlanThreads];
    __shared__ int32_t npos[kCostBuckets * kEClasses];
    __shared__ int32_t tpos[kCostBuckets * kEClasses];
    const int tid = threadIdx.x;
    const int per = (nbins + kPlanThreads - 1) / kPlanThreads;
    const int lo = tid * per, hi = min(lo + per, nbins);

    // exclusive scan of the bin counts
    int64_t s = 0;
    for (int b = lo; b < hi; b++) s += counts[b];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int b = lo; b < hi; b++) {
        out.offsets[b] = run;
        out.cursors[b] = run;
        run += counts[b];
    }

    // tiles per (cost bucket, E class): cost = length buckets x (2E+1), bucketed
    // by its bit length so that dispatch order is roughly longest first
    for (int i = tid; i < kCostBuckets * kEClasses; i += kPlanThreads) npos[i] = 0;
    __syncthreads();
    for (int b = lo; b < hi; b++) {
        const int c = counts[b];
        if (!c) continue;
        const int Ee = b % kBinE, mb = b / kBinE;
        const int cls = e_class(Ee);
        const uint32_t cost = (uint32_t)(mb + 1) * (uint32_t)(2 * Ee + 1);
        const int cb = kCostBuckets - 1 - min(kCostBuckets - 1, 31 - __builtin_clz(cost));
        atomicAdd(&npos[cls * kCostBuckets + cb], (c + kPairsPerWave - 1) / kPairsPerWave);
    }
    __syncthreads();
    if (tid < kEClasses) {
        int32_t acc = 0;
        for (int cb = 0; cb < kCostBuckets; cb++) {
            const int32_t v = npos[tid * kCostBuckets + cb];
            tpos[tid * kCostBuckets + cb] = acc;
            acc += v;
        }
        out.ntiles[tid] = acc;
    }
    __syncthreads();
    // the bin's first slot is carried in a register: reading it back from
    // offsets[] after each tile store would wait on memory once per tile
    int64_t first = part[tid] - s;
    for (int b = lo; b < hi; b++) {
        const int c = counts[b];
        const int64_t ob = first;
        first += c;
        if (!c) continue;
        const int Ee = b % kBinE, mb = b / kBinE;
        const int cls = e_class(Ee);
        const uint32_t cost = (uint32_t)(mb + 1) * (uint32_t)(2 * Ee + 1);
        const int cb = kCostBuckets - 1 - min(kCostBuckets - 1, 31 - __builtin_clz(cost));
        const int nt = (c + kPairsPerWave - 1) / kPairsPerWave;
        const int t0 = atomicAdd(&tpos[cls * kCostBuckets + cb], nt);
        int4 *tl = out.tiles[cls];
        for (int i = 0; i < nt; i++) {
            const int cnt = min(kPairsPerWave, c - i * kPairsPerWave);
            tl[t0 + i] = make_int4((int)(ob + (int64_t)i * kPairsPerWave), cnt, Ee, 0);
        }
    }
    (void)nbucket_len;
}

__global__ __launch_bounds__(256) void bin_scatter_kernel(ScatterParams prm) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < prm.n; p += stride) {
        const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
        const int e = prm.Ep[p];
        int bin, Ee;
        if (!pair_key(m, e, prm.max_len, prm.bw, bin, Ee)) {
            prm.out_accept[p] = 0xFF;
            if (prm.out_popcount) prm.out_popcount[p] = -1;
            continue;
        }
        const int64_t dst = (int64_t)atomicAdd((unsigned long long *)&prm.cursors[bin], 1ull);
        prm.bperm[dst] = p;
        prm.blens[dst] = m;
        prm.bE[dst] = e;
        const int nw = (m + kHalf - 1) / kHalf;
        for (int w = 0; w < nw; w++) {
            prm.breads[(int64_t)w * prm.bld + dst] = prm.reads[(int64_t)w * prm.ld + p];
            prm.brefs[(int64_t)w * prm.bld + dst] = prm.refs[(int64_t)w * prm.ld + p];
        }
    }
}

// Scatter staged through LDS.  A workgroup takes a chunk of CHUNK
// consecutive pairs, reserves one run per bin in the binned workspace (one
// global atomic per bin and chunk), ranks its pairs by bin in LDS, and then
// writes every word row, the lengths, thresholds and original indices in
// slot order, so consecutive threads write consecutive slots of a run.
// Reads of the input rows stay coalesced.  Needs nbins <= scatter_max_bins(CHUNK).
template <int CHUNK>
__global__ __launch_bounds__(kScatterThreads) void bin_scatter_lds_kernel(ScatterParams prm) {
    extern __shared__ int32_t sm[];
    const int nbins = prm.nbins;
    int32_t *cnt = sm;                                         // counts, then cursors
    int32_t *loff = cnt + nbins;                               // local run offsets
    int64_t *gbase = reinterpret_cast<int64_t *>(loff + nbins + (nbins & 1));
    uint16_t *slotbin = reinterpret_cast<uint16_t *>(gbase + nbins);
    uint16_t *slotsrc = slotbin + CHUNK;
    uint32_t *buf = reinterpret_cast<uint32_t *>(slotsrc + CHUNK);
    __shared__ int32_t part[kScatterThreads];
    static_assert(sizeof(part) == kScatterStaticLds, "the bin limit of the scatter counts this array");
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * CHUNK;
    constexpr int PER = CHUNK / kScatterThreads;

    for (int b = tid; b < nbins; b += kScatterThreads) cnt[b] = 0;
    __syncthreads();
    int bin[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t p = c0 + tid + (int64_t)i * kScatterThreads;
        bin[i] = -1;
        if (p >= prm.n) continue;
        const int m = prm.lengths ? prm.lengths[p] : prm.max_len;
        int b, Ee;
        if (pair_key(m, prm.Ep[p], prm.max_len, prm.bw, b, Ee)) {
            bin[i] = b;
            atomicAdd(&cnt[b], 1);
        } else {
            prm.out_accept[p] = 0xFF;
            if (prm.out_popcount) prm.out_popcount[p] = -1;
        }
    }
    __syncthreads();
    // reserve runs; exclusive scan of the counts over the bins
    const int per = (nbins + kScatterThreads - 1) / kScatterThreads;
    const int lo = tid * per, hi = min(lo + per, nbins);
    int32_t s = 0;
    for (int b = lo; b < hi; b++) {
        const int32_t c = cnt[b];
        if (c) gbase[b] = (int64_t)atomicAdd((unsigned long long *)&prm.cursors[b], (unsigned long long)c);
        s += c;
    }
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScatterThreads; off <<= 1) {
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    for (int b = lo; b < hi; b++) {
        loff[b] = run;
        const int32_t c = cnt[b];
        cnt[b] = run;                                          // becomes the slot cursor
        run += c;
    }
    __syncthreads();
    const int nvalid = part[kScatterThreads - 1];
    int slot[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        slot[i] = -1;
        if (bin[i] < 0) continue;
        slot[i] = atomicAdd(&cnt[bin[i]], 1);
        slotbin[slot[i]] = (uint16_t)bin[i];
        slotsrc[slot[i]] = (uint16_t)(tid + i * kScatterThreads);
    }
    __syncthreads();
    // per-pair metadata, in slot order
    for (int q = tid; q < nvalid; q += kScatterThreads) {
        const int b = slotbin[q];
        const int64_t dst = gbase[b] + (q - loff[b]);
        const int64_t src = c0 + slotsrc[q];
        prm.bperm[dst] = src;
        prm.blens[dst] = prm.lengths ? prm.lengths[src] : prm.max_len;
        prm.bE[dst] = prm.Ep[src];
    }
    // word rows, one at a time through the LDS buffer.  A bin's tiles read
    // no word past the longest length of its bucket (bucket b / kBinE holds
    // lengths up to (b / kBinE) * bw), so a pair's rows from there on are
    // neither loaded nor written.
    const int nw = (prm.max_len + kHalf - 1) / kHalf;
    int rows[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) rows[i] = bin[i] >= 0 ? ((bin[i] / kBinE) * prm.bw + kHalf - 1) / kHalf : 0;
    // rows of both sequences in turn; the loads of the next three rows are in
    // flight while the current one goes through LDS, so that the latency of
    // HBM under load is covered (one row ahead left each workgroup waiting on
    // its loads for most of every row)
    const int nrows = 2 * nw;
    uint32_t cur[PER], n1[PER], n2[PER], n3[PER];
    auto load_row = [&](int r, uint32_t (&v)[PER]) {
        const int w = r < nw ? r : r - nw;
        const uint32_t *in = r < nw ? prm.reads : prm.refs;
#pragma unroll
        for (int i = 0; i < PER; i++)
            v[i] = w < rows[i] ? in[(int64_t)w * prm.ld + c0 + tid + (int64_t)i * kScatterThreads] : 0u;
    };
    if (nrows > 0) load_row(0, cur);
    if (nrows > 1) load_row(1, n1);
    if (nrows > 2) load_row(2, n2);
    for (int r = 0; r < nrows; r++) {
        const int w = r < nw ? r : r - nw;
        uint32_t *outp = r < nw ? prm.breads : prm.brefs;
        if (r + 3 < nrows) load_row(r + 3, n3);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; i++)
            if (w < rows[i]) buf[slot[i]] = cur[i];
        __syncthreads();
        for (int q = tid; q < nvalid; q += kScatterThreads) {
            const int b = slotbin[q];
            if (w * kHalf < (b / kBinE) * prm.bw)
                outp[(int64_t)w * prm.bld + gbase[b] + (q - loff[b])] = buf[q];
        }
#pragma unroll
        for (int i = 0; i < PER; i++) {
            cur[i] = n1[i];
            n1[i] = n2[i];
            n2[i] = n3[i];
        }
    }
}

template __global__ void bin_scatter_lds_kernel<kScatterChunkLarge>(ScatterParams);
template __global__ void bin_scatter_lds_kernel<kScatterChunkSmall>(ScatterParams);

}  // namespace shouji
