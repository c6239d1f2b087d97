// Binning steps of the batched form (histogram, plan, scatter): constants,
// workspace layout and launch parameters shared by their kernels and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "shouji_internal.h"

namespace shouji {

constexpr int kMaxE = 31;                     // largest E (after clamping to m-1)
constexpr int kBinE = kMaxE + 1;              // E values per length bucket
constexpr int kPlanThreads = 1024;
constexpr int kCountThreads = 1024;           // histogram workgroup
constexpr int kCountGroups = 512;             // histogram workgroups at most
constexpr int kCountLds = 64 * 1024;          // LDS of the histogram copies at most
constexpr int kCostBuckets = 16;
// Tiles are launched per E class, each with the layout and LDS its largest E
// needs: Ee <= 13 takes the two-half layout (1024 pairs per wavefront), Ee <= 31
// the quarter layout (512 pairs per wavefront, two wavefronts per tile); both
// keep two wavefronts per SIMD.
constexpr int kEClasses = 2;
__host__ __device__ inline int e_class(int Ee) { return Ee <= 13 ? 0 : 1; }
__host__ __device__ inline int e_class_bound(int c) { return c == 0 ? 13 : 31; }
constexpr int kMinBinWidth = 4;
// The staged scatter takes chunks of 16,384 pairs per workgroup when its bin
// tables leave LDS room for them (longer runs per bin and chunk make longer
// writes), else chunks of 8,192 pairs.
constexpr int kScatterChunkLarge = 16384;
constexpr int kScatterChunkSmall = 8192;
constexpr int kScatterThreads = 1024;
inline size_t scatter_lds_bytes(int nbins, int chunk) {
    return (size_t)nbins * 4 * 2 + 8 + (size_t)nbins * 8 + (size_t)chunk * (2 + 2 + 4);
}
// LDS the staged scatter holds in static arrays (its scan's partial sums),
// beside the dynamic LDS of scatter_lds_bytes
constexpr size_t kScatterStaticLds = (size_t)kScatterThreads * 4;
// bins the staged scatter holds with chunks of `chunk` pairs (LDS of one CU):
// 1,791 with 16,384-pair chunks, 5,887 with 8,192
inline int scatter_max_bins(int chunk) {
    return (int)((kLdsPerCU - kScatterStaticLds - 8 - (size_t)chunk * 8) / 16);
}

struct PlanOut {
    int64_t *offsets;
    int64_t *cursors;
    int4 *tiles[kEClasses];
    int32_t *ntiles;          // kEClasses counts
};

struct ScatterParams {
    const uint32_t *reads;
    const uint32_t *refs;
    int64_t ld;
    const int32_t *lengths;
    const int32_t *Ep;
    int64_t n;
    int32_t max_len;
    int32_t bw;
    int64_t *cursors;
    int64_t *bperm;
    int32_t *blens;
    int32_t *bE;
    uint32_t *breads;
    uint32_t *brefs;
    int64_t bld;
    uint8_t *out_accept;
    int16_t *out_popcount;
    int32_t nbins;
};

// Byte offsets of the batched workspace regions (each 256-byte aligned).
struct BatchedLayout {
    size_t breads, brefs, blens, bE, bperm, counts, offsets, cursors, tiles[kEClasses], ntiles, total;
    int nbins, nw;
    int64_t max_tiles;
};
inline BatchedLayout batched_layout(int64_t n, int max_len, int bw) {
    BatchedLayout L;
    L.nw = (max_len + kHalf - 1) / kHalf;
    L.nbins = ((max_len + bw - 1) / bw + 1) * kBinE;
    L.max_tiles = L.nbins + (n + kPairsPerWave - 1) / kPairsPerWave;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    L.breads = take((size_t)L.nw * n * 4);
    L.brefs = take((size_t)L.nw * n * 4);
    L.blens = take((size_t)n * 4);
    L.bE = take((size_t)n * 4);
    L.bperm = take((size_t)n * 8);
    L.counts = take((size_t)L.nbins * 4);
    L.offsets = take((size_t)L.nbins * 8);
    L.cursors = take((size_t)L.nbins * 8);
    for (int c = 0; c < kEClasses; c++) L.tiles[c] = take((size_t)L.max_tiles * 16);
    L.ntiles = take(kEClasses * 4);
    L.total = off;
    return L;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v);
__global__ void bin_count_kernel(const int32_t *lengths, const int32_t *Ep, int64_t n, int max_len,
                                 int bw, int nbins, int ncopies, int32_t *counts);
__global__ void bin_plan_kernel(const int32_t *counts, int nbins, int nbucket_len, PlanOut out);
__global__ void bin_scatter_kernel(ScatterParams prm);
template <int CHUNK>
__global__ void bin_scatter_lds_kernel(ScatterParams prm);

}  // namespace shouji
