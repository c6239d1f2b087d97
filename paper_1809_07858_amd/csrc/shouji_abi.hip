// C ABI of the Shouji filter: argument checks, launch configuration, errors.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <utility>

#include "../../include/shouji.h"
#include "shouji_binning.h"
#include "shouji_launch.h"
#include "shouji_internal.h"

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace shouji {

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int clear_error() {
    g_err[0] = '\0';
    return SHOUJI_OK;
}

}  // namespace shouji

namespace {
template <typename... A>
inline int fail(int code, const char *fmt, A... a) { return shouji::set_error(code, fmt, a...); }
inline int ok() { return shouji::clear_error(); }
}  // namespace

extern "C" const char *shouji_last_error(void) { return g_err; }

namespace {
using shouji::LdsLimit;
using shouji::raise_lds_limit;
}  // namespace

extern "C" int shouji_version(void) { return 1 * 10000 + 0 * 100 + 0; }

namespace {
// Largest E at which the layout with 32 pair lanes per half keeps two
// wavefronts per SIMD: with a length array (ring, masks and length planes)
// and without one (ring only).  Above it the quarter layout is launched.
constexpr int kPlainHalfMaxE = 13;
constexpr int kRingOnlyHalfMaxE = 22;
// Wavefronts a CU holds with workgroups of wpg wavefronts of wl LDS bytes
// each (registers allow two per SIMD).
int waves_per_cu(size_t wl, int wpg) {
    const size_t w = shouji::kLdsPerCU / (wl * wpg) * wpg;
    return w > 8 ? 8 : (int)w;
}
// Ring slots of a plain launch with workgroups of wpg wavefronts: 8-aligned
// unless that lets a CU hold fewer wavefronts.
int plain_ring(int Ee, int wpg) {
    const int a = shouji::ring_slots_aligned(Ee), m = shouji::ring_slots(Ee);
    return waves_per_cu(shouji::plain_lds_wave_bytes(Ee, a), wpg) >=
                   waves_per_cu(shouji::plain_lds_wave_bytes(Ee, m), wpg)
               ? a
               : m;
}
}  // namespace

extern "C" int shouji_filter(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                             int32_t E, uint8_t *out_accept, int16_t *out_popcount,
                             int64_t n_pairs, int32_t max_len, int64_t ld, void *stream) {
    if (n_pairs < 0) return fail(SHOUJI_ERR_ARG, "n_pairs < 0 (%lld)", (long long)n_pairs);
    if (E < 0) return fail(SHOUJI_ERR_ARG, "E < 0 (%d)", E);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return fail(SHOUJI_ERR_RANGE, "max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    const int32_t Ee = max_len > 0 ? (E < max_len - 1 ? E : max_len - 1) : 0;
    if (Ee > SHOUJI_MAX_E)
        return fail(SHOUJI_ERR_RANGE, "E %d (clamped %d) above the supported maximum %d", E, Ee,
                    SHOUJI_MAX_E);
    if (n_pairs == 0) return ok();
    if (!reads || !refs || !out_accept) return fail(SHOUJI_ERR_NULL, "reads, refs and out_accept are required");
    if (ld < n_pairs) return fail(SHOUJI_ERR_ARG, "ld %lld < n_pairs %lld", (long long)ld, (long long)n_pairs);

    shouji::PlainParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.lengths = lengths;
    prm.max_len = max_len;
    prm.E = E;
    prm.Ee = Ee;
    prm.out_accept = out_accept;
    prm.out_popcount = out_popcount;
    prm.n = n_pairs;
    // Workgroups of 4 wavefronts (1024 pairs each); LDS and registers let a CU
    // hold two of them, i.e. two wavefronts per SIMD.  Without a length array
    // every pair has max_len bases: the boundary masks follow from the
    // positions, and a wavefront's LDS holds the pattern ring only (two
    // wavefronts per SIMD up to E = 22 instead of 13).  Above that (E >= 14
    // with lengths, E >= 23 without) the quarter layout (512 pairs per
    // wavefront, half the ring per wavefront) keeps two wavefronts per SIMD.
    prm.ring_only = lengths == nullptr ? 1 : 0;
    const bool quarter = prm.ring_only ? Ee > kRingOnlyHalfMaxE : Ee > kPlainHalfMaxE;
    prm.qh = shouji::quarter_h(Ee);
    size_t wave_lds;
    int64_t pairs_per_wave;
    if (quarter) {
        const int a = shouji::quarter_ring_slots_aligned(Ee), m = shouji::quarter_ring_slots(Ee);
        const bool ro = prm.ring_only != 0;
        prm.R = waves_per_cu(shouji::quarter_lds_wave_bytes(Ee, a, ro), shouji::kWavesPerGroup) >=
                        waves_per_cu(shouji::quarter_lds_wave_bytes(Ee, m, ro), shouji::kWavesPerGroup)
                    ? a
                    : m;
        wave_lds = shouji::quarter_lds_wave_bytes(Ee, prm.R, ro);
        pairs_per_wave = shouji::kQuarterPairs;
    } else {
        if (prm.ring_only) {
            const int a = shouji::ring_slots_aligned(Ee), m = shouji::ring_slots(Ee);
            prm.R = waves_per_cu(shouji::ring_lds_wave_bytes(a), shouji::kWavesPerGroup) >=
                            waves_per_cu(shouji::ring_lds_wave_bytes(m), shouji::kWavesPerGroup)
                        ? a
                        : m;
        } else {
            prm.R = plain_ring(Ee, shouji::kWavesPerGroup);
        }
        wave_lds = prm.ring_only ? shouji::ring_lds_wave_bytes(prm.R) : shouji::plain_lds_wave_bytes(Ee, prm.R);
        pairs_per_wave = shouji::kPairsPerWave;
    }
    const size_t lds = wave_lds * shouji::kWavesPerGroup;
    if (lds > shouji::kLdsPerCU) return fail(SHOUJI_ERR_RANGE, "E %d needs more LDS than one CU holds", E);
    const int64_t waves = (n_pairs + pairs_per_wave - 1) / pairs_per_wave;
    const int64_t grid = (waves + shouji::kWavesPerGroup - 1) / shouji::kWavesPerGroup;
    if (grid > 0x7fffffff) return fail(SHOUJI_ERR_ARG, "n_pairs too large");
    prm.lds_wave_bytes = (int32_t)wave_lds;
    static LdsLimit lds_limit[4];
    const int which = (quarter ? 2 : 0) + (prm.ring_only ? 1 : 0);
    const void *kernels[4] = {(const void *)shouji::shouji_plain_kernel, (const void *)shouji::shouji_plain_ring_kernel,
                              (const void *)shouji::shouji_plain_q_kernel,
                              (const void *)shouji::shouji_plain_ring_q_kernel};
    if (int rc = raise_lds_limit(kernels[which], lds_limit[which], lds)) return rc;
    const dim3 gdim((unsigned)grid), bdim(shouji::kWave * shouji::kWavesPerGroup);
    switch (which) {
        case 0: hipLaunchKernelGGL(shouji::shouji_plain_kernel, gdim, bdim, lds, (hipStream_t)stream, prm); break;
        case 1: hipLaunchKernelGGL(shouji::shouji_plain_ring_kernel, gdim, bdim, lds, (hipStream_t)stream, prm); break;
        case 2: hipLaunchKernelGGL(shouji::shouji_plain_q_kernel, gdim, bdim, lds, (hipStream_t)stream, prm); break;
        default: hipLaunchKernelGGL(shouji::shouji_plain_ring_q_kernel, gdim, bdim, lds, (hipStream_t)stream, prm);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SHOUJI_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

extern "C" int shouji_filter_local(const uint32_t *reads, const uint32_t *refs, const int32_t *read_lengths,
                                   const int32_t *ref_lengths, int32_t E, int32_t mode, uint8_t *out_accept,
                                   int16_t *out_popcount, int64_t n_pairs, int32_t max_len, int64_t ld,
                                   void *stream) {
    if (n_pairs < 0) return fail(SHOUJI_ERR_ARG, "n_pairs < 0 (%lld)", (long long)n_pairs);
    if (E < 0) return fail(SHOUJI_ERR_ARG, "E < 0 (%d)", E);
    if (mode < SHOUJI_COUNT_GLOBAL || mode > SHOUJI_COUNT_GLOCAL_END)
        return fail(SHOUJI_ERR_ARG, "counting mode %d is not one of 0..3", mode);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return fail(SHOUJI_ERR_RANGE, "max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    const int32_t Ee = max_len > 0 ? (E < max_len - 1 ? E : max_len - 1) : 0;
    if (Ee > SHOUJI_MAX_E)
        return fail(SHOUJI_ERR_RANGE, "E %d (clamped %d) above the supported maximum %d", E, Ee,
                    SHOUJI_MAX_E);
    if (n_pairs == 0) return ok();
    if (!reads || !refs || !out_accept || !read_lengths || !ref_lengths)
        return fail(SHOUJI_ERR_NULL, "reads, refs, both length arrays and out_accept are required");
    if (ld < n_pairs) return fail(SHOUJI_ERR_ARG, "ld %lld < n_pairs %lld", (long long)ld, (long long)n_pairs);

    shouji::LocalParams prm;
    prm.reads = reads;
    prm.refs = refs;
    prm.ld = ld;
    prm.read_lengths = read_lengths;
    prm.ref_lengths = ref_lengths;
    prm.max_len = max_len;
    prm.E = E;
    prm.Ee = Ee;
    prm.mode = mode;
    prm.out_accept = out_accept;
    prm.out_popcount = out_popcount;
    prm.n = n_pairs;
    // As many wavefronts per CU as LDS allows, up to two per SIMD: workgroups
    // of four wavefronts when two of them fit, else of one.
    int len_bits = 1;
    while ((1 << len_bits) <= max_len) len_bits++;   // bits of max_len
    prm.len_bits = len_bits;
    // the 8-aligned ring unless the minimal one lets a CU hold more wavefronts
    auto local_wpg = [](size_t wl) { return 8 * wl <= shouji::kLdsPerCU ? shouji::kWavesPerGroup : 1; };
    auto local_waves = [&](size_t wl) { return wl > shouji::kLdsPerCU ? 0 : waves_per_cu(wl, local_wpg(wl)); };
    prm.R = shouji::ring_slots(Ee);
    if (local_waves(shouji::local_lds_wave_bytes(Ee, len_bits, shouji::ring_slots_aligned(Ee))) >=
        local_waves(shouji::local_lds_wave_bytes(Ee, len_bits, prm.R)))
        prm.R = shouji::ring_slots_aligned(Ee);
    const size_t wave_lds = shouji::local_lds_wave_bytes(Ee, len_bits, prm.R);
    if (wave_lds > shouji::kLdsPerCU) return fail(SHOUJI_ERR_RANGE, "E %d needs more LDS than one CU holds", E);
    const int wpg = local_wpg(wave_lds);
    const size_t lds = wave_lds * wpg;
    const int64_t waves = (n_pairs + shouji::kPairsPerWave - 1) / shouji::kPairsPerWave;
    const int64_t grid = (waves + wpg - 1) / wpg;
    if (grid > 0x7fffffff) return fail(SHOUJI_ERR_ARG, "n_pairs too large");
    prm.waves_per_group = wpg;
    prm.lds_wave_bytes = (int32_t)wave_lds;
    static LdsLimit lds_limit;
    if (int rc = raise_lds_limit((const void *)shouji::shouji_local_kernel, lds_limit, lds)) return rc;
    hipLaunchKernelGGL(shouji::shouji_local_kernel, dim3((unsigned)grid), dim3(shouji::kWave * wpg), lds,
                       (hipStream_t)stream, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SHOUJI_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

// ---------------------------------------------------------------- batched form

namespace {

struct TuneKey {
    int len_bucket, n_log2;
    bool operator<(const TuneKey &o) const {
        return len_bucket != o.len_bucket ? len_bucket < o.len_bucket : n_log2 < o.n_log2;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, shouji_batched_config> g_tune;

TuneKey tune_key(int64_t n, int32_t max_len) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= n) lg++;
    return TuneKey{max_len / 64, lg};
}

bool valid_config(const shouji_batched_config &c) {
    return (c.bin_width == 4 || c.bin_width == 8 || c.bin_width == 16 || c.bin_width == 32) &&
           (c.waves_per_group == 1 || c.waves_per_group == 2 || c.waves_per_group == 4);
}

shouji_batched_config resolve_config(const shouji_batched_config *cfg, int64_t n, int32_t max_len) {
    if (cfg && (cfg->bin_width || cfg->waves_per_group)) {
        shouji_batched_config c = *cfg;
        if (!c.bin_width) c.bin_width = 8;
        if (!c.waves_per_group) c.waves_per_group = shouji::kWavesPerGroup;
        return c;
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(n, max_len));
    if (it != g_tune.end()) return it->second;
    return shouji_batched_config{8, shouji::kWavesPerGroup};
}

}  // namespace

extern "C" int64_t shouji_batched_workspace_bytes(int64_t n_pairs, int32_t max_len) {
    if (n_pairs < 0) return fail(SHOUJI_ERR_ARG, "n_pairs < 0");
    if (n_pairs > SHOUJI_MAX_BATCHED_PAIRS)
        return fail(SHOUJI_ERR_RANGE, "n_pairs %lld above the batched form's limit %lld", (long long)n_pairs,
                    (long long)SHOUJI_MAX_BATCHED_PAIRS);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return fail(SHOUJI_ERR_RANGE, "max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    ok();
    return (int64_t)shouji::batched_layout(n_pairs, max_len, shouji::kMinBinWidth).total;
}

extern "C" int shouji_filter_batched(const uint32_t *reads, const uint32_t *refs,
                                     const int32_t *lengths, const int32_t *E_per_pair,
                                     uint8_t *out_accept, int16_t *out_popcount, int64_t n_pairs,
                                     int32_t max_len, int64_t ld, void *workspace,
                                     int64_t workspace_bytes, const shouji_batched_config *config,
                                     void *stream) {
    if (n_pairs < 0) return fail(SHOUJI_ERR_ARG, "n_pairs < 0 (%lld)", (long long)n_pairs);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return fail(SHOUJI_ERR_RANGE, "max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    // bin counts, cursors within a bin and tile starts are 32-bit
    if (n_pairs > SHOUJI_MAX_BATCHED_PAIRS)
        return fail(SHOUJI_ERR_RANGE, "n_pairs %lld above the batched form's limit %lld", (long long)n_pairs,
                    (long long)SHOUJI_MAX_BATCHED_PAIRS);
    if (n_pairs == 0) return ok();
    if (!reads || !refs || !E_per_pair || !out_accept || !workspace)
        return fail(SHOUJI_ERR_NULL, "reads, refs, E_per_pair, out_accept and workspace are required");
    if (ld < n_pairs) return fail(SHOUJI_ERR_ARG, "ld %lld < n_pairs %lld", (long long)ld, (long long)n_pairs);
    const shouji_batched_config cfg = resolve_config(config, n_pairs, max_len);
    if (!valid_config(cfg))
        return fail(SHOUJI_ERR_ARG, "bad config (bin_width %d, waves_per_group %d)", cfg.bin_width,
                    cfg.waves_per_group);
    const shouji::BatchedLayout L = shouji::batched_layout(n_pairs, max_len, cfg.bin_width);
    const int64_t need = (int64_t)shouji::batched_layout(n_pairs, max_len, shouji::kMinBinWidth).total;
    if (workspace_bytes < need)
        return fail(SHOUJI_ERR_ARG, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes,
                    (long long)need);
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *counts = (int32_t *)(ws + L.counts);
    int32_t *ntiles = (int32_t *)(ws + L.ntiles);

    // 1. histogram of (length bucket, E)
    hipLaunchKernelGGL(shouji::fill_i32_kernel, dim3((L.nbins + 255) / 256), dim3(256), 0, st, counts,
                       (int64_t)L.nbins, 0);
    {
        const int64_t per = (int64_t)shouji::kCountThreads * 4;
        const int64_t blocks = (n_pairs + per - 1) / per;
        const int fit = (int)(shouji::kCountLds / ((size_t)L.nbins * 4));
        const int copies = fit < 1 ? 1 : (fit > shouji::kCountThreads / shouji::kWave ? shouji::kCountThreads / shouji::kWave : fit);
        hipLaunchKernelGGL(shouji::bin_count_kernel,
                           dim3((unsigned)(blocks < shouji::kCountGroups ? blocks : shouji::kCountGroups)),
                           dim3(shouji::kCountThreads), (size_t)L.nbins * 4 * copies, st, lengths, E_per_pair,
                           n_pairs, max_len, cfg.bin_width, L.nbins, copies, counts);
    }
    // 2. bin offsets and tile lists
    shouji::PlanOut po;
    po.offsets = (int64_t *)(ws + L.offsets);
    po.cursors = (int64_t *)(ws + L.cursors);
    for (int c = 0; c < shouji::kEClasses; c++) po.tiles[c] = (int4 *)(ws + L.tiles[c]);
    po.ntiles = ntiles;
    hipLaunchKernelGGL(shouji::bin_plan_kernel, dim3(1), dim3(shouji::kPlanThreads), 0, st, counts,
                       L.nbins, (max_len + cfg.bin_width - 1) / cfg.bin_width + 1, po);
    // 3. scatter into the binned workspace
    shouji::ScatterParams sp;
    sp.reads = reads;
    sp.refs = refs;
    sp.ld = ld;
    sp.lengths = lengths;
    sp.Ep = E_per_pair;
    sp.n = n_pairs;
    sp.max_len = max_len;
    sp.bw = cfg.bin_width;
    sp.cursors = po.cursors;
    sp.bperm = (int64_t *)(ws + L.bperm);
    sp.blens = (int32_t *)(ws + L.blens);
    sp.bE = (int32_t *)(ws + L.bE);
    sp.breads = (uint32_t *)(ws + L.breads);
    sp.brefs = (uint32_t *)(ws + L.brefs);
    sp.bld = n_pairs;
    sp.out_accept = out_accept;
    sp.out_popcount = out_popcount;
    sp.nbins = L.nbins;
    const int chunk = L.nbins <= shouji::scatter_max_bins(shouji::kScatterChunkLarge) ? shouji::kScatterChunkLarge
                                                                                        : shouji::kScatterChunkSmall;
    if (L.nbins <= shouji::scatter_max_bins(chunk)) {
        static LdsLimit slimit_large, slimit_small;
        const bool large = chunk == shouji::kScatterChunkLarge;
        const void *sk = large ? (const void *)shouji::bin_scatter_lds_kernel<shouji::kScatterChunkLarge>
                               : (const void *)shouji::bin_scatter_lds_kernel<shouji::kScatterChunkSmall>;
        const size_t slds = shouji::scatter_lds_bytes(L.nbins, chunk);
        if (int rc = raise_lds_limit(sk, large ? slimit_large : slimit_small, slds)) return rc;
        const int64_t chunks = (n_pairs + chunk - 1) / chunk;
        if (large)
            hipLaunchKernelGGL(shouji::bin_scatter_lds_kernel<shouji::kScatterChunkLarge>, dim3((unsigned)chunks),
                               dim3(shouji::kScatterThreads), slds, st, sp);
        else
            hipLaunchKernelGGL(shouji::bin_scatter_lds_kernel<shouji::kScatterChunkSmall>, dim3((unsigned)chunks),
                               dim3(shouji::kScatterThreads), slds, st, sp);
    } else {
        const int64_t blocks = (n_pairs + 255) / 256;
        hipLaunchKernelGGL(shouji::bin_scatter_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)),
                           dim3(256), 0, st, sp);
    }
    // 4. the filter over the tiles, largest E class first
    static LdsLimit tlimit;
    const int Emax_len = max_len > 0 ? max_len - 1 : 0;
    for (int c = shouji::kEClasses - 1; c >= 0; c--) {
        if (c > 0 && Emax_len <= shouji::e_class_bound(c - 1)) continue;   // the class is empty
        int Ecls = shouji::e_class_bound(c);
        if (Ecls > Emax_len) Ecls = Emax_len;
        shouji::TilesParams tp;
        tp.breads = sp.breads;
        tp.brefs = sp.brefs;
        tp.ld = n_pairs;
        tp.blens = sp.blens;
        tp.bE = sp.bE;
        tp.bperm = sp.bperm;
        tp.tiles = po.tiles[c];
        tp.ntiles = ntiles + c;
        tp.max_len = max_len;
        // the workgroup size (at most the configured one) that lets a CU hold
        // the most wavefronts (two per SIMD at most), with the 8-aligned ring
        // unless the minimal one lets it hold more
        auto best_group = [&](size_t wl, int &best_waves) {
            int wpg_ = 0;
            best_waves = 0;
            for (int g = cfg.waves_per_group; g >= 1; g >>= 1) {
                int waves = (int)(shouji::kLdsPerCU / (wl * g)) * g;
                if (waves > 8) waves = 8;
                if (waves > best_waves) { best_waves = waves; wpg_ = g; }
            }
            return wpg_;
        };
        // the large-E class runs the quarter layout (two wavefronts of 512
        // pairs per tile), which keeps two wavefronts per SIMD
        const bool quarter = c > 0;
        auto wave_bytes = [&](int R) {
            return quarter ? shouji::quarter_lds_wave_bytes(Ecls, R, false) : shouji::plain_lds_wave_bytes(Ecls, R);
        };
        const int Ra = quarter ? shouji::quarter_ring_slots_aligned(Ecls) : shouji::ring_slots_aligned(Ecls);
        const int Rm = quarter ? shouji::quarter_ring_slots(Ecls) : shouji::ring_slots(Ecls);
        int best_waves = 0, best_min = 0;
        int wpg = best_group(wave_bytes(Ra), best_waves);
        tp.R = Ra;
        const int wpg_min = best_group(wave_bytes(Rm), best_min);
        if (best_min > best_waves) {
            wpg = wpg_min;
            tp.R = Rm;
        }
        const size_t wave_lds = wave_bytes(tp.R);
        if (wpg == 0) return fail(SHOUJI_ERR_RANGE, "LDS too small for E %d", Ecls);
        tp.lds_wave_bytes = (int32_t)wave_lds;
        tp.waves_per_group = wpg;
        tp.qh = shouji::quarter_h(Ecls);
        tp.out_accept = out_accept;
        tp.out_popcount = out_popcount;
        const int64_t waves_needed = quarter ? 2 * L.max_tiles : L.max_tiles;
        const int64_t grid = (waves_needed + wpg - 1) / wpg;
        if (quarter) {
            static LdsLimit qlimit;
            if (int rc = raise_lds_limit((const void *)shouji::shouji_tiles_q_kernel, qlimit, wave_lds * wpg))
                return rc;
            hipLaunchKernelGGL(shouji::shouji_tiles_q_kernel, dim3((unsigned)grid), dim3(shouji::kWave * wpg),
                               wave_lds * wpg, st, tp);
        } else {
            if (int rc = raise_lds_limit((const void *)shouji::shouji_tiles_kernel, tlimit, wave_lds * wpg))
                return rc;
            hipLaunchKernelGGL(shouji::shouji_tiles_kernel, dim3((unsigned)grid), dim3(shouji::kWave * wpg),
                               wave_lds * wpg, st, tp);
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SHOUJI_ERR_DEVICE, "batched launch failed: %s", hipGetErrorString(e));
    return ok();
}

extern "C" int shouji_tune_batched(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                                   const int32_t *E_per_pair, uint8_t *out_accept,
                                   int16_t *out_popcount, int64_t n_pairs, int32_t max_len, int64_t ld,
                                   void *workspace, int64_t workspace_bytes, void *stream,
                                   shouji_batched_config *best, float *best_ms) {
    static const int widths[] = {4, 8, 16, 32};
    static const int wpgs[] = {2, 4};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(SHOUJI_ERR_DEVICE, "cannot create events");
    shouji_batched_config top{0, 0};
    float top_ms = 1e30f;
    int rc = SHOUJI_OK;
    for (int wi = 0; wi < 4 && rc == SHOUJI_OK; wi++) {
        for (int gi = 0; gi < 2 && rc == SHOUJI_OK; gi++) {
            const shouji_batched_config c{widths[wi], wpgs[gi]};
            rc = shouji_filter_batched(reads, refs, lengths, E_per_pair, out_accept, out_popcount,
                                       n_pairs, max_len, ld, workspace, workspace_bytes, &c, stream);
            if (rc) break;
            if (hipEventRecord(a, st) != hipSuccess) { rc = fail(SHOUJI_ERR_DEVICE, "tuning event failed"); break; }
            for (int r = 0; r < 3 && rc == SHOUJI_OK; r++)
                rc = shouji_filter_batched(reads, refs, lengths, E_per_pair, out_accept, out_popcount,
                                           n_pairs, max_len, ld, workspace, workspace_bytes, &c, stream);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                hipEventElapsedTime(&ms, a, b) != hipSuccess) {
                rc = fail(SHOUJI_ERR_DEVICE, "tuning run failed");
                break;
            }
            ms /= 3.f;
            if (ms < top_ms) { top_ms = ms; top = c; }
        }
    }
    // the events are released whatever the tuning runs returned; a failure
    // to release them does not change the tuned configuration
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[tune_key(n_pairs, max_len)] = top;
    }
    if (best) *best = top;
    if (best_ms) *best_ms = top_ms;
    return ok();
}

// ------------------------------------------- batched form without allocation

namespace {

// The binned copy of shouji_filter_batched_noalloc: a device array owned by
// the library (each GPU the library runs on holds its own copy until the
// process ends).  In host code `noalloc_scratch` names a host-side stand-in,
// never the device memory: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) unsigned char noalloc_scratch[SHOUJI_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device ordinal -> address of its copy

int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(SHOUJI_ERR_DEVICE, "no current HIP device: %s", hipGetErrorString(hipGetLastError()));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(SHOUJI_ERR_DEVICE, "cannot locate the scratch array on device %d: %s", dev,
                        hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return SHOUJI_OK;
}

}  // namespace

extern "C" int shouji_filter_batched_noalloc(const uint32_t *reads, const uint32_t *refs,
                                             const int32_t *lengths, const int32_t *E_per_pair,
                                             uint8_t *out_accept, int16_t *out_popcount, int64_t n_pairs,
                                             int32_t max_len, int64_t ld,
                                             const shouji_batched_config *config, void *stream) {
    // sizes first: nothing here touches the device before they are accepted
    if (n_pairs < 0) return fail(SHOUJI_ERR_ARG, "n_pairs < 0 (%lld)", (long long)n_pairs);
    if (max_len < 0 || max_len > SHOUJI_MAX_LEN)
        return fail(SHOUJI_ERR_RANGE, "max_len %d outside [0, %d]", max_len, SHOUJI_MAX_LEN);
    if (n_pairs > SHOUJI_MAX_BATCHED_PAIRS)
        return fail(SHOUJI_ERR_RANGE, "n_pairs %lld above the batched form's limit %lld", (long long)n_pairs,
                    (long long)SHOUJI_MAX_BATCHED_PAIRS);
    if (n_pairs == 0) return ok();
    const int64_t need = (int64_t)shouji::batched_layout(n_pairs, max_len, shouji::kMinBinWidth).total;
    if (need > SHOUJI_NOALLOC_SCRATCH_BYTES)
        return fail(SHOUJI_ERR_RANGE,
                    "%lld pairs of up to %d bases need %lld bytes of scratch, the library holds %lld: "
                    "call shouji_filter_batched with a workspace instead",
                    (long long)n_pairs, max_len, (long long)need, (long long)SHOUJI_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    // the same binning, scatter and tile kernels as the call with a workspace
    return shouji_filter_batched(reads, refs, lengths, E_per_pair, out_accept, out_popcount, n_pairs, max_len,
                                 ld, ws, SHOUJI_NOALLOC_SCRATCH_BYTES, config, stream);
}
