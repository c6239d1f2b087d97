// C ABI of the Shouji filter: argument checks, launch configuration, errors.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdint.h>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int ok() {
    g_err[0] = '\0';
    return SHOUJI_OK;
}

}  // namespace

extern "C" const char *shouji_last_error(void) { return g_err; }

extern "C" int shouji_version(void) { return 1 * 10000 + 0 * 100 + 0; }

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
    prm.R = shouji::ring_slots(Ee);
    prm.out_accept = out_accept;
    prm.out_popcount = out_popcount;
    prm.n = n_pairs;
    // Workgroups of 4 wavefronts (1024 pairs each); LDS and registers let a CU
    // hold two of them, i.e. two wavefronts per SIMD.
    const size_t wave_lds = shouji::plain_lds_wave_bytes(Ee);
    const size_t lds = wave_lds * shouji::kWavesPerGroup;
    if (lds > shouji::kLdsPerCU) return fail(SHOUJI_ERR_RANGE, "E %d needs more LDS than one CU holds", E);
    const int64_t waves = (n_pairs + shouji::kPairsPerWave - 1) / shouji::kPairsPerWave;
    const int64_t grid = (waves + shouji::kWavesPerGroup - 1) / shouji::kWavesPerGroup;
    if (grid > 0x7fffffff) return fail(SHOUJI_ERR_ARG, "n_pairs too large");
    prm.lds_wave_bytes = (int32_t)wave_lds;
    static bool attr_set = false;   // raise the dynamic LDS limit once per process
    if (!attr_set) {
        if (hipFuncSetAttribute((const void *)shouji::shouji_plain_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shouji::kLdsPerCU) != hipSuccess)
            return fail(SHOUJI_ERR_DEVICE, "cannot raise the LDS limit: %s",
                        hipGetErrorString(hipGetLastError()));
        attr_set = true;
    }
    hipLaunchKernelGGL(shouji::shouji_plain_kernel, dim3((unsigned)grid),
                       dim3(shouji::kWave * shouji::kWavesPerGroup), lds, (hipStream_t)stream, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SHOUJI_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}
