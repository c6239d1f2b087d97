// Host-side launch helper shared by the entry points: raising a kernel's
// dynamic LDS limit before a launch that needs more than the default.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <mutex>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace shouji {

// The largest dynamic LDS limit set so far for one kernel, per device (the
// attribute belongs to the kernel as loaded on the current device).
constexpr int kMaxDevices = 64;
struct LdsLimit {
    size_t bytes[kMaxDevices] = {};
};

// Raise `kernel`'s dynamic LDS limit on the current device to at least
// `bytes`.  Returns SHOUJI_OK or an error status with its text set.
inline int raise_lds_limit(const void *kernel, LdsLimit &limit, size_t bytes) {
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(SHOUJI_ERR_DEVICE, "no usable current HIP device");
    std::lock_guard<std::mutex> g(mu);
    if (bytes <= limit.bytes[dev]) return SHOUJI_OK;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "cannot raise the LDS limit to %zu bytes: %s", bytes,
                         hipGetErrorString(hipGetLastError()));
    limit.bytes[dev] = bytes;
    return SHOUJI_OK;
}

}  // namespace shouji
