// Host-side helpers shared by the C-ABI entry points: error state, launch
// checks and device limits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "aco.h"

namespace aco {

// Records a thread-local message for aco_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
void clear_error();

// Largest dynamic LDS allocation one workgroup may request on the current device.
size_t max_lds_per_block();
// Compute units of the current device.
int num_cus();

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Bytes of the per-ant visited bitmask (one bit per city).
inline size_t bitmask_bytes(int64_t n) { return (size_t)((n + 31) / 32) * 4; }

#define ACO_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::aco::fail(ACO_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define ACO_LAUNCH_CHECK(name)                                                           \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess)                                                            \
            return ::aco::fail(ACO_ERR_HIP, "launch of %s failed: %s", name,             \
                               hipGetErrorString(e_));                                   \
    } while (0)

#define ACO_REQUIRE(cond, ...)                                                           \
    do {                                                                                 \
        if (!(cond)) return ::aco::fail(ACO_ERR_INVALID_ARG, __VA_ARGS__);               \
    } while (0)

inline unsigned blocks_for(int64_t work, int threads)
{
    int64_t b = (work + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace aco
