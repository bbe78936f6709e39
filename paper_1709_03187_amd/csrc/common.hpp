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

// The device error word: guard bits (DeviceError, in device.hpp) that
// kernels set when device data breaks a stated precondition.

// Device address of the current device's error word (a `__device__` array of
// the library, located once per device; no allocation), or nullptr after a
// HIP error (message recorded).
uint32_t *device_error_word();
// Takes the error word (atomically reset to 0) in stream order, synchronises
// with `st` and returns ACO_ERR_DEVICE with a message naming the tripped
// guards, or ACO_OK.
int report_device_error(hipStream_t st);

// Copies the caller's parameters into `out`: only its struct_size bytes are
// read, later fields take their defaults.  INVALID_ARG when p is NULL or its
// struct_size does not cover the fields through seed.
int load_params(const aco_params_t *p, aco_params_t &out);

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
