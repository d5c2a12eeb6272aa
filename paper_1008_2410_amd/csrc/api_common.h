// Error reporting and device-allocation helpers shared by the sources of the C ABI
// (api.cpp, adaptive.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fmm2d.h"

namespace fmm {

// Sets the calling thread's message for fmm_last_error and returns code.
int fail(int code, const std::string &msg);
void clear_last_error();

// Coordinate scale of the near-field records: the pair kernel's exponent is -s (FP64,
// natural exp) or -s in base 2 (FP32) with s = |alpha dz|^2.
double record_alpha(double sigma, int precision);

inline int hip_fail(hipError_t e, const char *what)
{
    return fail(FMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
int dev_alloc(T **p, size_t count, const char *what)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FMM_ENOMEM, std::string("device allocation failed: ") + what);
    }
    return FMM_OK;
}

// Stream-ordered allocation from the device's default pool (see retain_pool).
template <typename T>
int dev_alloc_async(T **p, size_t count, const char *what, hipStream_t s)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMallocAsync((void **)p, count * sizeof(T), s);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FMM_ENOMEM, std::string("device allocation failed: ") + what);
    }
    return FMM_OK;
}

// Keep freed blocks of the device's default memory pool for reuse instead of returning
// them at every synchronisation, so that trees built and destroyed in a loop (time
// stepping) allocate from the pool.  Once per device.
void retain_pool(int device);
// Return the pool's unused memory to the device (after a fresh build, whose temporaries
// are freed, and when a tree is destroyed), so that what the pool holds follows what the
// library's trees and workspaces hold.  Synchronises the device first.
void trim_pool(int device);

template <typename T>
int upload(T **p, const std::vector<T> &h, const char *what)
{
    int rc = dev_alloc(p, h.size(), what);
    if (rc) return rc;
    if (!h.empty()) {
        hipError_t e = hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return FMM_OK;
}

// upload for host structs laid out as the device vector type D (HostD2 -> double2, ...)
template <typename D, typename H>
int upload_as(D **p, const std::vector<H> &h, const char *what)
{
    static_assert(sizeof(D) == sizeof(H), "host and device element layouts differ");
    int rc = dev_alloc(p, h.size(), what);
    if (rc) return rc;
    if (!h.empty()) {
        hipError_t e = hipMemcpy(*p, h.data(), h.size() * sizeof(D), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return FMM_OK;
}

}  // namespace fmm

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return fmm::hip_fail(e_, #expr);  \
    } while (0)
