// Building blocks shared by the device tree builds (tree_build.hip for the uniform tree,
// adaptive_build.hip for the adaptive one): stream-ordered temporaries, an error status,
// a device-wide exclusive scan, a stable radix sort and the bounding square.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/fmm2d.h"

namespace fmm {

inline unsigned grid_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// Device buffer owned for the duration of a build step.
template <typename T>
struct Buf {
    // stream-ordered: allocated and freed in the order of the build's stream, so a
    // temporary can be released while kernels that use it are still queued
    T *p = nullptr;
    hipStream_t s = nullptr;
    ~Buf()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
    hipError_t alloc(int64_t count, hipStream_t stream)
    {
        s = stream;
        return hipMallocAsync((void **)&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T), stream);
    }
    T *release()
    {
        T *q = p;
        p = nullptr;
        return q;
    }
};

struct Status {
    int code = FMM_OK;
    std::string msg;
    bool check(hipError_t e, const char *what)
    {
        if (e == hipSuccess) return true;
        if (code == FMM_OK) {
            code = e == hipErrorOutOfMemory ? FMM_ENOMEM : FMM_EDEVICE;
            msg = std::string(what) + ": " + hipGetErrorString(e);
        }
        return false;
    }
};

// Exclusive scan of n uint32 (totals below 2^32; in place allowed) on stream s;
// *total_host receives the sum (after a synchronisation of s) if non-null.
bool scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_host, hipStream_t s, Status &st);

// Stable LSD sort of (keys, vals) in place by the low `bits` bits of the keys, 8-bit digits.
bool radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s, Status &st);

// Staging slots of the two-pass permutations for the sorted order perm (sorted slot ->
// user index, device): bucket shift, gpos1 (user index -> staging slot), gpos2 (sorted
// slot -> staging slot of its user index) and a staging array st1 of n doubles, the three
// from the stream-ordered pool.  Buckets of 2^shift sorted slots, ordered by user index
// inside a bucket.
bool build_staging(const int *perm, int64_t n, hipStream_t s, Status &st, int &shift, int *&gpos1, int *&gpos2,
                   double *&st1);

// Root cell when none is given: {x0, y0, side} = (min x, min y, max(range x, range y) (1 + 2^-20)),
// side 1 for a single point; nonfinite when any coordinate is not finite.  Synchronises s.
bool bounding_square(const double2 *xy, int64_t n, hipStream_t s, Status &st, double box[3], bool &nonfinite);

}  // namespace fmm
