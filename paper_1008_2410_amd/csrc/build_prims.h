// Building blocks shared by the device tree builds (tree_build.hip for the uniform tree,
// adaptive_build.hip for the adaptive one): stream-ordered temporaries, an error status,
// a device-wide exclusive scan, a stable radix sort and the bounding square.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fmm2d.h"

namespace fmm {

inline unsigned grid_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// A region of device memory that is idle during a build (the per-call region of the
// evaluation workspace that a rebuilt tree takes over), lent to the build's temporaries
// as a stack: a block is taken at the top and the top moves back down when the topmost
// blocks have been given back.  All of a build's work runs on one stream, so a block
// given back while kernels that use it are still queued is only reused by kernels queued
// after them.  Requests that do not fit go to the stream-ordered pool.
struct BuildArena {
    char *base = nullptr;
    size_t cap = 0;
    struct Block {
        size_t off, end;
        bool live;
    };
    std::vector<Block> stack;
    void *take(size_t bytes)
    {
        const size_t off = stack.empty() ? 0 : (stack.back().end + 255) / 256 * 256;
        if (!base || off + bytes > cap) return nullptr;
        stack.push_back({off, off + bytes, true});
        return base + off;
    }
    void give(void *p)
    {
        for (Block &b : stack)
            if (base + b.off == (char *)p) b.live = false;
        while (!stack.empty() && !stack.back().live) stack.pop_back();
    }
};

// The arena of the build running on this host thread (null: temporaries from the pool).
inline thread_local BuildArena *t_build_arena = nullptr;

struct BuildArenaScope {
    BuildArena *prev;
    explicit BuildArenaScope(BuildArena *a) : prev(t_build_arena) { t_build_arena = a; }
    ~BuildArenaScope() { t_build_arena = prev; }
};

// Device buffer owned for the duration of a build step.
template <typename T>
struct Buf {
    // stream-ordered: allocated and freed in the order of the build's stream, so a
    // temporary can be released while kernels that use it are still queued
    T *p = nullptr;
    hipStream_t s = nullptr;
    BuildArena *arena = nullptr;  // the block came from this arena
    ~Buf()
    {
        if (!p) return;
        if (arena) arena->give(p);
        else (void)hipFreeAsync(p, s);
    }
    // kept: the buffer outlives the build (handed to the tree by release()), so it never
    // comes from the arena
    hipError_t alloc(int64_t count, hipStream_t stream, bool kept = false)
    {
        s = stream;
        const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        if (!kept && t_build_arena) {
            if (void *q = t_build_arena->take(bytes)) {
                p = (T *)q;
                arena = t_build_arena;
                return hipSuccess;
            }
        }
        return hipMallocAsync((void **)&p, bytes, stream);
    }
    // hands the buffer over (allocated with kept = true)
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
