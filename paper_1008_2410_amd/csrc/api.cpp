// C ABI of the gfx950 FMM library (include/fmm2d.h): argument checks, the host-side
// tree build (stages 1-3 of Fig. fmmStages), workspace management and the two-stream
// schedule of stages 4-10.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fmm2d.h"
#include "api_common.h"
#include "build_prims.h"
#include "fmm_internal.h"

using namespace fmm;

namespace {

thread_local std::string g_last_error;

// RAII guard for "one host thread per handle".
struct BusyGuard {
    fmm_tree *t;
    bool ok;
    explicit BusyGuard(fmm_tree *tree) : t(tree), ok(tree->busy.exchange(1) == 0) {}
    ~BusyGuard() { release(); }
    void release()
    {
        if (ok) t->busy.store(0);
        ok = false;
    }
};

// The workspace is allocated from the stream-ordered pool; callers have finished the
// device work that used it (destroy) or synchronised (reallocation).
void free_workspace(Workspace &ws, hipStream_t s)
{
    for (void *p : {ws.gam, (void *)ws.stage, (void *)ws.near, (void *)ws.mp_d, (void *)ws.lo_d, (void *)ws.mp_f,
                    (void *)ws.lo_f, (void *)ws.adj, (void *)ws.mp2_d, (void *)ws.lo2_d, (void *)ws.mp2_f,
                    (void *)ws.lo2_f, (void *)ws.rec2, ws.sums})
        if (p) hipFreeAsync(p, s);
    ws = Workspace{};
}

// The tree's device arrays (not its workspace, streams or events), freed in the order of
// stream fs; the caller has finished the work that used them.  Arrays of the device build
// come from the stream-ordered pool, those of the host build from hipMalloc; the
// near-field plan and the leaf-unit coordinates are always pooled.
void release_tree_arrays(fmm_tree *t, hipStream_t fs)
{
    auto release = [fs](auto *&p, bool pooled) {
        if (!p) return;
        if (pooled) hipFreeAsync((void *)p, fs);
        else hipFree((void *)p);
        p = nullptr;
    };
    release(t->d_perm, t->pooled);
    release(t->d_gpos1, t->pooled);
    release(t->d_gpos2, t->pooled);
    release(t->d_st1, t->pooled);
    release(t->d_leaf_of, t->pooled);
    release(t->d_xy, t->pooled);
    release(t->d_leaf_start, t->pooled);
    release(t->d_counts, t->pooled);
    release(t->d_lists, t->pooled);
    release(t->d_units, t->pooled);
    release(t->d_tile_start, t->pooled);
    release(t->d_tile_box, t->pooled);
    release(t->d_near_work, true);
    release(t->d_leaf_mask, true);
    release(t->d_pos[0], true);
    release(t->d_pos[1], true);
}

void free_tree(fmm_tree *t)
{
    hipStream_t fs = t->own_side;  // the caller has finished the work on the tree
    release_tree_arrays(t, fs);
    hipFree(t->d_flag);
    if (t->wsp.use_count() == 1) free_workspace(*t->wsp, fs);
    if (t->own_side) hipStreamDestroy(t->own_side);
    if (t->ev_fork) hipEventDestroy(t->ev_fork);
    if (t->ev_join) hipEventDestroy(t->ev_join);
    for (auto &evs : t->pending_timing)
        for (auto e : evs) hipEventDestroy(e);
    delete t;
}

// The mutual form is used when its plan has items; else the target-centric units alone.
bool use_mutual(const fmm_tree *t) { return t->near_mutual && t->nmut > 0; }

int effective_lc(const fmm_tree *t) { return std::min(t->lc, t->depth); }

// Last FP64 level: every level in FP64 precision; in mixed precision the coarse levels.
int split_level(const fmm_tree *t, int precision) { return precision == FMM_FP64 ? t->depth : effective_lc(t); }

// A workspace last used by another tree (a rebuild's hand-over, or a tree sharing it):
// multipoles of cells that are empty in this tree must read as zero (the M2L kernels
// read them unconditionally), so the multipole arrays are cleared.  Locals and
// per-particle arrays are written in full by every call before they are read.
int clear_multipoles(const fmm_tree *t, hipStream_t s)
{
    const Workspace &ws = *t->wsp;
    if (!ws.gam || t->depth < 2) return FMM_OK;
    const int64_t cells_d = level_base(std::min(ws.split, t->depth) + 1);
    const int64_t cells_f = level_base(t->depth + 1) - cells_d;
    const size_t bd = (cells_d * ws.p + kCoefPad) * sizeof(double2), bf = (cells_f * ws.p + kCoefPad) * sizeof(float2);
    for (double2 *m : {ws.mp_d, ws.mp2_d})
        if (m) HIP_TRY(hipMemsetAsync(m, 0, bd, s));
    for (float2 *m : {ws.mp_f, ws.mp2_f})
        if (m && cells_f > 0) HIP_TRY(hipMemsetAsync(m, 0, bf, s));
    return FMM_OK;
}

int ensure_workspace(fmm_tree *t, int p, int precision, bool backward, hipStream_t s)
{
    Workspace &ws = *t->wsp;
    const int split = split_level(t, precision);
    const int L = t->depth;
    if (ws.p != p || ws.precision != precision || ws.split != split) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        free_workspace(ws, s);
    }
    const int64_t n = t->n;
    const int64_t cells_d = level_base(std::min(split, L) + 1);
    const int64_t cells_f = level_base(L + 1) - cells_d;
    const size_t gam_bytes = precision == FMM_FP64 ? sizeof(double) : sizeof(float);
    int rc = FMM_OK;
    if (!ws.gam) {
        if ((rc = dev_alloc_async((char **)&ws.gam, n * gam_bytes, "circulations in tree order", s))) return rc;
        if ((rc = dev_alloc_async(&ws.stage, n, "velocities in tree order", s))) return rc;
        if ((rc = dev_alloc_async(&ws.near, n, "near field", s))) return rc;
        if (L >= 2) {
            if ((rc = dev_alloc_async(&ws.mp_d, cells_d * p + kCoefPad, "multipoles", s))) return rc;
            if ((rc = dev_alloc_async(&ws.lo_d, cells_d * p + kCoefPad, "locals", s))) return rc;
            if (cells_f > 0) {
                if ((rc = dev_alloc_async(&ws.mp_f, cells_f * p + kCoefPad, "multipoles", s))) return rc;
                if ((rc = dev_alloc_async(&ws.lo_f, cells_f * p + kCoefPad, "locals", s))) return rc;
            }
            // Empty cells are never written; the MFMA M2L reads them as zero rows.
            HIP_TRY(hipMemsetAsync(ws.mp_d, 0, (cells_d * p + kCoefPad) * sizeof(double2), s));
            HIP_TRY(hipMemsetAsync(ws.lo_d, 0, (cells_d * p + kCoefPad) * sizeof(double2), s));
            if (cells_f > 0) {
                HIP_TRY(hipMemsetAsync(ws.mp_f, 0, (cells_f * p + kCoefPad) * sizeof(float2), s));
                HIP_TRY(hipMemsetAsync(ws.lo_f, 0, (cells_f * p + kCoefPad) * sizeof(float2), s));
            }
        }
        ws.p = p;
        ws.precision = precision;
        ws.split = split;
        ws.owner = t->serial;  // zeroed just now
    }
    if (!ws.sums) {
        // the mutual slots, or the adjoint sums at 256-byte aligned offsets 0, A(32n), A(A(32n) + 8n)
        auto a256 = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t nn = (size_t)n;
        const size_t o_b = a256(32 * nn), o_src = a256(o_b + 8 * nn);
        const size_t bytes = std::max(9 * nn * (precision == FMM_FP64 ? 16 : 8), o_src + 32 * nn);
        if ((rc = dev_alloc_async((char **)&ws.sums, bytes, "near-field sums", s))) return rc;
        ws.sums_bytes = bytes;
        ws.slots = ws.sums;
        ws.bwd_near = (double4 *)ws.sums;
        ws.bwd_b = (double *)((char *)ws.sums + o_b);
        ws.bwd_src = (double4 *)((char *)ws.sums + o_src);
    }
    if (backward && !ws.adj) {
        if ((rc = dev_alloc_async(&ws.adj, n, "adjoint charges", s))) return rc;
        if (precision != FMM_FP64 && (rc = dev_alloc_async((float2 **)&ws.rec2, n, "adjoint charges (FP32)", s))) return rc;
        if (L >= 2) {
            // the far field of the charges q, computed beside that of the charges c
            if ((rc = dev_alloc_async(&ws.mp2_d, cells_d * p + kCoefPad, "adjoint multipoles", s))) return rc;
            if ((rc = dev_alloc_async(&ws.lo2_d, cells_d * p + kCoefPad, "adjoint locals", s))) return rc;
            HIP_TRY(hipMemsetAsync(ws.mp2_d, 0, (cells_d * p + kCoefPad) * sizeof(double2), s));
            if (cells_f > 0) {
                if ((rc = dev_alloc_async(&ws.mp2_f, cells_f * p + kCoefPad, "adjoint multipoles", s))) return rc;
                if ((rc = dev_alloc_async(&ws.lo2_f, cells_f * p + kCoefPad, "adjoint locals", s))) return rc;
                HIP_TRY(hipMemsetAsync(ws.mp2_f, 0, (cells_f * p + kCoefPad) * sizeof(float2), s));
            }
        }
    }
    if (ws.owner != t->serial) {
        int rc2 = clear_multipoles(t, s);
        if (rc2) return rc2;
        ws.owner = t->serial;
    }
    return FMM_OK;
}

// A handle whose arrays are there (see fmm_tree::released).
int check_tree(const fmm_tree *t)
{
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    if (t->released)
        return fail(FMM_ESTATE, "the tree's arrays were released by a failed rebuild: rebuild or destroy it");
    return FMM_OK;
}

int check_eval_args(fmm_tree *t, const double *gamma, double sigma, int p, int precision)
{
    if (int rc = check_tree(t)) return rc;
    if (!gamma) return fail(FMM_EINVAL, "gamma is NULL");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(FMM_EINVAL, "sigma must be finite and > 0");
    if (p < 1 || p > kMaxP) return fail(FMM_EINVAL, "p must be in [1, 32]");
    if (precision != FMM_FP64 && precision != FMM_MIXED) return fail(FMM_EINVAL, "unknown precision");
    return FMM_OK;
}


// FMM_OPT_VALIDATE: the circulations (and the cotangent of an adjoint call) are checked
// for NaN and infinities before any other work of the call; a bad value gives FMM_EINVAL
// naming the lowest particle index.  The check synchronises the main stream.
int validate_inputs(fmm_tree *t, const double *gamma, const double *dl_duv, hipStream_t s)
{
    if (!t->validate) return FMM_OK;
    int64_t bad = -1;
    HIP_TRY(find_nonfinite(gamma, t->n, 1, t->d_flag, s, bad));
    if (bad >= 0) return fail(FMM_EINVAL, "non-finite circulation (particle " + std::to_string(bad) + ")");
    if (dl_duv) {
        HIP_TRY(find_nonfinite(dl_duv, t->n, 2, t->d_flag, s, bad));
        if (bad >= 0) return fail(FMM_EINVAL, "non-finite dL/du (particle " + std::to_string(bad) + ")");
    }
    return FMM_OK;
}

FarArgs far_args(const fmm_tree *t, const Workspace &ws, int p, int precision, bool adjoint)
{
    FarArgs a{};
    a.t = t;
    a.p = p;
    a.split = ws.split;
    a.lc = effective_lc(t);
    a.mp_d = adjoint ? ws.mp2_d : ws.mp_d;
    a.lo_d = adjoint ? ws.lo2_d : ws.lo_d;
    a.mp_f = adjoint ? ws.mp2_f : ws.mp_f;
    a.lo_f = adjoint ? ws.lo2_f : ws.lo_f;
    a.pos = t->d_pos[precision == FMM_FP64];
    a.gam = ws.gam;
    a.rec_is_double = precision == FMM_FP64;
    a.charge_kind = adjoint ? 1 : 0;
    a.adj = adjoint ? ws.adj : nullptr;
    return a;
}

// Stage costs of the mixed form (p = 16) on one MI355X, in ms, fitted by the cost-model
// sweep of uniform particles (the complexity terms of section "Complexity Estimates"
// with the counts a launch pays for):
//   T_near = kNear0 + kNearPair pairs + kNearVisit 9 N_leaves,
//   T_far  = kFar0 + kFarCell C_fine + kFarCoarse C_coarse + kFarLevel (L - L_c).
constexpr double kNear0 = 0.070, kNearPair = 1.95e-10, kNearVisit = 1.74e-7;
constexpr double kFar0 = 0.268, kFarCell = 1.32e-6, kFarCoarse = 4.87e-5, kFarLevel = 0.00216;

// Predicted far-field / near-field time of the tree (the model above).
double far_near_ratio(const fmm_tree *t)
{
    const int lc = std::min(t->lc, t->depth);
    double fine = 0, coarse = 0;
    for (int l = 2; l <= t->depth; ++l) (l <= lc ? coarse : fine) += (double)t->list_len[l];
    const double near = kNear0 + kNearPair * (double)t->p2p_pairs + kNearVisit * 9.0 * (double)t->nonempty_leaves;
    const double far = kFar0 + kFarCell * fine + kFarCoarse * coarse + kFarLevel * (t->depth - lc);
    return far / near;
}

// Whether a call runs the far chain beside the near field (FMM_OPT_SCHEDULE 0), after it
// (1), or by the model (2, the default): both are throughput work on the same CUs.  In the
// mixed form, with the near field capped as below, overlapping measured faster than
// serialising up to a predicted far/near ratio of about 2.5 (uniform 2^18-2^22 particles,
// ratios 1.2-2.2: -7% to -15%; ratio 3.0: +2%), so only calls beyond it are serialised.
// FP64 calls overlap (the FP64 near field leaves issue slots that the far chain uses).
constexpr double kSerialRatio = 2.5;
bool call_overlaps(const fmm_tree *t, int precision)
{
    if (t->schedule != 2) return t->schedule == 0;
    if (precision == FMM_FP64 || t->depth < 2) return true;
    return far_near_ratio(t) <= kSerialRatio;
}

// In an overlapped call whose far chain is predicted clearly longer than the near field
// (r >= 1.4), the near field starts once P2M is done: beside the near field's workgroups
// P2M gets few slots, and the whole far chain waits for it (the 1024^2 lattice, depth 8,
// p = 12, coarse levels <= 5, r = 2.2: FP64 0.730 -> 0.705 ms, mixed 0.597 -> 0.573; uniform
// 2^20 particles at depths 7-9, r = 1.45-2.25: 0.23 ms less over the 12 points).  Nearer
// r = 1, P2M beside the near field costs less than the delay (uniform 2^22 particles at
// depth 10, r = 1.22: 3.65 against 3.88 ms with the wait), and far below it much less
// (2^24 patches, depth 10: 8.17 against 8.34 ms).
bool p2m_first(const fmm_tree *t) { return t->depth >= 2 && far_near_ratio(t) >= 1.4; }

// Near-field occupancy cap of a call (FMM_OPT_NEAR_OCCUPANCY), automatic from the tree:
//  - mixed, leaves of more than ~2500 near-field pairs per particle and a work list of at
//    least 64K entries (2^22-2^24 patch particles at depths 8-9): 3 wavefronts per SIMD, at
//    which the near field itself runs faster (2^24 patches at depth 9: 28.5 ms against 32.4
//    uncapped; 2^23: 8.1 against 9.1).  With fewer entries the cap idles the chip (uniform
//    2^22 particles at depth 6, 20K entries: 9.5 ms at cap 3 against 7.6 uncapped);
//  - mixed, by the predicted far/near ratio r (the far chain takes the slots the cap
//    leaves): r < 0.12 none, r < 0.9 six (2^24 patches at depth 10: 8.13 ms against 8.40
//    at five and 8.61 uncapped), 0.9 <= r <= 1.1 five, above four (uniform 2^20-2^22
//    particles at depths 7-10: four within 0.01 ms of the fastest cap);
//  - FP64 (at most 5 wavefronts per SIMD): 2 when the far field is the longer part (r >= 1:
//    the 1024^2 lattice, depth 8, p = 12, coarse levels <= 5 took 0.78 ms against 0.90
//    uncapped or serialised), else none.
int choose_occupancy(const fmm_tree *t, int precision, bool overlap)
{
    if (!overlap || t->depth < 2) return 0;
    if (t->near_occupancy >= 0) return t->near_occupancy;
    const double r = far_near_ratio(t);
    if (precision == FMM_FP64) return r >= 1.0 ? 2 : 0;
    const int64_t entries = use_mutual(t) ? t->nnear_work : t->nunits;
    if ((double)t->p2p_pairs >= 2500.0 * (double)t->n && entries >= 65536) return 3;
    if (r < 0.12) return 0;
    if (r < 0.9) return 6;
    if (r <= 1.1) return 5;
    return 4;
}

struct Timing {
    std::array<hipEvent_t, kNumEvents> ev{};
    bool on = false;
    int init(fmm_tree *t)
    {
        on = t->timing != 0;
        if (!on) return FMM_OK;
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        return FMM_OK;
    }
    void mark(int k, hipStream_t s)
    {
        if (on) hipEventRecord(ev[k], s);
    }
};

// The tree's leaf-unit coordinates in the precision of a call, made on its first use.
int ensure_positions(fmm_tree *t, int precision, hipStream_t s)
{
    const int d = precision == FMM_FP64;
    if (t->d_pos[d]) return FMM_OK;
    const int rc = dev_alloc_async((char **)&t->d_pos[d], (size_t)t->n * (d ? sizeof(double2) : sizeof(float2)),
                                   "leaf-unit coordinates", s);
    if (rc) return rc;
    launch_leaf_coords(t, d, t->d_pos[d], s);
    return FMM_OK;
}

// The per-call arrays of an evaluation carved from the static workspace (no allocation):
// circulations, staged velocities, near field, leaf-unit coordinates (in `sums`, when the
// tree has none yet), slots (mutual form), then the multipoles and locals of every level,
// each 256-byte aligned.  FMM_EINVAL when they do not fit, naming both sizes.
int static_ws(const fmm_tree *t, int p, int precision, Workspace &ws)
{
    char *base = nullptr;
    const int e = static_workspace(t->device, &base);
    if (e != 0) return hip_fail((hipError_t)e, "looking up the static workspace");
    const int split = split_level(t, precision);
    const int L = t->depth;
    const int64_t n = t->n;
    const int64_t cells_d = L >= 2 ? level_base(std::min(split, L) + 1) * p + kCoefPad : 0;
    const int64_t cells_f = L >= 2 && level_base(L + 1) > level_base(std::min(split, L) + 1)
                                ? (level_base(L + 1) - level_base(std::min(split, L) + 1)) * p + kCoefPad
                                : 0;
    const size_t real = precision == FMM_FP64 ? sizeof(double) : sizeof(float);
    const size_t slot = precision == FMM_FP64 ? sizeof(double2) : sizeof(float2);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return base + at;
    };
    ws = Workspace{};
    ws.p = p;
    ws.precision = precision;
    ws.split = split;
    ws.gam = take((size_t)n * real);
    ws.stage = (double2 *)take((size_t)n * sizeof(double2));
    ws.near = (double2 *)take((size_t)n * sizeof(double2));
    // the tree's leaf-unit coordinates when an allocating evaluation has not made them yet
    if (!t->d_pos[precision == FMM_FP64]) ws.sums = take((size_t)n * 2 * real);
    if (use_mutual(t)) ws.slots = take((size_t)9 * n * slot);
    ws.mp_d = (double2 *)take((size_t)cells_d * sizeof(double2));
    ws.lo_d = (double2 *)take((size_t)cells_d * sizeof(double2));
    ws.mp_f = (float2 *)take((size_t)cells_f * sizeof(float2));
    ws.lo_f = (float2 *)take((size_t)cells_f * sizeof(float2));
    if (off > kStaticWorkspaceBytes)
        return fail(FMM_EINVAL, "this evaluation needs " + std::to_string(off) + " bytes of device workspace, more "
                                "than the " + std::to_string(kStaticWorkspaceBytes) + " bytes of the static workspace");
    return FMM_OK;
}

// Stages 4-10.  noalloc: the per-call arrays in the static workspace (cleared where they
// must start at zero) and the tables already on the device; no allocation, no events.
int run_forward(fmm_tree *t, const double *gamma, double sigma, int p, int precision, void *main_stream,
                void *side_stream, double *uv, double *uv_near, double *uv_far, const double *base = nullptr,
                double h = 0.0, bool noalloc = false)
{
    int rc = check_eval_args(t, gamma, sigma, p, precision);
    if (rc) return rc;
    if (!uv && !(uv_near && uv_far)) return fail(FMM_EINVAL, "output is NULL");
    BusyGuard guard(t);
    if (!guard.ok) return fail(FMM_ESTATE, "tree handle in use by another thread");
    HIP_TRY(hipSetDevice(t->device));
    hipStream_t ms = (hipStream_t)main_stream;
    if ((rc = validate_inputs(t, gamma, nullptr, ms))) return rc;
    std::string err;
    Workspace local;
    if (noalloc) {
        if ((rc = shared_tables(t->device, p, &t->tabs, err, false)))
            return fail(FMM_ESTATE, err + " (an allocating evaluation with this p makes them)");
        if ((rc = static_ws(t, p, precision, local))) return rc;
        // multipoles of empty cells are read as zero rows by M2L
        if (local.mp_d) launch_zero(local.mp_d, (size_t)((char *)local.lo_d - (char *)local.mp_d), ms);
        if (local.mp_f) launch_zero(local.mp_f, (size_t)((char *)local.lo_f - (char *)local.mp_f), ms);
        if (local.sums) launch_leaf_coords(t, precision == FMM_FP64, local.sums, ms);
    } else {
        if ((rc = shared_tables(t->device, p, &t->tabs, err)))
            return fail(rc == -2 ? FMM_ENOMEM : FMM_EDEVICE, err);
        if ((rc = ensure_workspace(t, p, precision, false, ms)) || (rc = ensure_positions(t, precision, ms)))
            return rc;
    }
    Workspace &ws = noalloc ? local : *t->wsp;
    const void *pos = noalloc && local.sums ? local.sums : t->d_pos[precision == FMM_FP64];

    hipStream_t ss = side_stream ? (hipStream_t)side_stream : t->own_side;
    const bool overlap = call_overlaps(t, precision);
    if (!overlap) ss = ms;
    const double alpha = record_alpha(sigma, precision);
    const int is_double = precision == FMM_FP64;
    FarArgs a = far_args(t, ws, p, precision, false);
    a.pos = pos;
    a.gam = nullptr;  // P2M starts before the circulations are gathered: it reads the staging array
    t->occupancy_in_use = choose_occupancy(t, precision, overlap);
    // beside a capped near field the coarse kernel must fit in one wavefront per SIMD
    if (overlap && t->occupancy_in_use > 0) a.coarse_threads = 256;
    Timing tm;
    if (!noalloc && (rc = tm.init(t))) return rc;

    tm.mark(0, ms);
    launch_stage_in(t, gamma, ms);
    if (overlap) {  // the far chain needs only the staged circulations: it starts beside pack
        HIP_TRY(hipEventRecord(t->ev_fork, ms));
        HIP_TRY(hipStreamWaitEvent(ss, t->ev_fork, 0));
    }
    launch_pack(t, is_double, ws.gam, ms);
    tm.mark(1, ms);
    tm.mark(2, ss);
    if (overlap && p2m_first(t)) {
        // the far chain is the longer part: P2M, its first and widest kernel, runs beside
        // pack alone instead of being starved by the near field's workgroups
        launch_p2m(a, ss);
        HIP_TRY(hipEventRecord(t->ev_fork, ss));
        launch_far_chain(a, ss, false);
        HIP_TRY(hipStreamWaitEvent(ms, t->ev_fork, 0));
    } else {
        launch_far_chain(a, ss);
    }
    tm.mark(3, ss);
    if (overlap) HIP_TRY(hipEventRecord(t->ev_join, ss));
    void *slots = use_mutual(t) ? ws.slots : nullptr;
    tm.mark(4, ms);
    launch_p2p_forward(t, pos, ws.gam, is_double, alpha, ws.near, slots, ms);
    tm.mark(5, ms);
    if (overlap) HIP_TRY(hipStreamWaitEvent(ms, t->ev_join, 0));
    tm.mark(6, ms);
    launch_finalize(t, a, ws.near, slots, is_double, alpha, uv, uv_near, uv_far, ws.stage, base, h, ms);
    tm.mark(7, ms);
    HIP_TRY(hipGetLastError());
    if (tm.on) t->pending_timing.push_back(tm.ev);
    return FMM_OK;
}

}  // namespace

namespace {

// Argument checks shared by both builds; a new tree with device facts filled in.
int new_tree(const double *xy, int64_t n, int depth, const double *root_box, fmm_tree **out, fmm_tree *&t)
{
    g_last_error.clear();
    t = nullptr;
    if (!out) return fail(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!xy) return fail(FMM_EINVAL, "xy is NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FMM_EINVAL, "n must be in [1, 2^31)");
    if (depth < 1 || depth > kMaxDepth) return fail(FMM_EINVAL, "depth must be in [1, 12]");
    if (root_box && (!std::isfinite(root_box[0]) || !std::isfinite(root_box[1]) || !(root_box[2] > 0.0) ||
                     !std::isfinite(root_box[2])))
        return fail(FMM_EINVAL, "root_box must be finite with side > 0");
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return hip_fail(de, "hipGetDevice");
    retain_pool(dev);
    t = new fmm_tree();
    static std::atomic<uint64_t> next_serial{1};
    t->serial = next_serial.fetch_add(1);
    t->device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    t->num_cus = cus;
    t->n = n;
    t->depth = depth;
    return FMM_OK;
}

// Common end of both builds: the tree's side stream and events, the near-field plan
// (device) and the near-field work counter.
int finish_tree(fmm_tree *t, hipStream_t s)
{
    hipError_t e = hipStreamCreateWithFlags(&t->own_side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "creating stream/events");
    std::string err;
    const int rc = build_near_plan_device(t, s, err);
    if (rc) return fail(rc, err);
    return dev_alloc(&t->d_flag, 1, "input check flag");
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Stages 1-3: tree construction, binning, work lists -- on the device (default) or on
// the host (reference build; both give identical trees)
// ---------------------------------------------------------------------------------------
namespace {

// The device build; the options of `opts` (a tree being replaced) are taken over before
// the near-field plan is made, since that plan depends on them.  arena: device memory
// idle during the build that its temporaries may use; after_checks: see build_tree_device.
int build_device(const double *xy, int64_t n, int depth, const double *root_box, void *stream, const fmm_tree *opts,
                 fmm_tree **out, BuildArena *arena = nullptr, const std::function<void()> &after_checks = {})
{
    fmm_tree *t = nullptr;
    int rc = new_tree(xy, n, depth, root_box, out, t);
    if (rc) return rc;
    if (opts) {
        t->lc = opts->lc;
        t->schedule = opts->schedule;
        t->near_mutual = opts->near_mutual;
        t->dense_leaf = opts->dense_leaf;
        t->near_occupancy = opts->near_occupancy;
        t->timing = opts->timing;
        t->validate = opts->validate;
    }
    hipStream_t s = (hipStream_t)stream;
    std::string err;
    int64_t bad = -1;
    {
        BuildArenaScope scope(arena);
        rc = build_tree_device(t, xy, root_box, s, err, bad, after_checks);
        if (!rc) rc = finish_tree(t, s);
        else {
            if (bad >= 0) err += " (particle " + std::to_string(bad) + ")";
            fail(rc, err);
        }
    }
    if (rc) {
        free_tree(t);
        return rc;
    }
    if (!arena) trim_pool(t->device);  // the temporaries came from the pool
    *out = t;
    return FMM_OK;
}

}  // namespace

extern "C" int fmm_build_tree(const double *xy, int64_t n, int depth, const double *root_box, void *stream,
                              fmm_tree **out)
{
    return build_device(xy, n, depth, root_box, stream, nullptr, out);
}

extern "C" int fmm_rebuild_tree(fmm_tree *prev, const double *xy, int64_t n, const double *root_box, void *stream,
                                fmm_tree **out)
{
    g_last_error.clear();
    if (out) *out = nullptr;
    if (!prev) return fail(FMM_ESTATE, "null tree handle");
    if (n != prev->n) return fail(FMM_EINVAL, "n must equal the particle count of the tree being rebuilt");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != prev->device) return fail(FMM_EINVAL, "the current device is not the tree's");
    BusyGuard guard(prev);
    if (!guard.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    // Earlier calls on prev, or on a tree sharing its workspace, may still use the
    // workspace and prev's arrays.
    HIP_TRY(hipDeviceSynchronize());
    // One tree's arrays at a time: the build's temporaries go to the workspace's per-call
    // region (idle between calls), and prev's arrays are released once the positions have
    // passed their checks, before the new ones are allocated.
    BuildArena arena;
    arena.base = (char *)prev->wsp->sums;
    arena.cap = prev->wsp->sums ? prev->wsp->sums_bytes : 0;
    hipStream_t s = (hipStream_t)stream;
    auto release_prev = [prev, s]() {
        release_tree_arrays(prev, s);
        prev->released = true;
    };
    fmm_tree *t = nullptr;
    int rc = build_device(xy, n, prev->depth, root_box, stream, prev, &t, &arena, release_prev);
    if (rc) return rc;
    hipError_t e = hipDeviceSynchronize();  // the build used the workspace
    if (e != hipSuccess) {
        free_tree(t);
        return hip_fail(e, "hipDeviceSynchronize");
    }
    std::swap(t->wsp, prev->wsp);
    t->wsp->owner = kForeignOwner;  // cleared by the next call
    guard.release();
    free_tree(prev);
    *out = t;
    return FMM_OK;
}

extern "C" int fmm_build_tree_host(const double *xy, int64_t n, int depth, const double *root_box, void *stream,
                                   fmm_tree **out)
{
    fmm_tree *t = nullptr;
    int rc0 = new_tree(xy, n, depth, root_box, out, t);
    if (rc0) return rc0;
    try {
        hipStream_t s = (hipStream_t)stream;
        std::vector<double> h(2 * (size_t)n);
        hipError_t e = hipMemcpyAsync(h.data(), xy, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            free_tree(t);
            return hip_fail(e, "copying positions to the host");
        }
        UniformHostTree ht;
        int64_t bad = -1;
        std::string err;
        int rc = build_host_tree(h.data(), n, depth, root_box, ht, bad, err);
        if (rc) {
            free_tree(t);
            return fail(rc, err);
        }
        t->x0 = ht.x0;
        t->y0 = ht.y0;
        t->side = ht.side;
        t->stage_shift = ht.stage_shift;
        t->list_off = ht.list_off;
        t->list_len = ht.list_len;
        t->class_off = ht.class_off;
        t->p2p_pairs = ht.p2p_pairs;
        t->m2l_pairs = ht.m2l_pairs;
        t->nonempty_leaves = ht.nonempty_leaves;
        t->max_leaf = ht.max_leaf;
        t->nunits = (int64_t)ht.units.size();
        if (!rc) rc = upload(&t->d_perm, ht.perm, "permutation");
        if (!rc) rc = upload(&t->d_gpos1, ht.gpos1, "staging slots");
        if (!rc) rc = upload(&t->d_gpos2, ht.gpos2, "staging slots");
        if (!rc) rc = dev_alloc(&t->d_st1, n, "staging array");
        if (!rc) rc = upload(&t->d_leaf_of, ht.leaf_of, "leaf ids");
        if (!rc) rc = upload_as(&t->d_xy, ht.xy, "sorted positions");
        if (!rc) rc = upload(&t->d_leaf_start, ht.leaf_start, "leaf offsets");
        if (!rc) rc = upload(&t->d_counts, ht.counts, "cell counts");
        if (!rc) rc = upload(&t->d_lists, ht.lists, "cell lists");
        if (!rc) rc = upload_as(&t->d_units, ht.units, "P2P work units");
        if (!rc) rc = upload(&t->d_tile_start, ht.tile_start, "tile offsets");
        if (!rc) rc = upload_as(&t->d_tile_box, ht.tile_box, "tile boxes");
        if (!rc) rc = finish_tree(t, s);
        if (rc) {
            free_tree(t);
            return rc;
        }
    } catch (const std::bad_alloc &) {
        if (t) free_tree(t);
        return fail(FMM_ENOMEM, "host allocation failed while building the tree");
    }
    *out = t;
    return FMM_OK;
}

extern "C" int fmm_share_workspace(fmm_tree *t, fmm_tree *from)
{
    g_last_error.clear();
    if (!t || !from) return fail(FMM_ESTATE, "null tree handle");
    if (t == from) return FMM_OK;
    if (t->n != from->n || t->depth != from->depth || t->device != from->device)
        return fail(FMM_EINVAL, "trees sharing a workspace need the same n, depth and device");
    BusyGuard g1(t);
    if (!g1.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    BusyGuard g2(from);
    if (!g2.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    if (t->wsp == from->wsp) return FMM_OK;
    HIP_TRY(hipSetDevice(t->device));
    HIP_TRY(hipDeviceSynchronize());  // t's earlier calls may still use its workspace
    if (t->wsp.use_count() == 1) free_workspace(*t->wsp, t->own_side);
    t->wsp = from->wsp;
    return FMM_OK;
}

extern "C" int fmm_tree_info(const fmm_tree *t, int64_t *n, int *depth, double *root_box, int64_t *p2p_pairs,
                             int64_t *m2l_pairs, int64_t *nonempty_leaves, int64_t *max_leaf)
{
    if (int rc = check_tree(t)) return rc;
    if (n) *n = t->n;
    if (depth) *depth = t->depth;
    if (root_box) {
        root_box[0] = t->x0;
        root_box[1] = t->y0;
        root_box[2] = t->side;
    }
    if (p2p_pairs) *p2p_pairs = t->p2p_pairs;
    if (m2l_pairs) *m2l_pairs = t->m2l_pairs;
    if (nonempty_leaves) *nonempty_leaves = t->nonempty_leaves;
    if (max_leaf) *max_leaf = t->max_leaf;
    return FMM_OK;
}

namespace fmm {
void launch_widen_perm(const fmm_tree *t, int64_t *perm, int32_t *leaf, hipStream_t s);
}

extern "C" int fmm_tree_levels(const fmm_tree *t, int64_t *nonempty, int max_levels)
{
    if (int rc = check_tree(t)) return rc;
    if (!nonempty || max_levels < 1) return fail(FMM_EINVAL, "nonempty is NULL or max_levels < 1");
    std::vector<int> h((size_t)level_base(std::min(t->depth, 1) + 1));
    for (int l = 0; l < max_levels; ++l) nonempty[l] = 0;
    // levels 0 and 1 from the cell counts (they hold no expansions and have no list)
    const int top = std::min(t->depth, 1);
    if (hipMemcpy(h.data(), t->d_counts, h.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(FMM_EDEVICE, "reading cell counts");
    for (int l = 0; l <= top && l < max_levels; ++l)
        for (int64_t c = level_base(l); c < level_base(l + 1); ++c) nonempty[l] += h[c] > 0;
    for (int l = 2; l <= t->depth && l < max_levels; ++l) nonempty[l] = t->list_len[l];
    return FMM_OK;
}

extern "C" int fmm_tree_permutation(const fmm_tree *t, int64_t *perm, int32_t *leaf, void *stream)
{
    if (int rc = check_tree(t)) return rc;
    if (!perm) return fail(FMM_EINVAL, "perm is NULL");
    HIP_TRY(hipSetDevice(t->device));
    launch_widen_perm(t, perm, leaf, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FMM_OK;
}

extern "C" int fmm_velocity(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                            void *main_stream, void *side_stream, double *uv)
{
    g_last_error.clear();
    if (!uv) return fail(FMM_EINVAL, "uv is NULL");
    return run_forward(t, gamma, sigma, p, precision, main_stream, side_stream, uv, nullptr, nullptr);
}

extern "C" int fmm_velocity_noalloc(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                                    void *main_stream, void *side_stream, double *uv)
{
    g_last_error.clear();
    if (!uv) return fail(FMM_EINVAL, "uv is NULL");
    return run_forward(t, gamma, sigma, p, precision, main_stream, side_stream, uv, nullptr, nullptr, nullptr, 0.0,
                       true);
}

extern "C" int fmm_velocity_parts(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                                  void *main_stream, void *side_stream, double *uv_near, double *uv_far)
{
    g_last_error.clear();
    if (!uv_near || !uv_far) return fail(FMM_EINVAL, "uv_near / uv_far is NULL");
    return run_forward(t, gamma, sigma, p, precision, main_stream, side_stream, nullptr, uv_near, uv_far);
}

namespace {

// The adjoint of stages 4-10 for the cotangent scale * cot (user order), written as `out`
// says (see AdjointOut).
int run_backward(fmm_tree *t, const double *gamma, double sigma, int p, int precision, const double *cot,
                 double scale, void *main_stream, void *side_stream, const AdjointOut &out)
{
    int rc = check_eval_args(t, gamma, sigma, p, precision);
    if (rc) return rc;
    if (!cot) return fail(FMM_EINVAL, "dl_duv is NULL");
    if (!std::isfinite(scale)) return fail(FMM_EINVAL, "the cotangent scale must be finite");
    if (!out.dg && !out.dxe && !out.dxs && !out.dxy) return FMM_OK;
    BusyGuard guard(t);
    if (!guard.ok) return fail(FMM_ESTATE, "tree handle in use by another thread");
    HIP_TRY(hipSetDevice(t->device));
    if ((rc = validate_inputs(t, gamma, cot, (hipStream_t)main_stream))) return rc;
    std::string err;
    if ((rc = shared_tables(t->device, p, &t->tabs, err))) return fail(rc == -2 ? FMM_ENOMEM : FMM_EDEVICE, err);
    if ((rc = ensure_workspace(t, p, precision, true, (hipStream_t)main_stream)) ||
        (rc = ensure_positions(t, precision, (hipStream_t)main_stream)))
        return rc;
    Workspace &ws = *t->wsp;
    const bool need_src = out.dxs || out.dxy;
    const void *pos = t->d_pos[precision == FMM_FP64];

    hipStream_t ms = (hipStream_t)main_stream;
    hipStream_t ss = side_stream ? (hipStream_t)side_stream : t->own_side;
    const bool overlap = call_overlaps(t, precision);
    if (!overlap) ss = ms;
    t->occupancy_in_use = 0;  // the adjoint's near field is not capped
    const double alpha = record_alpha(sigma, precision);
    const int is_double = precision == FMM_FP64;
    FarArgs fc = far_args(t, ws, p, precision, false);
    fc.gam = nullptr;  // P2M of the charges c reads the staging array: it starts before pack
    const FarArgs fq = far_args(t, ws, p, precision, true);
    Timing tm;
    if ((rc = tm.init(t))) return rc;

    // The two far chains (the charges c: the derivative of their local expansion; the
    // charges q: the transpose pass A^T q = -A q) are independent: with the two streams the
    // chain of c runs on the side stream from the staged circulations on, beside the packing
    // and then the chain of q on the main stream, and the near field follows both.  (Beside
    // the adjoint's near field, which holds every wavefront slot, they would wait for it to
    // drain.)
    tm.mark(0, ms);
    launch_stage_in(t, gamma, ms);
    if (overlap) {
        HIP_TRY(hipEventRecord(t->ev_fork, ms));
        HIP_TRY(hipStreamWaitEvent(ss, t->ev_fork, 0));
    }
    tm.mark(2, ss);
    launch_far_chain(fc, ss);
    tm.mark(3, ss);
    if (overlap) HIP_TRY(hipEventRecord(t->ev_join, ss));
    launch_pack(t, is_double, ws.gam, ms);
    launch_pack_adjoint(t, cot, scale, ws.adj, ws.rec2, is_double, ws.stage, ms);  // stage: free until finalize
    tm.mark(1, ms);
    launch_far_chain(fq, ms);
    if (overlap) HIP_TRY(hipStreamWaitEvent(ms, t->ev_join, 0));
    tm.mark(4, ms);
    launch_p2p_backward(t, pos, ws.gam, is_double ? (const void *)ws.adj : ws.rec2, is_double, alpha, ws.bwd_near,
                        ws.bwd_b, need_src ? ws.bwd_src : nullptr, ms);
    tm.mark(5, ms);
    tm.mark(6, ms);
    // once the outputs fill the last-level cache they reach user order through staging slots, kept in
    // arrays this call no longer reads: dL/dGamma in the FP32 charges (mixed) or the FP64
    // circulations, the evaluation part in the forward's staged velocities, the source part
    // in the forward's near-field array
    const int64_t out_bytes = (out.dg ? 8 : 0) + ((out.dxe || out.dxy) ? 16 : 0) + ((out.dxs || out.dxy) ? 16 : 0);
    const bool staged = outputs_windowed(t->n, out_bytes);
    double *st_g = !staged ? nullptr : is_double ? (double *)ws.gam : (double *)ws.rec2;
    double *st_x = staged ? (double *)ws.stage : nullptr;
    double *st_s = staged ? (double *)ws.near : nullptr;
    launch_finalize_backward(t, fc, fq, ws.bwd_near, ws.bwd_b, ws.adj, ws.bwd_src, is_double, alpha, out, st_g, st_x,
                             st_s, ms);
    tm.mark(7, ms);
    HIP_TRY(hipGetLastError());
    if (tm.on) t->pending_timing.push_back(tm.ev);
    return FMM_OK;
}

}  // namespace

extern "C" int fmm_velocity_backward(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                                     const double *dl_duv, void *main_stream, void *side_stream, double *dl_dgamma,
                                     double *dl_dxeval, double *dl_dxsrc, double *dl_dxy)
{
    g_last_error.clear();
    AdjointOut out;
    out.dg = dl_dgamma;
    out.dxe = dl_dxeval;
    out.dxs = dl_dxsrc;
    out.dxy = dl_dxy;
    return run_backward(t, gamma, sigma, p, precision, dl_duv, 1.0, main_stream, side_stream, out);
}

extern "C" int fmm_transport_step(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                                  void *main_stream, void *side_stream, const double *x_base, double h, double *x_out)
{
    g_last_error.clear();
    if (!x_base || !x_out) return fail(FMM_EINVAL, "x_base / x_out is NULL");
    if (!std::isfinite(h)) return fail(FMM_EINVAL, "h must be finite");
    return run_forward(t, gamma, sigma, p, precision, main_stream, side_stream, x_out, nullptr, nullptr, x_base, h);
}

extern "C" int fmm_transport_vjp(fmm_tree *t, const double *gamma, double sigma, int p, int precision,
                                 const double *lam, double h, int flags, void *main_stream, void *side_stream,
                                 double *dl_dgamma, double *dl_dx)
{
    g_last_error.clear();
    if (flags & ~(FMM_ACC_GAMMA | FMM_ACC_X | FMM_IDENTITY)) return fail(FMM_EINVAL, "unknown flag");
    if (!lam) return fail(FMM_EINVAL, "lam is NULL");
    AdjointOut out;
    out.dg = dl_dgamma;
    out.dxy = dl_dx;
    out.lam = (flags & FMM_IDENTITY) ? lam : nullptr;
    out.acc_g = (flags & FMM_ACC_GAMMA) != 0;
    out.acc_xy = (flags & FMM_ACC_X) != 0;
    return run_backward(t, gamma, sigma, p, precision, lam, h, main_stream, side_stream, out);
}

extern "C" int fmm_set_option(fmm_tree *t, int key, int64_t value)
{
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    switch (key) {
    case FMM_OPT_SCHEDULE:
        if (value < 0 || value > 2) return fail(FMM_EINVAL, "schedule must be 0, 1 or 2");
        t->schedule = (int)value;
        return FMM_OK;
    case FMM_OPT_COARSE_LEVEL:
        if (value < 1 || value > t->depth) return fail(FMM_EINVAL, "coarse level must be in [1, depth]");
        t->lc = (int)value;
        return FMM_OK;
    case FMM_OPT_NEAR_MUTUAL:
    case FMM_OPT_DENSE_LEAF: {
        if (key == FMM_OPT_NEAR_MUTUAL && value != 0 && value != 1)
            return fail(FMM_EINVAL, "near mutual must be 0 or 1");
        if (key == FMM_OPT_DENSE_LEAF && (value < 1 || value > (int64_t(1) << 30)))
            return fail(FMM_EINVAL, "dense leaf must be in [1, 2^30]");
        if (int rc = check_tree(t)) return rc;  // the plan is made from the tree's arrays
        HIP_TRY(hipSetDevice(t->device));
        HIP_TRY(hipDeviceSynchronize());  // the plan's arrays may be in use
        if (key == FMM_OPT_NEAR_MUTUAL) t->near_mutual = (int)value;
        else t->dense_leaf = (int)value;
        std::string err;
        const int rc = build_near_plan_device(t, t->own_side, err);
        return rc ? fail(rc, err) : FMM_OK;
    }
    case FMM_OPT_NEAR_OCCUPANCY:
        if (value < -1 || value > 8) return fail(FMM_EINVAL, "near occupancy must be in [-1, 8]");
        t->near_occupancy = (int)value;
        return FMM_OK;
    case FMM_OPT_TIMING:
        if (value != 0 && value != 1) return fail(FMM_EINVAL, "timing must be 0 or 1");
        t->timing = (int)value;
        return FMM_OK;
    case FMM_OPT_VALIDATE:
        if (value != 0 && value != 1) return fail(FMM_EINVAL, "validate must be 0 or 1");
        t->validate = (int)value;
        return FMM_OK;
    case 4:
    case 5:
        return fail(FMM_EINVAL, "option withdrawn (persistent near-field grid, far-field grid cap)");
    default:
        return fail(FMM_EINVAL, "unknown option");
    }
}

extern "C" int fmm_near_plan_info(const fmm_tree *t, int64_t *mutual_items, int64_t *mutual_pairs,
                                  int64_t *target_units)
{
    if (int rc = check_tree(t)) return rc;
    const bool m = use_mutual(t);
    if (mutual_items) *mutual_items = m ? t->nmut : 0;
    if (mutual_pairs) *mutual_pairs = m ? t->mutual_pairs : 0;
    if (target_units) *target_units = m ? t->nunits_tc : t->nunits;
    return FMM_OK;
}

extern "C" int fmm_get_timings(fmm_tree *t, double *ms, int64_t *calls)
{
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    if (!ms) return fail(FMM_EINVAL, "ms is NULL");
    HIP_TRY(hipSetDevice(t->device));
    double acc[FMM_T_COUNT] = {};
    int64_t ncalls = 0;
    for (auto &ev : t->pending_timing) {
        HIP_TRY(hipEventSynchronize(ev[7]));
        HIP_TRY(hipEventSynchronize(ev[3]));
        float f;
        HIP_TRY(hipEventElapsedTime(&f, ev[0], ev[1]));
        acc[FMM_T_PACK] += f;
        HIP_TRY(hipEventElapsedTime(&f, ev[2], ev[3]));
        acc[FMM_T_FAR] += f;
        HIP_TRY(hipEventElapsedTime(&f, ev[4], ev[5]));
        acc[FMM_T_P2P] += f;
        HIP_TRY(hipEventElapsedTime(&f, ev[6], ev[7]));
        acc[FMM_T_FINAL] += f;
        HIP_TRY(hipEventElapsedTime(&f, ev[0], ev[7]));
        acc[FMM_T_TOTAL] += f;
        ++ncalls;
        for (auto e : ev) hipEventDestroy(e);
    }
    t->pending_timing.clear();
    for (int k = 0; k < FMM_T_COUNT; ++k) ms[k] = acc[k];
    if (calls) *calls = ncalls;
    return FMM_OK;
}

extern "C" int fmm_get_timeline(fmm_tree *t, double *ms, int count)
{
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    if (!ms || count < 1) return fail(FMM_EINVAL, "ms is NULL or count < 1");
    if (t->pending_timing.empty()) return fail(FMM_ESTATE, "no call recorded with FMM_OPT_TIMING since the last read");
    HIP_TRY(hipSetDevice(t->device));
    auto &ev = t->pending_timing.back();
    HIP_TRY(hipEventSynchronize(ev[7]));
    HIP_TRY(hipEventSynchronize(ev[3]));
    for (int k = 0; k < count; ++k) {
        ms[k] = 0.0;
        if (k >= kNumEvents) continue;
        float f = 0.0f;
        HIP_TRY(hipEventElapsedTime(&f, ev[0], ev[k]));
        ms[k] = f;
    }
    return FMM_OK;
}

extern "C" void fmm_destroy_tree(fmm_tree *t)
{
    if (!t) return;
    hipSetDevice(t->device);
    hipDeviceSynchronize();
    const int dev = t->device;
    free_tree(t);
    trim_pool(dev);
}

int fmm::fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

void fmm::clear_last_error() { g_last_error.clear(); }

void fmm::retain_pool(int device)
{
    static std::atomic<uint64_t> done{0};
    if (device < 0 || device >= 64 || ((done.load() >> device) & 1)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t threshold = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    (void)hipGetLastError();
    done.fetch_or(uint64_t(1) << device);
}

void fmm::trim_pool(int device)
{
    hipMemPool_t pool;
    if (hipDeviceSynchronize() == hipSuccess && hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess)
        (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
}

double fmm::record_alpha(double sigma, int precision)
{
    const double a = 1.0 / (sigma * std::sqrt(2.0));
    return precision == FMM_FP64 ? a : a * std::sqrt(1.4426950408889634073599246810019);
}

extern "C" const char *fmm_last_error(void) { return g_last_error.c_str(); }
