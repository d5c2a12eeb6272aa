// C ABI of the adaptive-tree variant (include/fmm2d_adaptive.h): the tree, its lists
// and work units built on the device (adaptive_build.hip) or, as the reference, on the
// host (here); the evaluation enqueued on the device (adaptive.hip).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fmm2d_adaptive.h"
#include "adaptive_internal.h"
#include "api_common.h"
#include "fmm_internal.h"

using namespace fmm;

namespace {

void free_ws(AtreeWs &w)
{
    hipFree(w.gam);
    hipFree(w.stage);
    hipFree(w.gamma);
    hipFree(w.near);
    hipFree(w.slots);
    hipFree(w.mp);
    hipFree(w.lo);
    hipFree(w.binom);
    hipFree(w.binom16);
    hipFree(w.binom32);
    hipFree(w.mp2);
    hipFree(w.lo2);
    hipFree(w.adj);
    hipFree(w.qt);
    hipFree(w.pa);
    hipFree(w.pb);
    hipFree(w.psrc);
    w = AtreeWs{};
}

void free_atree(fmm_atree *t)
{
    if (!t) return;
    AtreeDev &d = t->d;
    // the device build's arrays and the adjoint units come from the stream-ordered pool
    if (t->pooled || d.bwd_units || d.vslot) hipDeviceSynchronize();
    for (void *p : {(void *)d.bwd_units, (void *)d.m2l_targets, (void *)d.vslot})
        if (p) hipFreeAsync(p, nullptr);
    for (void *p : {(void *)d.perm, (void *)d.gpos1, (void *)d.gpos2, (void *)d.st1, (void *)d.leaf_of, (void *)d.xy, (void *)d.cell, (void *)d.range,
                    (void *)d.parent, (void *)d.child, (void *)d.u_off, (void *)d.u_idx, (void *)d.v_off,
                    (void *)d.v_idx, (void *)d.w_off, (void *)d.w_idx, (void *)d.x_off, (void *)d.x_idx,
                    (void *)d.p2m_cells, (void *)d.inner, (void *)d.tile_start, (void *)d.tile_box,
                    (void *)d.work, (void *)d.leaf_start, (void *)d.leaf_tile, (void *)d.tile_box_leaf,
                    (void *)d.mask}) {
        if (!p) continue;
        if (t->pooled)
            hipFreeAsync(p, nullptr);
        else
            hipFree(p);
    }
    if (t->wsp.use_count() == 1) free_ws(*t->wsp);
    for (void *q : t->d_pos) hipFree(q);
    if (t->d_flag) hipFree(t->d_flag);
    if (t->ev_fork) hipEventDestroy(t->ev_fork);
    if (t->ev_join) hipEventDestroy(t->ev_join);
    if (t->own_side) hipStreamDestroy(t->own_side);
    delete t;
}

struct HostCell {
    int level;
    uint64_t code;   // Morton index on its level
    int ix, iy;
    int first, count;
    int parent;
    int child[4];
    bool leaf;
};

// The tree and its lists, from the particles' Morton keys at depth L sorted ascending.
struct HostTree {
    int L = 0, smax = 1;
    std::vector<HostCell> cells;
    std::unordered_map<uint64_t, int> at;  // (level, ix, iy) -> cell
    std::vector<std::vector<int>> U, V, W, X;

    static uint64_t pos_key(int level, int ix, int iy)
    {
        return ((uint64_t)level << 40) | ((uint64_t)(uint32_t)ix << 20) | (uint64_t)(uint32_t)iy;
    }
    int find(int level, int ix, int iy) const
    {
        if (ix < 0 || iy < 0 || ix >= (1 << level) || iy >= (1 << level)) return -1;
        auto it = at.find(pos_key(level, ix, iy));
        return it == at.end() ? -1 : it->second;
    }
    // closed squares intersect, compared in units of the depth-L cell
    bool touch(int a, int b) const
    {
        const HostCell &A = cells[a], &B = cells[b];
        const int64_t sa = int64_t(1) << (L - A.level), sb = int64_t(1) << (L - B.level);
        return A.ix * sa <= (B.ix + 1) * sb && B.ix * sb <= (A.ix + 1) * sa && A.iy * sa <= (B.iy + 1) * sb &&
               B.iy * sb <= (A.iy + 1) * sa;
    }
    // same-level cells adjacent to cell k
    void neighbours(int k, std::vector<int> &out) const
    {
        out.clear();
        const HostCell &c = cells[k];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                const int j = find(c.level, c.ix + dx, c.iy + dy);
                if (j >= 0) out.push_back(j);
            }
    }

    void build(const std::vector<uint32_t> &keys, int n)
    {
        cells.clear();
        cells.push_back({0, 0, 0, 0, 0, n, -1, {-1, -1, -1, -1}, true});
        for (size_t k = 0; k < cells.size(); ++k) {
            const HostCell c = cells[k];
            if (c.count <= smax || c.level >= L) continue;
            cells[k].leaf = false;
            const int shift = 2 * (L - c.level - 1);
            int lo = c.first;
            const int end = c.first + c.count;
            for (int q = 0; q < 4; ++q) {
                const uint64_t next = c.code * 4 + q + 1;  // first key code of the next quadrant
                const int hi = (int)(std::partition_point(keys.begin() + lo, keys.begin() + end,
                                                          [&](uint32_t key) { return ((uint64_t)key >> shift) < next; }) -
                                     keys.begin());
                if (hi > lo) {
                    HostCell ch{c.level + 1, c.code * 4 + q, 2 * c.ix + (q & 1), 2 * c.iy + (q >> 1), lo, hi - lo,
                                (int)k, {-1, -1, -1, -1}, true};
                    cells[k].child[q] = (int)cells.size();
                    cells.push_back(ch);
                }
                lo = hi;
            }
        }
        at.reserve(cells.size() * 2);
        for (size_t k = 0; k < cells.size(); ++k) at[pos_key(cells[k].level, cells[k].ix, cells[k].iy)] = (int)k;
    }

    void lists()
    {
        const int K = (int)cells.size();
        U.assign(K, {});
        V.assign(K, {});
        W.assign(K, {});
        X.assign(K, {});
        std::vector<int> nb, nbp, stack;
        for (int k = 0; k < K; ++k) {
            const HostCell &c = cells[k];
            neighbours(k, nb);
            if (c.parent >= 0) {  // V: children of the parent's neighbours, not touching
                neighbours(c.parent, nbp);
                for (int P : nbp)
                    for (int ch : cells[P].child)
                        if (ch >= 0 && !touch(ch, k)) V[k].push_back(ch);
            }
            if (!c.leaf) continue;
            U[k].push_back(k);
            for (int C : nb) {  // leaves at or below the neighbours that touch; W
                stack.assign(1, C);
                while (!stack.empty()) {
                    const int d = stack.back();
                    stack.pop_back();
                    if (!touch(d, k)) {
                        W[k].push_back(d);  // its parent touches (C itself always does)
                        continue;
                    }
                    if (cells[d].leaf) {
                        U[k].push_back(d);
                        continue;
                    }
                    for (int q = 3; q >= 0; --q)
                        if (cells[d].child[q] >= 0) stack.push_back(cells[d].child[q]);
                }
            }
            for (int a = c.parent; a >= 0; a = cells[a].parent) {  // coarser leaves touching k
                neighbours(a, nbp);
                for (int C : nbp)
                    if (cells[C].leaf && touch(C, k)) U[k].push_back(C);
            }
        }
        for (int a = 0; a < K; ++a)
            for (int d : W[a]) X[d].push_back(a);
    }
};

template <typename T>
void flatten(const std::vector<std::vector<T>> &lists, std::vector<int> &off, std::vector<T> &idx)
{
    off.assign(lists.size() + 1, 0);
    for (size_t k = 0; k < lists.size(); ++k) off[k + 1] = off[k] + (int)lists[k].size();
    idx.clear();
    idx.reserve(off.back());
    for (const auto &l : lists) idx.insert(idx.end(), l.begin(), l.end());
}

struct Busy {
    fmm_atree *t;
    bool ok;
    explicit Busy(fmm_atree *tree) : t(tree), ok(tree->busy.exchange(1) == 0) {}
    ~Busy() { release(); }
    void release()
    {
        if (ok) t->busy.store(0);
        ok = false;
    }
};

// The tree's offsets z - c_leaf in the near field's precision, made on first use.
int ensure_coords(fmm_atree *t, int precision, hipStream_t s)
{
    const int k = precision == FMM_FP64;
    if (t->d_pos[k]) return FMM_OK;
    int rc = dev_alloc((char **)&t->d_pos[k], (size_t)t->n * (k ? sizeof(double2) : sizeof(float2)),
                       "leaf offsets of the particles");
    if (rc) return rc;
    launch_atree_coords(t, k, t->d_pos[k], s);
    HIP_TRY(hipGetLastError());
    return FMM_OK;
}

int ensure_ws(fmm_atree *t, int p, int precision)
{
    AtreeWs &w = *t->wsp;
    const size_t n = (size_t)t->n;
    const size_t coef = (size_t)t->ncells * p + kCoefPad;
    int rc;
    if (w.gam && w.p == p && w.precision == precision) {
        if (coef <= w.coef_cap) return FMM_OK;
        // a workspace handed over by fmm_atree_rebuild from a tree with fewer cells
        HIP_TRY(hipDeviceSynchronize());
        for (double2 **a : {&w.mp, &w.lo, &w.mp2, &w.lo2}) {
            hipFree(*a);
            *a = nullptr;
        }
        if ((rc = dev_alloc(&w.mp, coef, "multipoles")) || (rc = dev_alloc(&w.lo, coef, "locals"))) {
            free_ws(w);
            return rc;
        }
        w.coef_cap = coef;
        return FMM_OK;
    }
    if (w.gam) {
        HIP_TRY(hipDeviceSynchronize());  // earlier calls may still read the old workspace
        free_ws(w);
    }
    if ((rc = dev_alloc((char **)&w.gam, n * (precision == FMM_FP64 ? sizeof(double) : sizeof(float)),
                        "circulations in the near field's precision")) ||
        (rc = dev_alloc(&w.stage, n, "totals")) ||
        (rc = dev_alloc(&w.gamma, n, "circulations")) || (rc = dev_alloc(&w.near, n, "near field")) ||
        (rc = dev_alloc((char **)&w.slots, 9 * n * (precision == FMM_FP64 ? sizeof(double2) : sizeof(float2)),
                        "mutual near-field slots")) ||
        (rc = dev_alloc(&w.mp, coef, "multipoles")) || (rc = dev_alloc(&w.lo, coef, "locals"))) {
        free_ws(w);
        return rc;
    }
    w.coef_cap = coef;
    auto pascal = [](int nb) {
        std::vector<double> b((size_t)nb * nb, 0.0);
        for (int a = 0; a < nb; ++a) {
            b[(size_t)a * nb] = 1.0;
            for (int k = 1; k <= a; ++k)
                b[(size_t)a * nb + k] = b[(size_t)(a - 1) * nb + k - 1] + (k < a ? b[(size_t)(a - 1) * nb + k] : 0.0);
        }
        return b;
    };
    if ((rc = upload(&w.binom, pascal(2 * p + 1), "binomial table")) ||
        (rc = upload(&w.binom16, pascal(33), "binomial table")) ||
        (rc = upload(&w.binom32, pascal(65), "binomial table"))) {
        free_ws(w);
        return rc;
    }
    w.p = p;
    w.precision = precision;
    return FMM_OK;
}

// The adjoint's workspace beside the forward one (same p and precision); the
// source-position sums only when asked for.
int ensure_ws_backward(fmm_atree *t, bool src)
{
    AtreeWs &w = *t->wsp;
    const size_t n = (size_t)t->n;
    int rc = FMM_OK;
    // each group is allocated whole or not at all (a failed call leaves none of it)
    if (!w.mp2) {
        if ((rc = dev_alloc(&w.mp2, w.coef_cap, "adjoint multipoles")) ||
            (rc = dev_alloc(&w.lo2, w.coef_cap, "adjoint locals"))) {
            hipFree(w.mp2);
            w.mp2 = nullptr;
            return rc;
        }
    }
    if (!w.adj) {
        if ((rc = dev_alloc(&w.adj, n, "adjoint charges")) ||
            (rc = dev_alloc((char **)&w.qt, n * (w.precision == FMM_FP64 ? sizeof(double2) : sizeof(float2)),
                            "adjoint charges")) ||
            (rc = dev_alloc(&w.pa, n, "adjoint near sums")) || (rc = dev_alloc(&w.pb, n, "adjoint near sums"))) {
            for (void *q : {(void *)w.adj, w.qt, (void *)w.pa, (void *)w.pb}) hipFree(q);
            w.adj = nullptr;
            w.qt = nullptr;
            w.pa = nullptr;
            w.pb = nullptr;
            return rc;
        }
    }
    if (src && !w.psrc && (rc = dev_alloc(&w.psrc, n, "adjoint source-position sums"))) return rc;
    return FMM_OK;
}

// FMM_OPT_VALIDATE: circulations (and dL/du) checked for NaN / Inf first (synchronises s).
int validate_inputs(fmm_atree *t, const double *gamma, const double *dl_duv, hipStream_t s)
{
    if (!t->validate) return FMM_OK;
    int rc = FMM_OK;
    if (!t->d_flag && (rc = dev_alloc(&t->d_flag, 1, "input check flag"))) return rc;
    int64_t bad = -1;
    HIP_TRY(find_nonfinite(gamma, t->n, 1, t->d_flag, s, bad));
    if (bad >= 0) return fail(FMM_EINVAL, "non-finite circulation (particle " + std::to_string(bad) + ")");
    if (dl_duv) {
        HIP_TRY(find_nonfinite(dl_duv, t->n, 2, t->d_flag, s, bad));
        if (bad >= 0) return fail(FMM_EINVAL, "non-finite dL/du (particle " + std::to_string(bad) + ")");
    }
    return FMM_OK;
}

int check_eval(const fmm_atree *t, const double *gamma, double sigma, int p, int precision)
{
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    if (!gamma) return fail(FMM_EINVAL, "gamma is NULL");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(FMM_EINVAL, "sigma must be finite and > 0");
    if (p < 1 || p > kMaxP) return fail(FMM_EINVAL, "p must be in [1, 32]");
    if (precision != FMM_FP64 && precision != FMM_MIXED) return fail(FMM_EINVAL, "unknown precision");
    return FMM_OK;
}

// Near-field occupancy cap of a forward call (FMM_OPT_NEAR_OCCUPANCY), for the far chain
// on the other stream.  Without a cap the near-field workgroups take every wavefront slot
// and the far kernels wait for them to retire, so the two hardly overlap (2^24 particles:
// 9.78 ms beside each other against 9.83 ms one after the other).  Automatic (mixed
// precision): the stage times predicted from the tree's sizes (ms, fitted to the kernels
// run alone on Gaussian-patch and clustered trees of 2^24 particles, max_leaf 32..256),
//   near = kAtNearPair pairs + kAtNearU |U|,  far = kAtFar0 + kAtFarV |V| + kAtFarCell cells,
// and the cap 5 while the far field is comparable with the near field (0.4 <= far/near
// <= 1.6), else 6: on those eight trees this picks the fastest cap or one within 0.02 ms.
constexpr double kAtNearPair = 2.58e-10, kAtNearU = 2.4e-7;
constexpr double kAtFar0 = 0.08, kAtFarV = 1.0e-7, kAtFarCell = 1.5e-6;

int choose_occupancy(const fmm_atree *t, int precision, bool concurrent)
{
    if (!concurrent) return 0;
    if (t->near_occupancy >= 0) return t->near_occupancy;
    if (precision != FMM_MIXED || t->sizes[FMM_AT_DEEPEST] < 2) return 0;
    const double near = kAtNearPair * (double)t->sizes[FMM_AT_PAIRS] + kAtNearU * (double)t->sizes[FMM_AT_U];
    const double far = kAtFar0 + kAtFarV * (double)t->sizes[FMM_AT_V] + kAtFarCell * (double)t->sizes[FMM_AT_CELLS];
    const double ratio = far / near;
    return (ratio >= 0.4 && ratio <= 1.6) ? 5 : 6;
}

// Up to 16 terms the M2L runs on MFMA with the shared operator tables and the tree's M2L
// plan (made on the first such call, synchronising s); tabs stays NULL otherwise.
int ensure_m2l_plan(fmm_atree *t, int p, hipStream_t s, const Tables *&tabs)
{
    tabs = nullptr;
    if (p > 16 || t->sizes[FMM_AT_DEEPEST] < 2) return FMM_OK;
    std::string err;
    const Tables *tb = nullptr;
    int rc = shared_tables(t->device, p, &tb, err);
    if (rc) return fail(rc == -2 ? FMM_ENOMEM : FMM_EDEVICE, err);
    if (!t->m2l_plan && (rc = build_atree_m2l_plan(t, tb->mfma_entries, s, err))) return fail(rc, err);
    tabs = tb;
    return FMM_OK;
}

int run(fmm_atree *t, const double *gamma, double sigma, int p, int precision, void *main_stream, void *side_stream,
        double *uv, double *uv_near, double *uv_far, const double *base = nullptr, double h = 0.0)
{
    clear_last_error();
    if (t && !uv && !(uv_near && uv_far)) return fail(FMM_EINVAL, "output is NULL");
    int rc0 = check_eval(t, gamma, sigma, p, precision);
    if (rc0) return rc0;
    Busy guard(t);
    if (!guard.ok) return fail(FMM_ESTATE, "tree handle in use by another thread");
    HIP_TRY(hipSetDevice(t->device));
    int rc = validate_inputs(t, gamma, nullptr, (hipStream_t)main_stream);
    hipStream_t ms = (hipStream_t)main_stream;
    if (rc || (rc = ensure_ws(t, p, precision)) || (rc = ensure_coords(t, precision, ms))) return rc;
    hipStream_t ss = side_stream ? (hipStream_t)side_stream : t->own_side;
    const Tables *tabs = nullptr;
    if ((rc = ensure_m2l_plan(t, p, ms, tabs))) return rc;
    const AtreeCall c{t, p, precision == FMM_FP64, record_alpha(sigma, precision),
                      choose_occupancy(t, precision, ss != ms), tabs};
    launch_atree_pack(c, gamma, ms);
    HIP_TRY(hipEventRecord(t->ev_fork, ms));
    HIP_TRY(hipStreamWaitEvent(ss, t->ev_fork, 0));
    launch_atree_far(c, ss);  // P2M, M2M, M2L + P2L + L2L
    HIP_TRY(hipEventRecord(t->ev_join, ss));
    launch_atree_near(c, ms);  // P2P over U, beside the far field
    HIP_TRY(hipStreamWaitEvent(ms, t->ev_join, 0));
    launch_atree_finalize(c, uv, uv_near, uv_far, base, h, ms);  // L2P + M2P + sum
    HIP_TRY(hipGetLastError());
    return FMM_OK;
}

// The adjoint for the cotangent scale * dl_duv, written as `out` says (see AdjointOut).
int run_backward(fmm_atree *t, const double *gamma, double sigma, int p, int precision, const double *dl_duv,
                 double scale, void *main_stream, void *side_stream, const AdjointOut &out)
{
    int rc = check_eval(t, gamma, sigma, p, precision);
    if (rc) return rc;
    if (!dl_duv) return fail(FMM_EINVAL, "dl_duv is NULL");
    if (!std::isfinite(scale)) return fail(FMM_EINVAL, "the cotangent scale must be finite");
    if (!out.dg && !out.dxe && !out.dxs && !out.dxy) return FMM_OK;
    const bool src = out.dxs || out.dxy;
    Busy guard(t);
    if (!guard.ok) return fail(FMM_ESTATE, "tree handle in use by another thread");
    HIP_TRY(hipSetDevice(t->device));
    hipStream_t ms = (hipStream_t)main_stream;
    hipStream_t ss = side_stream ? (hipStream_t)side_stream : t->own_side;
    if ((rc = validate_inputs(t, gamma, dl_duv, ms))) return rc;
    if (t->nbwd_units < 0) {
        std::string err;
        if ((rc = build_atree_adjoint_units(t, ms, err))) return fail(rc, err);
    }
    const Tables *tabs = nullptr;
    if ((rc = ensure_ws(t, p, precision)) || (rc = ensure_ws_backward(t, src)) ||
        (rc = ensure_coords(t, precision, ms)) || (rc = ensure_m2l_plan(t, p, ms, tabs)))
        return rc;
    const AtreeCall c{t, p, precision == FMM_FP64, record_alpha(sigma, precision), 0, tabs};
    launch_atree_pack(c, gamma, ms);
    launch_atree_pack_adjoint(c, dl_duv, scale, ms);
    // The two far chains run beside each other, then the near field (which holds every
    // wavefront slot, so that far kernels beside it would wait for it to drain).
    HIP_TRY(hipEventRecord(t->ev_fork, ms));
    HIP_TRY(hipStreamWaitEvent(ss, t->ev_fork, 0));
    launch_atree_far(c, ss, true);   // the charges q: the transpose pass
    launch_atree_far(c, ms, false);  // the charges c: derivative W' at the particles
    HIP_TRY(hipEventRecord(t->ev_join, ss));
    HIP_TRY(hipStreamWaitEvent(ms, t->ev_join, 0));
    launch_atree_backward_near(c, src, ms);
    launch_atree_finalize_backward(c, out, ms);
    HIP_TRY(hipGetLastError());
    return FMM_OK;
}

// Argument checks shared by both builds; a new tree with the caller's parameters.
int new_atree(const double *xy, int64_t n, int max_leaf, int max_depth, const double *root_box, fmm_atree **out,
              fmm_atree *&t)
{
    clear_last_error();
    t = nullptr;
    if (!out) return fail(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!xy) return fail(FMM_EINVAL, "xy is NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(FMM_EINVAL, "n must be in [1, 2^31)");
    if (max_leaf < 1) return fail(FMM_EINVAL, "max_leaf must be >= 1");
    if (max_depth < 0 || max_depth > 15) return fail(FMM_EINVAL, "max_depth must be in [0, 15]");
    if (root_box && (!std::isfinite(root_box[0]) || !std::isfinite(root_box[1]) || !(root_box[2] > 0.0) ||
                     !std::isfinite(root_box[2])))
        return fail(FMM_EINVAL, "root_box must be finite with side > 0");
    t = new (std::nothrow) fmm_atree;
    if (!t) return fail(FMM_ENOMEM, "host allocation failed");
    t->n = n;
    t->max_leaf = max_leaf;
    t->max_depth = max_depth;
    const hipError_t e = hipGetDevice(&t->device);
    if (e != hipSuccess) {
        free_atree(t);
        t = nullptr;
        return hip_fail(e, "hipGetDevice");
    }
    return FMM_OK;
}

int finish_atree(fmm_atree *t)
{
    hipError_t e = hipStreamCreateWithFlags(&t->own_side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming);
    return e != hipSuccess ? hip_fail(e, "creating the side stream") : FMM_OK;
}

}  // namespace

extern "C" int fmm_atree_build(const double *xy, int64_t n, int max_leaf, int max_depth, const double *root_box,
                               void *stream, fmm_atree **out)
{
    fmm_atree *t = nullptr;
    int rc = new_atree(xy, n, max_leaf, max_depth, root_box, out, t);
    if (rc) return rc;
    retain_pool(t->device);
    std::string err;
    int64_t bad = -1;
    rc = build_atree_device(t, xy, root_box, (hipStream_t)stream, err, bad);
    if (rc) {
        if (bad >= 0) err += " (particle " + std::to_string(bad) + ")";
        fail(rc, err);
    } else {
        rc = finish_atree(t);
    }
    if (rc) {
        free_atree(t);
        return rc;
    }
    trim_pool(t->device);  // the build's temporaries
    *out = t;
    return FMM_OK;
}

extern "C" int fmm_atree_rebuild(fmm_atree *prev, const double *xy, int64_t n, const double *root_box, void *stream,
                                 fmm_atree **out)
{
    clear_last_error();
    if (out) *out = nullptr;
    if (!prev) return fail(FMM_ESTATE, "null tree handle");
    if (n != prev->n) return fail(FMM_EINVAL, "n must equal the particle count of the tree being rebuilt");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != prev->device) return fail(FMM_EINVAL, "the current device is not the tree's");
    Busy guard(prev);
    if (!guard.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    fmm_atree *t = nullptr;
    int rc = fmm_atree_build(xy, n, prev->max_leaf, prev->max_depth, root_box, stream, &t);
    if (rc) return rc;
    const hipError_t e = hipDeviceSynchronize();  // work of earlier calls on prev may still use its workspace
    if (e != hipSuccess) {
        free_atree(t);
        return hip_fail(e, "hipDeviceSynchronize");
    }
    std::swap(t->wsp, prev->wsp);
    t->near_occupancy = prev->near_occupancy;
    t->validate = prev->validate;
    guard.release();
    free_atree(prev);
    *out = t;
    return FMM_OK;
}

extern "C" int fmm_atree_build_host(const double *xy, int64_t n, int max_leaf, int max_depth, const double *root_box,
                                    void *stream, fmm_atree **out)
{
    fmm_atree *t = nullptr;
    int rc = new_atree(xy, n, max_leaf, max_depth, root_box, out, t);
    if (rc) return rc;
    try {
        std::vector<double> h(2 * (size_t)n);
        hipError_t e = hipMemcpyAsync(h.data(), xy, h.size() * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) {
            free_atree(t);
            return hip_fail(e, "copying positions to the host");
        }
        for (double v : h)
            if (!std::isfinite(v)) {
                free_atree(t);
                return fail(FMM_EINVAL, "non-finite particle position");
            }
        if (root_box) {
            t->x0 = root_box[0];
            t->y0 = root_box[1];
            t->side = root_box[2];
        } else {
            double xmin = h[0], xmax = h[0], ymin = h[1], ymax = h[1];
            for (int64_t i = 1; i < n; ++i) {
                xmin = std::min(xmin, h[2 * i]);
                xmax = std::max(xmax, h[2 * i]);
                ymin = std::min(ymin, h[2 * i + 1]);
                ymax = std::max(ymax, h[2 * i + 1]);
            }
            double side = std::max(xmax - xmin, ymax - ymin);
            if (side <= 0.0) side = 1.0;
            t->x0 = xmin;
            t->y0 = ymin;
            t->side = side * (1.0 + 1.0 / 1048576.0);
        }
        // binning at max_depth (as fmm_build_tree at that depth), Morton keys
        const int L = max_depth;
        const int64_t nside = int64_t(1) << L;
        const double w = t->side / (double)nside;
        std::vector<uint32_t> key((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            uint32_t c[2];
            for (int d = 0; d < 2; ++d) {
                const double v = (h[2 * i + d] - (d ? t->y0 : t->x0)) / w;
                if (!(v >= 0.0) || v > (double)nside) {
                    free_atree(t);
                    char buf[160];
                    snprintf(buf, sizeof buf, "particle %lld lies outside the root cell", (long long)i);
                    return fail(FMM_ERANGE, buf);
                }
                c[d] = (uint32_t)std::min<int64_t>((int64_t)std::floor(v), nside - 1);
            }
            key[i] = morton_encode(c[0], c[1]);
        }
        // stable LSD radix sort of the particles by key (two 16-bit digits)
        std::vector<int> order((size_t)n), tmp((size_t)n);
        for (int64_t i = 0; i < n; ++i) order[i] = (int)i;
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<int64_t> cnt(65537, 0);
            const int sh = 16 * pass;
            for (int64_t i = 0; i < n; ++i) cnt[((key[order[i]] >> sh) & 0xffff) + 1]++;
            for (int b = 0; b < 65536; ++b) cnt[b + 1] += cnt[b];
            for (int64_t i = 0; i < n; ++i) tmp[cnt[(key[order[i]] >> sh) & 0xffff]++] = order[i];
            order.swap(tmp);
        }
        std::vector<uint32_t> skey((size_t)n);
        for (int64_t j = 0; j < n; ++j) skey[j] = key[order[j]];

        HostTree ht;
        ht.L = L;
        ht.smax = max_leaf;
        ht.build(skey, (int)n);
        ht.lists();
        const int K = (int)ht.cells.size();
        t->ncells = K;

        // levels, leaves, sizes
        t->level_off.assign(L + 2, 0);
        t->inner_off.assign(L + 2, 0);
        std::vector<int> p2m, inner;
        std::vector<int4> cell(K);
        std::vector<int2> range(K);
        std::vector<int> parent(K), tile_start(K, 0), leaf_sorted((size_t)n);
        std::vector<int4> child(K);
        int64_t leaves = 0, deepest = 0, pairs = 0;
        for (int k = 0; k < K; ++k) {
            const HostCell &c = ht.cells[k];
            t->level_off[c.level + 1]++;
            cell[k] = make_int4(c.level, c.ix, c.iy, c.leaf ? 1 : 0);
            range[k] = make_int2(c.first, c.count);
            parent[k] = c.parent;
            child[k] = make_int4(c.child[0], c.child[1], c.child[2], c.child[3]);
            if (c.leaf) {
                leaves++;
                deepest = std::max<int64_t>(deepest, c.level);
                int64_t s = 0;
                for (int S : ht.U[k]) s += ht.cells[S].count;
                pairs += (int64_t)c.count * s - c.count;
                for (int j = c.first; j < c.first + c.count; ++j) leaf_sorted[j] = k;
                if (c.level >= 2) p2m.push_back(k);
            }
        }
        for (int l = 0; l <= L; ++l) t->level_off[l + 1] += t->level_off[l];
        for (int l = 0; l <= L; ++l) {
            t->inner_off[l] = (int)inner.size();
            for (int k = t->level_off[l]; k < t->level_off[l + 1]; ++k)
                if (!ht.cells[k].leaf && l >= 2) inner.push_back(k);
        }
        t->inner_off[L + 1] = (int)inner.size();
        int64_t lsum[4] = {0, 0, 0, 0};
        for (int k = 0; k < K; ++k) {
            lsum[0] += (int64_t)ht.U[k].size();
            lsum[1] += (int64_t)ht.V[k].size();
            lsum[2] += (int64_t)ht.W[k].size();
            lsum[3] += (int64_t)ht.X[k].size();
        }
        const int64_t sz[8] = {K, leaves, lsum[0], lsum[1], lsum[2], lsum[3], deepest, pairs};
        std::copy(sz, sz + 8, t->sizes);
        t->np2m = (int64_t)p2m.size();

        // 64-particle tiles of each leaf (leaves in sorted order) with their boxes: absolute
        // (relative to x0, y0) for the target-centric units, in leaf widths about the leaf
        // centre, rounded outwards to FP32, for the mutual items
        std::vector<double2> xs((size_t)n);
        for (int64_t j = 0; j < n; ++j) xs[j] = make_double2(h[2 * order[j]], h[2 * order[j] + 1]);
        std::vector<int> leaves_sorted;
        for (int k = 0; k < K; ++k)
            if (ht.cells[k].leaf) leaves_sorted.push_back(k);
        std::sort(leaves_sorted.begin(), leaves_sorted.end(),
                  [&](int a, int b) { return ht.cells[a].first < ht.cells[b].first; });
        const int NL = (int)leaves_sorted.size();
        std::vector<int> leaf_index(K, -1), leaf_start(NL + 1), leaf_tile(NL);
        std::vector<double4> boxes;
        std::vector<float4> boxes_leaf;
        for (int li = 0; li < NL; ++li) {
            const int k = leaves_sorted[li];
            const HostCell &c = ht.cells[k];
            leaf_index[k] = li;
            leaf_start[li] = c.first;
            leaf_tile[li] = tile_start[k] = (int)boxes.size();
            const double wl = t->side / (double)(int64_t(1) << c.level);
            const double cx = t->x0 + (c.ix + 0.5) * wl, cy = t->y0 + (c.iy + 0.5) * wl;
            for (int b = c.first; b < c.first + c.count; b += 64) {
                const int len = std::min(64, c.first + c.count - b);
                double4 bx = make_double4(1e300, 1e300, -1e300, -1e300);
                double4 bl = bx;
                for (int j = b; j < b + len; ++j) {
                    const double x = xs[j].x - t->x0, y = xs[j].y - t->y0;
                    bx.x = std::min(bx.x, x), bx.y = std::min(bx.y, y), bx.z = std::max(bx.z, x), bx.w = std::max(bx.w, y);
                    const double xl = (xs[j].x - cx) / wl, yl = (xs[j].y - cy) / wl;
                    bl.x = std::min(bl.x, xl), bl.y = std::min(bl.y, yl), bl.z = std::max(bl.z, xl), bl.w = std::max(bl.w, yl);
                }
                boxes.push_back(bx);
                boxes_leaf.push_back(make_float4(std::nextafter((float)bl.x, -INFINITY), std::nextafter((float)bl.y, -INFINITY),
                                                 std::nextafter((float)bl.z, INFINITY), std::nextafter((float)bl.w, INFINITY)));
            }
        }
        leaf_start[NL] = (int)n;

        // Near-field plan.  A leaf is dense with at least dense_leaf particles; every
        // unordered pair of adjacent dense leaves of one level, and every dense leaf with
        // itself, is one mutual item; the rest of U from the target end.  Costs as for the
        // uniform tree (mutual steps weight 3, target-centric 2).
        const int D = t->dense_leaf;
        std::vector<uint16_t> mask(K, 0);
        std::vector<int4> work;
        std::vector<int64_t> cost;
        const int up[4][2] = {{1, 0}, {-1, 1}, {0, 1}, {1, 1}};
        int64_t mpairs = 0, nmut = 0, ntc = 0;
        for (int li = 0; li < NL; ++li) {
            const int k = leaves_sorted[li];
            const HostCell &c = ht.cells[k];
            const bool dense = c.count >= D;
            uint32_t m = 0;
            int64_t nsrc = 0;
            for (int S : ht.U[k]) {
                const HostCell &cs = ht.cells[S];
                if (dense && cs.count >= D && cs.level == c.level)
                    m |= 1u << (3 * (cs.iy - c.iy + 1) + (cs.ix - c.ix + 1));
                else
                    nsrc += cs.count;
            }
            if (nsrc > 0) {
                m |= 1u << 9;
                for (int b = c.first; b < c.first + c.count; b += 64) {
                    const int len = std::min(64, c.first + c.count - b);
                    work.push_back(make_int4(k, b, len, at_log2_lanes(len) | (dense ? 16 : 0)));
                    cost.push_back(at_unit_cost(nsrc, len));
                    ++ntc;
                }
            }
            mask[k] = (uint16_t)m;
            if (!dense) continue;
            work.push_back(make_int4(li, li, 4 | (4 << 4), kMutualItem | (c.level << 9)));
            cost.push_back(at_self_cost(c.count));
            ++nmut;
            mpairs += (int64_t)c.count * (c.count - 1);
            for (const auto &o : up) {
                const int R = ht.find(c.level, c.ix + o[0], c.iy + o[1]);
                if (R < 0 || !ht.cells[R].leaf || ht.cells[R].count < D) continue;
                const int ds = 3 * (o[1] + 1) + (o[0] + 1);
                work.push_back(make_int4(li, leaf_index[R], ds | ((8 - ds) << 4), kMutualItem | (c.level << 9)));
                cost.push_back(3 * at_pair_steps(c.count, ht.cells[R].count));
                ++nmut;
                mpairs += 2 * (int64_t)c.count * ht.cells[R].count;
            }
        }
        std::vector<int> worder(work.size());
        for (size_t u = 0; u < work.size(); ++u) worder[u] = (int)u;
        std::stable_sort(worder.begin(), worder.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<int4> swork(work.size());
        for (size_t u = 0; u < work.size(); ++u) swork[u] = work[worder[u]];
        t->ntiles = (int64_t)boxes.size();
        t->nwork = (int64_t)swork.size();
        t->mutual_items = nmut;
        t->mutual_pairs = mpairs;
        t->target_units = ntc;

        std::vector<int> uo, ui, vo, vi, wo, wi, xo, xi;
        flatten(ht.U, uo, ui);
        flatten(ht.V, vo, vi);
        flatten(ht.W, wo, wi);
        flatten(ht.X, xo, xi);

        AtreeDev &d = t->d;
        hipError_t es = hipSetDevice(t->device);
        rc = es != hipSuccess ? hip_fail(es, "hipSetDevice") : upload(&d.perm, order, "permutation");
        if (!rc) {
            std::vector<int> g1, g2;
            host_staging(order, t->stage_shift, g1, g2);
            rc = upload(&d.gpos1, g1, "staging slots");
            if (!rc) rc = upload(&d.gpos2, g2, "staging slots");
            if (!rc) rc = dev_alloc(&d.st1, (size_t)t->n, "staging array");
        }
        if (!rc) rc = upload(&d.leaf_of, leaf_sorted, "leaf of each particle");
        if (!rc) rc = upload(&d.xy, xs, "sorted positions");
        if (!rc) rc = upload(&d.cell, cell, "cells");
        if (!rc) rc = upload(&d.range, range, "cell ranges");
        if (!rc) rc = upload(&d.parent, parent, "parents");
        if (!rc) rc = upload(&d.child, child, "children");
        if (!rc) rc = upload(&d.u_off, uo, "U list");
        if (!rc) rc = upload(&d.u_idx, ui, "U list");
        if (!rc) rc = upload(&d.v_off, vo, "V list");
        if (!rc) rc = upload(&d.v_idx, vi, "V list");
        if (!rc) rc = upload(&d.w_off, wo, "W list");
        if (!rc) rc = upload(&d.w_idx, wi, "W list");
        if (!rc) rc = upload(&d.x_off, xo, "X list");
        if (!rc) rc = upload(&d.x_idx, xi, "X list");
        if (!rc) rc = upload(&d.p2m_cells, p2m, "leaves with expansions");
        if (!rc) rc = upload(&d.inner, inner, "split cells");
        if (!rc) rc = upload(&d.tile_start, tile_start, "tiles");
        if (!rc) rc = upload(&d.tile_box, boxes, "tile boxes");
        if (!rc) rc = upload(&d.work, swork, "near-field work");
        if (!rc) rc = upload(&d.leaf_start, leaf_start, "leaf offsets");
        if (!rc) rc = upload(&d.leaf_tile, leaf_tile, "leaf tiles");
        if (!rc) rc = upload(&d.tile_box_leaf, boxes_leaf, "tile boxes");
        if (!rc) rc = upload(&d.mask, mask, "near-field mask");
        if (!rc) rc = finish_atree(t);
    } catch (const std::bad_alloc &) {
        rc = fail(FMM_ENOMEM, "host allocation failed while building the adaptive tree");
    }
    if (rc) {
        free_atree(t);
        return rc;
    }
    *out = t;
    return FMM_OK;
}

extern "C" int fmm_atree_share_workspace(fmm_atree *t, fmm_atree *from)
{
    clear_last_error();
    if (!t || !from) return fail(FMM_ESTATE, "null tree handle");
    if (t == from) return FMM_OK;
    if (t->n != from->n || t->device != from->device)
        return fail(FMM_EINVAL, "trees sharing a workspace need the same n and device");
    Busy g1(t);
    if (!g1.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    Busy g2(from);
    if (!g2.ok) return fail(FMM_ESTATE, "tree is in use by another call");
    if (t->wsp == from->wsp) return FMM_OK;
    HIP_TRY(hipSetDevice(t->device));
    HIP_TRY(hipDeviceSynchronize());  // t's earlier calls may still use its workspace
    if (t->wsp.use_count() == 1) free_ws(*t->wsp);
    t->wsp = from->wsp;
    return FMM_OK;
}

extern "C" int fmm_atree_info(const fmm_atree *t, int64_t *sizes, double *root_box)
{
    clear_last_error();
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    if (!sizes) return fail(FMM_EINVAL, "sizes is NULL");
    std::copy(t->sizes, t->sizes + FMM_AT_COUNT, sizes);
    if (root_box) {
        root_box[0] = t->x0;
        root_box[1] = t->y0;
        root_box[2] = t->side;
    }
    return FMM_OK;
}

extern "C" int fmm_atree_leaves(const fmm_atree *t, int32_t *level, int32_t *ix, int32_t *iy)
{
    clear_last_error();
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    try {
        std::vector<int> perm((size_t)t->n), leaf((size_t)t->n);
        std::vector<int4> cell((size_t)t->ncells);
        HIP_TRY(hipSetDevice(t->device));
        HIP_TRY(hipMemcpy(perm.data(), t->d.perm, perm.size() * sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(leaf.data(), t->d.leaf_of, leaf.size() * sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(cell.data(), t->d.cell, cell.size() * sizeof(int4), hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < t->n; ++j) {
            const int4 c = cell[leaf[j]];
            const int u = perm[j];
            if (level) level[u] = c.x;
            if (ix) ix[u] = c.y;
            if (iy) iy[u] = c.z;
        }
    } catch (const std::bad_alloc &) {
        return fail(FMM_ENOMEM, "host allocation failed");
    }
    return FMM_OK;
}

extern "C" int fmm_atree_velocity(fmm_atree *t, const double *gamma, double sigma, int p, int precision,
                                  void *main_stream, void *side_stream, double *uv)
{
    if (!uv) {
        clear_last_error();
        return fail(FMM_EINVAL, "uv is NULL");
    }
    return run(t, gamma, sigma, p, precision, main_stream, side_stream, uv, nullptr, nullptr);
}

extern "C" int fmm_atree_velocity_parts(fmm_atree *t, const double *gamma, double sigma, int p, int precision,
                                        void *main_stream, void *side_stream, double *uv_near, double *uv_far)
{
    if (!uv_near || !uv_far) {
        clear_last_error();
        return fail(FMM_EINVAL, "uv_near / uv_far is NULL");
    }
    return run(t, gamma, sigma, p, precision, main_stream, side_stream, nullptr, uv_near, uv_far);
}

extern "C" int fmm_atree_velocity_backward(fmm_atree *t, const double *gamma, double sigma, int p, int precision,
                                           const double *dl_duv, void *main_stream, void *side_stream,
                                           double *dl_dgamma, double *dl_dxeval, double *dl_dxsrc, double *dl_dxy)
{
    clear_last_error();
    AdjointOut out;
    out.dg = dl_dgamma;
    out.dxe = dl_dxeval;
    out.dxs = dl_dxsrc;
    out.dxy = dl_dxy;
    return run_backward(t, gamma, sigma, p, precision, dl_duv, 1.0, main_stream, side_stream, out);
}

extern "C" int fmm_atree_transport_step(fmm_atree *t, const double *gamma, double sigma, int p, int precision,
                                        void *main_stream, void *side_stream, const double *x_base, double h,
                                        double *x_out)
{
    clear_last_error();
    if (!x_base || !x_out) return fail(FMM_EINVAL, "x_base / x_out is NULL");
    if (!std::isfinite(h)) return fail(FMM_EINVAL, "h must be finite");
    return run(t, gamma, sigma, p, precision, main_stream, side_stream, x_out, nullptr, nullptr, x_base, h);
}

extern "C" int fmm_atree_transport_vjp(fmm_atree *t, const double *gamma, double sigma, int p, int precision,
                                       const double *lam, double h, int flags, void *main_stream, void *side_stream,
                                       double *dl_dgamma, double *dl_dx)
{
    clear_last_error();
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

extern "C" int fmm_atree_set_option(fmm_atree *t, int key, int64_t value)
{
    clear_last_error();
    if (!t) return fail(FMM_ESTATE, "null tree handle");
    switch (key) {
    case FMM_OPT_NEAR_OCCUPANCY:
        if (value < -1 || value > 8) return fail(FMM_EINVAL, "near occupancy must be in [-1, 8]");
        t->near_occupancy = (int)value;
        return FMM_OK;
    case FMM_OPT_VALIDATE:
        if (value != 0 && value != 1) return fail(FMM_EINVAL, "validate must be 0 or 1");
        t->validate = (int)value;
        return FMM_OK;
    default:
        return fail(FMM_EINVAL, "unknown option key for an adaptive tree");
    }
}

extern "C" void fmm_atree_destroy(fmm_atree *t)
{
    if (!t) return;
    hipSetDevice(t->device);
    const int dev = t->device;
    free_atree(t);
    trim_pool(dev);
}
