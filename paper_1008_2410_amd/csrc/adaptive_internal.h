// Internal layout of the adaptive tree (fmm2d_adaptive.h) and the launchers of its
// kernels (adaptive.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <cstdint>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

// Device arrays of one adaptive tree.  Cells are numbered level by level (the cells
// of level l are [level_off[l], level_off[l+1])), in Morton order inside a level;
// particles are sorted by their Morton key at max_depth, so every cell's particles
// are one contiguous range.  Lists are CSR over cells (int offsets, int cell ids).
struct AtreeDev {
    int *perm = nullptr;        // sorted slot -> user index
    // two-pass permutations between user and sorted order (buckets of 2^stage_shift sorted
    // slots): user index -> staging slot, sorted slot -> staging slot of its user index,
    // and the staging array of the circulations
    int *gpos1 = nullptr, *gpos2 = nullptr;
    double *st1 = nullptr;
    int *leaf_of = nullptr;     // sorted slot -> leaf cell
    double2 *xy = nullptr;      // positions, sorted
    int4 *cell = nullptr;       // {level, ix, iy, is_leaf}
    int2 *range = nullptr;      // {first sorted slot, count}
    int *parent = nullptr;      // -1 for the root
    int4 *child = nullptr;      // four quadrants (q = x bit | y bit << 1), -1 when empty
    int *u_off = nullptr, *u_idx = nullptr;
    int *v_off = nullptr, *v_idx = nullptr;
    int *w_off = nullptr, *w_idx = nullptr;
    int *x_off = nullptr, *x_idx = nullptr;
    int *p2m_cells = nullptr;   // leaves of level >= 2
    int *inner = nullptr;       // split cells of level >= 2, grouped by level (inner_off)
    int *tile_start = nullptr;  // per cell: first 64-particle tile of a leaf
    double4 *tile_box = nullptr;  // per tile: {xmin, ymin, xmax, ymax} relative to (x0, y0)
    // Near-field work, heaviest first: target-centric units {leaf cell, first, count,
    // log2 TP | 16 when the leaf is dense (its same-level dense neighbours are skipped)}
    // and mutual items {leaf index S, leaf index R, d_S | d_R << 4, kMutualItem | level << 9}
    // for same-level adjacent dense leaves (leaf index = position in sorted order).
    int4 *work = nullptr;
    int *leaf_start = nullptr;     // per leaf index: first sorted slot (nleaves + 1 entries)
    int *leaf_tile = nullptr;      // per leaf index: first tile
    float4 *tile_box_leaf = nullptr;  // per tile: box in leaf widths about the leaf centre
    uint16_t *mask = nullptr;      // per cell: slots d written by mutual items, bit 9 target-centric part
    // Adjoint near field: target-centric units over all of U, one per 64-particle tile
    // {leaf cell, first, count, log2 TP}, heaviest first (made on the first adjoint call).
    int4 *bwd_units = nullptr;
    // Translations on MFMA (made on the first evaluation with p <= 16): the cells of level
    // >= 2 grouped by level and, inside a level, by parity class (x bit | y bit << 1), and
    // per such cell (index - level_off[2]) the source cell of each of its class's 27
    // interaction offsets, -1 where V holds none.
    int *m2l_targets = nullptr;
    int *vslot = nullptr;
};

// Costs of near-field work (steps of the near kernel), for the heaviest-first order of
// the plan; the same functions serve the host and the device build.
__host__ __device__ inline int64_t at_chunks16(int64_t len) { return (len + 15) >> 4; }
// a mutual item between two leaves of cs and cr particles
__host__ __device__ inline int64_t at_pair_steps(int64_t cs, int64_t cr)
{
    const int64_t fs = cs / 64, fr = cr / 64, rs = cs % 64, rr = cr % 64;
    const int64_t a = at_chunks16(rs), b = at_chunks16(rr);
    return 16 * (fs * fr * 4 + fs * b + fr * a + (a < b ? a : b));
}
// the mutual item of a dense leaf with itself
__host__ __device__ inline int64_t at_self_cost(int64_t c)
{
    const int64_t f = c / 64, r = c % 64;
    const int64_t diag = 16 * (f * 4 + at_chunks16(r));
    const int64_t st = 16 * (f * (f - 1) / 2 * 4 + f * at_chunks16(r));
    return 3 * st + 2 * diag;
}
// log2 of the lanes per target of a target-centric unit of len targets (the smallest
// power of two >= len), and its cost over nsrc sources
__host__ __device__ inline int at_log2_lanes(int len)
{
    int l = 0;
    while ((1 << l) < len) ++l;
    return l;
}
__host__ __device__ inline int64_t at_unit_cost(int64_t nsrc, int len)
{
    const int64_t stride = 64 >> at_log2_lanes(len);
    return 2 * ((nsrc + stride - 1) / stride);
}

struct AtreeWs {
    int p = 0, precision = -1;
    size_t coef_cap = 0;        // elements of each expansion array (mp, lo, mp2, lo2)
    void *gam = nullptr;        // circulations, sorted, in the near field's precision (its records' Gamma)
    double2 *stage = nullptr;   // totals on their way to user order
    double *gamma = nullptr;    // circulations, sorted
    double2 *near = nullptr;    // near-field (u, v), sorted
    void *slots = nullptr;      // mutual form: 9 x n sums (dY, dX), float2 or double2
    double2 *mp = nullptr;      // multipoles a_m / w^m, cells x p
    double2 *lo = nullptr;      // locals b_l w^(l+1), cells x p
    // adjoint: expansions of the adjoint charges q, the charges (sorted, FP64, and in the
    // records' precision), the near sums {Phi, A (Re, Im / -2)}, B, and the source sums
    double2 *mp2 = nullptr, *lo2 = nullptr, *adj = nullptr;
    void *qt = nullptr;
    double4 *pa = nullptr, *psrc = nullptr;
    double *pb = nullptr;
    double *binom = nullptr;    // C(a, k), a, k <= 2p, row-major (2p + 1)^2
    double *binom16 = nullptr;  // the same for a, k <= 32 (33 x 33), and for a, k <= 64 (65 x 65):
    double *binom32 = nullptr;  // the M2L kernel runs 16 or 32 terms whatever p
};

}  // namespace fmm

struct fmm_atree {
    int device = 0;
    int64_t n = 0;
    int max_leaf = 0, max_depth = 0;
    double x0 = 0, y0 = 0, side = 1;
    int64_t sizes[8] = {};
    int64_t ncells = 0, ntiles = 0, nwork = 0, np2m = 0;
    int64_t mutual_items = 0, mutual_pairs = 0, target_units = 0;
    int64_t nbwd_units = -1;  // -1 until the adjoint units are made
    int dense_leaf = 32;
    int stage_shift = 0;
    int near_occupancy = -1;  // FMM_OPT_NEAR_OCCUPANCY: -1 automatic, 0 no cap, 1..8 the cap
    bool m2l_plan = false;    // d.m2l_targets and d.vslot made
    void *d_pos[2] = {};      // offsets z - c_leaf of the sorted particles, float2 / double2 (made on first use)
    std::vector<int> m2l_seg_off;  // segment 4 (level - 2) + class: start in d.m2l_targets
    int validate = 0;         // FMM_OPT_VALIDATE: check circulations (and dL/du) for NaN / Inf
    int *d_flag = nullptr;    // device result of that check
    std::vector<int> level_off;   // max_depth + 2 entries
    std::vector<int> inner_off;   // max_depth + 2 entries, into AtreeDev::inner
    bool pooled = false;  // device arrays from the stream-ordered pool (the device build)
    fmm::AtreeDev d;
    std::shared_ptr<fmm::AtreeWs> wsp = std::make_shared<fmm::AtreeWs>();  // shared by fmm_atree_share_workspace
    hipStream_t own_side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::atomic<int> busy{0};
};

namespace fmm {

struct AtreeCall {
    const fmm_atree *t;
    int p;
    int is_double;
    double alpha;   // record scale (as for the uniform tree)
    int near_occ = 0;  // forward near field: wavefronts per SIMD it may hold (0: no cap)
    const Tables *tabs = nullptr;  // with the M2L plan (p <= 16): the MFMA operators
};

// Stages 1-3 on the device (adaptive_build.hip): fills t->d and the host facts of t
// (n, max_leaf, max_depth and dense_leaf set by the caller) with the arrays the host build
// makes.  Returns FMM_OK or a status with err; bad_index names a particle outside the root
// cell or non-finite (else -1).
int build_atree_device(fmm_atree *t, const double *xy, const double *root_box, hipStream_t s, std::string &err,
                       int64_t &bad_index);

// The adjoint near-field units (d.bwd_units, nbwd_units) from the tree's arrays; either
// build.  Synchronises s.
int build_atree_adjoint_units(fmm_atree *t, hipStream_t s, std::string &err);

// The M2L plan of the MFMA path (d.m2l_targets, d.vslot, m2l_class_off) from the V lists
// and the interaction entries of the operator tables.  Synchronises s.
int build_atree_m2l_plan(fmm_atree *t, const int4 *entries, hipStream_t s, std::string &err);

void launch_atree_pack(const AtreeCall &c, const double *gamma, hipStream_t s);
// the particles' offsets from their leaves' centres in the near field's precision (d_pos)
void launch_atree_coords(const fmm_atree *t, int is_double, void *pos, hipStream_t s);
// adjoint false: the far field of the charges c (mp, lo); true: of the adjoint charges
// q (mp2, lo2)
void launch_atree_far(const AtreeCall &c, hipStream_t s, bool adjoint = false);
void launch_atree_pack_adjoint(const AtreeCall &c, const double *dl_duv, double scale, hipStream_t s);
void launch_atree_backward_near(const AtreeCall &c, bool src, hipStream_t s);
void launch_atree_finalize_backward(const AtreeCall &c, const AdjointOut &out, hipStream_t s);
void launch_atree_near(const AtreeCall &c, hipStream_t s);
// uv alone goes through the records as staging; with base, uv = base + h u
void launch_atree_finalize(const AtreeCall &c, double *uv, double *uv_near, double *uv_far, const double *base,
                           double h, hipStream_t s);

}  // namespace fmm
