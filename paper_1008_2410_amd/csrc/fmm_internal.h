// Internal declarations of the gfx950 FMM library: tree layout, workspace, and the
// kernel launchers implemented in kernels.hip.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <functional>
#include <memory>
#include <cstdint>
#include <string>
#include <vector>

#include "host_tree.h"
#include "morton.h"

namespace fmm {

constexpr int kMaxDepth = 12;
constexpr int kMaxP = 32;
constexpr int kNumEvents = 8;


// ---------------------------------------------------------------------------------
// Device-side tables for one expansion order p (radius-scaled operators, level
// independent).  All complex arrays are interleaved (re, im).
//   m2m[q][m][k]  = C(m,k) d_q^(m-k) 2^-k                 (k <= m, else 0)
//   l2l[q][k][l]  = C(l,k) d_q^(l-k) 2^-(k+1)             (l >= k, else 0)
//   m2l[o][m][l]  = (-1)^l C(l+m,m) delta^-(l+m+1), delta = (dx, dy) of offset o = (dx+3)*7 + (dy+3)
// with d_q = (c_child - c_parent)/w_parent = ((q&1) - 1/2)/2 + i((q>>1) - 1/2)/2.
// ---------------------------------------------------------------------------------
// mfma_f: the M2L and L2L operators as 2p x 2p real matrices (complex entries embedded
// with interleaved (re, im) rows and columns, zero-padded to 32 x 32) in the operand
// order of the MFMA M2L kernel: [slot][k / 16][column][k % 16], slots 0..48 the M2L
// offsets (index (dx+3)*7 + (dy+3)), 49..52 the L2L parities, 53..56 the M2M children.
// Built for p <= 16.
struct Tables {
    int p = 0;
    double2 *m2m_d = nullptr, *l2l_d = nullptr, *m2l_d = nullptr;
    float2 *m2m_f = nullptr, *l2l_f = nullptr, *m2l_f = nullptr;
    float *mfma_f = nullptr;
    double *mfma_d = nullptr;      // FP64 MFMA operand order: [slot][k / 8][column][k % 8]
    int4 *mfma_entries = nullptr;  // {dx, dy, slot, kind}: 4 x 28 M2L/L2L entries, then 4 M2M entries
    double *zero_row = nullptr;    // 128 zero doubles: the row read for absent source cells
};

// Coefficient arrays are allocated with this many extra elements at the end, so that
// fixed-length reads of a row never pass the allocation.
constexpr int64_t kCoefPad = 64;
// The number of XCDs that workgroups are dealt to round-robin.
constexpr int kXcds = 8;
constexpr int64_t kLastLevelCacheBytes = int64_t(256) << 20;  // MI355X Infinity Cache

// Whether a call's per-particle outputs (bytes_per_row each) reach user order through the
// staging windows (written by sorted bucket, then gathered in user order) rather than by
// random rows: once they fill the last-level cache.  At 2^24 patch particles (16-byte
// velocities: exactly the cache) the windows measured faster, 8.44 -> 8.36 ms per
// evaluation, and the adjoint's 24 (40) bytes 18.30 -> 18.15 (23.85 -> 23.50) ms.
inline bool outputs_windowed(int64_t n, int64_t bytes_per_row)
{
    return n * bytes_per_row >= kLastLevelCacheBytes;
}
// Flag (in w) of a mutual item in the near-field work list.
constexpr int kMutualItem = 256;

// Owner value of a workspace handed to a tree over other particles (clear before use).
constexpr uint64_t kForeignOwner = ~uint64_t(0);

// Coefficient storage for one (p, precision, split) configuration.  Levels 0..split
// are FP64, levels split+1..L are FP32; each level holds 4^l cells x p coefficients,
// multipoles (scaled a_m / w^m) and locals (scaled b_l w^(l+1)) in separate arrays.
struct Workspace {
    int p = 0, precision = -1, split = -1;
    // serial number of the tree whose call last wrote the multipoles (0: none yet, or
    // unknown after a hand-over): another tree must clear them first, since each call
    // writes only the cells that are non-empty in its own tree
    uint64_t owner = 0;
    void *gam = nullptr;          // circulations in tree order in the near field's precision, n
    double2 *stage = nullptr;     // n: the velocities in tree order before the permutation to user order
    double2 *near = nullptr;      // near-field (u, v) per sorted particle, n
    double2 *mp_d = nullptr, *lo_d = nullptr;  // FP64 levels
    float2 *mp_f = nullptr, *lo_f = nullptr;   // FP32 levels
    // backward pass
    double2 *adj = nullptr;       // per sorted particle: adjoint charge q (sorted order)
    double4 *bwd_near = nullptr;  // per sorted particle: near sums of Phi (2) and A (2)
    double *bwd_b = nullptr;      // per sorted particle: near sum of B
    double2 *mp2_d = nullptr, *lo2_d = nullptr;  // mp2_* = mp_* (the charges q reuse the multipoles)
    float2 *mp2_f = nullptr, *lo2_f = nullptr;
    void *rec2 = nullptr;         // adjoint charges q in FP32 for the mixed near field
    double4 *bwd_src = nullptr;   // per sorted particle: near sums of the source-position terms
    // One region for the per-particle sums of either call: the forward's mutual near-field
    // slots (9 x n float2 or double2) or the adjoint's near sums (bwd_near, bwd_b, bwd_src),
    // never live in the same call.
    void *sums = nullptr;
    size_t sums_bytes = 0;
    void *slots = nullptr;        // = sums
};

}  // namespace fmm

struct fmm_tree {
    int64_t n = 0;
    bool pooled = false;  // tree arrays from the stream-ordered pool (the device build)
    int depth = 0;
    double x0 = 0, y0 = 0, side = 1;
    int device = 0;
    int num_cus = 256;   // compute units of the device
    int lc = 3;          // coarse-level cutoff L_c
    int schedule = 2;    // 0 overlap, 1 serial, 2 by the cost model (FMM_OPT_SCHEDULE)
    int near_mutual = 1; // pairs of dense leaves evaluated once for both particles
    int dense_leaf = 32; // a leaf with at least this many particles is dense
    int near_occupancy = -1; // cap on forward near-field wavefronts per SIMD beside the far field
                             // (0: none, -1: chosen per call from the cost model)
    int occupancy_in_use = 0; // the cap of the current call (0 when serialised)
    int timing = 0;
    int validate = 0;    // FMM_OPT_VALIDATE: check circulations (and dL/du) for NaN / Inf first
    std::atomic<int> busy{0};
    // the tree's arrays were released by a rebuild that failed after the position checks:
    // only fmm_rebuild_tree and fmm_destroy_tree accept the handle
    bool released = false;

    // host statistics
    int64_t p2p_pairs = 0, m2l_pairs = 0, nonempty_leaves = 0, max_leaf = 0;
    int64_t nunits = 0;
    std::vector<int64_t> list_off;  // per level l: offset into d_lists; list_len[l] entries
    std::vector<int64_t> list_len;
    std::vector<int64_t> class_off; // per level l: 4 entries, start of each parity class inside the level list

    // device tree arrays
    int *d_perm = nullptr;        // sorted slot -> user index
    // Two-pass permutation of the circulations into sorted order through a staging array
    // cut into buckets of 2^stage_shift consecutive sorted slots (at most kStageBuckets):
    int stage_shift = 0;
    int *d_gpos1 = nullptr;       // user index -> staging slot (inside a bucket: by user index)
    int *d_gpos2 = nullptr;       // sorted slot -> staging slot of its user index
    double *d_st1 = nullptr;      // staging array, n FP64
    int *d_leaf_of = nullptr;     // sorted slot -> leaf Morton index
    double2 *d_xy = nullptr;      // sorted positions
    int *d_leaf_start = nullptr;  // CSR over Morton-ordered leaves, 4^L + 1
    int *d_counts = nullptr;      // particles per cell, all levels, global cell index
    int *d_lists = nullptr;       // non-empty cells per level (levels 2..L), parity-grouped
    int4 *d_units = nullptr;      // P2P work units {leaf, first, count, log2 lanes per target}
    // near-field plan of the mutual form (see build_near_plan)
    int64_t nunits_tc = 0, nmut = 0, nnear_work = 0;
    int64_t mutual_pairs = 0;     // ordered pairs (i != j) evaluated by the mutual items
    int4 *d_near_work = nullptr;  // mutual items and target-centric units, heaviest first
    uint16_t *d_leaf_mask = nullptr; // per leaf: bit d slot d written, bit 9 target-centric part
    int *d_tile_start = nullptr;  // per leaf: index of its first 64-particle tile, 4^L + 1
    float4 *d_tile_box = nullptr; // per tile: {xmin, ymin, xmax, ymax} in leaf units about the leaf centre
    int *d_flag = nullptr;        // result of the input check (FMM_OPT_VALIDATE)
    // leaf-unit coordinates xi = (z - c_leaf)/w_L of the sorted particles, float2 [0] and
    // double2 [1], each made on the first evaluation in that precision
    void *d_pos[2] = {nullptr, nullptr};

    hipStream_t own_side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    const fmm::Tables *tabs = nullptr;  // shared, never freed by the tree
    // evaluation workspace, shared by the trees of fmm_share_workspace (freed with the last)
    std::shared_ptr<fmm::Workspace> wsp = std::make_shared<fmm::Workspace>();
    uint64_t serial = 0;  // unique per tree of the process
    std::vector<std::array<hipEvent_t, fmm::kNumEvents>> pending_timing;
};

namespace fmm {

// Outputs of an adjoint call, in user order (device pointers, each may be null):
//   dg   dL/dGamma, added to the array when acc_g (else written);
//   dxe  dL/dx at the evaluation points, dxs dL/dx of the sources (written);
//   dxy  their sum, the derivative for particles moving as both, plus lam (when given: the
//        identity part of a transport stage x + h u(x)), added to the array when acc_xy.
// The cotangent is scaled before the sums, so every part but lam carries that scale.
struct AdjointOut {
    double *dg = nullptr, *dxe = nullptr, *dxs = nullptr, *dxy = nullptr;
    const double *lam = nullptr;
    int acc_g = 0, acc_xy = 0;
};

// Launch parameters shared by the forward and backward far-field chains.
struct FarArgs {
    const fmm_tree *t;
    int p;
    int split;                 // last FP64 level
    int lc;                    // coarse cutoff actually used (<= depth)
    double2 *mp_d, *lo_d;      // FP64 storage (levels 0..split)
    float2 *mp_f, *lo_f;       // FP32 storage (levels split+1..L)
    const void *pos;           // the tree's leaf-unit coordinates in the records' precision (or null)
    const void *gam;           // circulations in tree order in that precision (null: P2M reads the staging array)
    int rec_is_double;
    int charge_kind;           // 0: real Gamma in rec.z -> c = -i Gamma/(2 pi); 1: complex q from adj array
    const double2 *adj;        // complex charges in sorted order (charge_kind 1)
    int coarse_threads = 1024; // workgroup size of the coarse-level kernel (256 or 1024)
};

// Launchers (kernels.hip).  All are asynchronous on `s`.
// Stages 1-3 on the device (tree_build.hip); the near-field plan from the device leaf
// offsets (used by both builds).  FMM_* status; err / bad_index describe a failure.
// after_checks (if set) runs once the positions have passed their checks (inside the
// root cell, finite), before the sorted arrays are allocated: a rebuild releases the old
// tree's arrays there.
int build_tree_device(fmm_tree *t, const double *xy, const double *root_box, hipStream_t s, std::string &err,
                      int64_t &bad_index, const std::function<void()> &after_checks = {});
int build_near_plan_device(fmm_tree *t, hipStream_t s, std::string &err);

// Pass 1 of the circulations into tree order (the staging array, all P2M needs), then
// pass 2 with the near-field records.
void launch_stage_in(const fmm_tree *t, const double *gamma, hipStream_t s);
void launch_pack(const fmm_tree *t, int is_double, void *gam, hipStream_t s);
// The tree's leaf-unit coordinates (float2 or double2, n) into pos.
void launch_leaf_coords(const fmm_tree *t, int is_double, void *pos, hipStream_t s);
void launch_p2p_forward(const fmm_tree *t, const void *pos, const void *gam, int is_double, double alpha,
                        double2 *near, void *slots, hipStream_t s);
// Stages 4-7 (P2M, M2M, M2L, L2L), or 5-7 without P2M when it was launched on its own.
void launch_far_chain(const FarArgs &a, hipStream_t s, bool with_p2m = true);
void launch_p2m(const FarArgs &a, hipStream_t s);
// uv alone is written through `stage` (a buffer of n double2); with base, uv = base + h u.
void launch_finalize(const fmm_tree *t, const FarArgs &a, const double2 *near, const void *slots, int slots_double,
                     double alpha, double *uv, double *uv_near, double *uv_far, void *stage, const double *base,
                     double h, hipStream_t s);

// Backward
// The two passes between user and sorted order through bucket staging windows (gpos1,
// gpos2 and the shift of a sorted order): rows of one or two doubles from user order into
// their staging slots, and staged double2 rows out to user order (uv = base + h row with
// base, else the row).
void launch_stage_rows(int64_t n, int shift, const int *gpos1, const double *src, double *st, hipStream_t s);
void launch_stage_rows2(int64_t n, int shift, const int *gpos1, const double2 *src, double2 *st, hipStream_t s);
void launch_gather_rows(int64_t n, const int *gpos1, const double2 *staged, double *uv, const double *base, double h,
                        hipStream_t s);
void launch_pack_adjoint(const fmm_tree *t, const double *dl_duv, double scale, double2 *adj, void *qt, int is_double,
                         double2 *staging, hipStream_t s);
void launch_p2p_backward(const fmm_tree *t, const void *pos, const void *gam, const void *qv, int is_double,
                         double alpha, double4 *out_pa, double *out_b, double4 *out_src, hipStream_t s);
void launch_finalize_backward(const fmm_tree *t, const FarArgs &fc, const FarArgs &fq, const double4 *near_pa,
                              const double *near_b, const double2 *adj, const double4 *near_src, int is_double,
                              double alpha, const AdjointOut &out, double *stage_g, double *stage_x,
                              double *stage_s, hipStream_t s);

// Lowest index k of the n groups of `stride` doubles at a (device) that holds a NaN or an
// infinity, or -1 in bad; flag is a device int of the caller.  Synchronises s.
hipError_t find_nonfinite(const double *a, int64_t n, int stride, int *flag, hipStream_t s, int64_t &bad);

// Tables (host generation + upload), kernels.hip
int upload_tables(Tables &tb, int p, std::string &err);
void free_tables(Tables &tb);
// The tables of p-term expansions on a device (the current one): built on first use, shared
// by every tree of the process and kept until it ends.  Returns 0, -2 (no memory) or -3;
// with create false, -5 when they do not exist yet (nothing is allocated).
int shared_tables(int device, int p, const Tables **out, std::string &err, bool create = true);

// The library's static device workspace (fmm_velocity_noalloc): its address on the
// current device (looked up once per device) and its size in bytes.  hipError_t status.
constexpr size_t kStaticWorkspaceBytes = size_t(128) << 20;
int static_workspace(int device, char **base);
// Zero `bytes` (a multiple of 8) at p with a kernel (no memset node, no allocation).
void launch_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace fmm
