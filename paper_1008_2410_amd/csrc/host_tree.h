// The uniform tree (stages 1-3 of Fig. fmmStages) built on the host: plain C++ with no
// device types, so that the same code serves the library's host build
// (fmm_build_tree_host, the reference the device build is checked against) and a
// sanitizer build on the CPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fmm {

// Layout-compatible with double2, float4 and int4 of the device code.
struct HostD2 {
    double x, y;
};
struct HostF4 {
    float x, y, z, w;
};
struct HostI4 {
    int x, y, z, w;
};

// Staging buckets of the two-pass permutations between user and sorted order: at least
// 2^kStageShiftMin sorted slots per bucket and at most kStageBuckets buckets.  Small
// windows (2^14 slots: 256 KiB of double2 outputs) keep the random writes of a pass inside
// the L2 of the XCD that makes them until their lines are whole.
constexpr int kStageShiftMin = 14;
constexpr int kStageBucketsLog2 = 10;
constexpr int kStageBuckets = 1 << kStageBucketsLog2;

// Staging slots of a sorted order perm (sorted slot -> user index): the shift, gpos1
// (user index -> staging slot) and gpos2 (sorted slot -> staging slot of its user index).
void host_staging(const std::vector<int> &perm, int &shift, std::vector<int> &gpos1, std::vector<int> &gpos2);

struct UniformHostTree {
    double x0 = 0, y0 = 0, side = 1;  // root cell
    int stage_shift = 0;
    std::vector<int> perm;        // sorted slot -> user index
    std::vector<int> leaf_of;     // sorted slot -> leaf Morton index
    std::vector<int> gpos1;       // user index -> staging slot
    std::vector<int> gpos2;       // sorted slot -> staging slot of its user index
    std::vector<HostD2> xy;       // sorted positions
    std::vector<int> leaf_start;  // CSR over Morton-ordered leaves, 4^L + 1
    std::vector<int> tile_start;  // per leaf: first 64-particle tile, 4^L + 1
    std::vector<HostF4> tile_box; // per tile: {xmin, ymin, xmax, ymax} in leaf units, rounded outwards
    std::vector<int> counts;      // particles per cell, all levels, global cell index
    std::vector<int> lists;       // non-empty cells of levels 2..L, grouped by parity class
    std::vector<int64_t> list_off, list_len, class_off;
    std::vector<HostI4> units;    // near-field work units {leaf, first, count, log2 lanes}, heaviest first
    int64_t p2p_pairs = 0, m2l_pairs = 0, nonempty_leaves = 0, max_leaf = 0;
};

// Build the tree of depth L over n positions xy (host, n x 2, user order) in the root cell
// root_box {x0, y0, side} or, when NULL, the bounding square.  Returns 0, or FMM_EINVAL
// (non-finite position) / FMM_ERANGE (outside the root cell) with bad = the particle and
// err a message; std::bad_alloc propagates.
int build_host_tree(const double *xy, int64_t n, int depth, const double *root_box, UniformHostTree &t, int64_t &bad,
                    std::string &err);

}  // namespace fmm
