// Test driver (CPU): the library's host tree build (paper_1008_2410_amd/csrc/host_tree.cpp,
// stages 1-3 of Fig. fmmStages) on seeded inputs, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py, every array checked against
// definitions restated here: binning by floor and clamp, the sorted order, the staging
// permutation, tiles and their boxes, cell counts and lists, the near-field pair count
// (sum over leaves T of n_T times the particles of T's 3x3 neighbourhood, minus n), the
// work units; and the error returns for a non-finite position and a particle outside the
// root cell.  Prints one line per case and exits non-zero on the first mismatch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../include/fmm2d.h"
#include "../paper_1008_2410_amd/csrc/host_tree.h"
#include "../paper_1008_2410_amd/csrc/morton.h"

using namespace fmm;

static int g_fail = 0;
#define CHECK(cond)                                                                      \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::printf("  FAILED %s (line %d)\n", #cond, __LINE__);                     \
            g_fail = 1;                                                                  \
            return;                                                                      \
        }                                                                                \
    } while (0)

static void check_tree(const char *name, const std::vector<double> &xy, int depth, const double *root)
{
    const int64_t n = (int64_t)xy.size() / 2;
    UniformHostTree t;
    int64_t bad = -1;
    std::string err;
    const int rc = build_host_tree(xy.data(), n, depth, root, t, bad, err);
    std::printf("%s: n=%lld depth=%d rc=%d\n", name, (long long)n, depth, rc);
    CHECK(rc == FMM_OK);
    const int nside = 1 << depth;
    const int64_t nleaf = int64_t(1) << (2 * depth);
    const double w = t.side / nside;
    // binning of every particle by its definition
    std::vector<int> leaf_of_user(n);
    for (int64_t i = 0; i < n; ++i) {
        int c[2];
        for (int d = 0; d < 2; ++d) {
            const double v = (xy[2 * i + d] - (d ? t.y0 : t.x0)) / w;
            CHECK(v >= 0.0 && v <= nside);
            c[d] = std::min((int)std::floor(v), nside - 1);
        }
        leaf_of_user[i] = (int)morton_encode((uint32_t)c[0], (uint32_t)c[1]);
    }
    // the sorted order: a permutation, grouped by leaf in Morton order
    CHECK((int64_t)t.perm.size() == n && (int64_t)t.leaf_of.size() == n);
    std::vector<int> seen(n, 0);
    for (int64_t k = 0; k < n; ++k) {
        const int u = t.perm[k];
        CHECK(u >= 0 && u < n && !seen[u]);
        seen[u] = 1;
        CHECK(t.leaf_of[k] == leaf_of_user[u]);
        CHECK(k == 0 || t.leaf_of[k - 1] <= t.leaf_of[k]);
        CHECK(t.xy[k].x == xy[2 * u] && t.xy[k].y == xy[2 * u + 1]);
    }
    // leaf offsets
    CHECK((int64_t)t.leaf_start.size() == nleaf + 1 && t.leaf_start[0] == 0 && t.leaf_start[nleaf] == n);
    for (int64_t c = 0; c < nleaf; ++c)
        for (int k = t.leaf_start[c]; k < t.leaf_start[c + 1]; ++k) CHECK(t.leaf_of[k] == (int)c);
    // staging permutation: gpos1 a bijection onto [0, n), gpos2 = gpos1 o perm, buckets of
    // 2^shift sorted slots, inside a bucket by user index
    std::vector<int> hit(n, 0);
    for (int64_t u = 0; u < n; ++u) {
        CHECK(t.gpos1[u] >= 0 && t.gpos1[u] < n && !hit[t.gpos1[u]]);
        hit[t.gpos1[u]] = 1;
    }
    for (int64_t k = 0; k < n; ++k) {
        CHECK(t.gpos2[k] == t.gpos1[t.perm[k]]);
        CHECK((t.gpos2[k] >> t.stage_shift) == (int)(k >> t.stage_shift));
    }
    // tiles of 64 particles per leaf; boxes contain their particles (leaf units about the centre)
    CHECK((int64_t)t.tile_start.size() == nleaf + 1);
    for (int64_t c = 0; c < nleaf; ++c) {
        const int cnt = t.leaf_start[c + 1] - t.leaf_start[c];
        CHECK(t.tile_start[c + 1] - t.tile_start[c] == (cnt + 63) / 64);
        const double cx = t.x0 + (morton_x((uint32_t)c) + 0.5) * w, cy = t.y0 + (morton_y((uint32_t)c) + 0.5) * w;
        for (int k = t.leaf_start[c]; k < t.leaf_start[c + 1]; ++k) {
            const HostF4 b = t.tile_box[t.tile_start[c] + (k - t.leaf_start[c]) / 64];
            const double xl = (t.xy[k].x - cx) / w, yl = (t.xy[k].y - cy) / w;
            CHECK(b.x <= xl && xl <= b.z && b.y <= yl && yl <= b.w);
        }
    }
    // counts of every level, lists of non-empty cells by parity class
    for (int l = 0; l <= depth; ++l) {
        int64_t sum = 0;
        for (int64_t c = 0; c < (int64_t(1) << (2 * l)); ++c) sum += t.counts[level_base(l) + c];
        CHECK(sum == n);
    }
    for (int l = 2; l <= depth; ++l) {
        int64_t nonempty = 0;
        for (int64_t c = 0; c < (int64_t(1) << (2 * l)); ++c) nonempty += t.counts[level_base(l) + c] > 0;
        CHECK(t.list_len[l] == nonempty);
        for (int64_t k = 0; k < t.list_len[l]; ++k) {
            const int c = t.lists[t.list_off[l] + k];
            CHECK(t.counts[level_base(l) + c] > 0);
            const int par = c & 3;
            CHECK(k >= t.class_off[4 * l + par]);
            CHECK(par == 3 || k < t.class_off[4 * l + par + 1]);
        }
    }
    // near-field pairs by the direct-work sum
    int64_t pairs = 0, maxleaf = 0, nonempty = 0;
    for (int64_t c = 0; c < nleaf; ++c) {
        const int64_t nt = t.leaf_start[c + 1] - t.leaf_start[c];
        if (!nt) continue;
        ++nonempty;
        maxleaf = std::max(maxleaf, nt);
        const int x = (int)morton_x((uint32_t)c), y = (int)morton_y((uint32_t)c);
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int sx = x + dx, sy = y + dy;
                if (sx < 0 || sy < 0 || sx >= nside || sy >= nside) continue;
                const uint32_t S = morton_encode((uint32_t)sx, (uint32_t)sy);
                pairs += nt * (t.leaf_start[S + 1] - t.leaf_start[S]);
            }
    }
    CHECK(t.p2p_pairs == pairs - n && t.max_leaf == maxleaf && t.nonempty_leaves == nonempty);
    // work units cover every particle once, each inside its leaf, at most 64
    std::vector<int> cover(n, 0);
    for (const HostI4 &u : t.units) {
        CHECK(u.z >= 1 && u.z <= 64 && (1 << u.w) >= u.z && (u.w == 0 || (1 << (u.w - 1)) < u.z));
        CHECK(u.y >= t.leaf_start[u.x] && u.y + u.z <= t.leaf_start[u.x + 1]);
        for (int k = u.y; k < u.y + u.z; ++k) ++cover[k];
    }
    for (int64_t k = 0; k < n; ++k) CHECK(cover[k] == 1);
}

static void check_error(const char *name, const std::vector<double> &xy, int depth, const double *root, int want,
                        int64_t want_bad)
{
    UniformHostTree t;
    int64_t bad = -1;
    std::string err;
    const int rc = build_host_tree(xy.data(), (int64_t)xy.size() / 2, depth, root, t, bad, err);
    std::printf("%s: rc=%d bad=%lld (%s)\n", name, rc, (long long)bad, err.c_str());
    CHECK(rc == want && bad == want_bad);
}

int main()
{
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::normal_distribution<double> N(0.0, 1.0);
    const double unit[3] = {0.0, 0.0, 1.0};
    for (int depth : {1, 2, 4, 6}) {
        std::vector<double> xy(2 * 20000);
        for (double &v : xy) v = U(rng);
        check_tree(("uniform, depth " + std::to_string(depth)).c_str(), xy, depth, unit);
    }
    {  // clustered patches, bounding square, dense leaves of several tiles
        std::vector<double> xy(2 * 60000);
        for (size_t i = 0; i < xy.size() / 2; ++i) {
            const double c = (i % 3) * 0.3 + 0.2;
            xy[2 * i] = c + 0.01 * N(rng);
            xy[2 * i + 1] = 0.5 + 0.02 * N(rng);
        }
        check_tree("patches, bounding square, depth 7", xy, 7, nullptr);
    }
    {  // all in one leaf; one particle; particles on the top and right edges and on internal edges
        std::vector<double> xy(2 * 300);
        for (double &v : xy) v = 0.5 + 0.01 * U(rng);
        check_tree("one leaf", xy, 5, unit);
        check_tree("one particle", {0.3, 0.7}, 3, unit);
        check_tree("edges", {1.0, 1.0, 0.5, 0.5, 0.25, 0.75, 0.0, 1.0, 0.5, 0.5, 0.1, 0.9}, 3, unit);
        check_tree("coincident, bounding square", {0.25, 0.25, 0.25, 0.25}, 4, nullptr);
    }
    check_error("NaN position", {0.1, 0.2, 0.3, std::nan("")}, 3, unit, FMM_EINVAL, 1);
    check_error("outside the root cell", {0.1, 0.2, 1.5, 0.2, 2.0, 0.3}, 3, unit, FMM_ERANGE, 1);
    std::printf(g_fail ? "host tree checks FAILED\n" : "host tree checks passed\n");
    return g_fail;
}
