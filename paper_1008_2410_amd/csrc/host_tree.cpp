// Stages 1-3 of Fig. fmmStages on the host: the reference build of the uniform tree (see
// host_tree.h).  The device build (tree_build.hip) produces the same arrays.
#include "host_tree.h"

#include <algorithm>
#include <cmath>
#include <numeric>

#include "../../include/fmm2d.h"
#include "morton.h"

namespace fmm {

void host_staging(const std::vector<int> &perm, int &shift, std::vector<int> &gpos1, std::vector<int> &gpos2)
{
    // bucket = sorted slot >> shift, ordered by user index inside a bucket; a bucket's
    // segment of the staging array is the slot range of the bucket itself
    const int64_t n = (int64_t)perm.size();
    shift = kStageShiftMin;
    while ((((n - 1) >> shift) + 1) > kStageBuckets) ++shift;
    gpos1.assign((size_t)n, 0);
    gpos2.assign((size_t)n, 0);
    std::vector<int> inv((size_t)n);
    for (int64_t k = 0; k < n; ++k) inv[perm[k]] = (int)k;
    std::vector<int64_t> fill(kStageBuckets);
    for (int64_t b = 0; b < kStageBuckets; ++b) fill[b] = b << shift;
    for (int64_t u = 0; u < n; ++u) gpos1[u] = (int)fill[inv[u] >> shift]++;
    for (int64_t k = 0; k < n; ++k) gpos2[k] = gpos1[perm[k]];
}

int build_host_tree(const double *xy, int64_t n, int depth, const double *root_box, UniformHostTree &t, int64_t &bad,
                    std::string &err)
{
    bad = -1;
    const double *h = xy;
    for (int64_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(h[i])) {
            bad = i / 2;
            err = "non-finite particle position";
            return FMM_EINVAL;
        }
    if (root_box) {
        t.x0 = root_box[0];
        t.y0 = root_box[1];
        t.side = root_box[2];
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
        t.x0 = xmin;
        t.y0 = ymin;
        t.side = side * (1.0 + 1.0 / 1048576.0);
    }
    const int L = depth;
    const int nside = 1 << L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const double w = t.side / (double)nside;

    // Stage 2: leaf of each particle, floor binning clamped at the top edge; and a
    // sub-leaf key (Morton index in a 64 x 64 grid over the leaf) that orders the
    // particles inside a leaf so that 64-particle tiles are spatially compact.
    std::vector<uint32_t> key((size_t)n);
    std::vector<uint16_t> sub((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[2], f[2];
        for (int d = 0; d < 2; ++d) {
            const double v = (h[2 * i + d] - (d ? t.y0 : t.x0)) / w;
            if (!(v >= 0.0) || v > (double)nside) {
                bad = i;
                err = "particle " + std::to_string(i) + " lies outside the root cell";
                return FMM_ERANGE;
            }
            int64_t k = (int64_t)std::floor(v);
            c[d] = (uint32_t)std::min<int64_t>(k, nside - 1);
            f[d] = (uint32_t)std::min<int64_t>((int64_t)std::floor((v - c[d]) * 64.0), 63);
        }
        key[i] = morton_encode(c[0], c[1]);
        sub[i] = (uint16_t)morton_encode(f[0], f[1]);
    }
    // Stable counting sort by leaf Morton key.
    std::vector<int> &leaf_start = t.leaf_start;
    leaf_start.assign((size_t)nleaf + 1, 0);
    for (int64_t i = 0; i < n; ++i) leaf_start[key[i] + 1]++;
    for (int64_t c = 0; c < nleaf; ++c) leaf_start[c + 1] += leaf_start[c];
    std::vector<int> &perm = t.perm, &leaf_of = t.leaf_of;
    perm.assign((size_t)n, 0);
    leaf_of.assign((size_t)n, 0);
    {
        std::vector<int> fill(leaf_start.begin(), leaf_start.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            const int pos = fill[key[i]]++;
            perm[pos] = (int)i;
            leaf_of[pos] = (int)key[i];
        }
        // inside each leaf: by sub-leaf key, ties by user index
        for (int64_t c = 0; c < nleaf; ++c)
            if (leaf_start[c + 1] - leaf_start[c] > 1)
                std::stable_sort(perm.begin() + leaf_start[c], perm.begin() + leaf_start[c + 1],
                                 [&](int a, int b) { return sub[a] < sub[b]; });
    }
    host_staging(perm, t.stage_shift, t.gpos1, t.gpos2);
    std::vector<HostD2> &xys = t.xy;
    xys.assign((size_t)n, HostD2{});
    for (int64_t k = 0; k < n; ++k) {
        xys[k].x = h[2 * (size_t)perm[k]];
        xys[k].y = h[2 * (size_t)perm[k] + 1];
    }
    // 64-particle tiles of each leaf and their bounding boxes in leaf units about the
    // leaf centre, rounded outwards to FP32.
    std::vector<int> &tile_start = t.tile_start;
    tile_start.assign((size_t)nleaf + 1, 0);
    for (int64_t c = 0; c < nleaf; ++c)
        tile_start[c + 1] = tile_start[c] + (leaf_start[c + 1] - leaf_start[c] + 63) / 64;
    std::vector<HostF4> &tile_box = t.tile_box;
    tile_box.assign((size_t)tile_start[nleaf], HostF4{});
    for (int64_t c = 0; c < nleaf; ++c) {
        const double cx = t.x0 + (morton_x((uint32_t)c) + 0.5) * w;
        const double cy = t.y0 + (morton_y((uint32_t)c) + 0.5) * w;
        for (int b = leaf_start[c], tt = tile_start[c]; b < leaf_start[c + 1]; b += 64, ++tt) {
            double xmin = 1e300, ymin = 1e300, xmax = -1e300, ymax = -1e300;
            for (int k = b; k < std::min(b + 64, leaf_start[c + 1]); ++k) {
                const double xl = (xys[k].x - cx) / w, yl = (xys[k].y - cy) / w;
                xmin = std::min(xmin, xl);
                xmax = std::max(xmax, xl);
                ymin = std::min(ymin, yl);
                ymax = std::max(ymax, yl);
            }
            HostF4 bx;
            bx.x = std::nextafter((float)xmin, -INFINITY);
            bx.y = std::nextafter((float)ymin, -INFINITY);
            bx.z = std::nextafter((float)xmax, INFINITY);
            bx.w = std::nextafter((float)ymax, INFINITY);
            tile_box[tt] = bx;
        }
    }
    // Occupancy of every cell of every level (global cell index).
    std::vector<int> &counts = t.counts;
    counts.assign((size_t)level_base(L + 1), 0);
    for (int64_t c = 0; c < nleaf; ++c) counts[level_base(L) + c] = leaf_start[c + 1] - leaf_start[c];
    for (int l = L - 1; l >= 0; --l)
        for (int64_t c = 0; c < (int64_t(1) << (2 * l)); ++c) {
            const int *ch = &counts[level_base(l + 1) + 4 * c];
            counts[level_base(l) + c] = ch[0] + ch[1] + ch[2] + ch[3];
        }
    // Non-empty cells of levels 2..L, grouped by parity class (Morton & 3).
    std::vector<int> &lists = t.lists;
    lists.clear();
    t.list_off.assign(L + 1, 0);
    t.list_len.assign(L + 1, 0);
    t.class_off.assign(4 * (L + 1), 0);
    for (int l = 2; l <= L; ++l) {
        t.list_off[l] = (int64_t)lists.size();
        const int64_t nc = int64_t(1) << (2 * l);
        for (int par = 0; par < 4; ++par) {
            t.class_off[4 * l + par] = (int64_t)lists.size() - t.list_off[l];
            for (int64_t c = par; c < nc; c += 4)
                if (counts[level_base(l) + c] > 0) lists.push_back((int)c);
        }
        t.list_len[l] = (int64_t)lists.size() - t.list_off[l];
    }
    // Statistics: pairs (section "Complexity Estimates" direct work), M2L pairs.
    auto leaf_count = [&](int x, int y) -> int64_t {
        if (x < 0 || y < 0 || x >= nside || y >= nside) return 0;
        return counts[level_base(L) + morton_encode((uint32_t)x, (uint32_t)y)];
    };
    int64_t pairs = 0, nonempty = 0, maxleaf = 0;
    // Stage 9 work units: target chunks of <= 64 in each non-empty leaf.
    std::vector<HostI4> units;
    std::vector<int64_t> cost;
    for (int64_t c = 0; c < nleaf; ++c) {
        const int nt = leaf_start[c + 1] - leaf_start[c];
        if (nt == 0) continue;
        ++nonempty;
        maxleaf = std::max<int64_t>(maxleaf, nt);
        const int x = (int)morton_x((uint32_t)c), y = (int)morton_y((uint32_t)c);
        int64_t nsrc = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) nsrc += leaf_count(x + dx, y + dy);
        pairs += (int64_t)nt * nsrc;
        for (int c0 = 0; c0 < nt; c0 += 64) {
            const int cnt = std::min(64, nt - c0);
            int logtp = 0;
            while ((1 << logtp) < cnt) ++logtp;
            const int kstride = 64 >> logtp;
            HostI4 u;
            u.x = (int)c;
            u.y = leaf_start[c] + c0;
            u.z = cnt;
            u.w = logtp;
            units.push_back(u);
            cost.push_back((nsrc + kstride - 1) / kstride);
        }
    }
    t.p2p_pairs = pairs - n;
    t.nonempty_leaves = nonempty;
    t.max_leaf = maxleaf;
    int64_t m2l = 0;
    for (int l = 2; l <= L; ++l) {
        const int n1 = 1 << l;
        const int *lst = lists.data() + t.list_off[l];
        for (int64_t k = 0; k < t.list_len[l]; ++k) {
            const int tx = (int)morton_x((uint32_t)lst[k]), ty = (int)morton_y((uint32_t)lst[k]);
            const int qx = tx & 1, qy = ty & 1;
            for (int dy = -2 - qy; dy <= 3 - qy; ++dy)
                for (int dx = -2 - qx; dx <= 3 - qx; ++dx) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                    const int sx = tx + dx, sy = ty + dy;
                    if (sx < 0 || sy < 0 || sx >= n1 || sy >= n1) continue;
                    if (counts[level_base(l) + morton_encode((uint32_t)sx, (uint32_t)sy)] > 0) ++m2l;
                }
        }
    }
    t.m2l_pairs = m2l;
    // Heaviest units first so the tail of the launch is short.
    std::vector<int64_t> order(units.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    t.units.resize(units.size());
    for (size_t k = 0; k < order.size(); ++k) t.units[k] = units[order[k]];

    return FMM_OK;
}

}  // namespace fmm
