// Stages 1-3 of the adaptive tree on the GPU: keys on the finest grid, the stable sort,
// the cells level by level (a cell splits while it holds more than max_leaf particles
// and lies above max_depth), the same-level neighbours of every cell, the U, V, W and X
// lists, the leaves in sorted order with their 64-particle tiles and tile boxes, and
// the near-field plan.
//
// The arrays equal those of the host build (adaptive.cpp) element for element: cells
// are numbered level by level, in Morton order inside a level; every list is filled by
// the host build's traversal in the host build's order; tile boxes use the same double
// arithmetic (not contracted); and the sorts are stable on the same keys.  So the two
// builds give bit-identical evaluations.
//
// Neighbours come from the tree itself: the cell at (ix + dx, iy + dy) on level l is a
// child of the parent or of one of the parent's same-level neighbours, so each cell's
// eight neighbour slots follow from its parent's, level by level, without a search.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/fmm2d_adaptive.h"
#include "adaptive_internal.h"
#include "build_prims.h"
#include "fmm_internal.h"

namespace fmm {

namespace {

// Depth of the explicit stack of the U/W walk: it starts with one cell and each step
// that opens a cell replaces it by at most four children, so at most 1 + 3 * 15 entries.
constexpr int kWalkStack = 48;

// Slot of the same-level neighbour at (dx, dy) in {-1, 0, 1}^2 \ {(0, 0)}: the
// directions in the order dy = -1..1, dx = -1..1 with the centre left out (the order in
// which the host build visits neighbours).
__host__ __device__ inline int nb_slot(int dx, int dy)
{
    const int d = 3 * (dy + 1) + (dx + 1);
    return d < 4 ? d : d - 1;
}

__device__ inline int quadrant(const int4 &c, int q) { return q == 0 ? c.x : q == 1 ? c.y : q == 2 ? c.z : c.w; }

// Closed squares of cells a and b ({level, ix, iy, .}) intersect; in units of the
// finest cell.
__device__ inline bool touch(const int4 &a, const int4 &b, int L)
{
    const int64_t sa = int64_t(1) << (L - a.x), sb = int64_t(1) << (L - b.x);
    return a.y * sa <= (b.y + 1) * sb && b.y * sb <= (a.y + 1) * sa && a.z * sa <= (b.z + 1) * sb &&
           b.z * sb <= (a.z + 1) * sa;
}

// Finest-grid cell of every particle (floor binning, clamped at the top edge), as the
// host build: key = its Morton index, value = user index.  flags bit 0: outside the root
// cell, bit 1: non-finite; *first_bad: the lowest such index.
__global__ __launch_bounds__(256) void ak_keys(const double2 *__restrict__ xy, int64_t n, double x0, double y0,
                                                double w, int nside, uint64_t *__restrict__ key,
                                                uint32_t *__restrict__ val, int *__restrict__ flags,
                                                unsigned long long *__restrict__ first_bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 z = xy[i];
    uint32_t c[2] = {0, 0};
    bool bad = false;
    if (!isfinite(z.x) || !isfinite(z.y)) {
        atomicOr(flags, 2);
        bad = true;
    } else {
        for (int d = 0; d < 2; ++d) {
            const double v = ((d ? z.y : z.x) - (d ? y0 : x0)) / w;
            if (!(v >= 0.0) || v > (double)nside) {
                atomicOr(flags, 1);
                bad = true;
                break;
            }
            c[d] = (uint32_t)min((int64_t)floor(v), (int64_t)(nside - 1));
        }
    }
    if (bad) atomicMin(first_bad, (unsigned long long)i);
    key[i] = morton_encode(c[0], c[1]);
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void ak_sorted(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val,
                                                  const double2 *__restrict__ xy, int64_t n, int *__restrict__ perm,
                                                  uint32_t *__restrict__ skey, double2 *__restrict__ xs)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t u = val[j];
    perm[j] = (int)u;
    skey[j] = (uint32_t)key[j];
    xs[j] = xy[u];
}

__global__ void ak_root(int4 *cell, int2 *range, int *parent, int *coll, int n)
{
    cell[0] = make_int4(0, 0, 0, 0);
    range[0] = make_int2(0, n);
    parent[0] = -1;
    for (int j = 0; j < 8; ++j) coll[j] = -1;
}

// Cells [c0, c0 + m) of level l: the leaf flag; for a cell that splits, the ends of its
// four quadrants' particle ranges (stored in child until the children are numbered)
// and the number of non-empty quadrants.
__global__ __launch_bounds__(256) void ak_split(int4 *__restrict__ cell, const int2 *__restrict__ range,
                                                 int4 *__restrict__ child, const uint32_t *__restrict__ skey, int c0,
                                                 int m, int l, int L, int smax, uint32_t *__restrict__ nchild,
                                                 unsigned int *__restrict__ nsplit)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int c = c0 + i;
    const int2 r = range[c];
    int4 cc = cell[c];
    const bool split = r.y > smax && l < L;
    cc.w = split ? 0 : 1;
    cell[c] = cc;
    if (!split) {
        child[c] = make_int4(-1, -1, -1, -1);
        nchild[i] = 0;
        return;
    }
    atomicAdd(nsplit, 1u);
    const int shift = 2 * (L - l - 1);
    const uint64_t code = morton_encode((uint32_t)cc.y, (uint32_t)cc.z);
    const int end = r.x + r.y;
    int b[4];
    int lo = r.x;
    for (int q = 0; q < 3; ++q) {
        const uint64_t next = code * 4 + q + 1;  // first code of the next quadrant
        int a = lo, e = end;
        while (a < e) {
            const int mid = a + (e - a) / 2;
            if (((uint64_t)skey[mid] >> shift) < next)
                a = mid + 1;
            else
                e = mid;
        }
        b[q] = a;
        lo = a;
    }
    b[3] = end;
    uint32_t k = 0;
    int prev = r.x;
    for (int q = 0; q < 4; ++q) {
        k += b[q] > prev;
        prev = b[q];
    }
    child[c] = make_int4(b[0], b[1], b[2], b[3]);
    nchild[i] = k;
}

// Children of the split cells of level l, numbered from `base` in the order of their
// parents with quadrants ascending (Morton order on level l + 1).
__global__ __launch_bounds__(256) void ak_children(int4 *__restrict__ cell, int2 *__restrict__ range,
                                                    int *__restrict__ parent, int4 *__restrict__ child, int c0, int m,
                                                    int l, const uint32_t *__restrict__ offs, int base)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int c = c0 + i;
    const int4 cc = cell[c];
    if (cc.w) return;  // a leaf: child is already -1
    const int4 b = child[c];
    const int2 r = range[c];
    int idx = base + (int)offs[i];
    int prev = r.x;
    int ch[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int hi = quadrant(b, q);
        if (hi > prev) {
            cell[idx] = make_int4(l + 1, 2 * cc.y + (q & 1), 2 * cc.z + (q >> 1), 0);
            range[idx] = make_int2(prev, hi - prev);
            parent[idx] = c;
            ch[q] = idx++;
        } else {
            ch[q] = -1;
        }
        prev = hi;
    }
    child[c] = make_int4(ch[0], ch[1], ch[2], ch[3]);
}

// Same-level neighbours of the cells [c0, c0 + m) of level l >= 1 (slot order of nb_slot,
// -1 where there is no cell).
__global__ __launch_bounds__(256) void ak_neighbours(const int4 *__restrict__ cell, const int *__restrict__ parent,
                                                      const int4 *__restrict__ child, int *__restrict__ coll, int c0,
                                                      int m, int l)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int c = c0 + i;
    const int4 cc = cell[c];
    const int P = parent[c];
    const int nside = 1 << l, pix = cc.y >> 1, piy = cc.z >> 1;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy) continue;
            const int nx = cc.y + dx, ny = cc.z + dy;
            int r = -1;
            if (nx >= 0 && ny >= 0 && nx < nside && ny < nside) {
                const int qx = (nx >> 1) - pix, qy = (ny >> 1) - piy;
                const int PP = (!qx && !qy) ? P : coll[(int64_t)P * 8 + nb_slot(qx, qy)];
                if (PP >= 0) r = quadrant(child[PP], (nx & 1) | ((ny & 1) << 1));
            }
            coll[(int64_t)c * 8 + nb_slot(dx, dy)] = r;
        }
}

// V list of every cell: children of the parent's neighbours that do not touch it.
// Counting pass (FILL false, K + 1 counts with the last 0) and filling pass.
template <bool FILL>
__global__ __launch_bounds__(256) void ak_vlist(const int4 *__restrict__ cell, const int *__restrict__ parent,
                                                 const int4 *__restrict__ child, const int *__restrict__ coll, int K,
                                                 uint32_t *__restrict__ cnt, const int *__restrict__ off,
                                                 int *__restrict__ idx)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    if (k == K) {
        if (!FILL) cnt[K] = 0;
        return;
    }
    const int P = parent[k];
    int nv = 0;
    const int o = FILL ? off[k] : 0;
    if (P >= 0) {
        const int4 ck = cell[k];
        for (int j = 0; j < 8; ++j) {
            const int PN = coll[(int64_t)P * 8 + j];
            if (PN < 0) continue;
            const int4 ch = child[PN];
            for (int q = 0; q < 4; ++q) {
                const int d = quadrant(ch, q);
                if (d < 0) continue;
                const int4 cd = cell[d];
                if (abs(cd.y - ck.y) > 1 || abs(cd.z - ck.z) > 1) {
                    if (FILL) idx[o + nv] = d;
                    ++nv;
                }
            }
        }
    }
    if (!FILL) cnt[k] = (uint32_t)nv;
}

// U and W lists of every leaf k: k itself; then, below each same-level neighbour, the
// leaves that touch k (U) and the cells that do not touch k while their parents do (W),
// depth first with quadrants ascending; then the coarser leaves that touch k among the
// neighbours of its ancestors, nearest ancestor first.  W entries carry their owner.
template <bool FILL>
__global__ __launch_bounds__(256) void ak_uwlist(const int4 *__restrict__ cell, const int *__restrict__ parent,
                                                  const int4 *__restrict__ child, const int *__restrict__ coll, int K,
                                                  int L, uint32_t *__restrict__ ucnt, uint32_t *__restrict__ wcnt,
                                                  const int *__restrict__ uoff, const int *__restrict__ woff,
                                                  int *__restrict__ uidx, int *__restrict__ widx,
                                                  uint32_t *__restrict__ wown, int *__restrict__ err)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    if (k == K) {
        if (!FILL) ucnt[K] = wcnt[K] = 0;
        return;
    }
    const int4 ck = cell[k];
    if (!ck.w) {
        if (!FILL) ucnt[k] = wcnt[k] = 0;
        return;
    }
    int nu = 0, nw = 0;
    const int uo = FILL ? uoff[k] : 0, wo = FILL ? woff[k] : 0;
    if (FILL) uidx[uo] = k;
    ++nu;
    int st[kWalkStack];
    for (int j = 0; j < 8; ++j) {
        const int C = coll[(int64_t)k * 8 + j];
        if (C < 0) continue;
        int sp = 0;
        st[sp++] = C;
        while (sp > 0) {
            const int d = st[--sp];
            const int4 cd = cell[d];
            if (!touch(cd, ck, L)) {
                if (FILL) {
                    widx[wo + nw] = d;
                    wown[wo + nw] = (uint32_t)k;
                }
                ++nw;
                continue;
            }
            if (cd.w) {
                if (FILL) uidx[uo + nu] = d;
                ++nu;
                continue;
            }
            if (sp + 4 > kWalkStack) {  // cannot happen for depth <= 15; reported, never overrun
                atomicOr(err, 1);
                break;
            }
            const int4 ch = child[d];
            if (ch.w >= 0) st[sp++] = ch.w;
            if (ch.z >= 0) st[sp++] = ch.z;
            if (ch.y >= 0) st[sp++] = ch.y;
            if (ch.x >= 0) st[sp++] = ch.x;
        }
    }
    for (int a = parent[k]; a >= 0; a = parent[a])
        for (int j = 0; j < 8; ++j) {
            const int C = coll[(int64_t)a * 8 + j];
            if (C < 0) continue;
            const int4 cc = cell[C];
            if (cc.w && touch(cc, ck, L)) {
                if (FILL) uidx[uo + nu] = C;
                ++nu;
            }
        }
    if (!FILL) {
        ucnt[k] = (uint32_t)nu;
        wcnt[k] = (uint32_t)nw;
    }
}

// X list counts: X(d) holds every a with d in W(a).
__global__ __launch_bounds__(256) void ak_xcount(const int *__restrict__ widx, int64_t nw, uint32_t *__restrict__ xcnt)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nw) atomicAdd(&xcnt[widx[u]], 1u);
}

__global__ __launch_bounds__(256) void ak_xkeys(const int *__restrict__ widx, int64_t nw, uint64_t *__restrict__ key)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nw) key[u] = (uint64_t)widx[u];
}

// First sorted slot of every leaf gets flag 1 (flag zeroed beforehand).
__global__ __launch_bounds__(256) void ak_leaf_marks(const int4 *__restrict__ cell, const int2 *__restrict__ range, int K,
                                                      uint32_t *__restrict__ flag)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K && cell[k].w) flag[range[k].x] = 1;
}

// Leaf index (position in sorted order) of every leaf; deepest leaf level.
__global__ __launch_bounds__(256) void ak_leaf_index(const int4 *__restrict__ cell, const int2 *__restrict__ range,
                                                      int K, const uint32_t *__restrict__ e,
                                                      int *__restrict__ leaf_index, int *__restrict__ leaves,
                                                      int *__restrict__ leaf_start, unsigned int *__restrict__ deepest)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int4 c = cell[k];
    if (!c.w) {
        leaf_index[k] = -1;
        return;
    }
    const int first = range[k].x;
    const int li = (int)e[first];
    leaf_index[k] = li;
    leaves[li] = k;
    leaf_start[li] = first;
    atomicMax(deepest, (unsigned int)c.x);
}

// Leaf of every sorted particle: the leaf whose first slot is the last flagged slot <= j.
__global__ __launch_bounds__(256) void ak_leaf_of(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ e,
                                                   const int *__restrict__ leaves, int64_t n, int *__restrict__ leaf_of)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) leaf_of[j] = leaves[e[j] + flag[j] - 1];
}

__global__ void ak_set(int *p, int v) { *p = v; }

// Tiles per leaf (NL + 1 entries, the last 0).
__global__ __launch_bounds__(256) void ak_leaf_ntiles(const int *__restrict__ leaves, const int2 *__restrict__ range,
                                                       int NL, uint32_t *__restrict__ nt)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li > NL) return;
    nt[li] = li == NL ? 0u : (uint32_t)((range[leaves[li]].y + 63) / 64);
}

// First tile of every leaf cell (tile_start zeroed beforehand) and the leaf of every tile.
__global__ __launch_bounds__(256) void ak_tiles(const int *__restrict__ leaves, const int *__restrict__ leaf_tile, int NL,
                                                 int *__restrict__ tile_start, int *__restrict__ tile_leaf)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= NL) return;
    const int t0 = leaf_tile[li], t1 = leaf_tile[li + 1];
    tile_start[leaves[li]] = t0;
    for (int t = t0; t < t1; ++t) tile_leaf[t] = li;
}

// Box of every tile: {xmin, ymin, xmax, ymax} relative to (x0, y0), and in leaf widths
// about the leaf centre rounded outwards to FP32; the host build's arithmetic, with
// no fused multiply-adds.
__global__ __launch_bounds__(256) void ak_tile_box(const int *__restrict__ tile_leaf, const int *__restrict__ leaves,
                                                    const int *__restrict__ leaf_tile, const int4 *__restrict__ cell,
                                                    const int2 *__restrict__ range, const double2 *__restrict__ xs,
                                                    int64_t ntiles, double x0, double y0, double side,
                                                    double4 *__restrict__ box, float4 *__restrict__ box_leaf)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int li = tile_leaf[t];
    const int k = leaves[li];
    const int4 c = cell[k];
    const int2 r = range[k];
    const int b = r.x + 64 * (int)(t - leaf_tile[li]);
    const int e = min(b + 64, r.x + r.y);
    const double wl = side / (double)(int64_t(1) << c.x);
    const double cx = x0 + (c.y + 0.5) * wl, cy = y0 + (c.z + 0.5) * wl;
    double4 bx = make_double4(1e300, 1e300, -1e300, -1e300), bl = bx;
    for (int j = b; j < e; ++j) {
        const double2 z = xs[j];
        const double x = z.x - x0, y = z.y - y0;
        bx.x = x < bx.x ? x : bx.x;
        bx.y = y < bx.y ? y : bx.y;
        bx.z = bx.z < x ? x : bx.z;
        bx.w = bx.w < y ? y : bx.w;
        const double xl = (z.x - cx) / wl, yl = (z.y - cy) / wl;
        bl.x = xl < bl.x ? xl : bl.x;
        bl.y = yl < bl.y ? yl : bl.y;
        bl.z = bl.z < xl ? xl : bl.z;
        bl.w = bl.w < yl ? yl : bl.w;
    }
    box[t] = bx;
    box_leaf[t] = make_float4(nextafterf((float)bl.x, -INFINITY), nextafterf((float)bl.y, -INFINITY),
                              nextafterf((float)bl.z, INFINITY), nextafterf((float)bl.w, INFINITY));
}

// Statistics gathered by the plan's counting pass.
enum { kStPairs = 0, kStMutualPairs, kStMutualItems, kStUnits, kStMaxCost, kStCount };

// Near-field plan, per leaf in sorted order: target-centric units (one per 64-particle
// tile) when some of U is left to them, then for a dense leaf its mutual item with
// itself and with each dense same-level leaf at (1, 0), (-1, 1), (0, 1), (1, 1); the slot
// mask of every leaf.  Counting pass (NL + 1 counts, the last 0; statistics) and
// filling pass (entries, costs, largest cost).
template <bool FILL>
__global__ __launch_bounds__(256) void ak_plan(const int *__restrict__ leaves, const int *__restrict__ leaf_index, int NL,
                                                const int4 *__restrict__ cell, const int2 *__restrict__ range,
                                                const int *__restrict__ coll, const int *__restrict__ u_off,
                                                const int *__restrict__ u_idx, int D, uint32_t *__restrict__ cnt,
                                                const int *__restrict__ off, int4 *__restrict__ work,
                                                uint64_t *__restrict__ cost, uint16_t *__restrict__ mask,
                                                unsigned long long *__restrict__ stats)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li > NL) return;
    if (li == NL) {
        if (!FILL) cnt[NL] = 0;
        return;
    }
    const int k = leaves[li];
    const int4 c = cell[k];
    const int2 r = range[k];
    const bool dense = r.y >= D;
    uint32_t m = 0;
    int64_t nsrc = 0, usum = 0;
    for (int u = u_off[k]; u < u_off[k + 1]; ++u) {
        const int S = u_idx[u];
        const int4 cs = cell[S];
        const int ns = range[S].y;
        usum += ns;
        if (dense && ns >= D && cs.x == c.x)
            m |= 1u << (3 * (cs.z - c.z + 1) + (cs.y - c.y + 1));
        else
            nsrc += ns;
    }
    int ne = 0;
    const int o = FILL ? off[li] : 0;
    uint64_t cmax = 0;
    auto put = [&](int4 item, int64_t cst) {
        if (FILL) {
            work[o + ne] = item;
            cost[o + ne] = (uint64_t)cst;
            cmax = cmax > (uint64_t)cst ? cmax : (uint64_t)cst;
        }
        ++ne;
    };
    int64_t units = 0, items = 0, mp = 0;
    if (nsrc > 0) {
        m |= 1u << 9;
        for (int b = r.x; b < r.x + r.y; b += 64) {
            const int len = min(64, r.x + r.y - b);
            put(make_int4(k, b, len, at_log2_lanes(len) | (dense ? 16 : 0)), at_unit_cost(nsrc, len));
            ++units;
        }
    }
    if (dense) {
        put(make_int4(li, li, 4 | (4 << 4), kMutualItem | (c.x << 9)), at_self_cost(r.y));
        ++items;
        mp += (int64_t)r.y * (r.y - 1);
        const int up[4][2] = {{1, 0}, {-1, 1}, {0, 1}, {1, 1}};
        for (int q = 0; q < 4; ++q) {
            const int R = coll[(int64_t)k * 8 + nb_slot(up[q][0], up[q][1])];
            if (R < 0 || !cell[R].w || range[R].y < D) continue;
            const int ds = 3 * (up[q][1] + 1) + (up[q][0] + 1);
            put(make_int4(li, leaf_index[R], ds | ((8 - ds) << 4), kMutualItem | (c.x << 9)),
                3 * at_pair_steps(r.y, range[R].y));
            ++items;
            mp += 2 * (int64_t)r.y * range[R].y;
        }
    }
    if (!FILL) {
        cnt[li] = (uint32_t)ne;
        mask[k] = (uint16_t)m;
        atomicAdd(&stats[kStPairs], (unsigned long long)((int64_t)r.y * usum - r.y));
        if (mp) atomicAdd(&stats[kStMutualPairs], (unsigned long long)mp);
        if (items) atomicAdd(&stats[kStMutualItems], (unsigned long long)items);
        if (units) atomicAdd(&stats[kStUnits], (unsigned long long)units);
    } else if (ne) {
        atomicMax(&stats[kStMaxCost], (unsigned long long)cmax);
    }
}

// Sort keys of the plan: heaviest first, so key = largest cost - cost (ascending).
__global__ __launch_bounds__(256) void ak_cost_keys(uint64_t *__restrict__ cost, int64_t nwork, uint64_t cmax,
                                                     uint32_t *__restrict__ val)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nwork) return;
    cost[u] = cmax - cost[u];
    val[u] = (uint32_t)u;
}

__global__ __launch_bounds__(256) void ak_gather_work(const int4 *__restrict__ src, const uint32_t *__restrict__ order,
                                                       int64_t nwork, int4 *__restrict__ dst)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nwork) dst[u] = src[order[u]];
}

// Flags of the leaves of level >= 2 (multipoles from particles) and of the split cells
// of level >= 2 (multipoles from children); K + 1 entries, the last 0.
__global__ __launch_bounds__(256) void ak_cell_flags(const int4 *__restrict__ cell, int K, uint32_t *__restrict__ fleaf,
                                                      uint32_t *__restrict__ finner)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    if (k == K) {
        fleaf[K] = finner[K] = 0;
        return;
    }
    const int4 c = cell[k];
    fleaf[k] = c.w && c.x >= 2;
    finner[k] = !c.w && c.x >= 2;
}

__global__ __launch_bounds__(256) void ak_compact(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                                                   int K, int *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K && flag[k]) out[pos[k]] = k;
}

// Adjoint near-field units, one per 64-particle tile of every leaf (leaf index li in
// sorted order; tile t = leaf_tile[li] + tile within the leaf): {leaf cell, first, count,
// log2 TP}, cost over all of U(leaf) as for the forward target-centric units.
__global__ __launch_bounds__(256) void ak_adj_units(const int *__restrict__ leaf_start, const int *__restrict__ leaf_of,
                                                     const int *__restrict__ leaf_tile, int NL,
                                                     const int2 *__restrict__ range, const int *__restrict__ u_off,
                                                     const int *__restrict__ u_idx, int4 *__restrict__ units,
                                                     uint64_t *__restrict__ cost, uint32_t *__restrict__ order,
                                                     unsigned long long *__restrict__ cmax)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= NL) return;
    const int k = leaf_of[leaf_start[li]];
    const int2 r = range[k];
    int64_t usum = 0;
    for (int e = u_off[k]; e < u_off[k + 1]; ++e) usum += range[u_idx[e]].y;
    uint64_t m = 0;
    int t = leaf_tile[li];
    for (int b = r.x; b < r.x + r.y; b += 64, ++t) {
        const int len = min(64, r.x + r.y - b);
        units[t] = make_int4(k, b, len, at_log2_lanes(len));
        const uint64_t c = (uint64_t)at_unit_cost(usum, len);
        cost[t] = c;
        order[t] = (uint32_t)t;
        m = m > c ? m : c;
    }
    atomicMax(cmax, (unsigned long long)m);
}

__global__ __launch_bounds__(256) void ak_desc_keys(uint64_t *__restrict__ key, int64_t n, uint64_t cmax)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) key[u] = cmax - key[u];
}

// The per-cell arrays while the levels are made: grown by doubling, first `used`
// entries kept.  Released to the tree (cell, range, parent, child) or freed.
struct CellStore {
    int4 *cell = nullptr;
    int2 *range = nullptr;
    int *parent = nullptr;
    int4 *child = nullptr;
    int *coll = nullptr;  // 8 neighbour slots per cell
    int64_t cap = 0;
    hipStream_t s = nullptr;

    ~CellStore()
    {
        for (void *p : {(void *)cell, (void *)range, (void *)parent, (void *)child, (void *)coll})
            if (p) (void)hipFreeAsync(p, s);
    }
    template <typename T>
    bool regrow(T *&p, int64_t ncap, int64_t used, int per, Status &st)
    {
        T *q = nullptr;
        if (!st.check(hipMallocAsync((void **)&q, (size_t)ncap * per * sizeof(T), s), "adaptive tree cells")) return false;
        if (used > 0 && !st.check(hipMemcpyAsync(q, p, (size_t)used * per * sizeof(T), hipMemcpyDeviceToDevice, s),
                                  "adaptive tree cells")) {
            (void)hipFreeAsync(q, s);
            return false;
        }
        if (p) (void)hipFreeAsync(p, s);
        p = q;
        return true;
    }
    bool reserve(int64_t need, int64_t used, Status &st)
    {
        if (need <= cap) return true;
        const int64_t ncap = std::max<int64_t>(need, 2 * cap);
        if (!regrow(cell, ncap, used, 1, st) || !regrow(range, ncap, used, 1, st) || !regrow(parent, ncap, used, 1, st) ||
            !regrow(child, ncap, used, 1, st) || !regrow(coll, ncap, used, 8, st))
            return false;
        cap = ncap;
        return true;
    }
};

template <typename T>
bool alloc_to(T *&p, int64_t count, hipStream_t s, Status &st, const char *what)
{
    return st.check(hipMallocAsync((void **)&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T), s), what);
}

bool read_back(void *dst, const void *src, size_t bytes, hipStream_t s, Status &st)
{
    return st.check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "adaptive tree build") &&
           st.check(hipStreamSynchronize(s), "adaptive tree build");
}

int bits_for(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

}  // namespace

int build_atree_device(fmm_atree *t, const double *xy, const double *root_box, hipStream_t s, std::string &err,
                       int64_t &bad_index)
{
    t->pooled = true;
    Status st;
    auto failed = [&]() {
        err = st.msg;
        return st.code;
    };
    bad_index = -1;
    const int64_t n = t->n;
    const int L = t->max_depth;
    const int smax = t->max_leaf;
    const double2 *xy2 = (const double2 *)xy;
    AtreeDev &d = t->d;

    // Stage 1: root cell.
    if (root_box) {
        t->x0 = root_box[0];
        t->y0 = root_box[1];
        t->side = root_box[2];
    } else {
        double box[3];
        bool nonfinite = false;
        if (!bounding_square(xy2, n, s, st, box, nonfinite)) return failed();
        if (nonfinite) {
            err = "non-finite particle position";
            return FMM_EINVAL;
        }
        t->x0 = box[0];
        t->y0 = box[1];
        t->side = box[2];
    }
    // Stage 2: keys on the finest grid and the stable sort by key (ties by user index).
    const int nside = 1 << L;
    const double w = t->side / (double)nside;
    Buf<uint64_t> key;
    Buf<uint32_t> val, skey;
    Buf<int> flags;
    Buf<unsigned long long> first_bad;
    if (!st.check(key.alloc(n, s), "adaptive tree build") || !st.check(val.alloc(n, s), "adaptive tree build") ||
        !st.check(skey.alloc(n, s), "adaptive tree build") || !st.check(flags.alloc(1, s), "adaptive tree build") ||
        !st.check(first_bad.alloc(1, s), "adaptive tree build") ||
        !st.check(hipMemsetAsync(flags.p, 0, sizeof(int), s), "adaptive tree build") ||
        !st.check(hipMemsetAsync(first_bad.p, 0xff, sizeof(unsigned long long), s), "adaptive tree build"))
        return failed();
    ak_keys<<<grid_for(n, 256), 256, 0, s>>>(xy2, n, t->x0, t->y0, w, nside, key.p, val.p, flags.p, first_bad.p);
    {
        int hf = 0;
        unsigned long long hb = 0;
        if (!st.check(hipMemcpyAsync(&hf, flags.p, sizeof(int), hipMemcpyDeviceToHost, s), "adaptive tree build") ||
            !read_back(&hb, first_bad.p, sizeof hb, s, st))
            return failed();
        if (hf) {
            bad_index = (int64_t)hb;
            err = (hf & 2) ? "non-finite particle position" : "particle lies outside the root cell";
            return (hf & 2) ? FMM_EINVAL : FMM_ERANGE;
        }
    }
    if (!radix_sort(key.p, val.p, n, 2 * L, s, st)) return failed();
    if (!alloc_to(d.perm, n, s, st, "permutation") || !alloc_to(d.xy, n, s, st, "sorted positions") ||
        !alloc_to(d.leaf_of, n, s, st, "leaf of each particle"))
        return failed();
    ak_sorted<<<grid_for(n, 256), 256, 0, s>>>(key.p, val.p, xy2, n, d.perm, skey.p, d.xy);

    // Stage 3a: cells, level by level.
    CellStore cs;
    cs.s = s;
    Buf<unsigned int> nsplit;
    if (!cs.reserve(std::max<int64_t>(1024, 4 * (n / (smax + 1)) + 64), 0, st) ||
        !st.check(nsplit.alloc(L + 1, s), "adaptive tree build") ||
        !st.check(hipMemsetAsync(nsplit.p, 0, (L + 1) * sizeof(unsigned int), s), "adaptive tree build"))
        return failed();
    ak_root<<<1, 1, 0, s>>>(cs.cell, cs.range, cs.parent, cs.coll, (int)n);
    std::vector<int> level_off(L + 2, 0);
    level_off[1] = 1;
    int begin = 0, end = 1, l = 0;
    for (;; ++l) {
        const int m = end - begin;
        Buf<uint32_t> nchild;
        if (!st.check(nchild.alloc(m, s), "adaptive tree build")) return failed();
        ak_split<<<grid_for(m, 256), 256, 0, s>>>(cs.cell, cs.range, cs.child, skey.p, begin, m, l, L, smax, nchild.p,
                                                  nsplit.p + l);
        if (l == L) break;
        uint32_t total = 0;
        if (!scan_exclusive(nchild.p, nchild.p, m, &total, s, st)) return failed();
        if (total == 0) break;
        if ((int64_t)end + total >= (int64_t(1) << 31)) {
            err = "adaptive tree: too many cells";
            return FMM_ENOMEM;
        }
        if (!cs.reserve((int64_t)end + total, end, st)) return failed();
        ak_children<<<grid_for(m, 256), 256, 0, s>>>(cs.cell, cs.range, cs.parent, cs.child, begin, m, l, nchild.p, end);
        ak_neighbours<<<grid_for(total, 256), 256, 0, s>>>(cs.cell, cs.parent, cs.child, cs.coll, end, (int)total, l + 1);
        if (!st.check(hipGetLastError(), "adaptive tree build")) return failed();
        begin = end;
        end += (int)total;
        level_off[l + 2] = end;
    }
    for (int k = l + 2; k <= L + 1; ++k) level_off[k] = end;
    const int K = end;
    t->ncells = K;
    t->level_off = level_off;
    std::vector<unsigned int> splits(L + 1);
    if (!read_back(splits.data(), nsplit.p, (L + 1) * sizeof(unsigned int), s, st)) return failed();
    t->inner_off.assign(L + 2, 0);
    for (int k = 0; k <= L; ++k) t->inner_off[k + 1] = t->inner_off[k] + (k >= 2 ? (int)splits[k] : 0);

    // Stage 3b: lists.
    Buf<int> werr;
    Buf<uint32_t> ucnt, wcnt, vcnt;
    if (!st.check(werr.alloc(1, s), "adaptive tree build") ||
        !st.check(hipMemsetAsync(werr.p, 0, sizeof(int), s), "adaptive tree build") ||
        !st.check(ucnt.alloc(K + 1, s, true), "adaptive tree lists") || !st.check(wcnt.alloc(K + 1, s, true), "adaptive tree lists") ||
        !st.check(vcnt.alloc(K + 1, s, true), "adaptive tree lists"))
        return failed();
    ak_vlist<false><<<grid_for(K + 1, 256), 256, 0, s>>>(cs.cell, cs.parent, cs.child, cs.coll, K, vcnt.p, nullptr,
                                                         nullptr);
    ak_uwlist<false><<<grid_for(K + 1, 256), 256, 0, s>>>(cs.cell, cs.parent, cs.child, cs.coll, K, L, ucnt.p, wcnt.p,
                                                          nullptr, nullptr, nullptr, nullptr, nullptr, werr.p);
    uint32_t nv = 0, nu = 0, nw = 0;
    if (!scan_exclusive(vcnt.p, vcnt.p, K + 1, nullptr, s, st) || !scan_exclusive(ucnt.p, ucnt.p, K + 1, nullptr, s, st) ||
        !scan_exclusive(wcnt.p, wcnt.p, K + 1, nullptr, s, st) ||
        !st.check(hipMemcpyAsync(&nv, vcnt.p + K, sizeof nv, hipMemcpyDeviceToHost, s), "adaptive tree lists") ||
        !st.check(hipMemcpyAsync(&nu, ucnt.p + K, sizeof nu, hipMemcpyDeviceToHost, s), "adaptive tree lists") ||
        !read_back(&nw, wcnt.p + K, sizeof nw, s, st))
        return failed();
    // the scanned counts are the CSR offsets (totals below 2^31)
    d.v_off = (int *)vcnt.release();
    d.u_off = (int *)ucnt.release();
    d.w_off = (int *)wcnt.release();
    Buf<uint32_t> wown;
    if (!alloc_to(d.v_idx, nv, s, st, "V list") || !alloc_to(d.u_idx, nu, s, st, "U list") ||
        !alloc_to(d.w_idx, nw, s, st, "W list") || !st.check(wown.alloc(nw, s, true), "W list"))
        return failed();
    ak_vlist<true><<<grid_for(K + 1, 256), 256, 0, s>>>(cs.cell, cs.parent, cs.child, cs.coll, K, nullptr, d.v_off,
                                                        d.v_idx);
    ak_uwlist<true><<<grid_for(K + 1, 256), 256, 0, s>>>(cs.cell, cs.parent, cs.child, cs.coll, K, L, nullptr, nullptr,
                                                         d.u_off, d.w_off, d.u_idx, d.w_idx, wown.p, werr.p);
    // X: the W entries (in owner order) stably sorted by the cell they name.
    {
        Buf<uint32_t> xcnt;
        Buf<uint64_t> xkey;
        if (!st.check(xcnt.alloc(K + 1, s, true), "X list") ||
            !st.check(hipMemsetAsync(xcnt.p, 0, (K + 1) * sizeof(uint32_t), s), "X list") ||
            !st.check(xkey.alloc(nw, s), "X list"))
            return failed();
        ak_xcount<<<grid_for(nw, 256), 256, 0, s>>>(d.w_idx, nw, xcnt.p);
        ak_xkeys<<<grid_for(nw, 256), 256, 0, s>>>(d.w_idx, nw, xkey.p);
        if (!scan_exclusive(xcnt.p, xcnt.p, K + 1, nullptr, s, st) ||
            !radix_sort(xkey.p, wown.p, nw, bits_for((uint64_t)K), s, st))
            return failed();
        d.x_off = (int *)xcnt.release();
        d.x_idx = (int *)wown.release();
    }
    {
        int he = 0;
        if (!read_back(&he, werr.p, sizeof he, s, st)) return failed();
        if (he) {
            err = "adaptive tree: list walk deeper than the stack";
            return FMM_EDEVICE;
        }
    }

    // Stage 3c: leaves in sorted order, the leaf of every particle, tiles and their boxes.
    Buf<uint32_t> lflag, lscan;
    Buf<int> leaf_index, leaves;
    Buf<unsigned int> deepest;
    uint32_t NL = 0;
    if (!st.check(lflag.alloc(n, s), "adaptive tree leaves") || !st.check(lscan.alloc(n, s), "adaptive tree leaves") ||
        !st.check(hipMemsetAsync(lflag.p, 0, n * sizeof(uint32_t), s), "adaptive tree leaves") ||
        !st.check(leaf_index.alloc(K, s), "adaptive tree leaves") ||
        !st.check(deepest.alloc(1, s), "adaptive tree leaves") ||
        !st.check(hipMemsetAsync(deepest.p, 0, sizeof(unsigned int), s), "adaptive tree leaves"))
        return failed();
    ak_leaf_marks<<<grid_for(K, 256), 256, 0, s>>>(cs.cell, cs.range, K, lflag.p);
    if (!scan_exclusive(lflag.p, lscan.p, n, &NL, s, st)) return failed();
    if (!st.check(leaves.alloc(NL, s), "adaptive tree leaves") ||
        !alloc_to(d.leaf_start, (int64_t)NL + 1, s, st, "leaf offsets"))
        return failed();
    ak_leaf_index<<<grid_for(K, 256), 256, 0, s>>>(cs.cell, cs.range, K, lscan.p, leaf_index.p, leaves.p, d.leaf_start,
                                                   deepest.p);
    ak_set<<<1, 1, 0, s>>>(d.leaf_start + NL, (int)n);
    ak_leaf_of<<<grid_for(n, 256), 256, 0, s>>>(lflag.p, lscan.p, leaves.p, n, d.leaf_of);
    uint32_t ntiles = 0;
    {
        Buf<uint32_t> nt;
        if (!st.check(nt.alloc((int64_t)NL + 1, s, true), "tiles")) return failed();
        ak_leaf_ntiles<<<grid_for((int64_t)NL + 1, 256), 256, 0, s>>>(leaves.p, cs.range, (int)NL, nt.p);
        if (!scan_exclusive(nt.p, nt.p, (int64_t)NL + 1, &ntiles, s, st)) return failed();
        d.leaf_tile = (int *)nt.release();  // NL + 1 entries, the last = ntiles
    }
    Buf<int> tile_leaf;
    if (!alloc_to(d.tile_start, K, s, st, "tiles") ||
        !st.check(hipMemsetAsync(d.tile_start, 0, (size_t)K * sizeof(int), s), "tiles") ||
        !st.check(tile_leaf.alloc(ntiles, s), "tiles") || !alloc_to(d.tile_box, ntiles, s, st, "tile boxes") ||
        !alloc_to(d.tile_box_leaf, ntiles, s, st, "tile boxes"))
        return failed();
    ak_tiles<<<grid_for(NL, 256), 256, 0, s>>>(leaves.p, d.leaf_tile, (int)NL, d.tile_start, tile_leaf.p);
    ak_tile_box<<<grid_for(ntiles, 256), 256, 0, s>>>(tile_leaf.p, leaves.p, d.leaf_tile, cs.cell, cs.range, d.xy,
                                                      ntiles, t->x0, t->y0, t->side, d.tile_box, d.tile_box_leaf);

    // Stage 3d: the near-field plan, heaviest first.
    Buf<uint32_t> pcnt;
    Buf<unsigned long long> stats;
    uint32_t nwork = 0;
    if (!st.check(pcnt.alloc((int64_t)NL + 1, s), "near-field plan") ||
        !alloc_to(d.mask, K, s, st, "near-field mask") ||
        !st.check(hipMemsetAsync(d.mask, 0, (size_t)K * sizeof(uint16_t), s), "near-field mask") ||
        !st.check(stats.alloc(kStCount, s), "near-field plan") ||
        !st.check(hipMemsetAsync(stats.p, 0, kStCount * sizeof(unsigned long long), s), "near-field plan"))
        return failed();
    ak_plan<false><<<grid_for((int64_t)NL + 1, 256), 256, 0, s>>>(leaves.p, leaf_index.p, (int)NL, cs.cell, cs.range,
                                                                   cs.coll, d.u_off, d.u_idx, t->dense_leaf, pcnt.p,
                                                                   nullptr, nullptr, nullptr, d.mask, stats.p);
    if (!scan_exclusive(pcnt.p, pcnt.p, (int64_t)NL + 1, &nwork, s, st)) return failed();
    Buf<int4> work;
    Buf<uint64_t> cost;
    Buf<uint32_t> order;
    if (!st.check(work.alloc(nwork, s), "near-field plan") || !st.check(cost.alloc(nwork, s), "near-field plan") ||
        !st.check(order.alloc(nwork, s), "near-field plan"))
        return failed();
    ak_plan<true><<<grid_for((int64_t)NL + 1, 256), 256, 0, s>>>(leaves.p, leaf_index.p, (int)NL, cs.cell, cs.range,
                                                                  cs.coll, d.u_off, d.u_idx, t->dense_leaf, nullptr,
                                                                  (const int *)pcnt.p, work.p, cost.p, nullptr, stats.p);
    unsigned long long hs[kStCount];
    if (!read_back(hs, stats.p, sizeof hs, s, st)) return failed();
    if (!alloc_to(d.work, nwork, s, st, "near-field work")) return failed();
    ak_cost_keys<<<grid_for(nwork, 256), 256, 0, s>>>(cost.p, nwork, hs[kStMaxCost], order.p);
    if (!radix_sort(cost.p, order.p, nwork, bits_for(hs[kStMaxCost]), s, st)) return failed();
    ak_gather_work<<<grid_for(nwork, 256), 256, 0, s>>>(work.p, order.p, nwork, d.work);

    // Leaves and split cells of level >= 2, in cell order.
    uint32_t np2m = 0, ninner = 0;
    {
        Buf<uint32_t> fl, fi, pl, pi;
        if (!st.check(fl.alloc(K + 1, s), "adaptive tree build") || !st.check(fi.alloc(K + 1, s), "adaptive tree build") ||
            !st.check(pl.alloc(K + 1, s), "adaptive tree build") || !st.check(pi.alloc(K + 1, s), "adaptive tree build"))
            return failed();
        ak_cell_flags<<<grid_for(K + 1, 256), 256, 0, s>>>(cs.cell, K, fl.p, fi.p);
        if (!scan_exclusive(fl.p, pl.p, K + 1, nullptr, s, st) || !scan_exclusive(fi.p, pi.p, K + 1, nullptr, s, st) ||
            !st.check(hipMemcpyAsync(&np2m, pl.p + K, sizeof np2m, hipMemcpyDeviceToHost, s), "adaptive tree build") ||
            !read_back(&ninner, pi.p + K, sizeof ninner, s, st))
            return failed();
        if (!alloc_to(d.p2m_cells, np2m, s, st, "leaves with expansions") || !alloc_to(d.inner, ninner, s, st, "split cells"))
            return failed();
        ak_compact<<<grid_for(K, 256), 256, 0, s>>>(fl.p, pl.p, K, d.p2m_cells);
        ak_compact<<<grid_for(K, 256), 256, 0, s>>>(fi.p, pi.p, K, d.inner);
    }
    unsigned int hdeep = 0;
    if (!read_back(&hdeep, deepest.p, sizeof hdeep, s, st) || !st.check(hipGetLastError(), "adaptive tree build"))
        return failed();
    if ((int64_t)ninner != (int64_t)t->inner_off[L + 1]) {
        err = "adaptive tree: inconsistent split-cell count";
        return FMM_EDEVICE;
    }

    // Staging slots of the two-pass permutations between user and sorted order.
    if (!build_staging(d.perm, n, s, st, t->stage_shift, d.gpos1, d.gpos2, d.st1)) {
        err = st.msg;
        return st.code;
    }

    // The cell arrays pass to the tree; the neighbour slots were the build's alone.
    d.cell = cs.cell;
    d.range = cs.range;
    d.parent = cs.parent;
    d.child = cs.child;
    cs.cell = nullptr;
    cs.range = nullptr;
    cs.parent = nullptr;
    cs.child = nullptr;

    const int64_t sz[FMM_AT_COUNT] = {K, (int64_t)NL, (int64_t)nu, (int64_t)nv, (int64_t)nw, (int64_t)nw, (int64_t)hdeep,
                                      (int64_t)hs[kStPairs]};
    std::copy(sz, sz + FMM_AT_COUNT, t->sizes);
    t->np2m = np2m;
    t->ntiles = ntiles;
    t->nwork = nwork;
    t->mutual_items = (int64_t)hs[kStMutualItems];
    t->mutual_pairs = (int64_t)hs[kStMutualPairs];
    t->target_units = (int64_t)hs[kStUnits];
    return FMM_OK;
}

int build_atree_adjoint_units(fmm_atree *t, hipStream_t s, std::string &err)
{
    Status st;
    const int64_t nt = t->ntiles;
    const int NL = (int)t->sizes[FMM_AT_LEAVES];
    Buf<int4> units;
    Buf<uint64_t> cost;
    Buf<uint32_t> order;
    Buf<unsigned long long> cmax;
    int4 *out = nullptr;
    if (!st.check(units.alloc(nt, s), "adjoint units") || !st.check(cost.alloc(nt, s), "adjoint units") ||
        !st.check(order.alloc(nt, s), "adjoint units") || !st.check(cmax.alloc(1, s), "adjoint units") ||
        !st.check(hipMemsetAsync(cmax.p, 0, sizeof(unsigned long long), s), "adjoint units")) {
        err = st.msg;
        return st.code;
    }
    ak_adj_units<<<grid_for(NL, 256), 256, 0, s>>>(t->d.leaf_start, t->d.leaf_of, t->d.leaf_tile, NL, t->d.range,
                                                   t->d.u_off, t->d.u_idx, units.p, cost.p, order.p, cmax.p);
    unsigned long long hm = 0;
    if (!read_back(&hm, cmax.p, sizeof hm, s, st)) {
        err = st.msg;
        return st.code;
    }
    ak_desc_keys<<<grid_for(nt, 256), 256, 0, s>>>(cost.p, nt, hm);
    if (!radix_sort(cost.p, order.p, nt, bits_for(hm), s, st) ||
        !st.check(hipMallocAsync((void **)&out, (size_t)std::max<int64_t>(nt, 1) * sizeof(int4), s), "adjoint units")) {
        err = st.msg;
        return st.code;
    }
    ak_gather_work<<<grid_for(nt, 256), 256, 0, s>>>(units.p, order.p, nt, out);
    if (!st.check(hipGetLastError(), "adjoint units") || !st.check(hipStreamSynchronize(s), "adjoint units")) {
        (void)hipFreeAsync(out, s);
        err = st.msg;
        return st.code;
    }
    t->d.bwd_units = out;
    t->nbwd_units = nt;
    return FMM_OK;
}

// M2L plan of the MFMA path: segment key 4 (level - 2) + parity class and cell of every
// cell of level >= 2, and the counts per segment (count[0 .. 4 nlev - 1]).
__global__ __launch_bounds__(256) void ak_m2l_keys(const int4 *__restrict__ cell, int first, int ncl, int nseg,
                                                   uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                                                   unsigned int *__restrict__ count)
{
    __shared__ unsigned int bc[64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < nseg) bc[threadIdx.x] = 0;
    __syncthreads();
    if (i < ncl) {
        const int4 c = cell[first + i];
        const int sg = 4 * (c.x - 2) + ((c.y & 1) | ((c.z & 1) << 1));
        key[i] = (uint64_t)sg;
        val[i] = (uint32_t)(first + i);
        atomicAdd(&bc[sg], 1u);
    }
    __syncthreads();
    if (threadIdx.x < nseg && bc[threadIdx.x]) atomicAdd(&count[threadIdx.x], bc[threadIdx.x]);
}

// Source cell of each interaction offset {dx, dy} of the cell's class (entries 28 q ..
// 28 q + 26 of the operator tables) from its V list; a V member of another level or at an
// offset outside the class's 27 counts into *bad.
__global__ __launch_bounds__(256) void ak_vslot(const int4 *__restrict__ cell, int first, int ncl,
                                                const int *__restrict__ v_off, const int *__restrict__ v_idx,
                                                const int4 *__restrict__ entries, int *__restrict__ vslot,
                                                unsigned int *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int k = first + i;
    const int4 c = cell[k];
    const int q = (c.y & 1) | ((c.z & 1) << 1);
    int *vs = vslot + (int64_t)i * 27;
    for (int j = 0; j < 27; ++j) vs[j] = -1;
    for (int e = v_off[k]; e < v_off[k + 1]; ++e) {
        const int S = v_idx[e];
        const int4 cs = cell[S];
        const int dx = cs.y - c.y, dy = cs.z - c.z;
        int slot = -1;
        for (int j = 0; j < 27; ++j) {
            const int4 en = entries[28 * q + j];
            if (en.x == dx && en.y == dy) slot = j;
        }
        if (slot < 0 || cs.x != c.x) atomicAdd(bad, 1u);
        else vs[slot] = S;
    }
}

int build_atree_m2l_plan(fmm_atree *t, const int4 *entries, hipStream_t s, std::string &err)
{
    Status st;
    const int deepest = (int)t->sizes[FMM_AT_DEEPEST];
    t->m2l_seg_off.assign(1, 0);
    if (deepest < 2) {
        t->m2l_plan = true;
        return FMM_OK;
    }
    const int first = t->level_off[2], ncl = t->level_off[deepest + 1] - first;
    const int nseg = 4 * (deepest - 1);  // <= 56
    Buf<uint64_t> key;
    Buf<uint32_t> val;
    Buf<unsigned int> cnt;
    int *targets = nullptr, *vslot = nullptr;
    auto failed = [&]() {
        if (targets) (void)hipFreeAsync(targets, s);
        if (vslot) (void)hipFreeAsync(vslot, s);
        err = st.msg;
        return st.code;
    };
    if (!st.check(key.alloc(ncl, s), "M2L plan") || !st.check(val.alloc(ncl, s), "M2L plan") ||
        !st.check(cnt.alloc(nseg + 1, s), "M2L plan") ||
        !st.check(hipMemsetAsync(cnt.p, 0, (nseg + 1) * sizeof(unsigned int), s), "M2L plan") ||
        !st.check(hipMallocAsync((void **)&targets, (size_t)std::max(ncl, 1) * sizeof(int), s), "M2L plan") ||
        !st.check(hipMallocAsync((void **)&vslot, (size_t)std::max(ncl, 1) * 27 * sizeof(int), s), "M2L plan"))
        return failed();
    ak_m2l_keys<<<grid_for(ncl, 256), 256, 0, s>>>(t->d.cell, first, ncl, nseg, key.p, val.p, cnt.p);
    ak_vslot<<<grid_for(ncl, 256), 256, 0, s>>>(t->d.cell, first, ncl, t->d.v_off, t->d.v_idx, entries, vslot,
                                                cnt.p + nseg);
    // stable by segment: Morton order inside a class as inside a level
    if (!radix_sort(key.p, val.p, ncl, 6, s, st) ||
        !st.check(hipMemcpyAsync(targets, val.p, (size_t)ncl * sizeof(int), hipMemcpyDeviceToDevice, s), "M2L plan"))
        return failed();
    std::vector<unsigned int> hc((size_t)nseg + 1);
    if (!read_back(hc.data(), cnt.p, hc.size() * sizeof(unsigned int), s, st)) return failed();
    if (hc[nseg] != 0) {
        st.code = FMM_EDEVICE;
        st.msg = "M2L plan: " + std::to_string(hc[nseg]) + " V-list entries outside the interaction offsets";
        return failed();
    }
    t->m2l_seg_off.assign((size_t)nseg + 1, 0);
    for (int q = 0; q < nseg; ++q) t->m2l_seg_off[q + 1] = t->m2l_seg_off[q] + (int)hc[q];
    t->d.m2l_targets = targets;
    t->d.vslot = vslot;
    t->m2l_plan = true;
    return FMM_OK;
}

}  // namespace fmm
