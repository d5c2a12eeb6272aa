// Stages 1-3 of Fig. fmmStages on the GPU: root cell, binning, Morton sort, leaf
// offsets, per-level occupancy, interaction-list cell lists, near-field work lists and
// the statistics of fmm_tree_info.
//
// The arrays equal those of the host build of api.cpp element for element (same
// arithmetic for the binning and tile boxes, stable sorts with the same keys), so either
// build gives bit-identical evaluations.  The building blocks are a stable LSD radix
// sort of (64-bit key, 32-bit value) pairs with 8-bit digits and a device-wide
// exclusive scan, both written here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fmm2d.h"
#include "build_prims.h"
#include "fmm_internal.h"

namespace fmm {

namespace {

// ---------------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 (totals below 2^32).  Tiles of 2048: each
// thread scans 8 consecutive elements, the block scans the thread totals; tile sums
// are scanned by a single workgroup and added back.  In place is allowed.
// ---------------------------------------------------------------------------------
constexpr int kScanTile = 2048;

__device__ inline uint32_t block_exclusive_sum(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wid) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(256) void scan_tile_sums(const uint32_t *__restrict__ in, int64_t n,
                                                       uint32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 8;
    uint32_t s = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (base + e < n) s += in[base + e];
    uint32_t total;
    block_exclusive_sum(s, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile sums in place, grand total to *total.
__global__ __launch_bounds__(256) void scan_sums(uint32_t *__restrict__ sums, int64_t nb, uint32_t *__restrict__ total)
{
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanTile) {
        const int64_t b = base + (int64_t)threadIdx.x * 8;
        uint32_t v[8], s = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[e] = b + e < nb ? sums[b + e] : 0u;
            s += v[e];
        }
        uint32_t tot;
        uint32_t run = carry + block_exclusive_sum(s, tot);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (b + e < nb) {
                sums[b + e] = run;
                run += v[e];
            }
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_tiles(const uint32_t *in, uint32_t *out, int64_t n,
                                                   const uint32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        v[e] = base + e < n ? in[base + e] : 0u;
        s += v[e];
    }
    uint32_t tot;
    uint32_t run = sums[blockIdx.x] + block_exclusive_sum(s, tot);
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (base + e < n) {
            out[base + e] = run;
            run += v[e];
        }
}

// ---------------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the key,
// 8-bit digits.  Per pass: per-tile digit histograms (digit-major), their exclusive
// scan, then a scatter in which each tile of 2048 pairs is taken in 8 rounds of 256;
// inside a wavefront the lanes with the same digit find each other with 8 ballots
// (rank = lanes below with the same digit), across wavefronts and rounds the digit
// counts accumulate in LDS, so equal digits keep their input order.
// ---------------------------------------------------------------------------------
constexpr int kRsTile = 2048;

__global__ __launch_bounds__(256) void rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                uint32_t *__restrict__ counts, int nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsTile / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                   uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                                                   int shift, const uint32_t *__restrict__ offs, int nb)
{
    __shared__ uint32_t start[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    start[t] = offs[(int64_t)t * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsTile / 256; ++r) {
        wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0;
        __syncthreads();
        const int64_t i = base + r * 256 + t;
        const bool valid = i < n;
        uint64_t key = 0;
        uint32_t val = 0, d = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            d = (uint32_t)(key >> shift) & 255u;
        }
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bm = __ballot(valid && bit);
            m &= bit ? bm : ~bm;
        }
        const uint64_t below = m & ((1ull << lane) - 1ull);
        if (valid && below == 0) wcnt[wid][d] = (uint32_t)__popcll(m);  // lowest lane of its digit group
        __syncthreads();
        if (valid) {
            uint32_t pos = start[d] + (uint32_t)__popcll(below);
            for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        start[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    }
}

// ---------------------------------------------------------------------------------
// Tree kernels
// ---------------------------------------------------------------------------------
// Per-block min/max of the coordinates; flags bit 1: a non-finite coordinate.
__global__ __launch_bounds__(256) void k_minmax(const double2 *__restrict__ xy, int64_t n, double4 *__restrict__ part,
                                                 int *__restrict__ flags)
{
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 z = xy[i];
        if (!isfinite(z.x) || !isfinite(z.y)) {
            bad = true;
            continue;
        }
        xmin = fmin(xmin, z.x);
        xmax = fmax(xmax, z.x);
        ymin = fmin(ymin, z.y);
        ymax = fmax(ymax, z.y);
    }
    if (bad) atomicOr(flags, 2);
    for (int o = 32; o > 0; o >>= 1) {
        xmin = fmin(xmin, __shfl_xor(xmin, o));
        xmax = fmax(xmax, __shfl_xor(xmax, o));
        ymin = fmin(ymin, __shfl_xor(ymin, o));
        ymax = fmax(ymax, __shfl_xor(ymax, o));
    }
    __shared__ double4 w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = make_double4(xmin, xmax, ymin, ymax);
    __syncthreads();
    if (threadIdx.x == 0) {
        double4 r = w[0];
        for (int k = 1; k < 4; ++k) {
            r.x = fmin(r.x, w[k].x);
            r.y = fmax(r.y, w[k].y);
            r.z = fmin(r.z, w[k].z);
            r.w = fmax(r.w, w[k].w);
        }
        part[blockIdx.x] = r;
    }
}

// Leaf (floor binning, clamped at the top edge) and sub-leaf key (64 x 64 grid over the
// leaf), as in the host build.  key = leaf Morton << 12 | sub-leaf Morton, value = index.
// flags bit 0: outside the root cell, bit 1: non-finite; *first_bad: lowest such index.
__global__ __launch_bounds__(256) void k_keys(const double2 *__restrict__ xy, int64_t n, double x0, double y0,
                                               double w, int nside, uint64_t *__restrict__ key,
                                               uint32_t *__restrict__ val, int *__restrict__ flags,
                                               unsigned long long *__restrict__ first_bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 z = xy[i];
    uint32_t c[2] = {0, 0}, f[2] = {0, 0};
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
            const int64_t k = (int64_t)floor(v);
            c[d] = (uint32_t)min(k, (int64_t)(nside - 1));
            f[d] = (uint32_t)min((int64_t)floor((v - (double)c[d]) * 64.0), (int64_t)63);
        }
    }
    if (bad) atomicMin(first_bad, (unsigned long long)i);
    key[i] = ((uint64_t)morton_encode(c[0], c[1]) << 12) | morton_encode(f[0], f[1]);
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_sorted(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val,
                                                 const double2 *__restrict__ xy, int64_t n, int *__restrict__ perm,
                                                 int *__restrict__ leaf_of, double2 *__restrict__ xys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t u = val[i];
    perm[i] = (int)u;
    leaf_of[i] = (int)(key[i] >> 12);
    xys[i] = xy[u];
}

// leaf_start[c] = first sorted slot with leaf >= c, c = 0..nleaf: a binary search per
// leaf (a fill between consecutive occupied leaves would leave one thread to write each
// run of empty leaves, long for clustered particles).
__global__ __launch_bounds__(256) void k_leaf_start(const int *__restrict__ leaf_of, int64_t n, int64_t nleaf,
                                                     int *__restrict__ ls)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nleaf) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (leaf_of[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    ls[c] = (int)lo;
}

// Occupancy of every cell of every level (global cell index (4^l - 1)/3 + Morton).
__global__ __launch_bounds__(256) void k_counts(const int *__restrict__ ls, int L, int64_t ncells,
                                                 int *__restrict__ counts)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncells) return;
    int l = 0;
    while (level_base(l + 1) <= g) ++l;
    const int64_t c = g - level_base(l);
    const int sh = 2 * (L - l);
    counts[g] = ls[(c + 1) << sh] - ls[c << sh];
}

__global__ __launch_bounds__(256) void k_leaf_tiles(const int *__restrict__ ls, int64_t nleaf,
                                                     uint32_t *__restrict__ ntile)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nleaf) return;
    ntile[c] = c == nleaf ? 0u : (uint32_t)((ls[c + 1] - ls[c] + 63) / 64);
}

__global__ __launch_bounds__(256) void k_tile_leaf(const uint32_t *__restrict__ tile_start, int64_t nleaf,
                                                    int *__restrict__ tile_leaf)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nleaf) return;
    for (uint32_t t = tile_start[c]; t < tile_start[c + 1]; ++t) tile_leaf[t] = (int)c;
}

// Bounding box of each 64-particle tile in leaf units about the leaf centre, rounded
// outwards to FP32 (as the host build).
__global__ __launch_bounds__(256) void k_tile_box(const int *__restrict__ tile_leaf,
                                                   const uint32_t *__restrict__ tile_start,
                                                   const int *__restrict__ ls, const double2 *__restrict__ xys,
                                                   int64_t ntiles, double x0, double y0, double w,
                                                   float4 *__restrict__ box)
{
    const int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= ntiles) return;
    const uint32_t c = (uint32_t)tile_leaf[tt];
    const double cx = x0 + (morton_x(c) + 0.5) * w;
    const double cy = y0 + (morton_y(c) + 0.5) * w;
    const int b = ls[c] + 64 * (int)(tt - tile_start[c]);
    const int e = min(b + 64, ls[c + 1]);
    double xmin = 1e300, ymin = 1e300, xmax = -1e300, ymax = -1e300;
    for (int k = b; k < e; ++k) {
        const double xl = (xys[k].x - cx) / w, yl = (xys[k].y - cy) / w;
        xmin = fmin(xmin, xl);
        xmax = fmax(xmax, xl);
        ymin = fmin(ymin, yl);
        ymax = fmax(ymax, yl);
    }
    box[tt] = make_float4(nextafterf((float)xmin, -INFINITY), nextafterf((float)ymin, -INFINITY),
                          nextafterf((float)xmax, INFINITY), nextafterf((float)ymax, INFINITY));
}

// Cell lists of levels 2..L grouped by parity class: index k runs over the levels in
// order, inside a level over the classes q = 0..3, inside a class over the cells
// c = 4j + q in increasing order.
__device__ inline void list_cell(int64_t k, int &l, int64_t &c)
{
    l = 2;
    int64_t base = 0;
    while (base + (int64_t(1) << (2 * l)) <= k) {
        base += int64_t(1) << (2 * l);
        ++l;
    }
    const int64_t kk = k - base, quarter = int64_t(1) << (2 * l - 2);
    c = 4 * (kk % quarter) + kk / quarter;
}

__global__ __launch_bounds__(256) void k_list_flags(const int *__restrict__ counts, int64_t nflags,
                                                     uint32_t *__restrict__ flag)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nflags) return;
    int l;
    int64_t c;
    list_cell(k, l, c);
    flag[k] = counts[level_base(l) + c] > 0 ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_list_scatter(const int *__restrict__ counts, int64_t nflags,
                                                       const uint32_t *__restrict__ pos, int *__restrict__ lists)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nflags) return;
    int l;
    int64_t c;
    list_cell(k, l, c);
    if (counts[level_base(l) + c] > 0) lists[pos[k]] = (int)c;
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const int64_t *__restrict__ idx, int m,
                              uint32_t *__restrict__ dst)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = src[idx[k]];
}

__device__ inline int leaf_count(const int *__restrict__ ls, int nside, int x, int y)
{
    if (x < 0 || y < 0 || x >= nside || y >= nside) return 0;
    const uint32_t c = morton_encode((uint32_t)x, (uint32_t)y);
    return ls[c + 1] - ls[c];
}

// Per leaf: near-field pair sum, occupancy statistics, and the target-centric work
// units (one per 64-particle tile, cost = source steps) with their sort keys.
__global__ __launch_bounds__(256) void k_leaf_stats(const int *__restrict__ ls, int L,
                                                     const uint32_t *__restrict__ tile_start,
                                                     unsigned long long *__restrict__ stats, int4 *__restrict__ units,
                                                     uint64_t *__restrict__ ukey, uint32_t *__restrict__ uval)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nside = 1 << L;
    if (c >= (int64_t(1) << (2 * L))) return;
    const int nt = ls[c + 1] - ls[c];
    if (nt == 0) return;
    const int x = (int)morton_x((uint32_t)c), y = (int)morton_y((uint32_t)c);
    int64_t nsrc = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) nsrc += leaf_count(ls, nside, x + dx, y + dy);
    atomicAdd(&stats[0], (unsigned long long)((int64_t)nt * nsrc));
    atomicAdd(&stats[1], 1ull);
    atomicMax(&stats[2], (unsigned long long)nt);
    uint32_t tt = tile_start[c];
    for (int c0 = 0; c0 < nt; c0 += 64, ++tt) {
        const int cnt = min(64, nt - c0);
        int logtp = 0;
        while ((1 << logtp) < cnt) ++logtp;
        const int kstride = 64 >> logtp;
        units[tt] = make_int4((int)c, ls[c] + c0, cnt, logtp);
        const uint64_t cost = (uint64_t)((nsrc + kstride - 1) / kstride);
        ukey[tt] = 0xffffffffull - min(cost, 0xffffffffull);  // heaviest first
        uval[tt] = tt;
    }
}

// Non-empty (target, source) cell pairs of the interaction lists at one level.
__global__ __launch_bounds__(256) void k_m2l_count(const int *__restrict__ lst, int64_t len, int l,
                                                    const int *__restrict__ counts,
                                                    unsigned long long *__restrict__ stats)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    const int n1 = 1 << l;
    const int tx = (int)morton_x((uint32_t)lst[k]), ty = (int)morton_y((uint32_t)lst[k]);
    const int qx = tx & 1, qy = ty & 1;
    unsigned long long m = 0;
    for (int dy = -2 - qy; dy <= 3 - qy; ++dy)
        for (int dx = -2 - qx; dx <= 3 - qx; ++dx) {
            if (abs(dx) <= 1 && abs(dy) <= 1) continue;
            const int sx = tx + dx, sy = ty + dy;
            if (sx < 0 || sy < 0 || sx >= n1 || sy >= n1) continue;
            if (counts[level_base(l) + morton_encode((uint32_t)sx, (uint32_t)sy)] > 0) ++m;
        }
    if (m) atomicAdd(&stats[3], m);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T *__restrict__ src, const uint32_t *__restrict__ idx, int64_t m,
                                                 T *__restrict__ dst)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = src[idx[k]];
}

// Staging slots of the two-pass permutation of the circulations (see pack_kernel):
// sort key of user index u = bucket of its sorted slot.
__global__ __launch_bounds__(256) void k_stage_keys(const int *__restrict__ perm, int64_t n, int shift,
                                                     uint64_t *__restrict__ key, uint32_t *__restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[perm[i]] = (uint64_t)(i >> shift);  // the sorted slot of user index perm[i] is i
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_gpos(const uint32_t *__restrict__ sorted_users, int64_t n,
                                               int *__restrict__ gpos1)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    gpos1[sorted_users[k]] = (int)k;
}

__global__ __launch_bounds__(256) void k_gpos2(const int *__restrict__ gpos1, const int *__restrict__ perm, int64_t n,
                                                int *__restrict__ gpos2)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) gpos2[k] = gpos1[perm[k]];
}

// ---------------------------------------------------------------------------------
// Near-field plan (the mutual form; see build_near_plan in api.cpp for its meaning).
// Per leaf: its entries (target-centric units, then the self item, then the items of
// its dense upper neighbours), their costs, the slot mask; then a stable sort by cost.
// ---------------------------------------------------------------------------------
__device__ inline int64_t nch16(int len) { return (len + 15) >> 4; }

__device__ inline int64_t block_steps(int cs, int cr)
{
    const int64_t fs = cs / 64, fr = cr / 64;
    const int rs = cs % 64, rr = cr % 64;
    return 16 * (fs * fr * 4 + fs * nch16(rr) + fr * nch16(rs) + min(nch16(rs), nch16(rr)));
}

__constant__ int kUp[4][2] = {{1, 0}, {-1, 1}, {0, 1}, {1, 1}};

__global__ __launch_bounds__(256) void k_plan_count(const int *__restrict__ ls, int L, int D,
                                                     uint32_t *__restrict__ nentries, uint16_t *__restrict__ mask,
                                                     unsigned long long *__restrict__ stats)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nleaf = int64_t(1) << (2 * L);
    if (c > nleaf) return;
    if (c == nleaf) {
        nentries[c] = 0;
        return;
    }
    const int nside = 1 << L;
    const int nt = ls[c + 1] - ls[c];
    if (nt == 0) {
        nentries[c] = 0;
        mask[c] = 0;
        return;
    }
    const int x = (int)morton_x((uint32_t)c), y = (int)morton_y((uint32_t)c);
    const bool dense = nt >= D;
    int64_t nsrc = 0;
    uint32_t m = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ns = leaf_count(ls, nside, x + dx, y + dy);
            if (ns == 0) continue;
            if (dense && ns >= D) m |= 1u << (3 * (dy + 1) + (dx + 1));
            else nsrc += ns;
        }
    uint32_t cnt = 0;
    if (nsrc > 0) {
        m |= 1u << 9;
        cnt += (uint32_t)((nt + 63) / 64);
        atomicAdd(&stats[0], (unsigned long long)((nt + 63) / 64));
    }
    mask[c] = (uint16_t)m;
    if (dense) {
        int64_t pairs = (int64_t)nt * (nt - 1);
        uint32_t items = 1;
        for (int k = 0; k < 4; ++k) {
            const int nr = leaf_count(ls, nside, x + kUp[k][0], y + kUp[k][1]);
            if (nr >= D) {
                ++items;
                pairs += 2 * (int64_t)nt * nr;
            }
        }
        cnt += items;
        atomicAdd(&stats[1], (unsigned long long)items);
        atomicAdd(&stats[2], (unsigned long long)pairs);
    }
    nentries[c] = cnt;
}

__global__ __launch_bounds__(256) void k_plan_fill(const int *__restrict__ ls, int L, int D,
                                                    const uint32_t *__restrict__ off, int4 *__restrict__ work,
                                                    uint64_t *__restrict__ key, uint32_t *__restrict__ val)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t(1) << (2 * L))) return;
    const int nside = 1 << L;
    const int nt = ls[c + 1] - ls[c];
    if (nt == 0) return;
    const int x = (int)morton_x((uint32_t)c), y = (int)morton_y((uint32_t)c);
    const bool dense = nt >= D;
    int64_t nsrc = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ns = leaf_count(ls, nside, x + dx, y + dy);
            if (ns == 0) continue;
            if (!(dense && ns >= D)) nsrc += ns;
        }
    uint32_t o = off[c];
    const uint64_t kMax = (1ull << 40) - 1;
    auto put = [&](int4 e, int64_t cost) {
        work[o] = e;
        key[o] = kMax - min((uint64_t)cost, kMax);  // heaviest first
        val[o] = o;
        ++o;
    };
    if (nsrc > 0)
        for (int c0 = 0; c0 < nt; c0 += 64) {
            const int cnt = min(64, nt - c0);
            int logtp = 0;
            while ((1 << logtp) < cnt) ++logtp;
            const int kstride = 64 >> logtp;
            put(make_int4((int)c, ls[c] + c0, cnt, logtp | (dense ? 16 : 0)), 2 * ((nsrc + kstride - 1) / kstride));
        }
    if (!dense) return;
    const int64_t f = nt / 64;
    const int r = nt % 64;
    const int64_t diag = 16 * (f * 4 + nch16(r));
    const int64_t st = 16 * (f * (f - 1) / 2 * 4 + f * nch16(r));
    put(make_int4((int)c, (int)c, 4 | (4 << 4), kMutualItem), 3 * st + 2 * diag);
    for (int k = 0; k < 4; ++k) {
        const int nr = leaf_count(ls, nside, x + kUp[k][0], y + kUp[k][1]);
        if (nr < D) continue;
        const int ds = 3 * (kUp[k][1] + 1) + (kUp[k][0] + 1);
        put(make_int4((int)c, (int)morton_encode((uint32_t)(x + kUp[k][0]), (uint32_t)(y + kUp[k][1])),
                      ds | ((8 - ds) << 4), kMutualItem),
            3 * block_steps(nt, nr));
    }
}

}  // namespace

// Exclusive scan of n uint32 (in place allowed); *total_host receives the sum if non-null.
bool scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_host, hipStream_t s, Status &st)
{
    const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
    Buf<uint32_t> sums, total;
    if (!st.check(sums.alloc(nb, s), "scan workspace") || !st.check(total.alloc(1, s), "scan workspace")) return false;
    scan_tile_sums<<<(unsigned)nb, 256, 0, s>>>(in, n, sums.p);
    scan_sums<<<1, 256, 0, s>>>(sums.p, nb, total.p);
    scan_tiles<<<(unsigned)nb, 256, 0, s>>>(in, out, n, sums.p);
    if (!st.check(hipGetLastError(), "scan launch")) return false;
    if (total_host) {
        if (!st.check(hipMemcpyAsync(total_host, total.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "scan total") ||
            !st.check(hipStreamSynchronize(s), "scan total"))
            return false;
    }
    return true;
}

// Sort (keys, vals) in place by the low `bits` bits of the keys (stable).
bool radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s, Status &st)
{
    if (n <= 1 || bits <= 0) return true;
    const int nb = (int)((n + kRsTile - 1) / kRsTile);
    Buf<uint64_t> k2;
    Buf<uint32_t> v2, counts;
    if (!st.check(k2.alloc(n, s), "sort workspace") || !st.check(v2.alloc(n, s), "sort workspace") ||
        !st.check(counts.alloc((int64_t)256 * nb, s), "sort workspace"))
        return false;
    uint64_t *ka = keys, *kb = k2.p;
    uint32_t *va = vals, *vb = v2.p;
    for (int shift = 0; shift < bits; shift += 8) {
        rs_hist<<<nb, 256, 0, s>>>(ka, n, shift, counts.p, nb);
        if (!scan_exclusive(counts.p, counts.p, (int64_t)256 * nb, nullptr, s, st)) return false;
        rs_scatter<<<nb, 256, 0, s>>>(ka, va, kb, vb, n, shift, counts.p, nb);
        if (!st.check(hipGetLastError(), "sort launch")) return false;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        if (!st.check(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s), "sort copy") ||
            !st.check(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "sort copy"))
            return false;
    }
    return true;
}


bool bounding_square(const double2 *xy, int64_t n, hipStream_t s, Status &st, double box[3], bool &nonfinite)
{
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    Buf<double4> part;
    Buf<int> flags;
    std::vector<double4> h(nb);
    int hf = 0;
    if (!st.check(part.alloc(nb, s), "bounding square") || !st.check(flags.alloc(1, s), "bounding square") ||
        !st.check(hipMemsetAsync(flags.p, 0, sizeof(int), s), "bounding square"))
        return false;
    k_minmax<<<nb, 256, 0, s>>>(xy, n, part.p, flags.p);
    if (!st.check(hipMemcpyAsync(h.data(), part.p, nb * sizeof(double4), hipMemcpyDeviceToHost, s), "bounding square") ||
        !st.check(hipMemcpyAsync(&hf, flags.p, sizeof(int), hipMemcpyDeviceToHost, s), "bounding square") ||
        !st.check(hipStreamSynchronize(s), "bounding square"))
        return false;
    nonfinite = (hf & 2) != 0;
    double xmin = h[0].x, xmax = h[0].y, ymin = h[0].z, ymax = h[0].w;
    for (int b = 1; b < nb; ++b) {
        xmin = std::min(xmin, h[b].x);
        xmax = std::max(xmax, h[b].y);
        ymin = std::min(ymin, h[b].z);
        ymax = std::max(ymax, h[b].w);
    }
    double side = std::max(xmax - xmin, ymax - ymin);
    if (side <= 0.0) side = 1.0;
    box[0] = xmin;
    box[1] = ymin;
    box[2] = side * (1.0 + 1.0 / 1048576.0);
    return true;
}


// ---------------------------------------------------------------------------------
// Near-field plan of the mutual form (stage 9), from the device leaf offsets (both
// builds use it).  A leaf is dense when it holds at least dense_leaf particles.  Every
// unordered pair of neighbouring dense leaves, and every dense leaf with itself, is one
// mutual item; every other ordered (target leaf, source leaf) pair is evaluated by the
// target-centric units, whose flag makes dense target leaves skip their dense
// neighbours.  leaf_mask[leaf]: bit d (direction d = 3(dy+1) + (dx+1) of a neighbour)
// when the particles' slot d is written, bit 9 when a target-centric unit writes their
// near-field sum.  With the mutual form off the plan is empty and the target-centric
// units cover every pair.
// ---------------------------------------------------------------------------------
int build_near_plan_device(fmm_tree *t, hipStream_t s, std::string &err)
{
    if (t->d_near_work || t->d_leaf_mask) {  // a rebuild (option change): the old plan may be in use
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            err = std::string("near-field plan: ") + hipGetErrorString(e);
            return FMM_EDEVICE;
        }
        if (t->d_near_work) hipFreeAsync(t->d_near_work, s);
        if (t->d_leaf_mask) hipFreeAsync(t->d_leaf_mask, s);
    }
    t->d_near_work = nullptr;
    t->d_leaf_mask = nullptr;
    t->nunits_tc = t->nmut = t->nnear_work = t->mutual_pairs = 0;
    if (!t->near_mutual) return FMM_OK;
    Status st;
    const int L = t->depth;
    const int64_t nleaf = int64_t(1) << (2 * L);
    Buf<uint32_t> nent;
    Buf<uint16_t> mask;
    Buf<unsigned long long> stats;
    if (!st.check(nent.alloc(nleaf + 1, s), "near-field plan") || !st.check(mask.alloc(nleaf, s, true), "near-field plan") ||
        !st.check(stats.alloc(4, s), "near-field plan") ||
        !st.check(hipMemsetAsync(stats.p, 0, 4 * sizeof(unsigned long long), s), "near-field plan")) {
        err = st.msg;
        return st.code;
    }
    k_plan_count<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(t->d_leaf_start, L, t->dense_leaf, nent.p, mask.p, stats.p);
    uint32_t total = 0;
    if (!scan_exclusive(nent.p, nent.p, nleaf + 1, &total, s, st)) {
        err = st.msg;
        return st.code;
    }
    unsigned long long hs[4];
    if (!st.check(hipMemcpyAsync(hs, stats.p, sizeof hs, hipMemcpyDeviceToHost, s), "near-field plan") ||
        !st.check(hipStreamSynchronize(s), "near-field plan")) {
        err = st.msg;
        return st.code;
    }
    Buf<int4> work, sorted;
    Buf<uint64_t> key;
    Buf<uint32_t> val;
    if (!st.check(work.alloc(total, s), "near-field plan") || !st.check(sorted.alloc(total, s, true), "near-field plan") ||
        !st.check(key.alloc(total, s), "near-field plan") || !st.check(val.alloc(total, s), "near-field plan")) {
        err = st.msg;
        return st.code;
    }
    k_plan_fill<<<grid_for(nleaf, 256), 256, 0, s>>>(t->d_leaf_start, L, t->dense_leaf, nent.p, work.p, key.p, val.p);
    if (!st.check(hipGetLastError(), "near-field plan") || !radix_sort(key.p, val.p, total, 40, s, st)) {
        err = st.msg;
        return st.code;
    }
    k_gather<int4><<<grid_for(total, 256), 256, 0, s>>>(work.p, val.p, total, sorted.p);
    if (!st.check(hipStreamSynchronize(s), "near-field plan")) {
        err = st.msg;
        return st.code;
    }
    t->d_near_work = total ? sorted.release() : nullptr;
    t->d_leaf_mask = mask.release();
    t->nunits_tc = (int64_t)hs[0];
    t->nmut = (int64_t)hs[1];
    t->mutual_pairs = (int64_t)hs[2];
    t->nnear_work = total;
    return FMM_OK;
}

// ---------------------------------------------------------------------------------
// Stages 1-3 on the device.  xy: device (n, 2) user order.  On success every device
// array of the tree and its host-side counts are set; bad_index receives the first
// offending particle for FMM_EINVAL / FMM_ERANGE.
// ---------------------------------------------------------------------------------
int build_tree_device(fmm_tree *t, const double *xy, const double *root_box, hipStream_t s, std::string &err,
                      int64_t &bad_index, const std::function<void()> &after_checks)
{
    t->pooled = true;
    Status st;
    auto failed = [&]() {
        err = st.msg;
        return st.code;
    };
    const int64_t n = t->n;
    const int L = t->depth;
    const int nside = 1 << L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const double2 *xy2 = (const double2 *)xy;
    bad_index = -1;
    Buf<int> flags;
    Buf<unsigned long long> first_bad;
    if (!st.check(flags.alloc(1, s), "tree build") || !st.check(first_bad.alloc(1, s), "tree build") ||
        !st.check(hipMemsetAsync(flags.p, 0, sizeof(int), s), "tree build") ||
        !st.check(hipMemsetAsync(first_bad.p, 0xff, sizeof(unsigned long long), s), "tree build"))
        return failed();
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
    const double w = t->side / (double)nside;
    // Stage 2: keys, then the stable sort by (leaf, sub-leaf key), ties by user index.
    Buf<uint64_t> key;
    Buf<uint32_t> val;
    if (!st.check(key.alloc(n, s), "tree build") || !st.check(val.alloc(n, s), "tree build")) return failed();
    k_keys<<<grid_for(n, 256), 256, 0, s>>>(xy2, n, t->x0, t->y0, w, nside, key.p, val.p, flags.p, first_bad.p);
    {
        int hf = 0;
        unsigned long long hb = 0;
        if (!st.check(hipMemcpyAsync(&hf, flags.p, sizeof(int), hipMemcpyDeviceToHost, s), "tree build") ||
            !st.check(hipMemcpyAsync(&hb, first_bad.p, sizeof hb, hipMemcpyDeviceToHost, s), "tree build") ||
            !st.check(hipStreamSynchronize(s), "tree build"))
            return failed();
        if (hf) {
            bad_index = (int64_t)hb;
            err = (hf & 2) ? "non-finite particle position" : "particle lies outside the root cell";
            return (hf & 2) ? FMM_EINVAL : FMM_ERANGE;
        }
    }
    if (after_checks) after_checks();
    if (!radix_sort(key.p, val.p, n, 2 * L + 12, s, st)) return failed();
    if (!st.check(hipMallocAsync((void **)&t->d_perm, n * sizeof(int), s), "permutation") ||
        !st.check(hipMallocAsync((void **)&t->d_leaf_of, n * sizeof(int), s), "leaf ids") ||
        !st.check(hipMallocAsync((void **)&t->d_xy, n * sizeof(double2), s), "sorted positions") ||
        !st.check(hipMallocAsync((void **)&t->d_leaf_start, (nleaf + 1) * sizeof(int), s), "leaf offsets"))
        return failed();
    k_sorted<<<grid_for(n, 256), 256, 0, s>>>(key.p, val.p, xy2, n, t->d_perm, t->d_leaf_of, t->d_xy);
    k_leaf_start<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(t->d_leaf_of, n, nleaf, t->d_leaf_start);
    // Occupancy of all levels.
    const int64_t ncells = level_base(L + 1);
    if (!st.check(hipMallocAsync((void **)&t->d_counts, ncells * sizeof(int), s), "cell counts")) return failed();
    k_counts<<<grid_for(ncells, 256), 256, 0, s>>>(t->d_leaf_start, L, ncells, t->d_counts);
    // Tiles and their boxes.
    uint32_t ntiles = 0;
    Buf<uint32_t> tstart;
    if (!st.check(tstart.alloc(nleaf + 1, s, true), "tile offsets")) return failed();
    k_leaf_tiles<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(t->d_leaf_start, nleaf, tstart.p);
    if (!scan_exclusive(tstart.p, tstart.p, nleaf + 1, &ntiles, s, st)) return failed();
    Buf<int> tile_leaf;
    if (!st.check(tile_leaf.alloc(ntiles, s), "tile leaves") ||
        !st.check(hipMallocAsync((void **)&t->d_tile_box, std::max<size_t>(ntiles, 1) * sizeof(float4), s), "tile boxes"))
        return failed();
    k_tile_leaf<<<grid_for(nleaf, 256), 256, 0, s>>>(tstart.p, nleaf, tile_leaf.p);
    k_tile_box<<<grid_for(ntiles, 256), 256, 0, s>>>(tile_leaf.p, tstart.p, t->d_leaf_start, t->d_xy, ntiles, t->x0,
                                                      t->y0, w, t->d_tile_box);
    t->d_tile_start = (int *)tstart.release();
    // Cell lists of levels 2..L by parity class.
    t->list_off.assign(L + 1, 0);
    t->list_len.assign(L + 1, 0);
    t->class_off.assign(4 * (L + 1), 0);
    int64_t nflags = 0;
    for (int l = 2; l <= L; ++l) nflags += int64_t(1) << (2 * l);
    uint32_t nlist = 0;
    if (nflags > 0) {
        Buf<uint32_t> pos;
        if (!st.check(pos.alloc(nflags + 1, s), "cell lists")) return failed();
        k_list_flags<<<grid_for(nflags, 256), 256, 0, s>>>(t->d_counts, nflags, pos.p);
        if (!scan_exclusive(pos.p, pos.p, nflags, &nlist, s, st)) return failed();
        if (!st.check(hipMallocAsync((void **)&t->d_lists, std::max<size_t>(nlist, 1) * sizeof(int), s), "cell lists"))
            return failed();
        k_list_scatter<<<grid_for(nflags, 256), 256, 0, s>>>(t->d_counts, nflags, pos.p, t->d_lists);
        // list offsets at the level and class boundaries
        std::vector<int64_t> idx;
        int64_t base = 0;
        for (int l = 2; l <= L; ++l) {
            const int64_t nc = int64_t(1) << (2 * l);
            for (int q = 0; q < 4; ++q) idx.push_back(base + q * (nc / 4));
            base += nc;
        }
        Buf<int64_t> didx;
        Buf<uint32_t> dval;
        std::vector<uint32_t> hv(idx.size());
        const int m = (int)idx.size();
        if (!st.check(didx.alloc(m, s), "cell lists") || !st.check(dval.alloc(m, s), "cell lists") ||
            !st.check(hipMemcpyAsync(didx.p, idx.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s), "cell lists"))
            return failed();
        k_gather_u32<<<1, 256, 0, s>>>(pos.p, didx.p, m, dval.p);
        if (!st.check(hipMemcpyAsync(hv.data(), dval.p, m * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "cell lists") ||
            !st.check(hipStreamSynchronize(s), "cell lists"))
            return failed();
        for (int l = 2; l <= L; ++l) {
            const int64_t off = hv[4 * (l - 2)];
            t->list_off[l] = off;
            for (int q = 0; q < 4; ++q) t->class_off[4 * l + q] = (int64_t)hv[4 * (l - 2) + q] - off;
            t->list_len[l] = (l < L ? (int64_t)hv[4 * (l - 1)] : (int64_t)nlist) - off;
        }
    } else if (!st.check(hipMallocAsync((void **)&t->d_lists, sizeof(int), s), "cell lists")) {
        return failed();
    }
    // Statistics and the target-centric units, heaviest first.
    Buf<unsigned long long> stats;
    Buf<int4> units;
    Buf<uint64_t> ukey;
    Buf<uint32_t> uval;
    if (!st.check(stats.alloc(4, s), "statistics") ||
        !st.check(hipMemsetAsync(stats.p, 0, 4 * sizeof(unsigned long long), s), "statistics") ||
        !st.check(units.alloc(ntiles, s), "work units") || !st.check(ukey.alloc(ntiles, s), "work units") ||
        !st.check(uval.alloc(ntiles, s), "work units"))
        return failed();
    k_leaf_stats<<<grid_for(nleaf, 256), 256, 0, s>>>(t->d_leaf_start, L, (const uint32_t *)t->d_tile_start, stats.p,
                                                       units.p, ukey.p, uval.p);
    for (int l = 2; l <= L; ++l)
        if (t->list_len[l] > 0)
            k_m2l_count<<<grid_for(t->list_len[l], 256), 256, 0, s>>>(t->d_lists + t->list_off[l], t->list_len[l], l,
                                                                       t->d_counts, stats.p);
    if (!radix_sort(ukey.p, uval.p, ntiles, 32, s, st)) return failed();
    if (!st.check(hipMallocAsync((void **)&t->d_units, std::max<size_t>(ntiles, 1) * sizeof(int4), s), "work units"))
        return failed();
    k_gather<int4><<<grid_for(ntiles, 256), 256, 0, s>>>(units.p, uval.p, ntiles, t->d_units);
    {
        unsigned long long hs[4];
        if (!st.check(hipMemcpyAsync(hs, stats.p, sizeof hs, hipMemcpyDeviceToHost, s), "statistics") ||
            !st.check(hipStreamSynchronize(s), "statistics"))
            return failed();
        t->p2p_pairs = (int64_t)hs[0] - n;
        t->nonempty_leaves = (int64_t)hs[1];
        t->max_leaf = (int64_t)hs[2];
        t->m2l_pairs = (int64_t)hs[3];
    }
    t->nunits = ntiles;
    // Staging slots of the two-pass permutations between user and sorted order.
    if (!build_staging(t->d_perm, n, s, st, t->stage_shift, t->d_gpos1, t->d_gpos2, t->d_st1)) return failed();
    if (!st.check(hipGetLastError(), "tree build") || !st.check(hipStreamSynchronize(s), "tree build"))
        return failed();
    return FMM_OK;
}

bool build_staging(const int *perm, int64_t n, hipStream_t s, Status &st, int &shift, int *&gpos1, int *&gpos2,
                   double *&st1)
{
    shift = kStageShiftMin;
    while ((((n - 1) >> shift) + 1) > kStageBuckets) ++shift;
    Buf<uint64_t> key;
    Buf<uint32_t> val;
    if (!st.check(key.alloc(n, s), "staging slots") || !st.check(val.alloc(n, s), "staging slots") ||
        !st.check(hipMallocAsync((void **)&gpos1, n * sizeof(int), s), "staging slots") ||
        !st.check(hipMallocAsync((void **)&gpos2, n * sizeof(int), s), "staging slots") ||
        !st.check(hipMallocAsync((void **)&st1, n * sizeof(double), s), "staging array"))
        return false;
    k_stage_keys<<<grid_for(n, 256), 256, 0, s>>>(perm, n, shift, key.p, val.p);
    if (!radix_sort(key.p, val.p, n, kStageBucketsLog2, s, st)) return false;
    k_gpos<<<grid_for(n, 256), 256, 0, s>>>(val.p, n, gpos1);
    k_gpos2<<<grid_for(n, 256), 256, 0, s>>>(gpos1, perm, n, gpos2);
    return st.check(hipGetLastError(), "staging slots");
}

}  // namespace fmm
