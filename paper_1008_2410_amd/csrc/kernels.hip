// gfx950 kernels of the FMM evaluation phase (stages 4-10 of Fig. fmmStages of
// Knepley, arXiv:1008.2410) and their host launchers.
//
// Conventions (shared with the host code in api.cpp / tree.cpp):
//  - Particles are in leaf-Morton order ("sorted"); d_perm maps a sorted slot to the
//    user index, d_leaf_of to its leaf.
//  - Complex charge c_j = -i Gamma_j / (2 pi) (the factor of the multipole
//    coefficients, section "Complexity Estimates"); conjugate velocity W = u - i v.
//  - Expansions are radius-scaled so every translation operator is level independent:
//    multipole a_m / w^m, local b_l w^(l+1), with w the cell width of the level.
//  - Complex numbers are interleaved (re, im) float2 / double2.
#include "fmm_internal.h"
#include "device_common.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <type_traits>

namespace fmm {
namespace {

// ---------------------------------------------------------------------------------
// Circulations from user order into tree order in two passes.  The user order is
// arbitrary (a random shuffle in the benchmark), so a direct gather makes one random
// memory access per element.  Instead, with buckets of 2^S consecutive sorted slots:
//   pass 1 (stage_in_kernel) reads a contiguous chunk of user indices, sorts it in LDS
//          by bucket and writes each bucket's elements as one run into that bucket's
//          segment of a staging array (inside a bucket, slots follow user index, so a
//          chunk's elements of one bucket are one contiguous run);
//   pass 2 (in pack_kernel) walks the sorted slots and gathers from the current
//          bucket's segment, a window small enough to stay in one XCD's L2.
// gpos1[user index] = staging slot; gpos2[sorted slot] = staging slot of its user index.
// S is chosen with the tree so that there are at most kStageBuckets.  Blocks are remapped
// so that each XCD (workgroups are dealt to XCDs round-robin) walks one contiguous index
// range, which keeps its live windows few.
// ---------------------------------------------------------------------------------
constexpr int kStageE = 4;  // elements per thread in pass 1 (chunk of 1024)

template <typename V>
__global__ __launch_bounds__(256) void stage_in_kernel(int n, int shift, int nxcd, const int *__restrict__ gpos1,
                                                        const V *__restrict__ src, V *__restrict__ st)
{
    constexpr int C = 256 * kStageE;
    __shared__ int cnt[kStageBuckets], lo[kStageBuckets], off[kStageBuckets];
    __shared__ V val[C];
    __shared__ int dst[C];
    const int t = threadIdx.x;
    const int nb = ((n - 1) >> shift) + 1;  // buckets in use, <= kStageBuckets by the choice of shift
    for (int b = t; b < nb; b += 256) {
        cnt[b] = 0;
        lo[b] = INT_MAX;
    }
    __syncthreads();
    const int64_t k0 = (int64_t)xcd_block(nxcd) * C;
    int q[kStageE];
    V v[kStageE];
#pragma unroll
    for (int e = 0; e < kStageE; ++e) {
        const int64_t k = k0 + e * 256 + t;
        q[e] = -1;
        v[e] = V{};
        if (k < n) {
            q[e] = gpos1[k];
            v[e] = src[k];
            const int bk = q[e] >> shift;
            atomicAdd(&cnt[bk], 1);
            atomicMin(&lo[bk], q[e]);
        }
    }
    __syncthreads();
    if (t < 64) {  // exclusive scan of the bucket counts by one wavefront, a run of buckets per lane
        const int per = (nb + 63) / 64;
        const int b0 = t * per, b1 = min(b0 + per, nb);
        int sum = 0;
        for (int b = b0; b < b1; ++b) sum += cnt[b];
        int incl = sum;
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d);
            if (t >= d) incl += o;
        }
        int run = incl - sum;
        for (int b = b0; b < b1; ++b) {
            off[b] = run;
            run += cnt[b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kStageE; ++e)
        if (q[e] >= 0) {
            const int bk = q[e] >> shift;
            const int slot = off[bk] + (q[e] - lo[bk]);  // < C: the bucket's run is contiguous
            val[slot] = v[e];
            dst[slot] = q[e];
        }
    __syncthreads();
    const int m = (int)min((int64_t)C, (int64_t)n - k0);
    for (int j = t; j < m; j += 256) st[dst[j]] = val[j];
}

// Pass 2 of the user-to-tree permutation: the circulation of sorted particle i, read from
// the staging array at gpos2[i] and rounded to the near field's precision (the near-field
// records' Gamma; the positions of the records are the tree's, in leaf units).
template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(int n, int nxcd, const int *__restrict__ gpos2,
                                                    const double *__restrict__ gamma_st, T *__restrict__ gam)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gam[i] = (T)gamma_st[gpos2[i]];
}

// Leaf-unit coordinates xi = (z - c_leaf)/w_L of the sorted particles (the tree's, made once
// per precision): the near-field records are xi scaled by alpha w_L on load, and L2P and
// P2M evaluate their series at xi.
template <typename T>
__global__ __launch_bounds__(256) void leaf_coords_kernel(int n, const int *__restrict__ leaf_of,
                                                           const double2 *__restrict__ xy, double x0, double y0,
                                                           double w, c2<T> *__restrict__ pos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t leaf = (uint32_t)leaf_of[i];
    const double cx = x0 + (morton_x(leaf) + 0.5) * w;
    const double cy = y0 + (morton_y(leaf) + 0.5) * w;
    const double2 z = xy[i];
    pos[i] = mk<T>((T)((z.x - cx) / w), (T)((z.y - cy) / w));
}


// ---------------------------------------------------------------------------------
// Stage 9, P2P (near field), target-centric: every pair is evaluated from the target's
// end, so no output is shared between work-items (the paper computes each pair from
// both ends to avoid memory contention).  One wavefront per work unit
// {leaf T, first target, count nt <= 64, log2 TP}: lane = k*TP + t handles target t
// and, of every 64-source tile of the 3x3 leaf neighbourhood, the sources k, k+K, ...
// (K = 64/TP), so sparse leaves still fill the wavefront.
//
// Source tiles are the 64-particle, leaf-aligned chunks of the sorted order (particles
// inside a leaf are ordered by a finer Morton key, so a tile is spatially compact).
// Each tile is staged in LDS (one coalesced load, then broadcast reads) and tested
// against the bounding box of the target chunk: when every pair of the tile has
// s >= cut, 1 - exp(-s) rounds to exactly 1 in T and the exponential is skipped --
// the result is bit-identical to evaluating it.
// Per-leaf partial sums are kept in T and folded into FP64; the K partial sums of a
// target are combined by lane shuffles.
//   velocity u = -(alpha/2pi) sum Gamma g dY/s,  v = (alpha/2pi) sum Gamma g dX/s
// ---------------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void p2p_forward_unit(const int4 u, rec_t<T> *tile, const SoaRec<T> &rec,
                                                 const int *__restrict__ leaf_start,
                                                 const int *__restrict__ tile_start,
                                                 const float4 *__restrict__ tile_box, int nside, T step,
                                                 float cut_leaf2, double scale, int dense,
                                                 double2 *__restrict__ near)
{
    const int lane = threadIdx.x;
    const int logtp = u.w & 15;
    const bool skip_dense = (u.w >> 4) != 0;  // pairs with dense leaves go to the mutual form
    const int tp = 1 << logtp;
    const int t = lane & (tp - 1);
    const int k = lane >> logtp;
    const int i = u.y + min(t, u.z - 1);
    const rec_t<T> ri = rec(i);
    const int ix = (int)morton_x((uint32_t)u.x), iy = (int)morton_y((uint32_t)u.x);
    const float4 tbox = tile_box[tile_start[u.x] + ((u.y - leaf_start[u.x]) >> 6)];
    double au = 0.0, av = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int ny = iy + dy;
        if (ny < 0 || ny >= nside) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int nx = ix + dx;
            if (nx < 0 || nx >= nside) continue;
            const uint32_t S = morton_encode((uint32_t)nx, (uint32_t)ny);
            const int s0 = leaf_start[S], s1 = leaf_start[S + 1];
            if (skip_dense && s1 - s0 >= dense) continue;
            // target relative to the centre of leaf S: z_i - c_S = (z_i - c_T) + (c_T - c_S)
            const T tx = ri.x - (T)dx * step;
            const T ty = ri.y - (T)dy * step;
            T fu = 0, fv = 0;
            int tt = tile_start[S];
            for (int base = s0; base < s1; base += 64, ++tt) {
                const int len = min(64, s1 - base);
                __syncthreads();
                if (lane < len) tile[lane] = rec(base + lane);
                const bool far = box_gap2(tbox, (float)-dx, (float)-dy, tile_box[tt]) >= cut_leaf2;
                __syncthreads();
                switch (logtp) {
                case 6: p2p_tile_any<T, 1>(tile, len, k, tx, ty, fu, fv, far); break;
                case 5: p2p_tile_any<T, 2>(tile, len, k, tx, ty, fu, fv, far); break;
                case 4: p2p_tile_any<T, 4>(tile, len, k, tx, ty, fu, fv, far); break;
                case 3: p2p_tile_any<T, 8>(tile, len, k, tx, ty, fu, fv, far); break;
                case 2: p2p_tile_any<T, 16>(tile, len, k, tx, ty, fu, fv, far); break;
                case 1: p2p_tile_any<T, 32>(tile, len, k, tx, ty, fu, fv, far); break;
                default: p2p_tile_any<T, 64>(tile, len, k, tx, ty, fu, fv, far); break;
                }
            }
            au += (double)fu;
            av += (double)fv;
        }
    }
    for (int o = tp; o < 64; o <<= 1) {
        au += __shfl_xor(au, o);
        av += __shfl_xor(av, o);
    }
    if (k == 0 && t < u.z) near[i] = make_double2(-scale * au, scale * av);
}

// Near-field grid (stage 9): one list of work entries, each one wavefront's work:
//   mutual items {S, R, d_S | d_R << 4, kMutualItem}, d_S = direction of R seen from S
//   and d_R = 8 - d_S, writing the slots (9 x n sums (dY, dX) in the records'
//   precision, unscaled);
//   target-centric units {leaf, first, count, log2 TP | 16 if dense neighbours are
//   skipped}, writing near.
// The list is sorted by estimated cost, heaviest first, and launched as one workgroup
// per entry: the hardware dispatcher hands them out in order.  Each entry writes only
// its own outputs, so the result does not depend on which wavefront takes which entry.

template <typename T>
__device__ __forceinline__ void near_entry(const int4 u, rec_t<T> *tile_a, rec_t<T> *tile_b,
                                           const SoaRec<T> &rec, const int *__restrict__ leaf_start,
                                           const int *__restrict__ tile_start, const float4 *__restrict__ tile_box,
                                           int nside, T step, float cut_leaf2, double scale, int dense, int64_t n,
                                           double2 *__restrict__ near, c2<T> *__restrict__ slots)
{
    if (u.w & kMutualItem)
        mutual_item_src<T, SoaRec<T>>(u, tile_a, tile_b, rec, leaf_start, tile_start, tile_box, step, cut_leaf2, n,
                                      slots);
    else
        p2p_forward_unit<T>(u, tile_a, rec, leaf_start, tile_start, tile_box, nside, step, cut_leaf2, scale, dense,
                            near);
}

template <typename T>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 8 : 5) void p2p_near_kernel(
    const int4 *__restrict__ work, const c2<T> *__restrict__ pos, const T *__restrict__ gam,
    const int *__restrict__ leaf_start, const int *__restrict__ tile_start, const float4 *__restrict__ tile_box,
    int nside, T step, float cut_leaf2, double scale, int dense, int64_t n, double2 *__restrict__ near,
    c2<T> *__restrict__ slots)
{
    __shared__ rec_t<T> tile_a[128], tile_b[128];
    const SoaRec<T> rec{pos, gam, step};
    near_entry<T>(work[blockIdx.x], tile_a, tile_b, rec, leaf_start, tile_start, tile_box, nside, step, cut_leaf2,
                  scale, dense, n, near, slots);
}

// Sum over the 64 lanes of each of NC values (NC = 32 or 64) by recursive halving: at
// offset o a lane keeps the half of its values that its lane bit o selects and adds its
// partner's copy of that half.  Returns the total of value lane >> 1 (NC = 32; lanes 2c
// and 2c + 1 both hold it) or of value lane (NC = 64).  Shuffles only: no LDS, so the
// kernel fits beside near-field workgroups that hold the LDS.
template <typename TC, int NC, int W, int O>
__device__ __forceinline__ void lane_halve(TC (&v)[NC], int lane)
{
    if constexpr (O >= 1) {
        if constexpr (W > 1) {
            const bool hi = (lane & O) != 0;
#pragma unroll
            for (int k = 0; k < W / 2; ++k) {
                const TC send = hi ? v[k] : v[k + W / 2];
                const TC keep = hi ? v[k + W / 2] : v[k];
                v[k] = keep + __shfl_xor(send, O);
            }
            lane_halve<TC, NC, W / 2, O / 2>(v, lane);
        } else {
            v[0] += __shfl_xor(v[0], O);
            lane_halve<TC, NC, 1, O / 2>(v, lane);
        }
    }
}
template <typename TC, int NC>
__device__ __forceinline__ TC lane_reduce_scatter(TC (&v)[NC], int lane)
{
    static_assert(NC == 32 || NC == 64, "32 or 64 values");
    lane_halve<TC, NC, NC, 32>(v, lane);
    return v[0];
}

template <typename TR, typename TC, int PMAX>
__global__ __launch_bounds__(64) void p2m_kernel(const int *__restrict__ leaves, int nleaves,
                                                  const int *__restrict__ leaf_start,
                                                  const double2 *__restrict__ xy, const c2<TC> *__restrict__ pos,
                                                  const int *__restrict__ gpos2, const double *__restrict__ gamma_st,
                                                  const typename RecScalar<TR>::type *__restrict__ gam,
                                                  const double2 *__restrict__ adj, double x0, double y0, double w,
                                                  int p, c2<TC> *__restrict__ out, int nxcd)
{
    constexpr int NC = 2 * PMAX;             // partial sums per lane (re, im interleaved)
    const int lane = threadIdx.x;
    // each XCD takes a contiguous run of leaves, so the staging windows its circulation
    // reads fall in stay in its own L2
    for (int li = xcd_block(nxcd); li < nleaves; li += gridDim.x) {
    const uint32_t leaf = (uint32_t)leaves[li];
    const int s0 = leaf_start[leaf], s1 = leaf_start[leaf + 1];
    const double cx = x0 + (morton_x(leaf) + 0.5) * w;
    const double cy = y0 + (morton_y(leaf) + 0.5) * w;
    c2<TC> acc[PMAX];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) acc[m] = mk<TC>(0, 0);
    for (int j = s0 + lane; j < s1; j += 64) {
        c2<TC> xi;
        if (pos) {
            xi = pos[j];  // the tree's leaf-unit coordinates, made by the same formula
        } else {
            const double2 z = xy[j];
            xi = mk<TC>((TC)((z.x - cx) / w), (TC)((z.y - cy) / w));
        }
        c2<TC> pw;
        if (adj) {
            const double2 q = adj[j];
            pw = mk<TC>((TC)q.x, (TC)q.y);
        } else {
            // the circulation as the records hold it (rounded to their precision): from the
            // gathered circulations, or from the staging array when P2M starts before them
            const double gj = gam ? (double)gam[j] : (double)(typename RecScalar<TR>::type)gamma_st[gpos2[j]];
            pw = mk<TC>(0, (TC)(-gj * kInv2Pi));
        }
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            if (m < p) {
                acc[m].x += pw.x;
                acc[m].y += pw.y;
                pw = cmul<TC>(pw, xi);
            }
        }
    }
    TC v[NC];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) {
        v[2 * m] = acc[m].x;
        v[2 * m + 1] = acc[m].y;
    }
    const TC sum = lane_reduce_scatter<TC, NC>(v, lane);
    const int c = NC == 64 ? lane : lane >> 1;  // the value this lane holds
    if ((NC == 64 || (lane & 1) == 0) && c < 2 * p) ((TC *)out)[(int64_t)leaf * 2 * p + c] = sum;
    }
}

// ---------------------------------------------------------------------------------
// Stage 5, M2M: coefficient m of parent P from its non-empty children,
//   A_m = sum_q sum_{k<=m} C(m,k) d_q^(m-k) 2^-k a_k(child q)      (scaled form)
// ---------------------------------------------------------------------------------
template <typename TC, typename TP>
__device__ __forceinline__ void m2m_one(int P, int m, int p, const int *__restrict__ child_count,
                                        const c2<TC> *__restrict__ child, c2<TP> *__restrict__ parent,
                                        const c2<TP> *__restrict__ tab)
{
    c2<TP> acc = mk<TP>(0, 0);
    for (int q = 0; q < 4; ++q) {
        const int ch = 4 * P + q;
        if (child_count[ch] == 0) continue;
        const c2<TC> *a = child + (int64_t)ch * p;
        const c2<TP> *row = tab + (q * p + m) * p;
        for (int k = 0; k <= m; ++k) acc = cmac<TP>(acc, row[k], cvt<TP, TC>(a[k]));
    }
    parent[(int64_t)P * p + m] = acc;
}

// ---------------------------------------------------------------------------------
// Stages 6 + 7 fused per cell: local coefficient l of cell T at level `level`,
//   b_l(T) = sum_{S in IL(T), S non-empty} sum_m (-1)^l C(l+m,m) delta^-(l+m+1) a_m(S)
//          + sum_{k>=l} C(k,l) d_q^(k-l) 2^-(l+1) b_k(parent(T))   (levels >= 3)
// IL(T) = children of the parent's neighbours that are not neighbours of T: for the
// parity class (qx, qy) = (tx & 1, ty & 1) the source offsets are
// dx in [-2-qx, 3-qx], dy in [-2-qy, 3-qy] minus the 3x3 block (27 cells).
// ---------------------------------------------------------------------------------
template <typename T, typename TPar>
__device__ __forceinline__ void m2l_one(int Tm, int lo, int p, int level, const int *__restrict__ count_l,
                                        const c2<T> *__restrict__ mp_l, c2<T> *__restrict__ lo_l,
                                        const c2<T> *__restrict__ m2l_tab, const c2<TPar> *__restrict__ loc_par,
                                        const c2<TPar> *__restrict__ l2l_tab)
{
    const int tx = (int)morton_x((uint32_t)Tm), ty = (int)morton_y((uint32_t)Tm);
    const int qx = tx & 1, qy = ty & 1;
    const int nside = 1 << level;
    c2<T> acc = mk<T>(0, 0);
    for (int dy = -2 - qy; dy <= 3 - qy; ++dy) {
        const int sy = ty + dy;
        if (sy < 0 || sy >= nside) continue;
        for (int dx = -2 - qx; dx <= 3 - qx; ++dx) {
            if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
            const int sx = tx + dx;
            if (sx < 0 || sx >= nside) continue;
            const uint32_t S = morton_encode((uint32_t)sx, (uint32_t)sy);
            if (count_l[S] == 0) continue;
            const c2<T> *a = mp_l + (int64_t)S * p;
            // delta = (c_T - c_S)/w = (-dx, -dy)
            const c2<T> *tab = m2l_tab + ((3 - dx) * 7 + (3 - dy)) * p * p + lo;
            for (int m = 0; m < p; ++m) acc = cmac<T>(acc, tab[m * p], a[m]);
        }
    }
    if (loc_par) {
        const int P = Tm >> 2, q = Tm & 3;
        const c2<TPar> *b = loc_par + (int64_t)P * p;
        const c2<TPar> *row = l2l_tab + (q * p + lo) * p;
        c2<TPar> acc2 = mk<TPar>(0, 0);
        for (int k = lo; k < p; ++k) acc2 = cmac<TPar>(acc2, row[k], b[k]);
        acc.x += (T)acc2.x;
        acc.y += (T)acc2.y;
    }
    lo_l[(int64_t)Tm * p + lo] = acc;
}

// ---------------------------------------------------------------------------------
// Stages 6 + 7 on MFMA (FP32, p <= 16).  For a target cell T of parity class q the
// local expansion is a sum of 28 dense products of 2p-vectors with 2p x 2p real
// matrices (the complex operators embedded with interleaved (re, im) rows/columns):
//   L(T) = sum_{o in IL offsets of q} M(T + o) R_o  +  L(parent(T)) R^{L2L}_q.
// All targets of one parity class share the 28 matrices, so each wavefront takes 4
// tiles of 32 same-class targets and accumulates 32 x 32 output tiles with
// v_mfma_f32_32x32x2f32 (16 instructions per offset and tile, K = 32).  Empty and
// out-of-domain source cells contribute zero rows (multipoles of empty cells are
// kept at zero).  Operand layouts of the 32x32x2 instruction:
//   A: lane l holds A[row l%32][k l/32]     B: lane l holds B[k l/32][col l%32]
//   D: lane l, register r holds D[8(r/4) + 4(l/32) + r%4][l%32]
// K is permuted so that step s uses k = 16(l/32) + s: a lane then reads 16
// contiguous floats of its row, and the table stores B as [slot][l/32][col][s].
// ---------------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));


// a[s] = row[k0 + s] for k0 + s < two_p, else 0.  Every coefficient array carries a
// tail pad of 64 elements and absent sources read a zero row, so the 16 reads of a
// half row never leave their allocation.
__device__ __forceinline__ void load_half_row(float (&a)[16], const float *row, int k0, int two_p)
{
    const float *r = row + k0;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const float v = r[s];
        a[s] = (k0 + s < two_p) ? v : 0.0f;
    }
}
__device__ __forceinline__ void load_half_row(float (&a)[16], const double *row, int k0, int two_p)
{
    const double *r = row + k0;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const double v = r[s];
        a[s] = (k0 + s < two_p) ? (float)v : 0.0f;
    }
}

// One 32-target tile per wavefront: the 28 (M2L) or 4 (M2M) products of a tile run as
// one chain of 16-instruction groups.  Entries {dx, dy, slot, kind} of a class:
//   kind 0: M2L source cell (tx + dx, ty + dy) of the same level (skipped if outside)
//   kind 1: L2L from the parent's local expansion
//   kind 2: M2M from child dx (cell 4 T + dx of the next finer level)
// Operands of one gather-GEMM entry {dx, dy, slot, kind} for this lane: b = the 16
// table values of column `row`, half kh; a = 16 values of the source row.
template <typename TPar>
__device__ __forceinline__ void gemm_load_entry(int4 en, int kh, int row, int tx, int ty, int tcell, bool tvalid,
                                                int nside, int k0, int two_p, int p,
                                                const float *__restrict__ src_same,
                                                const float *__restrict__ src_child,
                                                const c2<TPar> *__restrict__ loc_par, const float *__restrict__ tab,
                                                const double *__restrict__ zero, float (&a)[16], float (&b)[16])
{
    const float4 *bsrc = (const float4 *)(tab + ((size_t)(en.z * 2 + kh) * 32 + row) * 16);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float4 t4 = bsrc[v];
        b[4 * v] = t4.x;
        b[4 * v + 1] = t4.y;
        b[4 * v + 2] = t4.z;
        b[4 * v + 3] = t4.w;
    }
    if (en.w == 1) {
        load_half_row(a, (tvalid && loc_par) ? (const TPar *)(loc_par + (size_t)(tcell >> 2) * p) : (const TPar *)zero,
                      k0, two_p);
    } else {
        const float *src = (const float *)zero;
        if (en.w == 0) {
            const int sx = tx + en.x, sy = ty + en.y;
            if (tvalid && sx >= 0 && sy >= 0 && sx < nside && sy < nside)
                src = src_same + (size_t)morton_encode((uint32_t)sx, (uint32_t)sy) * two_p;
        } else if (tvalid) {
            src = src_child + (size_t)(4 * tcell + en.x) * two_p;
        }
        load_half_row(a, src, k0, two_p);
    }
}

template <typename TPar, typename TOut>
__global__ __launch_bounds__(256, 4) void gather_gemm_kernel(
    const int *__restrict__ targets, int4 class_start, int4 class_len, int4 class_wave0, int4 class_entry,
    int4 class_nentry, int nwaves, int p, int level, const int4 *__restrict__ entries, const float *__restrict__ src_same,
    const float *__restrict__ src_child, const c2<TPar> *__restrict__ loc_par, TOut *__restrict__ out,
    const float *__restrict__ tab, const double *__restrict__ zero)
{
    const int lane = threadIdx.x & 63;
    const int wave_step = (int)((gridDim.x * blockDim.x) >> 6);
    for (int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); wave < nwaves; wave += wave_step) {
    const int q = wave >= class_wave0.w ? 3 : wave >= class_wave0.z ? 2 : wave >= class_wave0.y ? 1 : 0;
    const int cstart = q == 0 ? class_start.x : q == 1 ? class_start.y : q == 2 ? class_start.z : class_start.w;
    const int clen = q == 0 ? class_len.x : q == 1 ? class_len.y : q == 2 ? class_len.z : class_len.w;
    const int cw0 = q == 0 ? class_wave0.x : q == 1 ? class_wave0.y : q == 2 ? class_wave0.z : class_wave0.w;
    const int e0 = q == 0 ? class_entry.x : q == 1 ? class_entry.y : q == 2 ? class_entry.z : class_entry.w;
    const int ne = q == 0 ? class_nentry.x : q == 1 ? class_nentry.y : q == 2 ? class_nentry.z : class_nentry.w;
    const int base = (wave - cw0) * 32;
    const int row = lane & 31, kh = lane >> 5;
    const int two_p = 2 * p;
    const int nside = 1 << level;
    const int k0 = 16 * kh;

    const int li = base + row;
    const bool tvalid = li < clen;
    const int tcell = tvalid ? targets[cstart + li] : 0;
    const int tx = (int)morton_x((uint32_t)tcell), ty = (int)morton_y((uint32_t)tcell);

    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int e = 0; e < ne; ++e) {
        float a[16], b[16];
        gemm_load_entry<TPar>(entries[e0 + e], kh, row, tx, ty, tcell, tvalid, nside, k0, two_p, p, src_same,
                              src_child, loc_par, tab, zero, a, b);
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], acc, 0, 0, 0);
    }
    // Store: lane holds column `row` of rows 8(r/4) + 4 kh + r%4; the cell of output row
    // o is the target of lane o.
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int orow = 8 * (r >> 2) + 4 * kh + (r & 3);
        const int cell = __shfl(tcell, orow);
        if (row < two_p && base + orow < clen) out[(size_t)cell * two_p + row] = (TOut)acc[r];
    }
    }
}

// ---------------------------------------------------------------------------------
// The same gather-GEMM in FP64 on v_mfma_f64_16x16x4f64 (tiles of 16 targets, two
// 16-column output blocks).  Operand layouts of the 16x16x4 instruction:
//   A: lane l holds A[row l%16][k l/16]     B: lane l holds B[k l/16][col l%16]
//   D: lane l, register r holds D[l/16 + 4r][l%16]
// K is permuted so that step s uses k = 8(l/16) + s; the table stores B as
// [slot][l/16][column][s].
// ---------------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));

// a[s] = row[k0 + s] for k0 + s < two_p, else 0 (rows padded as for load_half_row).
__device__ __forceinline__ void load_row8(double (&a)[8], const double *row, int k0, int two_p)
{
    const double *r = row + k0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double v = r[s];
        a[s] = (k0 + s < two_p) ? v : 0.0;
    }
}

// One wavefront: the 16 targets tlist[base .. base + 15] (clen entries valid).
__device__ __forceinline__ void gemm_tile_f64(const int *__restrict__ tlist, int clen, int base,
                                              const int4 *__restrict__ ents, int ne, int p, int level,
                                              const double *__restrict__ src_same,
                                              const double *__restrict__ src_child,
                                              const double *__restrict__ loc_par, double *__restrict__ out,
                                              const double *__restrict__ tab, const double *__restrict__ zero)
{
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    const int two_p = 2 * p;
    const int k0 = 8 * kq;
    const int nside = 1 << level;
    const int li = base + row;
    const bool tvalid = li < clen;
    const int tcell = tvalid ? tlist[li] : 0;
    const int tx = (int)morton_x((uint32_t)tcell), ty = (int)morton_y((uint32_t)tcell);
    doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < ne; ++e) {
        const int4 en = ents[e];
        const double *b0p = tab + (((size_t)en.z * 4 + kq) * 32 + row) * 8;
        const double *b1p = b0p + 16 * 8;
        double a[8], b0[8], b1[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double2 u0 = ((const double2 *)b0p)[v], u1 = ((const double2 *)b1p)[v];
            b0[2 * v] = u0.x;
            b0[2 * v + 1] = u0.y;
            b1[2 * v] = u1.x;
            b1[2 * v + 1] = u1.y;
        }
        const double *src = zero;
        if (en.w == 0) {
            const int sx = tx + en.x, sy = ty + en.y;
            if (tvalid && sx >= 0 && sy >= 0 && sx < nside && sy < nside)
                src = src_same + (size_t)morton_encode((uint32_t)sx, (uint32_t)sy) * two_p;
        } else if (en.w == 1) {
            if (tvalid && loc_par) src = loc_par + (size_t)(tcell >> 2) * two_p;
        } else {
            if (tvalid) src = src_child + (size_t)(4 * tcell + en.x) * two_p;
        }
        load_row8(a, src, k0, two_p);
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b0[st], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b1[st], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = base + kq + 4 * r;
        if (lo < clen) {
            double *o = out + (size_t)tlist[lo] * two_p;
            if (row < two_p) o[row] = acc0[r];
            if (16 + row < two_p) o[16 + row] = acc1[r];
        }
    }
}

// Out-of-line copy for the coarse kernel, which calls it from two loops.
__device__ __noinline__ void gemm_tile_f64_call(const int *__restrict__ tlist, int clen, int base,
                                                const int4 *__restrict__ ents, int ne, int p, int level,
                                                const double *__restrict__ src_same,
                                                const double *__restrict__ src_child,
                                                const double *__restrict__ loc_par, double *__restrict__ out,
                                                const double *__restrict__ tab, const double *__restrict__ zero)
{
    gemm_tile_f64(tlist, clen, base, ents, ne, p, level, src_same, src_child, loc_par, out, tab, zero);
}

struct LevelClasses {
    int start[4], len[4], wave0[4];
    int waves;
};

// Wide FP64 launch over one level: wavefront w takes tile w of its class.
__global__ __launch_bounds__(256, 4) void gather_gemm_f64_kernel(const int *__restrict__ targets, LevelClasses lc,
                                                              int4 class_entry, int ne_l2l, int ne_m2m, int mode,
                                                              int p, int level, const int4 *__restrict__ entries,
                                                              const double *__restrict__ src_same,
                                                              const double *__restrict__ src_child,
                                                              const double *__restrict__ loc_par,
                                                              double *__restrict__ out, const double *__restrict__ tab,
                                                              const double *__restrict__ zero)
{
    const int wave_step = (int)((gridDim.x * blockDim.x) >> 6);
    for (int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); wave < lc.waves; wave += wave_step) {
        int q = 0;
        for (int c = 1; c < 4; ++c)
            if (wave >= lc.wave0[c]) q = c;
        const int e0 = q == 0 ? class_entry.x : q == 1 ? class_entry.y : q == 2 ? class_entry.z : class_entry.w;
        const int ne = mode == 2 ? ne_m2m : ne_l2l;
        gemm_tile_f64(targets + lc.start[q], lc.len[q], (wave - lc.wave0[q]) * 16, entries + e0, ne, p, level,
                      src_same, src_child, loc_par, out, tab, zero);
    }
}

template <typename TC, typename TP>
__global__ __launch_bounds__(256) void m2m_kernel(const int *__restrict__ parents, int nparents, int p,
                                                   const int *__restrict__ child_count,
                                                   const c2<TC> *__restrict__ child, c2<TP> *__restrict__ parent,
                                                   const c2<TP> *__restrict__ tab)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = g / p;
    if (cell >= nparents) return;
    const int m = (int)(g - cell * p);
    m2m_one<TC, TP>(parents[cell], m, p, child_count, child, parent, tab);
}

template <typename T, typename TPar>
__global__ __launch_bounds__(256) void m2l_kernel(const int *__restrict__ targets, int ntargets, int p, int level,
                                                   const int *__restrict__ count_l, const c2<T> *__restrict__ mp_l,
                                                   c2<T> *__restrict__ lo_l, const c2<T> *__restrict__ m2l_tab,
                                                   const c2<TPar> *__restrict__ loc_par,
                                                   const c2<TPar> *__restrict__ l2l_tab)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = g / p;
    if (cell >= ntargets) return;
    const int lo = (int)(g - cell * p);
    m2l_one<T, TPar>(targets[cell], lo, p, level, count_l, mp_l, lo_l, m2l_tab, loc_par, l2l_tab);
}

// ---------------------------------------------------------------------------------
// Coarse levels (<= L_c) in one workgroup: M2M into levels L_c-1..2, then M2L + L2L
// for levels 2..L_c, in FP64 on MFMA (16 wavefronts, one 16-target tile each per
// pass).  These levels hold too few cells to fill the chip; the paper assigns them to
// a single thread group and covers their latency with the near-field work (section
// "Concurrency").
// ---------------------------------------------------------------------------------
// One workgroup of up to 16 wavefronts (four per SIMD of its CU): each level's tiles are
// dealt to the wavefronts, so a level of 1024 cells takes four rounds of gathers with 16
// wavefronts instead of 16 rounds with 4.  Beside a near field capped below the full
// occupancy only one wavefront per SIMD fits in the registers it leaves, so the kernel is
// then launched with 4 (FarArgs::coarse_threads).
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseMaxLevel = 4;

struct CoarseArgs {
    int p, lc;
    const int *lists;
    int64_t list_off[kMaxDepth + 1];
    int64_t list_len[kMaxDepth + 1];
    int64_t class_off[4 * (kMaxDepth + 1)];
    double2 *mp, *lo;   // FP64 storage from level 0
    const int4 *entries;
    const double *tab;
    const double *zero;
};

__global__ __launch_bounds__(kCoarseThreads) void coarse_kernel(CoarseArgs a)
{
    const int p = a.p;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int l = a.lc - 1; l >= 2; --l) {
        const int n = (int)a.list_len[l];
        const int *lst = a.lists + a.list_off[l];
        for (int tile = wave; tile * 16 < n; tile += nw)
            gemm_tile_f64_call(lst, n, tile * 16, a.entries + 112, 4, p, l, nullptr,
                          (const double *)(a.mp + level_base(l + 1) * p), nullptr,
                          (double *)(a.mp + level_base(l) * p), a.tab, a.zero);
        __syncthreads();
    }
    for (int l = 2; l <= a.lc; ++l) {
        const int n = (int)a.list_len[l];
        const int *lst = a.lists + a.list_off[l];
        const int64_t *co = &a.class_off[4 * l];
        // tiles of the four parity classes, numbered consecutively
        int ntile[4], tot = 0;
        for (int q = 0; q < 4; ++q) {
            const int len = (int)((q < 3 ? co[q + 1] : n) - co[q]);
            ntile[q] = (len + 15) / 16;
            tot += ntile[q];
        }
        for (int tile = wave; tile < tot; tile += nw) {
            int q = 0, tq = tile;
            while (tq >= ntile[q]) {
                tq -= ntile[q];
                ++q;
            }
            const int len = (int)((q < 3 ? co[q + 1] : n) - co[q]);
            gemm_tile_f64_call(lst + co[q], len, tq * 16, a.entries + 28 * q, l >= 3 ? 28 : 27, p, l,
                          (const double *)(a.mp + level_base(l) * p), nullptr,
                          l >= 3 ? (const double *)(a.lo + level_base(l - 1) * p) : nullptr,
                          (double *)(a.lo + level_base(l) * p), a.tab, a.zero);
        }
        __syncthreads();
    }
}

// VALU form of the coarse-level kernel for p > 16 (no MFMA tables).
struct CoarseValuArgs {
    int p, lc;
    const int *counts;  // global cell index
    const int *lists;
    int64_t list_off[kMaxDepth + 1];
    int64_t list_len[kMaxDepth + 1];
    double2 *mp, *lo;   // FP64 storage from level 0
    const double2 *m2m_tab, *m2l_tab, *l2l_tab;
};

__global__ __launch_bounds__(1024) void coarse_valu_kernel(CoarseValuArgs a)
{
    const int p = a.p;
    for (int l = a.lc - 1; l >= 2; --l) {
        const int n = (int)a.list_len[l];
        const int *lst = a.lists + a.list_off[l];
        for (int g = threadIdx.x; g < n * p; g += blockDim.x) {
            const int c = g / p, m = g - c * p;
            m2m_one<double, double>(lst[c], m, p, a.counts + level_base(l + 1), a.mp + level_base(l + 1) * p,
                                    a.mp + level_base(l) * p, a.m2m_tab);
        }
        __syncthreads();
    }
    for (int l = 2; l <= a.lc; ++l) {
        const int n = (int)a.list_len[l];
        const int *lst = a.lists + a.list_off[l];
        for (int g = threadIdx.x; g < n * p; g += blockDim.x) {
            const int c = g / p, lo = g - c * p;
            m2l_one<double, double>(lst[c], lo, p, l, a.counts + level_base(l), a.mp + level_base(l) * p,
                                    a.lo + level_base(l) * p, a.m2l_tab,
                                    l >= 3 ? a.lo + level_base(l - 1) * p : nullptr, a.l2l_tab);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// Stages 8 + 10: L2P from the leaf's local expansion (Horner in xi = (z - c)/w_L,
// W_far = (1/w_L) sum_l b_l xi^l), plus the near field, scattered to user order:
// (u, v) = (u_near + Re W_far, v_near - Im W_far).  (A two-pass scatter through a
// staging array, as for the circulations, measured no faster for (u, v) pairs.)
// ---------------------------------------------------------------------------------
// Near field of a particle: with the mutual form (mask != NULL), the target-centric
// part (if mask bit 9 of its leaf) plus the slots d with mask bit d, in order d = 0..8.
template <typename TL, typename TS>
__global__ __launch_bounds__(256) void finalize_kernel(int n, const int *__restrict__ perm,
                                                        const int *__restrict__ leaf_of,
                                                        const double2 *__restrict__ xy,
                                                        const double2 *__restrict__ near,
                                                        const uint16_t *__restrict__ mask,
                                                        const c2<TS> *__restrict__ slots, double scale,
                                                        const c2<TL> *__restrict__ loc, const c2<TL> *__restrict__ pos,
                                                        int p, int has_far, double x0,
                                                        double y0, double w, double *__restrict__ uv,
                                                        double *__restrict__ uv_near, double *__restrict__ uv_far,
                                                        double2 *__restrict__ staged, const int *__restrict__ gpos2,
                                                        int nxcd)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = staged ? 0 : perm[i];  // issued with the first loads
    const uint32_t leaf = (uint32_t)leaf_of[i];
    const double2 nr = mask ? near_from_slots<TS>(i, n, mask[leaf], near, slots, scale) : near[i];
    double fu = 0.0, fv = 0.0;
    if (has_far) {
        const double cx = x0 + (morton_x(leaf) + 0.5) * w;
        const double cy = y0 + (morton_y(leaf) + 0.5) * w;
        c2<TL> xi;
        if (pos) {
            xi = pos[i];  // the tree's leaf-unit coordinates, made by the same formula
        } else {
            const double2 z = xy[i];
            xi = mk<TL>((TL)((z.x - cx) / w), (TL)((z.y - cy) / w));
        }
        const c2<TL> acc = horner_prefetch<TL>(loc + (int64_t)leaf * p, p, xi);
        fu = (double)acc.x / w;
        fv = -(double)acc.y / w;
    }
    if (staged) {  // at gpos2[i], inside its bucket's window, or else at i
        staged[gpos2 ? gpos2[i] : i] = make_double2(nr.x + fu, nr.y + fv);
        return;
    }
    if (uv) {
        uv[2 * o] = nr.x + fu;
        uv[2 * o + 1] = nr.y + fv;
    }
    if (uv_near) {
        uv_near[2 * o] = nr.x;
        uv_near[2 * o + 1] = nr.y;
    }
    if (uv_far) {
        uv_far[2 * o] = fu;
        uv_far[2 * o + 1] = fv;
    }
}

// Pass 2 of the tree-to-user permutation for large n (the mirror of the circulations'
// two passes): finalize wrote each total at gpos2[i], inside the window of its sorted
// bucket, where the random writes merge in L2; here user row u reads its slot gpos1[u]
// (a chunk of users reads one short run per bucket) and the rows go out in user order.
// The direct scatter to user order (scatter_rows_kernel) makes one random 16-byte write
// per row, which is cheaper while the output is smaller than the chip's 256 MiB last-level
// cache; for 2^25 rows (537 MB) the scatter alone took 1.12 ms, and the windows save 0.3 ms
// per evaluation.  With windows of 2^14 slots (1024 buckets at 2^24 rows) the writes of a
// window stay in the XCD's L2 until their lines are whole: 2^24 patches, 8.35 -> 8.29 ms
// per evaluation against windows of 2^17.
__global__ __launch_bounds__(256) void gather_rows_kernel(int n, int nxcd, const int *__restrict__ gpos1,
                                                          const double2 *__restrict__ staged,
                                                          double *__restrict__ uv, const double *__restrict__ base,
                                                          double h)
{
    const int u = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (u >= n) return;
    store_velocity(uv, u, staged[gpos1[u]], base, h);
}

inline unsigned blocks_for(int64_t work, int per_block) { return (unsigned)((work + per_block - 1) / per_block); }

// A grid of whole rounds over the XCDs, for kernels that index blocks with xcd_block.
inline unsigned xcd_grid(int64_t work, int per_block) { return fmm::xcd_grid(work, per_block, kXcds); }


template <typename T> c2<T> *level_ptr(const FarArgs &a, int l, bool local);
template <> double2 *level_ptr<double>(const FarArgs &a, int l, bool local)
{
    return (local ? a.lo_d : a.mp_d) + level_base(l) * a.p;
}
template <> float2 *level_ptr<float>(const FarArgs &a, int l, bool local)
{
    return (local ? a.lo_f : a.mp_f) + (level_base(l) - level_base(a.split + 1)) * a.p;
}

const int *level_list(const fmm_tree *t, int l) { return t->d_lists + t->list_off[l]; }

template <typename TR, typename TC>
void p2m_launch(const FarArgs &a, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int L = t->depth;
    const int64_t nl = t->list_len[L];
    if (nl == 0) return;
    const double w = t->side / (double)(1 << L);
    c2<TC> *out = level_ptr<TC>(a, L, false);
    // one leaf per workgroup, contiguous per XCD
    const unsigned g = xcd_grid(nl, 1);
    const int nxcd = kXcds;
    // the leaf-unit coordinates when they are in the precision of the expansions
    using TRs = typename RecScalar<TR>::type;
    const c2<TC> *pos = std::is_same<TRs, TC>::value ? (const c2<TC> *)a.pos : nullptr;
    const TRs *gam = (const TRs *)a.gam;
    if (a.p <= 16)
        p2m_kernel<TR, TC, 16><<<g, 64, 0, s>>>(level_list(t, L), (int)nl, t->d_leaf_start, t->d_xy, pos,
                                                t->d_gpos2, t->d_st1, gam, a.adj, t->x0, t->y0, w, a.p, out, nxcd);
    else
        p2m_kernel<TR, TC, 32><<<g, 64, 0, s>>>(level_list(t, L), (int)nl, t->d_leaf_start, t->d_xy, pos,
                                                t->d_gpos2, t->d_st1, gam, a.adj, t->x0, t->y0, w, a.p, out, nxcd);
}

template <typename TC, typename TP>
void m2m_launch(const FarArgs &a, int l, const c2<TP> *tab, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int64_t n = t->list_len[l];
    if (n == 0) return;
    m2m_kernel<TC, TP><<<blocks_for(n * a.p, 256), 256, 0, s>>>(
        level_list(t, l), (int)n, a.p, t->d_counts + level_base(l + 1), level_ptr<TC>(a, l + 1, false),
        level_ptr<TP>(a, l, false), tab);
}

// Split a level list into up to four classes of 32-target tiles (one wavefront each).
struct ClassTiles {
    int start[4], len[4], wave0[4], waves;
};

ClassTiles class_tiles(const int64_t *class_off, int64_t n, int nclass)
{
    ClassTiles c{};
    for (int q = 0; q < 4; ++q) {
        if (q < nclass) {
            c.start[q] = (int)class_off[q];
            c.len[q] = (int)((q + 1 < nclass ? class_off[q + 1] : n) - class_off[q]);
        } else {
            c.start[q] = (int)n;
            c.len[q] = 0;
        }
        c.wave0[q] = c.waves;
        c.waves += (c.len[q] + 31) / 32;
    }
    return c;
}

inline int4 i4(const int (&v)[4]) { return make_int4(v[0], v[1], v[2], v[3]); }

// Stages 6 + 7 at level l on MFMA: local expansions of the non-empty cells.
template <typename TPar>
void m2l_mfma_launch(const FarArgs &a, int l, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int64_t n = t->list_len[l];
    if (n == 0) return;
    const ClassTiles c = class_tiles(&t->class_off[4 * l], n, 4);
    const c2<TPar> *par = l >= 3 ? level_ptr<TPar>(a, l - 1, true) : nullptr;
    const int ne = par ? 28 : 27;  // the L2L entry is last in each class
    gather_gemm_kernel<TPar, float><<<blocks_for(c.waves, 4), 256, 0, s>>>(
        level_list(t, l), i4(c.start), i4(c.len), i4(c.wave0), make_int4(0, 28, 56, 84), make_int4(ne, ne, ne, ne),
        c.waves, a.p, l, t->tabs->mfma_entries, (const float *)level_ptr<float>(a, l, false), nullptr, par,
        (float *)level_ptr<float>(a, l, true), t->tabs->mfma_f, t->tabs->zero_row);
}

// Stage 5 into level l on MFMA from the FP32 child level l + 1.
template <typename TP>
void m2m_mfma_launch(const FarArgs &a, int l, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int64_t n = t->list_len[l];
    if (n == 0) return;
    const int64_t one_class[1] = {0};
    const ClassTiles c = class_tiles(one_class, n, 1);
    gather_gemm_kernel<float, TP><<<blocks_for(c.waves, 4), 256, 0, s>>>(
        level_list(t, l), i4(c.start), i4(c.len), i4(c.wave0), make_int4(112, 112, 112, 112), make_int4(4, 0, 0, 0),
        c.waves, a.p, l, t->tabs->mfma_entries, nullptr, (const float *)level_ptr<float>(a, l + 1, false), nullptr,
        (TP *)level_ptr<TP>(a, l, false), t->tabs->mfma_f, t->tabs->zero_row);
}

LevelClasses level_classes(const int64_t *class_off, int64_t n, int nclass)
{
    LevelClasses c{};
    for (int q = 0; q < 4; ++q) {
        if (q < nclass) {
            c.start[q] = (int)class_off[q];
            c.len[q] = (int)((q + 1 < nclass ? class_off[q + 1] : n) - class_off[q]);
        } else {
            c.start[q] = (int)n;
            c.len[q] = 0;
        }
        c.wave0[q] = c.waves;
        c.waves += (c.len[q] + 15) / 16;
    }
    return c;
}

// FP64 stages 6 + 7 (mode 0) or stage 5 (mode 2) at level l on MFMA.
void gemm_f64_launch(const FarArgs &a, int l, int mode, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int64_t n = t->list_len[l];
    if (n == 0) return;
    const int64_t one_class[1] = {0};
    const LevelClasses c = mode == 2 ? level_classes(one_class, n, 1) : level_classes(&t->class_off[4 * l], n, 4);
    const int p = a.p;
    gather_gemm_f64_kernel<<<blocks_for(c.waves, 4), 256, 0, s>>>(
        level_list(t, l), c, mode == 2 ? make_int4(112, 112, 112, 112) : make_int4(0, 28, 56, 84), l >= 3 ? 28 : 27, 4,
        mode, p, l, t->tabs->mfma_entries, mode == 0 ? (const double *)(a.mp_d + level_base(l) * p) : nullptr,
        mode == 2 ? (const double *)(a.mp_d + level_base(l + 1) * p) : nullptr,
        (mode == 0 && l >= 3) ? (const double *)(a.lo_d + level_base(l - 1) * p) : nullptr,
        (double *)((mode == 0 ? a.lo_d : a.mp_d) + level_base(l) * p), t->tabs->mfma_d, t->tabs->zero_row);
}

template <typename T, typename TPar>
void m2l_launch(const FarArgs &a, int l, const c2<T> *m2l_tab, const c2<TPar> *l2l_tab, hipStream_t s)
{
    const fmm_tree *t = a.t;
    const int64_t n = t->list_len[l];
    if (n == 0) return;
    const c2<TPar> *par = l >= 3 ? level_ptr<TPar>(a, l - 1, true) : nullptr;
    m2l_kernel<T, TPar><<<blocks_for(n * a.p, 256), 256, 0, s>>>(
        level_list(t, l), (int)n, a.p, l, t->d_counts + level_base(l), level_ptr<T>(a, l, false),
        level_ptr<T>(a, l, true), m2l_tab, par, l2l_tab);
}

// ---------------------------------------------------------------------------------
// Backward pass (adjoint of stages 4-10 for a loss L(u)).
// q_i = dL/du_i + i dL/dv_i.  With W = A c and A antisymmetric (A_ij = -A_ji),
//   dL/dGamma_j = -Im((A q)_j)/(2 pi)
// and, with the sources held fixed, dW_i/dx_i = A_i + B_i + W'_far, dW_i/dy_i = i(A_i - B_i + W'_far),
//   A_i = sum_j c_j conj(dz)^2 f'(s),  B_i = sum_j c_j g'(s),   f = g/s, s = |dz|^2,
// so dL/dx_i = Re(q_i (A+B+W')), dL/dy_i = -Im(q_i (A-B+W')).  The particle's own blob
// (dz = 0) contributes B = c_i/(2 sigma^2) and nothing else.
// In the scaled variable s' = alpha^2 |dz|^2 (alpha as in the forward records) and with
// lambda = 1 (FP64, base e) or ln 2 (FP32, base 2):
//   Phi_near = alpha sum_j q_j (g/s') conj(dz'),
//   A = -i alpha^2/(2 pi) sum_j Gamma_j conj(dz')^2 (lambda e s' - g)/s'^2,
//   B = -i alpha^2 lambda/(2 pi) sum_j Gamma_j e,        e = exp(-|dz|^2/(2 sigma^2)), g = 1 - e.
// ---------------------------------------------------------------------------------
// The cotangent reaches tree order as the circulations do: staged by bucket (stage_in_kernel
// on rows of two doubles), then gathered by sorted slot here.
template <typename T>
__global__ __launch_bounds__(256) void pack_adjoint_kernel(int n, int nxcd, const int *__restrict__ gpos2,
                                                            const double2 *__restrict__ dl_st, double scale,
                                                            double2 *__restrict__ adj, c2<T> *__restrict__ qt)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 d = dl_st[gpos2[i]];
    const double2 q = make_double2(scale * d.x, scale * d.y);
    adj[i] = q;
    if (qt) qt[i] = mk<T>((T)q.x, (T)q.y);
}

// Adjoint near field of one work unit, organised as the forward P2P (LDS tiles,
// exponential skipped on far tiles).  With SRC the source-position sums (At, Bt) go to
// out_src.
template <typename T, bool SRC>
__device__ __forceinline__ void p2p_backward_unit(const int4 u, rec_t<T> *tile, c2<T> *qtile,
                                                  const SoaRec<T> &rec, const c2<T> *__restrict__ qv,
                                                  const int *__restrict__ leaf_start,
                                                  const int *__restrict__ tile_start,
                                                  const float4 *__restrict__ tile_box, int nside, T step,
                                                  float cut_leaf2, float series_leaf2, T lambda,
                                                  double4 *__restrict__ out_pa, double *__restrict__ out_b,
                                                  double4 *__restrict__ out_src)
{
    constexpr int NA = SRC ? 9 : 5;
    const int lane = threadIdx.x;
    const int logtp = u.w;
    const int tp = 1 << logtp;
    const int t = lane & (tp - 1);
    const int k = lane >> logtp;
    const int i = u.y + min(t, u.z - 1);
    const rec_t<T> ri = rec(i);
    const int ix = (int)morton_x((uint32_t)u.x), iy = (int)morton_y((uint32_t)u.x);
    const float4 tbox = tile_box[tile_start[u.x] + ((u.y - leaf_start[u.x]) >> 6)];
    double sum[NA] = {};
    for (int dy = -1; dy <= 1; ++dy) {
        const int ny = iy + dy;
        if (ny < 0 || ny >= nside) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int nx = ix + dx;
            if (nx < 0 || nx >= nside) continue;
            const uint32_t S = morton_encode((uint32_t)nx, (uint32_t)ny);
            const int s0 = leaf_start[S], s1 = leaf_start[S + 1];
            const T tx = ri.x - (T)dx * step;
            const T ty = ri.y - (T)dy * step;
            T acc[NA] = {};
            int tt = tile_start[S];
            for (int base = s0; base < s1; base += 64, ++tt) {
                const int len = min(64, s1 - base);
                __syncthreads();
                if (lane < len) {
                    tile[lane] = rec(base + lane);
                    qtile[lane] = qv[base + lane];
                }
                const float gap2 = box_gap2(tbox, (float)-dx, (float)-dy, tile_box[tt]);
                const int cls = gap2 >= cut_leaf2 ? 2 : gap2 >= series_leaf2 ? 1 : 0;
                __syncthreads();
                switch (logtp) {
                case 6: p2p_bwd_tile_any<T, 1, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                case 5: p2p_bwd_tile_any<T, 2, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                case 4: p2p_bwd_tile_any<T, 4, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                case 3: p2p_bwd_tile_any<T, 8, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                case 2: p2p_bwd_tile_any<T, 16, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                case 1: p2p_bwd_tile_any<T, 32, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                default: p2p_bwd_tile_any<T, 64, SRC>(tile, qtile, len, k, tx, ty, lambda, acc, cls); break;
                }
            }
#pragma unroll
            for (int c = 0; c < NA; ++c) sum[c] += (double)acc[c];
        }
    }
    for (int o = tp; o < 64; o <<= 1)
#pragma unroll
        for (int c = 0; c < NA; ++c) sum[c] += __shfl_xor(sum[c], o);
    if (k == 0 && t < u.z) {
        out_pa[i] = make_double4(sum[0], sum[1], sum[2], sum[3]);
        out_b[i] = sum[4];
        if constexpr (SRC) out_src[i] = make_double4(sum[5], sum[6], sum[7], sum[8]);
    }
}

// Adjoint near-field grid: one workgroup per target-centric unit.
template <typename T, bool SRC>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? (SRC ? 5 : 6) : 2) void p2p_backward_kernel(
    const int4 *__restrict__ units, const c2<T> *__restrict__ pos, const T *__restrict__ gam,
    const c2<T> *__restrict__ qv, const int *__restrict__ leaf_start, const int *__restrict__ tile_start,
    const float4 *__restrict__ tile_box, int nside, T step, float cut_leaf2, float series_leaf2, T lambda,
    double4 *__restrict__ out_pa, double *__restrict__ out_b, double4 *__restrict__ out_src)
{
    __shared__ rec_t<T> tile[64];
    __shared__ c2<T> qtile[64];
    const SoaRec<T> rec{pos, gam, step};
    p2p_backward_unit<T, SRC>(units[blockIdx.x], tile, qtile, rec, qv, leaf_start, tile_start, tile_box, nside, step,
                              cut_leaf2, series_leaf2, lambda, out_pa, out_b, out_src);
}

// Adjoint finalize: far parts from the q-field locals (Phi_far, by L2P) and the c-field
// locals (W'_far = (1/w^2) sum_l l b_l xi^(l-1)), combined with the near sums.
// Source positions (near_src != NULL): with c = -i Gamma/(2 pi),
//   At = alpha^2 (near sum) + Phi'_far,  Bt = alpha^2 lambda (near sum),
//   dL/dx_src = -Re(c (At + Bt)),  dL/dy_src = Im(c (At - Bt)),
// Phi'_far = (1/w^2) sum_l l b_l(q) xi^(l-1) the derivative of the q-field's local
// expansion (the far operator is antisymmetric).  gamma_st[gpos2[i]] is Gamma of
// sorted particle i (the staged circulations).
template <typename TL>
__global__ __launch_bounds__(256) void finalize_backward_kernel(
    int n, const int *__restrict__ perm, const int *__restrict__ leaf_of, const double2 *__restrict__ xy,
    const double4 *__restrict__ near_pa, const double *__restrict__ near_b, const double2 *__restrict__ adj,
    const c2<TL> *__restrict__ loc_c, const c2<TL> *__restrict__ loc_q, const c2<TL> *__restrict__ pos, int p,
    int has_far, double x0, double y0,
    double w, double alpha, double lambda, AdjointOut out, const double4 *__restrict__ near_src,
    const int *__restrict__ gpos2, const double *__restrict__ gamma_st, double *__restrict__ stage_g,
    double *__restrict__ stage_x, double *__restrict__ stage_s, int nxcd)
{
    const bool stage = stage_x != nullptr;
    const bool need_x = out.dxe || out.dxy, need_s = out.dxs || out.dxy;
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the user row, or with stage the staging slot inside the window of the sorted bucket
    const int64_t o = stage ? gpos2[i] : perm[i];  // issued with the first loads
    const double4 a = near_pa[i];
    const double sb = near_b[i];
    double phi = alpha * a.y;  // only Im(Phi) enters dL/dGamma
    const double ka = alpha * alpha * kInv2Pi;
    // A = -i ka (a.z + i a.w') with a.w' = -2 a.w (the near sums hold Im A / -2):
    // A = ka (a.w', -a.z);  B = -i ka lambda sb
    double Ar = ka * (-2.0 * a.w), Ai = -ka * a.z;
    const double Bi = -ka * lambda * sb;
    double dwr = 0.0, dwi = 0.0, dpr = 0.0, dpi = 0.0;
    if (has_far) {
        const uint32_t leaf = (uint32_t)leaf_of[i];
        const double cx = x0 + (morton_x(leaf) + 0.5) * w;
        const double cy = y0 + (morton_y(leaf) + 0.5) * w;
        c2<TL> xi;
        if (pos) {
            xi = pos[i];
        } else {
            const double2 z = xy[i];
            xi = mk<TL>((TL)((z.x - cx) / w), (TL)((z.y - cy) / w));
        }
        const c2<TL> *bq = loc_q + (int64_t)leaf * p;
        const c2<TL> *bc = loc_c + (int64_t)leaf * p;
        const c2<TL> accq = horner_prefetch<TL>(bq, p, xi);
        phi += (double)accq.y / w;
        if (p >= 2) {
            const c2<TL> accd = horner_weighted_prefetch<TL>(bc, p, xi, 1, 0);
            dwr = (double)accd.x / (w * w);
            dwi = (double)accd.y / (w * w);
            if (need_s) {
                const c2<TL> accp = horner_weighted_prefetch<TL>(bq, p, xi, 1, 0);
                dpr = (double)accp.x / (w * w);
                dpi = (double)accp.y / (w * w);
            }
        }
    }
    const double g = -phi * kInv2Pi;
    double ex = 0.0, ey = 0.0, sx = 0.0, sy = 0.0;
    if (need_x) {
        const double2 q = adj[i];
        // D1 = A + B + W', D2 = A - B + W'  (B purely imaginary)
        const double d1r = Ar + dwr, d1i = Ai + Bi + dwi;
        const double d2r = Ar + dwr, d2i = Ai - Bi + dwi;
        ex = q.x * d1r - q.y * d1i;
        ey = -(q.x * d2i + q.y * d2r);
    }
    if (need_s) {
        const double4 ns = near_src[i];
        const double a2 = alpha * alpha;
        const double atr = a2 * ns.x + dpr, ati = a2 * ns.y + dpi;
        const double btr = a2 * lambda * ns.z, bti = a2 * lambda * ns.w;
        const double G = gamma_st[gpos2[i]] * kInv2Pi;  // c = -i G: Re(c w) = G Im w, Im(c w) = -G Re w
        sx = -G * (ati + bti);
        sy = -G * (atr - btr);
    }
    if (stage) {  // by staging slot: dL/dGamma, evaluation part, source part
        if (out.dg) stage_g[o] = g;
        if (need_x) {
            stage_x[2 * o] = ex;
            stage_x[2 * o + 1] = ey;
        }
        if (need_s) {
            stage_s[2 * o] = sx;
            stage_s[2 * o + 1] = sy;
        }
        return;
    }
    store_adjoint(out, o, g, ex, ey, sx, sy);
}

// The adjoint outputs from their staging slots (written by finalize_backward_kernel for n
// above the last-level cache) to user order, as gather_rows_kernel does for velocities.
__global__ __launch_bounds__(256) void gather_adjoint_kernel(int n, int nxcd, const int *__restrict__ gpos1,
                                                             const double *__restrict__ stage_g,
                                                             const double *__restrict__ stage_x,
                                                             const double *__restrict__ stage_s, AdjointOut out)
{
    const int u = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int64_t k = gpos1[u];
    const bool need_x = out.dxe || out.dxy, need_s = out.dxs || out.dxy;
    const double g = out.dg ? stage_g[k] : 0.0;
    const double ex = need_x ? stage_x[2 * k] : 0.0, ey = need_x ? stage_x[2 * k + 1] : 0.0;
    const double sx = need_s ? stage_s[2 * k] : 0.0, sy = need_s ? stage_s[2 * k + 1] : 0.0;
    store_adjoint(out, u, g, ex, ey, sx, sy);
}

// Input check (FMM_OPT_VALIDATE): the lowest particle index whose `stride` values hold a
// NaN or an infinity, by atomic minimum into *first (which starts at INT_MAX).
__global__ void int_fill_kernel(int *p, int v) { *p = v; }

__global__ __launch_bounds__(256) void nonfinite_kernel(int64_t count, int stride, const double *__restrict__ a,
                                                         int *__restrict__ first)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += step)
        if (!__builtin_isfinite(a[k])) atomicMin(first, (int)(k / stride));
}

__global__ __launch_bounds__(256) void widen_perm_kernel(int n, const int *__restrict__ perm,
                                                          const int *__restrict__ leaf_of, int64_t *__restrict__ out,
                                                          int32_t *__restrict__ leaf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = perm[i];
    if (leaf) leaf[i] = leaf_of[i];
}

}  // namespace

hipError_t find_nonfinite(const double *a, int64_t n, int stride, int *flag, hipStream_t s, int64_t &bad)
{
    bad = -1;
    const int64_t count = n * stride;
    int_fill_kernel<<<1, 1, 0, s>>>(flag, INT_MAX);
    const unsigned g = (unsigned)std::min<int64_t>(blocks_for(count, 256), 4096);
    nonfinite_kernel<<<g, 256, 0, s>>>(count, stride, a, flag);
    int h = INT_MAX;
    hipError_t e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && h != INT_MAX) bad = h;
    return e;
}

// ---------------------------------------------------------------------------------
// The static workspace of fmm_velocity_noalloc: per-particle arrays, slots and
// expansions of one call carved from a file-scope device array, for callers that cannot
// allocate.  Host code never uses the array's name as an address: the device address is
// looked up once per device and kept.
// ---------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
__global__ __launch_bounds__(256) void zero_kernel(uint64_t *__restrict__ p, int64_t count)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += step) p[k] = 0;
}
}  // namespace

int static_workspace(int device, char **base)
{
    static std::mutex mu;
    static char *ptr[64] = {};
    *base = nullptr;
    if (device < 0 || device >= 64) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
        if (e != hipSuccess) return (int)e;
        ptr[device] = (char *)p;
    }
    *base = ptr[device];
    return (int)hipSuccess;
}

void launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t count = (int64_t)(bytes / 8);
    if (count == 0) return;
    zero_kernel<<<(unsigned)std::min<int64_t>(blocks_for(count, 256), 2048), 256, 0, s>>>((uint64_t *)p, count);
}

void launch_widen_perm(const fmm_tree *t, int64_t *perm, int32_t *leaf, hipStream_t s)
{
    const int n = (int)t->n;
    widen_perm_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, t->d_perm, t->d_leaf_of, perm, leaf);
}

// Grids of the permutation kernels: a multiple of the XCD count (see xcd_block).

void launch_stage_rows(int64_t n, int shift, const int *gpos1, const double *src, double *st, hipStream_t s)
{
    stage_in_kernel<double><<<xcd_grid(n, 256 * kStageE), 256, 0, s>>>((int)n, shift, kXcds, gpos1, src, st);
}

void launch_stage_rows2(int64_t n, int shift, const int *gpos1, const double2 *src, double2 *st, hipStream_t s)
{
    stage_in_kernel<double2><<<xcd_grid(n, 256 * kStageE), 256, 0, s>>>((int)n, shift, kXcds, gpos1, src, st);
}

void launch_gather_rows(int64_t n, const int *gpos1, const double2 *staged, double *uv, const double *base, double h,
                        hipStream_t s)
{
    gather_rows_kernel<<<xcd_grid(n, 256), 256, 0, s>>>((int)n, kXcds, gpos1, staged, uv, base, h);
}

void launch_stage_in(const fmm_tree *t, const double *gamma, hipStream_t s)
{
    launch_stage_rows(t->n, t->stage_shift, t->d_gpos1, gamma, t->d_st1, s);
}

void launch_pack(const fmm_tree *t, int is_double, void *gam, hipStream_t s)
{
    const int n = (int)t->n;
    if (is_double)
        pack_kernel<double><<<xcd_grid(n, 256), 256, 0, s>>>(n, kXcds, t->d_gpos2, t->d_st1, (double *)gam);
    else
        pack_kernel<float><<<xcd_grid(n, 256), 256, 0, s>>>(n, kXcds, t->d_gpos2, t->d_st1, (float *)gam);
}

void launch_leaf_coords(const fmm_tree *t, int is_double, void *pos, hipStream_t s)
{
    const int n = (int)t->n;
    const double w = t->side / (double)(1 << t->depth);
    if (is_double)
        leaf_coords_kernel<double><<<blocks_for(n, 256), 256, 0, s>>>(n, t->d_leaf_of, t->d_xy, t->x0, t->y0, w,
                                                                      (double2 *)pos);
    else
        leaf_coords_kernel<float><<<blocks_for(n, 256), 256, 0, s>>>(n, t->d_leaf_of, t->d_xy, t->x0, t->y0, w,
                                                                     (float2 *)pos);
}

// Exponential skipped where every pair has s >= cut: FP32 base 2, 1 - 2^-s rounds to 1
// for s >= 26; FP64 base e, 1 - e^-s rounds to 1 for s >= 37.5.  One unit of margin
// covers the rounding of the records and of the box test (boxes in leaf units).
inline float near_cut_leaf2(const fmm_tree *t, int is_double, double alpha)
{
    const double step = alpha * t->side / (double)(1 << t->depth);
    const double cut = is_double ? 39.0 : 27.0;
    return (float)(cut / (step * step));
}

// Dynamic LDS reserved by each near-field workgroup (one wavefront) so that at most
// near_occupancy wavefronts per SIMD are resident (160 KiB of LDS per CU, 4 SIMDs),
// leaving room for the far-field kernels on the other stream.  Serial schedule: no cap.
inline size_t near_lds_reserve(const fmm_tree *t, size_t static_bytes)
{
    if (t->occupancy_in_use <= 0 || t->depth < 2) return 0;
    const size_t per_wave = (size_t)160 * 1024 / (4 * (size_t)t->occupancy_in_use);
    return per_wave > static_bytes ? per_wave - static_bytes : 0;
}

void launch_p2p_forward(const fmm_tree *t, const void *pos, const void *gam, int is_double, double alpha,
                        double2 *near, void *slots, hipStream_t s)
{
    const bool mutual = slots != nullptr;
    const int64_t nwork = mutual ? t->nnear_work : t->nunits;
    const int4 *work = mutual ? t->d_near_work : t->d_units;
    if (nwork == 0) return;
    const int nside = 1 << t->depth;
    const double w = t->side / (double)nside;
    const double scale = alpha * kInv2Pi;
    const double step = alpha * w;
    const float cut_leaf2 = near_cut_leaf2(t, is_double, alpha);
    const unsigned grid = (unsigned)nwork;
    if (is_double)
        p2p_near_kernel<double><<<grid, 64, near_lds_reserve(t, 256 * sizeof(double4)), s>>>(
            work, (const double2 *)pos, (const double *)gam, t->d_leaf_start, t->d_tile_start,
            t->d_tile_box, nside, step, cut_leaf2, scale, t->dense_leaf, t->n, near, (double2 *)slots);
    else
        p2p_near_kernel<float><<<grid, 64, near_lds_reserve(t, 256 * sizeof(float4)), s>>>(
            work, (const float2 *)pos, (const float *)gam, t->d_leaf_start, t->d_tile_start,
            t->d_tile_box, nside, (float)step, cut_leaf2, scale, t->dense_leaf, t->n, near, (float2 *)slots);
}

void launch_p2m(const FarArgs &a, hipStream_t s)
{
    if (a.t->depth < 2) return;
    if (a.t->depth <= a.split) {
        if (a.rec_is_double) p2m_launch<double4, double>(a, s);
        else p2m_launch<float4, double>(a, s);
    } else {
        if (a.rec_is_double) p2m_launch<double4, float>(a, s);
        else p2m_launch<float4, float>(a, s);
    }
}

void launch_far_chain(const FarArgs &a, hipStream_t s, bool with_p2m)
{
    const fmm_tree *t = a.t;
    const int L = t->depth;
    if (L < 2) return;
    const Tables &tb = *t->tabs;
    const bool fine_is_double = a.split >= L;  // FP64 precision: every level double
    // Stage 4: P2M into the leaf level.
    if (with_p2m) launch_p2m(a, s);
    // Levels <= lw run in the one-workgroup coarse kernel: the coarse levels up to 256
    // cells (level 4), one round of gathers for its 16 wavefronts.  Coarse levels above that
    // (L_c = 5: 1024 cells, 64 tiles) keep FP64 and the side stream but run as wide launches
    // like the fine levels: on one CU their MFMA work alone takes longer than the near field.
    const int lw = std::min(a.lc, kCoarseMaxLevel);
    // Stage 5 on the fine levels: parents L-1 .. max(lw, 2).
    for (int l = L - 1; l >= 2 && l >= lw; --l) {
        const bool child_d = (l + 1) <= a.split, parent_d = l <= a.split;
        if (child_d && parent_d && a.p <= 16) gemm_f64_launch(a, l, 2, s);
        else if (child_d && parent_d) m2m_launch<double, double>(a, l, tb.m2m_d, s);
        else if (a.p <= 16 && parent_d) m2m_mfma_launch<double>(a, l, s);
        else if (a.p <= 16) m2m_mfma_launch<float>(a, l, s);
        else if (parent_d) m2m_launch<float, double>(a, l, tb.m2m_d, s);
        else m2m_launch<float, float>(a, l, tb.m2m_f, s);
    }
    // Coarse levels 2..lw in one workgroup (stages 5, 6, 7 there).
    if (lw >= 2 && a.p > 16) {
        CoarseValuArgs c{};
        c.p = a.p;
        c.lc = lw;
        c.counts = t->d_counts;
        c.lists = t->d_lists;
        for (int l = 0; l <= kMaxDepth; ++l) {
            c.list_off[l] = l <= L ? t->list_off[l] : 0;
            c.list_len[l] = l <= L ? t->list_len[l] : 0;
        }
        c.mp = a.mp_d;
        c.lo = a.lo_d;
        c.m2m_tab = tb.m2m_d;
        c.m2l_tab = tb.m2l_d;
        c.l2l_tab = tb.l2l_d;
        coarse_valu_kernel<<<1, 1024, 0, s>>>(c);
    } else if (lw >= 2) {
        CoarseArgs c{};
        c.p = a.p;
        c.lc = lw;
        c.lists = t->d_lists;
        for (int l = 0; l <= kMaxDepth; ++l) {
            c.list_off[l] = l <= L ? t->list_off[l] : 0;
            c.list_len[l] = l <= L ? t->list_len[l] : 0;
            for (int q = 0; q < 4; ++q) c.class_off[4 * l + q] = l <= L ? t->class_off[4 * l + q] : 0;
        }
        c.mp = a.mp_d;
        c.lo = a.lo_d;
        c.entries = tb.mfma_entries;
        c.tab = tb.mfma_d;
        c.zero = tb.zero_row;
        coarse_kernel<<<1, a.coarse_threads, 0, s>>>(c);
    }
    // Stages 6 + 7 on the fine levels.
    for (int l = (lw + 1 > 2 ? lw + 1 : 2); l <= L; ++l) {
        const bool here_d = l <= a.split, par_d = (l - 1) <= a.split;
        if (here_d && a.p <= 16) gemm_f64_launch(a, l, 0, s);
        else if (here_d) m2l_launch<double, double>(a, l, tb.m2l_d, tb.l2l_d, s);
        else if (a.p <= 16 && par_d) m2l_mfma_launch<double>(a, l, s);
        else if (a.p <= 16) m2l_mfma_launch<float>(a, l, s);
        else if (par_d) m2l_launch<float, double>(a, l, tb.m2l_f, tb.l2l_d, s);
        else m2l_launch<float, float>(a, l, tb.m2l_f, tb.l2l_f, s);
    }
    (void)fine_is_double;
}

void launch_finalize(const fmm_tree *t, const FarArgs &a, const double2 *near, const void *slots, int slots_double,
                     double alpha, double *uv, double *uv_near, double *uv_far, void *stage, const double *base,
                     double h, hipStream_t s)
{
    // uv alone: the totals go to stage (n double2), then out in user order; through the
    // staging windows once the output outgrows the last-level cache
    double2 *staged = uv && !uv_near && !uv_far ? (double2 *)stage : nullptr;
    const bool windowed = outputs_windowed(t->n, sizeof(double2));
    double *uv_direct = staged ? nullptr : uv;
    const int L = t->depth;
    const int n = (int)t->n;
    const double w = t->side / (double)(1 << L);
    const int has_far = L >= 2;
    const uint16_t *mask = slots ? t->d_leaf_mask : nullptr;
    const double scale = alpha * kInv2Pi;
    const dim3 g(xcd_grid(n, 256));
    const int *gp = windowed ? t->d_gpos2 : nullptr;
    // L2P at the tree's leaf-unit coordinates when they are in the precision of the locals
    if (!has_far || L <= a.split) {
        const double2 *loc = has_far ? level_ptr<double>(a, L, true) : nullptr;
        const double2 *pos = a.rec_is_double ? (const double2 *)a.pos : nullptr;
        if (slots_double)
            finalize_kernel<double, double><<<g, 256, 0, s>>>(n, t->d_perm, t->d_leaf_of, t->d_xy, near, mask,
                                                              (const double2 *)slots, scale, loc, pos, a.p, has_far,
                                                              t->x0, t->y0, w, uv_direct, uv_near, uv_far, staged, gp,
                                                              kXcds);
        else
            finalize_kernel<double, float><<<g, 256, 0, s>>>(n, t->d_perm, t->d_leaf_of, t->d_xy, near, mask,
                                                             (const float2 *)slots, scale, loc, pos, a.p, has_far,
                                                             t->x0, t->y0, w, uv_direct, uv_near, uv_far, staged, gp,
                                                             kXcds);
    } else {
        const float2 *loc = level_ptr<float>(a, L, true);
        const float2 *pos = a.rec_is_double ? nullptr : (const float2 *)a.pos;
        if (slots_double)
            finalize_kernel<float, double><<<g, 256, 0, s>>>(n, t->d_perm, t->d_leaf_of, t->d_xy, near, mask,
                                                             (const double2 *)slots, scale, loc, pos, a.p, has_far,
                                                             t->x0, t->y0, w, uv_direct, uv_near, uv_far, staged, gp,
                                                             kXcds);
        else
            finalize_kernel<float, float><<<g, 256, 0, s>>>(n, t->d_perm, t->d_leaf_of, t->d_xy, near, mask,
                                                            (const float2 *)slots, scale, loc, pos, a.p, has_far,
                                                            t->x0, t->y0, w, uv_direct, uv_near, uv_far, staged, gp,
                                                            kXcds);
    }
    if (staged && windowed) gather_rows_kernel<<<g, 256, 0, s>>>(n, kXcds, t->d_gpos1, staged, uv, base, h);
    else if (staged) scatter_rows_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, t->d_perm, staged, uv, base, h);
}
void launch_pack_adjoint(const fmm_tree *t, const double *dl_duv, double scale, double2 *adj, void *qt, int is_double,
                         double2 *staging, hipStream_t s)
{
    const int n = (int)t->n;
    launch_stage_rows2(n, t->stage_shift, t->d_gpos1, (const double2 *)dl_duv, staging, s);
    if (is_double)
        pack_adjoint_kernel<double><<<xcd_grid(n, 256), 256, 0, s>>>(n, kXcds, t->d_gpos2, staging, scale, adj,
                                                                      nullptr);
    else
        pack_adjoint_kernel<float><<<xcd_grid(n, 256), 256, 0, s>>>(n, kXcds, t->d_gpos2, staging, scale, adj,
                                                                     (float2 *)qt);
}

void launch_p2p_backward(const fmm_tree *t, const void *pos, const void *gam, const void *qv, int is_double,
                         double alpha,
                         double4 *out_pa, double *out_b, double4 *out_src, hipStream_t s)
{
    if (t->nunits == 0) return;
    const int nside = 1 << t->depth;
    const double w = t->side / (double)nside;
    const double step = alpha * w;
    const double cut = is_double ? 39.0 : 27.0;
    const float cut_leaf2 = (float)(cut / (step * step));
    const unsigned grid = (unsigned)t->nunits;
    const double ln2 = 0.69314718055994530942;
    // the series of the pair code applies below s' = (0.125 / ln 2) in FP32 (natural exponent
    // 0.125) and 1e-3 in FP64; tiles whose boxes are twice that apart skip the test
    const double series_s = is_double ? 1e-3 : 0.125 / ln2;
    const float series_leaf2 = (float)(2.0 * series_s / (step * step));
    if (is_double) {
        if (out_src)
            p2p_backward_kernel<double, true><<<grid, 64, 0, s>>>(
                t->d_units, (const double2 *)pos, (const double *)gam, (const double2 *)qv, t->d_leaf_start,
                t->d_tile_start, t->d_tile_box, nside, step, cut_leaf2, series_leaf2, 1.0, out_pa, out_b, out_src);
        else
            p2p_backward_kernel<double, false><<<grid, 64, 0, s>>>(
                t->d_units, (const double2 *)pos, (const double *)gam, (const double2 *)qv, t->d_leaf_start,
                t->d_tile_start, t->d_tile_box, nside, step, cut_leaf2, series_leaf2, 1.0, out_pa, out_b, nullptr);
    } else {
        if (out_src)
            p2p_backward_kernel<float, true><<<grid, 64, 0, s>>>(
                t->d_units, (const float2 *)pos, (const float *)gam, (const float2 *)qv, t->d_leaf_start,
                t->d_tile_start, t->d_tile_box, nside, (float)step, cut_leaf2, series_leaf2, (float)ln2, out_pa,
                out_b, out_src);
        else
            p2p_backward_kernel<float, false><<<grid, 64, 0, s>>>(
                t->d_units, (const float2 *)pos, (const float *)gam, (const float2 *)qv, t->d_leaf_start,
                t->d_tile_start, t->d_tile_box, nside, (float)step, cut_leaf2, series_leaf2, (float)ln2, out_pa,
                out_b, nullptr);
    }
}

void launch_finalize_backward(const fmm_tree *t, const FarArgs &fc, const FarArgs &fq, const double4 *near_pa,
                              const double *near_b, const double2 *adj, const double4 *near_src, int is_double,
                              double alpha, const AdjointOut &out, double *stage_g, double *stage_x,
                              double *stage_s, hipStream_t s)
{
    const int L = t->depth;
    const int n = (int)t->n;
    const dim3 g(xcd_grid(n, 256));
    const double w = t->side / (double)(1 << L);
    const int has_far = L >= 2;
    const double lambda = is_double ? 1.0 : 0.69314718055994530942;
    if (!has_far || L <= fc.split)
        finalize_backward_kernel<double><<<g, 256, 0, s>>>(
            n, t->d_perm, t->d_leaf_of, t->d_xy, near_pa, near_b, adj,
            has_far ? level_ptr<double>(fc, L, true) : nullptr, has_far ? level_ptr<double>(fq, L, true) : nullptr,
            fc.rec_is_double ? (const double2 *)fc.pos : nullptr, fc.p, has_far, t->x0, t->y0, w, alpha, lambda, out, near_src, t->d_gpos2, t->d_st1, stage_g, stage_x,
            stage_s, kXcds);
    else
        finalize_backward_kernel<float><<<g, 256, 0, s>>>(
            n, t->d_perm, t->d_leaf_of, t->d_xy, near_pa, near_b, adj, level_ptr<float>(fc, L, true),
            level_ptr<float>(fq, L, true), fc.rec_is_double ? nullptr : (const float2 *)fc.pos, fc.p, has_far, t->x0, t->y0, w, alpha, lambda, out, near_src, t->d_gpos2,
            t->d_st1, stage_g, stage_x, stage_s, kXcds);
    if (stage_x) gather_adjoint_kernel<<<g, 256, 0, s>>>(n, kXcds, t->d_gpos1, stage_g, stage_x, stage_s, out);
}


}  // namespace fmm
