// gfx950 kernels of the adaptive-tree variant (fmm2d_adaptive.h): the evaluation
// stages of Fig. fmmStages over the four lists of the adaptive FMM.
//
// Expansions are radius-scaled as in the uniform kernels (multipole a_m / w^m, local
// b_l w^(l+1), w the cell's width), so the translations between a cell and its parent
// and the M2L between cells of one level do not depend on the level.  Every expansion
// is FP64; the near field runs in the records' precision (FP32 for the mixed form).
// Complex charge c_j = -i Gamma_j / (2 pi); conjugate velocity W = u - i v.
#include "adaptive_internal.h"
#include "device_common.h"

#include <cmath>

namespace fmm {
namespace {

__device__ __forceinline__ double2 cell_centre(double x0, double y0, double side, int4 c)
{
    const double w = ldexp(side, -c.x);
    return make_double2(x0 + (c.y + 0.5) * w, y0 + (c.z + 0.5) * w);
}

__device__ __forceinline__ double2 cinv(double2 a)
{
    const double r = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * r, -a.y * r);
}

// Records {alpha (z - c_leaf), Gamma, 0} for the near field and the circulations in
// sorted order for the expansions.
// The circulation of sorted particle i from its staging slot gpos2[i] (the circulations
// staged by bucket beforehand): in the near field's precision for its records, in FP64
// for the expansions.
template <typename T>
__global__ __launch_bounds__(256) void at_pack_kernel(int n, int nxcd, const int *__restrict__ gpos2,
                                                       const double *__restrict__ gamma_st, T *__restrict__ gam,
                                                       double *__restrict__ gamma_sorted)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = gamma_st[gpos2[i]];
    gam[i] = (T)g;
    gamma_sorted[i] = g;
}

// The offsets z - c_leaf of the sorted particles from their leaves' centres, in the near
// field's precision (made once per tree and precision): the near field's records are
// these offsets scaled by alpha on load (SoaRec) and the circulations.
template <typename T>
__global__ __launch_bounds__(256) void at_coords_kernel(int n, const int *__restrict__ leaf_of,
                                                         const int4 *__restrict__ cell, const double2 *__restrict__ xy,
                                                         double x0, double y0, double side, c2<T> *__restrict__ pos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 c = cell_centre(x0, y0, side, cell[leaf_of[i]]);
    const double2 z = xy[i];
    pos[i] = mk<T>((T)(z.x - c.x), (T)(z.y - c.y));
}

// One step of a wavefront butterfly over all N coefficients (independent shuffles).
template <int N>
__device__ __forceinline__ void butterfly_step(double2 (&acc)[N], int o)
{
    double sx[N], sy[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        sx[m] = __shfl_xor(acc[m].x, o);
        sy[m] = __shfl_xor(acc[m].y, o);
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {
        acc[m].x += sx[m];
        acc[m].y += sy[m];
    }
}

// Charge of sorted particle j: c_j = -i Gamma_j / (2 pi), or (CPLX) the complex charge
// q_j of the adjoint pass.
template <bool CPLX>
__device__ __forceinline__ double2 charge(const double *__restrict__ gamma, const double2 *__restrict__ q, int j)
{
    if constexpr (CPLX) return q[j];
    else return make_double2(0.0, -gamma[j] * kInv2Pi);
}

// P2M (stage 4) at the leaves of level >= 2, G lanes per leaf (64/G leaves per
// wavefront):
//   a_m / w^m = sum_j c_j xi_j^m,  xi_j = (z_j - c)/w,
// the G lanes over the leaf's particles, then a butterfly over the G lanes per
// coefficient (log2 G steps of independent shuffles).
template <int PMAX, bool CPLX, int G>
__global__ __launch_bounds__(64) void at_p2m_kernel(const int *__restrict__ cells, int ncells,
                                                     const int4 *__restrict__ cell, const int2 *__restrict__ range,
                                                     const double2 *__restrict__ xy, const double *__restrict__ gamma,
                                                     const double2 *__restrict__ q, double x0, double y0, double side,
                                                     int p, double2 *__restrict__ mp)
{
    const int lane = threadIdx.x, g = lane % G;
    const int idx = blockIdx.x * (64 / G) + lane / G;
    const bool valid = idx < ncells;  // a group past the end idles (its shuffles stay inside it)
    const int k = valid ? cells[idx] : 0;
    const int4 c = cell[k];
    const int2 r = valid ? range[k] : make_int2(0, 0);
    const double w = ldexp(side, -c.x);
    const double rw = 1.0 / w;
    const double2 ctr = cell_centre(x0, y0, side, c);
    // PMAX coefficients throughout (those at m >= p are never stored): no branches on
    // p, so the butterfly below runs step by step over all coefficients at once
    double2 acc[PMAX];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) acc[m] = make_double2(0.0, 0.0);
    for (int j = r.x + g; j < r.x + r.y; j += G) {
        const double2 z = xy[j];
        const double2 xi = make_double2((z.x - ctr.x) * rw, (z.y - ctr.y) * rw);
        double2 pw = charge<CPLX>(gamma, q, j);
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            acc[m].x += pw.x;
            acc[m].y += pw.y;
            pw = cmul<double>(pw, xi);
        }
    }
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) butterfly_step<PMAX>(acc, o);
    // every lane of the group holds the sums; its first lane stores them (constant
    // indices: a lane-dependent pick would make the compiler address the array in
    // scratch memory)
    if (valid && g == 0)
#pragma unroll
        for (int m = 0; m < PMAX; ++m)
            if (m < p) mp[(int64_t)k * p + m] = acc[m];
}

// M2M (stage 5) into the split cells of one level, one thread per (cell, m):
//   A_m = sum_children sum_{k<=m} C(m,k) d^(m-k) 2^-k a_k,  d = (c_child - c_parent)/w_parent.
__global__ __launch_bounds__(256) void at_m2m_kernel(const int *__restrict__ cells, int ncells,
                                                      const int4 *__restrict__ child, const double *__restrict__ binom,
                                                      int nb, int p, double2 *__restrict__ mp)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * p) return;
    const int k = cells[t / p], m = t % p;
    const int4 ch = child[k];
    const int cq[4] = {ch.x, ch.y, ch.z, ch.w};
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < 4; ++q) {
        const int c = cq[q];
        if (c < 0) continue;
        const double2 d = make_double2(((q & 1) - 0.5) * 0.5, ((q >> 1) - 0.5) * 0.5);
        double2 pw = make_double2(1.0, 0.0);
        for (int kk = m; kk >= 0; --kk) {
            const double f = binom[m * nb + kk] * ldexp(1.0, -kk);
            const double2 a = mp[(int64_t)c * p + kk];
            const double2 term = cmul<double>(a, pw);
            acc.x = fma(f, term.x, acc.x);
            acc.y = fma(f, term.y, acc.y);
            pw = cmul<double>(pw, d);
        }
    }
    mp[(int64_t)k * p + m] = acc;
}

// Stage 6 for every cell of level >= 2 in one launch (its sources need only the
// multipoles, complete after the upward pass), one thread per cell, PMAX terms
// (coefficients m >= p enter as zero; the binomial table is sized for PMAX):
// M2L from V, with u = 1/delta, delta = (c - c_S)/w and a~_m = u^m a_m(S),
//   b_l = sum_S (-1)^l u^(l+1) sum_m C(l+m,m) a~_m;
// P2L from X,  b_l += -sum_{j in A} c_j u_j^(l+1),  u_j = w/(z_j - c).
// Up to 16 terms the cell's locals, the scaled source coefficients and the loads in flight
// fit in 168 VGPRs with a 40-byte spill: 3 wavefronts per SIMD instead of 2 hide more of
// the gather latency (clustered tree, 2^24 particles: 6.02 against 6.18 ms per evaluation).
template <int PMAX, bool CPLX>
__global__ __launch_bounds__(64, PMAX <= 16 ? 3 : 1) void at_m2l_kernel(int first, int ncells, const int4 *__restrict__ cell,
                                                     const int *__restrict__ v_off, const int *__restrict__ v_idx,
                                                     const int *__restrict__ x_off, const int *__restrict__ x_idx,
                                                     const int2 *__restrict__ range, const double2 *__restrict__ xy,
                                                     const double *__restrict__ gamma, const double2 *__restrict__ q,
                                                     double x0, double y0, double side,
                                                     const double *__restrict__ binom, int p,
                                                     const double2 *__restrict__ mp, double2 *__restrict__ lo)
{
    constexpr int NB = 2 * PMAX + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells) return;
    const int k = first + t;
    const int4 c = cell[k];
    double2 b[PMAX];
#pragma unroll
    for (int l = 0; l < PMAX; ++l) b[l] = make_double2(0.0, 0.0);
    for (int e = v_off[k]; e < v_off[k + 1]; ++e) {
        const int S = v_idx[e];
        const int4 cs = cell[S];
        const double2 u = cinv(make_double2((double)(c.y - cs.y), (double)(c.z - cs.z)));
        const double2 *a = mp + (int64_t)S * p;
        double2 at[PMAX];
        double2 pw = make_double2(1.0, 0.0);
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            const double2 am = m < p ? a[m] : make_double2(0.0, 0.0);
            at[m] = cmul<double>(am, pw);
            pw = cmul<double>(pw, u);
        }
        double2 ul = u;
#pragma unroll
        for (int l = 0; l < PMAX; ++l) {
            double2 sum = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < PMAX; ++m) {
                const double cb = binom[(l + m) * NB + m];
                sum.x = fma(cb, at[m].x, sum.x);
                sum.y = fma(cb, at[m].y, sum.y);
            }
            const double2 tv = cmul<double>(ul, sum);
            const double sg = (l & 1) ? -1.0 : 1.0;
            b[l].x = fma(sg, tv.x, b[l].x);
            b[l].y = fma(sg, tv.y, b[l].y);
            ul = cmul<double>(ul, u);
        }
    }
    if (x_off[k] < x_off[k + 1]) {
        const double rw = 1.0 / ldexp(side, -c.x);
        const double2 ctr = cell_centre(x0, y0, side, c);
        for (int e = x_off[k]; e < x_off[k + 1]; ++e) {
            const int2 r = range[x_idx[e]];
            for (int j = r.x; j < r.x + r.y; ++j) {
                const double2 z = xy[j];
                const double2 u = cinv(make_double2((z.x - ctr.x) * rw, (z.y - ctr.y) * rw));
                const double2 cj = charge<CPLX>(gamma, q, j);
                double2 ul = cmul<double>(cj, u);  // c_j u^(l+1)
#pragma unroll
                for (int l = 0; l < PMAX; ++l) {
                    b[l].x -= ul.x;
                    b[l].y -= ul.y;
                    ul = cmul<double>(ul, u);
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < PMAX; ++l)
        if (l < p) lo[(int64_t)k * p + l] = b[l];
}

// Stages 5-7 on v_mfma_f64_16x16x4f64 for p <= 16.  With radius-scaled coefficients
// every translation is a fixed 2p x 2p real operator per offset, shared with the uniform
// tree (its tables and interaction entries):
//  - mode 0 (stages 6 + 7) over the cells of one level, grouped by parity class q: the
//    M2L from V, whose cells sit at the class's 27 interaction offsets (vslot: the source
//    cell per offset, -1 where V has none), plus the L2L from the parent's locals (levels
//    >= 3), added to the P2L sums of the cells with an X list (written before);
//  - mode 1 (stage 5) over the split cells of one level: the M2M from the four children.
// A wavefront takes 16 targets; per operator it gathers their 16 source rows (a zero row
// where a target has no source; an operator no target of the tile uses is skipped).
// Operand layouts as for the uniform tree's FP64 gather-GEMM:
//   A: lane l holds A[row l%16][k l/16]     B: lane l holds B[k l/16][col l%16]
//   D: lane l, register r holds D[l/16 + 4r][l%16]
// with K permuted so that step s uses k = 8(l/16) + s.
typedef double doublex4 __attribute__((ext_vector_type(4)));

struct AtGemm {
    const int *targets;          // the launch's targets, by class (mode 0) or one list (mode 1)
    int cstart[4], clen[4], cwave0[4];
    int nwaves, mode, first, p;
    const int *vslot;            // mode 0: 27 source cells per cell of level >= 2 (index - first)
    const int *x_off;            // mode 0: cells with an X list start from their P2L sums
    const int *parent;           // mode 0: the L2L source (with par)
    const int4 *child;           // mode 1: the four children
    const int4 *entries;         // {dx, dy, slot, kind}: 4 x 28 M2L/L2L, then 4 M2M
    const double *src;           // multipoles (M2L and M2M sources)
    const double *par;           // mode 0: locals of the parents' level, NULL at level 2
    double *out;                 // locals (mode 0) or multipoles (mode 1)
    const double *tab, *zero;
};

__global__ __launch_bounds__(256, 4) void at_gemm_kernel(AtGemm a)
{
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    const int two_p = 2 * a.p;
    const int k0 = 8 * kq;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (wave >= a.nwaves) return;  // whole wavefronts
    int q = 0;
    for (int c = 1; c < 4; ++c)
        if (wave >= a.cwave0[c]) q = c;
    const int cs = a.cstart[q], cl = a.clen[q];
    const int base = (wave - a.cwave0[q]) * 16;
    const int li = base + row;
    const bool tvalid = li < cl;
    const int tcell = tvalid ? a.targets[cs + li] : -1;
    doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    if (a.mode == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = base + kq + 4 * r;
            if (o < cl) {
                const int k = a.targets[cs + o];
                if (a.x_off[k] < a.x_off[k + 1]) {
                    const double *b = a.out + (size_t)k * two_p;
                    if (row < two_p) acc0[r] = b[row];
                    if (16 + row < two_p) acc1[r] = b[16 + row];
                }
            }
        }
    }
    const int ne = a.mode == 0 ? 28 : 4;
    for (int e = 0; e < ne; ++e) {
        int S = -1, en_idx;
        const double *sbase = a.src;
        if (a.mode == 1) {
            en_idx = 112 + e;
            if (tvalid) {
                const int4 ch = a.child[tcell];
                S = e == 0 ? ch.x : e == 1 ? ch.y : e == 2 ? ch.z : ch.w;
            }
        } else if (e < 27) {
            en_idx = 28 * q + e;
            if (tvalid) S = a.vslot[(int64_t)(tcell - a.first) * 27 + e];
        } else {
            en_idx = 28 * q + 27;  // L2L from the parent (child quadrant q)
            sbase = a.par;
            if (tvalid && a.par) S = a.parent[tcell];
        }
        if (!__any(S >= 0)) continue;  // wavefront-uniform
        const int4 en = a.entries[en_idx];
        const double *b0p = a.tab + (((size_t)en.z * 4 + kq) * 32 + row) * 8;
        const double *b1p = b0p + 16 * 8;
        double av[8], b0[8], b1[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double2 u0 = ((const double2 *)b0p)[v], u1 = ((const double2 *)b1p)[v];
            b0[2 * v] = u0.x;
            b0[2 * v + 1] = u0.y;
            b1[2 * v] = u1.x;
            b1[2 * v + 1] = u1.y;
        }
        // rows carry a tail pad and absent sources read the zero row: the 8 reads stay inside
        const double *src = S >= 0 ? sbase + (size_t)S * two_p + k0 : a.zero + k0;
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const double v = src[st];
            av[st] = (k0 + st < two_p) ? v : 0.0;
        }
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], b0[st], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], b1[st], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = base + kq + 4 * r;
        if (o < cl) {
            double *out = a.out + (size_t)a.targets[cs + o] * two_p;
            if (row < two_p) out[row] = acc0[r];
            if (16 + row < two_p) out[16 + row] = acc1[r];
        }
    }
}

// P2L from X before the MFMA translations, one thread per cell with a non-empty X list,
// written to its locals (the level's gather-GEMM adds M2L and L2L to them):
//   b_l = -sum_{j in A} c_j u_j^(l+1),  u_j = w/(z_j - c).
template <int PMAX, bool CPLX>
__global__ __launch_bounds__(64) void at_p2l_kernel(int first, int ncells, const int4 *__restrict__ cell,
                                                     const int *__restrict__ x_off, const int *__restrict__ x_idx,
                                                     const int2 *__restrict__ range, const double2 *__restrict__ xy,
                                                     const double *__restrict__ gamma,
                                                     const double2 *__restrict__ q, double x0, double y0,
                                                     double side, int p, double2 *__restrict__ lo)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells) return;
    const int k = first + t;
    if (x_off[k] == x_off[k + 1]) return;
    const int4 c = cell[k];
    double2 b[PMAX];
#pragma unroll
    for (int l = 0; l < PMAX; ++l) b[l] = make_double2(0.0, 0.0);
    const double rw = 1.0 / ldexp(side, -c.x);
    const double2 ctr = cell_centre(x0, y0, side, c);
    for (int e = x_off[k]; e < x_off[k + 1]; ++e) {
        const int2 r = range[x_idx[e]];
        for (int j = r.x; j < r.x + r.y; ++j) {
            const double2 z = xy[j];
            const double2 u = cinv(make_double2((z.x - ctr.x) * rw, (z.y - ctr.y) * rw));
            const double2 cj = charge<CPLX>(gamma, q, j);
            double2 ul = cmul<double>(cj, u);  // c_j u^(l+1)
#pragma unroll
            for (int l = 0; l < PMAX; ++l) {
                b[l].x -= ul.x;
                b[l].y -= ul.y;
                ul = cmul<double>(ul, u);
            }
        }
    }
#pragma unroll
    for (int l = 0; l < PMAX; ++l)
        if (l < p) lo[(int64_t)k * p + l] = b[l];
}

// Stage 7 into the cells of one level l >= 3 (parents of level >= 2), one thread per
// (cell, k), by Horner in d = (c - c_parent)/w_parent:
//   b_k += 2^-(k+1) sum_{j>=k} C(j,k) d^(j-k) b_j(parent).
__global__ __launch_bounds__(256) void at_l2l_kernel(int first, int ncells, const int4 *__restrict__ cell,
                                                      const int *__restrict__ parent,
                                                      const double *__restrict__ binom, int nb, int p,
                                                      double2 *__restrict__ lo)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * p) return;
    const int k = first + t / p, kk = t % p;
    const int4 c = cell[k];
    const double2 *bp = lo + (int64_t)parent[k] * p;
    const double2 d = make_double2(((c.y & 1) - 0.5) * 0.5, ((c.z & 1) - 0.5) * 0.5);
    const double c0 = binom[(p - 1) * nb + kk];
    double2 acc = make_double2(c0 * bp[p - 1].x, c0 * bp[p - 1].y);
    for (int j = p - 2; j >= kk; --j) {
        acc = cmul<double>(acc, d);
        const double cj = binom[j * nb + kk];
        acc.x = fma(cj, bp[j].x, acc.x);
        acc.y = fma(cj, bp[j].y, acc.y);
    }
    const double f = ldexp(1.0, -(kk + 1));
    double2 &out = lo[(int64_t)k * p + kk];
    out.x = fma(f, acc.x, out.x);
    out.y = fma(f, acc.y, out.y);
}

// Near field (stage 9) over U.  One wavefront per work entry:
//  - a mutual item (two adjacent dense leaves of one level, or a dense leaf with itself)
//    evaluates each unordered pair once for both particles (the kernel is odd), as for
//    the uniform tree, with that level's leaf width; sums go to the per-direction slots;
//  - a target-centric unit {leaf A, first, count <= 64, log2 TP | 16 if dense} takes
//    every source leaf S of U(A) (but the same-level dense ones when flagged) in
//    64-particle tiles staged in LDS, the target moved into S's frame
//    (alpha (z_i - c_S) = record_i + alpha (c_A - c_S)).  A source tile whose bounding box
//    is at least the cut from the unit's box skips the exponential (1 - e rounds to 1).
template <typename T>
__device__ __forceinline__ void at_target_unit(const int4 u, rec_t<T> *tile, const int4 *__restrict__ cell,
                                               const int2 *__restrict__ range, const int *__restrict__ u_off,
                                               const int *__restrict__ u_idx, const int *__restrict__ tile_start,
                                               const double4 *__restrict__ tile_box,
                                               const SoaRec<T> &rec, double x0, double y0, double side,
                                               double alpha, double cut, double scale, int dense,
                                               double2 *__restrict__ near)
{
    const int lane = threadIdx.x;
    const int logtp = u.w & 15;
    const bool skip_dense = (u.w >> 4) != 0;
    const int tp = 1 << logtp;
    const int t = lane & (tp - 1);
    const int k = lane >> logtp;
    const int i = u.y + min(t, u.z - 1);
    const rec_t<T> ri = rec(i);
    const int A = u.x;
    const int4 cla = cell[A];
    const double2 ca = cell_centre(x0, y0, side, cla);
    const double4 tb = tile_box[tile_start[A] + ((u.y - range[A].x) >> 6)];
    const double a2 = alpha * alpha;
    double au = 0.0, av = 0.0;
    for (int e = u_off[A]; e < u_off[A + 1]; ++e) {
        const int S = u_idx[e];
        const int4 cls = cell[S];
        const int2 r = range[S];
        if (skip_dense && cls.x == cla.x && r.y >= dense) continue;  // in a mutual item
        const double2 cs = cell_centre(x0, y0, side, cls);
        const T tx = ri.x + (T)(alpha * (ca.x - cs.x));
        const T ty = ri.y + (T)(alpha * (ca.y - cs.y));
        T fu = 0, fv = 0;
        int tt = tile_start[S];
        for (int base = r.x; base < r.x + r.y; base += 64, ++tt) {
            const int len = min(64, r.x + r.y - base);
            __syncthreads();
            if (lane < len) tile[lane] = rec(base + lane);
            const double4 sb = tile_box[tt];
            const double gx = fmax(0.0, fmax(sb.x - tb.z, tb.x - sb.z));
            const double gy = fmax(0.0, fmax(sb.y - tb.w, tb.y - sb.w));
            const bool far = (gx * gx + gy * gy) * a2 >= cut;
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
    for (int o = tp; o < 64; o <<= 1) {
        au += __shfl_xor(au, o);
        av += __shfl_xor(av, o);
    }
    if (k == 0 && t < u.z) near[i] = make_double2(-scale * au, scale * av);
}

template <typename T>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 8 : 4) void at_near_kernel(
    const int4 *__restrict__ work, const int4 *__restrict__ cell, const int2 *__restrict__ range,
    const int *__restrict__ u_off, const int *__restrict__ u_idx, const int *__restrict__ tile_start,
    const double4 *__restrict__ tile_box, const int *__restrict__ leaf_start, const int *__restrict__ leaf_tile,
    const float4 *__restrict__ tile_box_leaf, const c2<T> *__restrict__ pos, const T *__restrict__ gam, double x0,
    double y0, double side, double alpha, double cut, double scale, int dense, int64_t n,
    double2 *__restrict__ near, c2<T> *__restrict__ slots)
{
    __shared__ rec_t<T> tile_a[128], tile_b[128];
    const SoaRec<T> rec{pos, gam, (T)alpha};  // records alpha (z - c_leaf), Gamma
    const int4 u = work[blockIdx.x];
    if (u.w & kMutualItem) {
        const double step = alpha * ldexp(side, -(u.w >> 9));
        mutual_item_src<T, SoaRec<T>>(u, tile_a, tile_b, rec, leaf_start, leaf_tile, tile_box_leaf, (T)step,
                                      (float)(cut / (step * step)), n, slots);
    } else {
        at_target_unit<T>(u, tile_a, cell, range, u_off, u_idx, tile_start, tile_box, rec, x0, y0, side, alpha, cut,
                          scale, dense, near);
    }
}

// Stages 8 + 10: L2P from the leaf's local expansion (level >= 2),
//   W += (1/w) sum_l b_l xi^l;  M2P from W(leaf),  W += (1/w_D) sum_m a_m zeta^-(m+1);
// (u, v) = near + (Re W, -Im W), scattered to user order.
template <typename TS>
__global__ __launch_bounds__(256) void at_finalize_kernel(int n, const int *__restrict__ perm,
                                                           const int *__restrict__ leaf_of,
                                                           const int4 *__restrict__ cell,
                                                           const double2 *__restrict__ xy,
                                                           const int *__restrict__ w_off,
                                                           const int *__restrict__ w_idx,
                                                           const double2 *__restrict__ mp,
                                                           const double2 *__restrict__ lo, int p, double x0,
                                                           double y0, double side, const double2 *__restrict__ near,
                                                           const uint16_t *__restrict__ mask,
                                                           const c2<TS> *__restrict__ slots, double scale,
                                                           double *__restrict__ uv, double *__restrict__ uv_near,
                                                           double *__restrict__ uv_far, double2 *__restrict__ staged,
                                                           const int *__restrict__ gpos2, int nxcd)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = staged ? (gpos2 ? gpos2[i] : i) : perm[i];  // issued with the first loads
    const int A = leaf_of[i];
    // near field: the target-centric part (mask bit 9) plus the slots of the mutual
    // items (bits d), in order d = 0..8 (first, so that its loads overlap the far part's)
    const double2 nr = near_from_slots<TS>(i, n, mask[A], near, slots, scale);
    const int4 c = cell[A];
    const double2 z = xy[i];
    double2 W = make_double2(0.0, 0.0);
    if (c.x >= 2) {
        const double w = ldexp(side, -c.x);
        const double2 ctr = cell_centre(x0, y0, side, c);
        const double2 xi = make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w);
        const double2 acc = horner_prefetch<double>(lo + (int64_t)A * p, p, xi);
        W = make_double2(acc.x / w, acc.y / w);
    }
    for (int e = w_off[A]; e < w_off[A + 1]; ++e) {
        const int D = w_idx[e];
        const int4 cd = cell[D];
        const double w = ldexp(side, -cd.x);
        const double2 ctr = cell_centre(x0, y0, side, cd);
        const double2 inv = cinv(make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w));
        const double2 acc = cmul<double>(horner_prefetch<double>(mp + (int64_t)D * p, p, inv), inv);
        W.x += acc.x / w;
        W.y += acc.y / w;
    }
    if (staged) {  // at its staging slot (windows) or in sorted order
        staged[o] = make_double2(nr.x + W.x, nr.y - W.y);
        return;
    }
    if (uv) {
        uv[2 * o] = nr.x + W.x;
        uv[2 * o + 1] = nr.y - W.y;
    }
    if (uv_near) {
        uv_near[2 * o] = nr.x;
        uv_near[2 * o + 1] = nr.y;
    }
    if (uv_far) {
        uv_far[2 * o] = W.x;
        uv_far[2 * o + 1] = -W.y;
    }
}

// ---------------------------------------------------------------------------------
// Adjoint (fmm_atree_velocity_backward).  q_i = dL/du_i + i dL/dv_i.  The adaptive
// operator is antisymmetric (odd near kernel over symmetric U lists, M2L over symmetric V
// lists, M2P over W the transpose of P2L over X at equal truncation), so, as for the
// uniform tree, dL/dGamma = -Im(Phi)/(2 pi) with Phi the same evaluation with charges q,
// the evaluation-position derivative comes from the near sums A, B and the derivative W'
// of the far field of the charges c, and the source-position derivative from the near
// sums with the charges q and the derivative Phi' of the far field of the charges q.
// ---------------------------------------------------------------------------------

// Adjoint charges in sorted order, FP64 and in the records' precision.
template <typename T>
__global__ __launch_bounds__(256) void at_pack_adjoint_kernel(int n, int nxcd, const int *__restrict__ gpos2,
                                                               const double2 *__restrict__ dl_st, double scale,
                                                               double2 *__restrict__ adj, c2<T> *__restrict__ qt)
{
    const int i = xcd_block(nxcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 d = dl_st[gpos2[i]];  // the cotangent staged by bucket
    const double2 q = make_double2(scale * d.x, scale * d.y);
    adj[i] = q;
    qt[i] = mk<T>((T)q.x, (T)q.y);
}

// Adjoint near field of one unit {leaf A, first, count <= 64, log2 TP}: every source leaf
// of U(A) in 64-particle tiles (records and adjoint charges staged in LDS), the target
// moved into the source leaf's frame, the exponential skipped on far tiles; the sums of
// the uniform tree's adjoint pair kernel, FP64 per source leaf.
template <typename T, bool SRC>
__device__ __forceinline__ void at_backward_unit(const int4 u, rec_t<T> *tile, c2<T> *qtile,
                                                 const int4 *__restrict__ cell, const int2 *__restrict__ range,
                                                 const int *__restrict__ u_off, const int *__restrict__ u_idx,
                                                 const int *__restrict__ tile_start,
                                                 const double4 *__restrict__ tile_box,
                                                 const SoaRec<T> &rec, const c2<T> *__restrict__ qt,
                                                 double x0, double y0, double side, double alpha, double cut,
                                                 T lambda, double4 *__restrict__ out_pa, double *__restrict__ out_b,
                                                 double4 *__restrict__ out_src)
{
    constexpr int NA = SRC ? 9 : 5;
    const int lane = threadIdx.x;
    const int logtp = u.w & 15;
    const int tp = 1 << logtp;
    const int t = lane & (tp - 1);
    const int k = lane >> logtp;
    const int i = u.y + min(t, u.z - 1);
    const rec_t<T> ri = rec(i);
    const int A = u.x;
    const int4 cla = cell[A];
    const double2 ca = cell_centre(x0, y0, side, cla);
    const double4 tb = tile_box[tile_start[A] + ((u.y - range[A].x) >> 6)];
    const double a2 = alpha * alpha;
    double sum[NA] = {};
    for (int e = u_off[A]; e < u_off[A + 1]; ++e) {
        const int S = u_idx[e];
        const int2 r = range[S];
        const double2 cs = cell_centre(x0, y0, side, cell[S]);
        const T tx = ri.x + (T)(alpha * (ca.x - cs.x));
        const T ty = ri.y + (T)(alpha * (ca.y - cs.y));
        T acc[NA] = {};
        int tt = tile_start[S];
        for (int base = r.x; base < r.x + r.y; base += 64, ++tt) {
            const int len = min(64, r.x + r.y - base);
            __syncthreads();
            if (lane < len) {
                tile[lane] = rec(base + lane);
                qtile[lane] = qt[base + lane];
            }
            const double4 sb = tile_box[tt];
            const double gx = fmax(0.0, fmax(sb.x - tb.z, tb.x - sb.z));
            const double gy = fmax(0.0, fmax(sb.y - tb.w, tb.y - sb.w));
            // beyond the exponential's cut: point-vortex terms; beyond twice the series cut: no
            // per-pair series test
            const double g2 = (gx * gx + gy * gy) * a2;
            const int cls = g2 >= cut ? 2 : g2 >= 2.0 * (double)series_cut<T>() / (double)lambda ? 1 : 0;
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
    for (int o = tp; o < 64; o <<= 1)
#pragma unroll
        for (int c = 0; c < NA; ++c) sum[c] += __shfl_xor(sum[c], o);
    if (k == 0 && t < u.z) {
        out_pa[i] = make_double4(sum[0], sum[1], sum[2], sum[3]);
        out_b[i] = sum[4];
        if constexpr (SRC) out_src[i] = make_double4(sum[5], sum[6], sum[7], sum[8]);
    }
}

// FP32: 6 wavefronts per SIMD (5 with the source sums), as the uniform tree's adjoint.
template <typename T, bool SRC>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? (SRC ? 5 : 6) : 2) void at_backward_kernel(
    const int4 *__restrict__ units, const int4 *__restrict__ cell, const int2 *__restrict__ range,
    const int *__restrict__ u_off, const int *__restrict__ u_idx, const int *__restrict__ tile_start,
    const double4 *__restrict__ tile_box, const c2<T> *__restrict__ pos, const T *__restrict__ gam,
    const c2<T> *__restrict__ qt, double x0, double y0, double side, double alpha, double cut, T lambda,
    double4 *__restrict__ out_pa, double *__restrict__ out_b, double4 *__restrict__ out_src)
{
    __shared__ rec_t<T> tile[64];
    __shared__ c2<T> qtile[64];
    const SoaRec<T> rec{pos, gam, (T)alpha};
    at_backward_unit<T, SRC>(units[blockIdx.x], tile, qtile, cell, range, u_off, u_idx, tile_start, tile_box, rec, qt,
                             x0, y0, side, alpha, cut, lambda, out_pa, out_b, out_src);
}

// Far field of scaled expansions at z in leaf A and its derivative (FP64):
//   L2P  (1/w) sum_l b_l xi^l,             derivative (1/w^2) sum_{l>=1} l b_l xi^(l-1);
//   M2P  (1/w_D) sum_m a_m zeta^-(m+1),     derivative -(1/w_D^2) sum_m (m+1) a_m zeta^-(m+2),
// over D in W(A), xi = (z - c_A)/w, zeta = (z - c_D)/w_D.  DERIV false: the value only.
template <bool VALUE, bool DERIV>
__device__ __forceinline__ void far_value_deriv(int A, int4 c, double2 z, const int *__restrict__ w_off,
                                                const int *__restrict__ w_idx, const int4 *__restrict__ cell,
                                                const double2 *__restrict__ mp, const double2 *__restrict__ lo, int p,
                                                double x0, double y0, double side, double2 &val, double2 &der)
{
    val = make_double2(0.0, 0.0);
    der = make_double2(0.0, 0.0);
    if (c.x >= 2) {
        const double w = ldexp(side, -c.x);
        const double2 ctr = cell_centre(x0, y0, side, c);
        const double2 xi = make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w);
        const double2 *b = lo + (int64_t)A * p;
        if (VALUE) {
            const double2 acc = horner_prefetch<double>(b, p, xi);
            val = make_double2(acc.x / w, acc.y / w);
        }
        if (DERIV && p >= 2) {
            const double2 acc = horner_weighted_prefetch<double>(b, p, xi, 1, 0);
            der = make_double2(acc.x / (w * w), acc.y / (w * w));
        }
    }
    for (int e = w_off[A]; e < w_off[A + 1]; ++e) {
        const int D = w_idx[e];
        const int4 cd = cell[D];
        const double w = ldexp(side, -cd.x);
        const double2 ctr = cell_centre(x0, y0, side, cd);
        const double2 inv = cinv(make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w));
        const double2 *a = mp + (int64_t)D * p;
        if (VALUE) {
            const double2 acc = cmul<double>(horner_prefetch<double>(a, p, inv), inv);
            val.x += acc.x / w;
            val.y += acc.y / w;
        }
        if (DERIV) {
            const double2 acc = cmul<double>(horner_weighted_prefetch<double>(a, p, inv, 0, 1), cmul<double>(inv, inv));
            der.x -= acc.x / (w * w);
            der.y -= acc.y / (w * w);
        }
    }
}

// Adjoint finalize: the near sums (record units: Phi scaled by alpha, A and B by
// alpha^2 / (2 pi), as for the uniform tree) combined with the far parts:
//   dL/dGamma = -Im(Phi_near + Phi_far)/(2 pi),
//   dL/dx_eval = Re(q (A + B + W')), dL/dy_eval = -Im(q (A - B + W'))   (B imaginary),
//   dL/dx_src = -Re(c (At + Bt)),     dL/dy_src = Im(c (At - Bt)),  At = near + Phi'.
template <bool SRC>
__global__ __launch_bounds__(256) void at_finalize_backward_kernel(
    int n, const int *__restrict__ perm, const int *__restrict__ leaf_of, const int4 *__restrict__ cell,
    const double2 *__restrict__ xy, const int *__restrict__ w_off, const int *__restrict__ w_idx,
    const double2 *__restrict__ mp, const double2 *__restrict__ lo, const double2 *__restrict__ mp2,
    const double2 *__restrict__ lo2, int p, double x0, double y0, double side, const double4 *__restrict__ near_pa,
    const double *__restrict__ near_b, const double4 *__restrict__ near_src, const double2 *__restrict__ adj,
    const double *__restrict__ gamma, double alpha, double lambda, AdjointOut out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the per-particle loads first, in flight during the far-field work
    const int64_t o = perm[i];
    const double4 a = near_pa[i];
    const double sb = near_b[i];
    const int A = leaf_of[i];
    const int4 c = cell[A];
    const double2 z = xy[i];
    double2 wv, dw, phi, dphi;
    far_value_deriv<false, true>(A, c, z, w_off, w_idx, cell, mp, lo, p, x0, y0, side, wv, dw);
    far_value_deriv<true, SRC>(A, c, z, w_off, w_idx, cell, mp2, lo2, p, x0, y0, side, phi, dphi);
    const double ka = alpha * alpha * kInv2Pi;
    const double Ar = ka * (-2.0 * a.w), Ai = -ka * a.z;
    const double Bi = -ka * lambda * sb;
    const double g = -(alpha * a.y + phi.y) * kInv2Pi;
    double ex = 0.0, ey = 0.0, sx = 0.0, sy = 0.0;
    if (out.dxe || out.dxy) {
        const double2 q = adj[i];
        const double d1r = Ar + dw.x, d1i = Ai + Bi + dw.y;
        const double d2r = Ar + dw.x, d2i = Ai - Bi + dw.y;
        ex = q.x * d1r - q.y * d1i;
        ey = -(q.x * d2i + q.y * d2r);
    }
    if constexpr (SRC) {
        const double4 ns = near_src[i];
        const double a2 = alpha * alpha;
        const double atr = a2 * ns.x + dphi.x, ati = a2 * ns.y + dphi.y;
        const double btr = a2 * lambda * ns.z, bti = a2 * lambda * ns.w;
        const double G = gamma[i] * kInv2Pi;  // c = -i G: Re(c w) = G Im w, Im(c w) = -G Re w
        sx = -G * (ati + bti);
        sy = -G * (atr - btr);
    }
    store_adjoint(out, o, g, ex, ey, sx, sy);
}

inline unsigned blocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

void launch_atree_pack(const AtreeCall &c, const double *gamma, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    launch_stage_rows(n, t->stage_shift, t->d.gpos1, gamma, t->d.st1, s);
    const unsigned g = xcd_grid(n, 256, kXcds);
    if (c.is_double)
        at_pack_kernel<double><<<g, 256, 0, s>>>(n, kXcds, t->d.gpos2, t->d.st1, (double *)t->wsp->gam,
                                                 t->wsp->gamma);
    else
        at_pack_kernel<float><<<g, 256, 0, s>>>(n, kXcds, t->d.gpos2, t->d.st1, (float *)t->wsp->gam,
                                                t->wsp->gamma);
}

void launch_atree_coords(const fmm_atree *t, int is_double, void *pos, hipStream_t s)
{
    const int n = (int)t->n;
    if (is_double)
        at_coords_kernel<double><<<blocks(n, 256), 256, 0, s>>>(n, t->d.leaf_of, t->d.cell, t->d.xy, t->x0, t->y0,
                                                                t->side, (double2 *)pos);
    else
        at_coords_kernel<float><<<blocks(n, 256), 256, 0, s>>>(n, t->d.leaf_of, t->d.cell, t->d.xy, t->x0, t->y0,
                                                               t->side, (float2 *)pos);
}

// One gather-GEMM launch over up to four target lists (classes).
void at_gemm_launch(AtGemm a, const int *seg_off, int nlists, hipStream_t s)
{
    a.nwaves = 0;
    for (int k = 0; k < 4; ++k) {
        a.cstart[k] = k < nlists ? seg_off[k] : 0;
        a.clen[k] = k < nlists ? seg_off[k + 1] - seg_off[k] : 0;
        a.cwave0[k] = a.nwaves;
        a.nwaves += (a.clen[k] + 15) / 16;
    }
    if (a.nwaves > 0) at_gemm_kernel<<<(unsigned)((a.nwaves + 3) / 4), 256, 0, s>>>(a);
}

template <bool CPLX>
void far_chain(const AtreeCall &c, double2 *mp, double2 *lo, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int deepest = (int)t->sizes[6];
    if (deepest < 2) return;
    const int p = c.p, nb = 2 * p + 1;
    const double2 *q = t->wsp->adj;
    const bool gemm = c.tabs && t->m2l_plan;  // p <= 16: stages 5-7 on MFMA
    if (t->np2m > 0) {
        // 16 lanes per leaf, four leaves per wavefront
        const int np = (int)t->np2m;
        const unsigned g = (unsigned)((np + 3) / 4);
        if (p <= 16)
            at_p2m_kernel<16, CPLX, 16><<<g, 64, 0, s>>>(t->d.p2m_cells, np, t->d.cell, t->d.range, t->d.xy,
                                                         t->wsp->gamma, q, t->x0, t->y0, t->side, p, mp);
        else
            at_p2m_kernel<32, CPLX, 16><<<g, 64, 0, s>>>(t->d.p2m_cells, np, t->d.cell, t->d.range, t->d.xy,
                                                         t->wsp->gamma, q, t->x0, t->y0, t->side, p, mp);
    }
    AtGemm a{};
    if (gemm) {
        a.first = t->level_off[2];
        a.p = p;
        a.vslot = t->d.vslot;
        a.x_off = t->d.x_off;
        a.parent = t->d.parent;
        a.child = t->d.child;
        a.entries = c.tabs->mfma_entries;
        a.src = (const double *)mp;
        a.tab = c.tabs->mfma_d;
        a.zero = c.tabs->zero_row;
    }
    for (int l = deepest - 1; l >= 2; --l) {
        const int cnt = t->inner_off[l + 1] - t->inner_off[l];
        if (cnt == 0) continue;
        if (gemm) {
            a.mode = 1;
            a.targets = t->d.inner + t->inner_off[l];
            a.out = (double *)mp;
            const int one[2] = {0, cnt};
            at_gemm_launch(a, one, 1, s);
        } else {
            at_m2m_kernel<<<blocks((int64_t)cnt * p, 256), 256, 0, s>>>(t->d.inner + t->inner_off[l], cnt,
                                                                        t->d.child, t->wsp->binom, nb, p, mp);
        }
    }
    const int first = t->level_off[2], cnt = t->level_off[deepest + 1] - first;
    if (cnt > 0 && gemm) {
        // P2L into the locals of the cells with an X list, then level by level the M2L
        // from V and the L2L from the parent added to them
        if (t->sizes[5] > 0)  // |X|
            at_p2l_kernel<16, CPLX><<<blocks(cnt, 64), 64, 0, s>>>(first, cnt, t->d.cell, t->d.x_off, t->d.x_idx,
                                                                   t->d.range, t->d.xy, t->wsp->gamma, q, t->x0,
                                                                   t->y0, t->side, p, lo);
        a.mode = 0;
        a.targets = t->d.m2l_targets;
        a.out = (double *)lo;
        for (int l = 2; l <= deepest; ++l) {
            a.par = l >= 3 ? (const double *)lo : nullptr;
            at_gemm_launch(a, &t->m2l_seg_off[4 * (l - 2)], 4, s);
        }
        return;
    }
    // M2L + P2L for every cell of level >= 2 at once, then L2L level by level
    if (cnt > 0) {
        if (p <= 16)
            at_m2l_kernel<16, CPLX><<<blocks(cnt, 64), 64, 0, s>>>(first, cnt, t->d.cell, t->d.v_off, t->d.v_idx,
                                                                   t->d.x_off, t->d.x_idx, t->d.range, t->d.xy,
                                                                   t->wsp->gamma, q, t->x0, t->y0, t->side,
                                                                   t->wsp->binom16, p, mp, lo);
        else
            at_m2l_kernel<32, CPLX><<<blocks(cnt, 64), 64, 0, s>>>(first, cnt, t->d.cell, t->d.v_off, t->d.v_idx,
                                                                   t->d.x_off, t->d.x_idx, t->d.range, t->d.xy,
                                                                   t->wsp->gamma, q, t->x0, t->y0, t->side,
                                                                   t->wsp->binom32, p, mp, lo);
    }
    for (int l = 3; l <= deepest; ++l) {
        const int f = t->level_off[l], nc = t->level_off[l + 1] - f;
        if (nc == 0) continue;
        at_l2l_kernel<<<blocks((int64_t)nc * p, 256), 256, 0, s>>>(f, nc, t->d.cell, t->d.parent, t->wsp->binom, nb, p,
                                                                   lo);
    }
}

void launch_atree_far(const AtreeCall &c, hipStream_t s, bool adjoint)
{
    if (adjoint)
        far_chain<true>(c, c.t->wsp->mp2, c.t->wsp->lo2, s);
    else
        far_chain<false>(c, c.t->wsp->mp, c.t->wsp->lo, s);
}

void launch_atree_near(const AtreeCall &c, hipStream_t s)
{
    const fmm_atree *t = c.t;
    if (t->nwork == 0) return;
    const double scale = c.alpha * kInv2Pi;
    // exponent at which 1 - e rounds to 1: FP32 base 2 at 26, FP64 base e at 37.5, one
    // unit of margin for the rounding of the records and the boxes
    const double cut = c.is_double ? 39.0 : 27.0;
    // Occupancy cap: each workgroup (one wavefront) reserves LDS so that at most near_occ
    // of them fit on a SIMD (160 KiB per CU, 4 SIMDs); the far chain on the other stream
    // takes the wavefront slots left over.
    const size_t static_lds = 256 * (c.is_double ? sizeof(double4) : sizeof(float4));
    const size_t per_wave = c.near_occ > 0 ? (size_t)160 * 1024 / (4 * (size_t)c.near_occ) : 0;
    const size_t dyn = per_wave > static_lds ? per_wave - static_lds : 0;
    if (c.is_double)
        at_near_kernel<double><<<(unsigned)t->nwork, 64, dyn, s>>>(
            t->d.work, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            t->d.leaf_start, t->d.leaf_tile, t->d.tile_box_leaf, (const double2 *)t->d_pos[1],
            (const double *)t->wsp->gam, t->x0, t->y0, t->side,
            c.alpha, cut, scale, t->dense_leaf, t->n, t->wsp->near, (double2 *)t->wsp->slots);
    else
        at_near_kernel<float><<<(unsigned)t->nwork, 64, dyn, s>>>(
            t->d.work, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            t->d.leaf_start, t->d.leaf_tile, t->d.tile_box_leaf, (const float2 *)t->d_pos[0],
            (const float *)t->wsp->gam, t->x0, t->y0, t->side,
            c.alpha, cut, scale, t->dense_leaf, t->n, t->wsp->near, (float2 *)t->wsp->slots);
}

void launch_atree_finalize(const AtreeCall &c, double *uv, double *uv_near, double *uv_far, const double *base,
                           double h, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    const double scale = c.alpha * kInv2Pi;
    // uv alone: the totals go to the staging array (n double2), then to user order:
    // through the staging windows once the output fills the last-level cache, else in
    // sorted order and scattered
    double2 *staged = uv && !uv_near && !uv_far ? t->wsp->stage : nullptr;
    const bool windowed = staged && outputs_windowed(n, sizeof(double2));
    const int *gp = windowed ? t->d.gpos2 : nullptr;
    double *uv_direct = staged ? nullptr : uv;
    const unsigned g = xcd_grid(n, 256, kXcds);
    if (c.is_double)
        at_finalize_kernel<double><<<g, 256, 0, s>>>(
            n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, t->d.w_off, t->d.w_idx, t->wsp->mp, t->wsp->lo, c.p, t->x0,
            t->y0, t->side, t->wsp->near, t->d.mask, (const double2 *)t->wsp->slots, scale, uv_direct, uv_near, uv_far,
            staged, gp, kXcds);
    else
        at_finalize_kernel<float><<<g, 256, 0, s>>>(
            n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, t->d.w_off, t->d.w_idx, t->wsp->mp, t->wsp->lo, c.p, t->x0,
            t->y0, t->side, t->wsp->near, t->d.mask, (const float2 *)t->wsp->slots, scale, uv_direct, uv_near, uv_far,
            staged, gp, kXcds);
    if (windowed) launch_gather_rows(n, t->d.gpos1, staged, uv, base, h, s);
    else if (staged) scatter_rows_kernel<<<blocks(n, 256), 256, 0, s>>>(n, t->d.perm, staged, uv, base, h);
}

void launch_atree_pack_adjoint(const AtreeCall &c, const double *dl_duv, double scale, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    // the forward's near-field array (n double2) is free during the adjoint: the staging
    double2 *st = t->wsp->near;
    launch_stage_rows2(n, t->stage_shift, t->d.gpos1, (const double2 *)dl_duv, st, s);
    const unsigned g = xcd_grid(n, 256, kXcds);
    if (c.is_double)
        at_pack_adjoint_kernel<double><<<g, 256, 0, s>>>(n, kXcds, t->d.gpos2, st, scale, t->wsp->adj,
                                                         (double2 *)t->wsp->qt);
    else
        at_pack_adjoint_kernel<float><<<g, 256, 0, s>>>(n, kXcds, t->d.gpos2, st, scale, t->wsp->adj,
                                                        (float2 *)t->wsp->qt);
}

void launch_atree_backward_near(const AtreeCall &c, bool src, hipStream_t s)
{
    const fmm_atree *t = c.t;
    if (t->nbwd_units <= 0) return;
    const double cut = c.is_double ? 39.0 : 27.0;  // as for the forward near field
    const unsigned g = (unsigned)t->nbwd_units;
    const AtreeDev &d = t->d;
    const AtreeWs &w = *t->wsp;
    if (c.is_double) {
        auto k = src ? at_backward_kernel<double, true> : at_backward_kernel<double, false>;
        k<<<g, 64, 0, s>>>(d.bwd_units, d.cell, d.range, d.u_off, d.u_idx, d.tile_start, d.tile_box,
                           (const double2 *)t->d_pos[1], (const double *)w.gam, (const double2 *)w.qt, t->x0,
                           t->y0, t->side, c.alpha, cut, 1.0,
                           w.pa, w.pb, src ? w.psrc : nullptr);
    } else {
        auto k = src ? at_backward_kernel<float, true> : at_backward_kernel<float, false>;
        k<<<g, 64, 0, s>>>(d.bwd_units, d.cell, d.range, d.u_off, d.u_idx, d.tile_start, d.tile_box,
                           (const float2 *)t->d_pos[0], (const float *)w.gam, (const float2 *)w.qt, t->x0,
                           t->y0, t->side, c.alpha, cut,
                           0.69314718055994530942f, w.pa, w.pb, src ? w.psrc : nullptr);
    }
}

void launch_atree_finalize_backward(const AtreeCall &c, const AdjointOut &out, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    const double lambda = c.is_double ? 1.0 : 0.69314718055994530942;
    const AtreeDev &d = t->d;
    const AtreeWs &w = *t->wsp;
    auto k = (out.dxs || out.dxy) ? at_finalize_backward_kernel<true> : at_finalize_backward_kernel<false>;
    k<<<blocks(n, 256), 256, 0, s>>>(n, d.perm, d.leaf_of, d.cell, d.xy, d.w_off, d.w_idx, w.mp, w.lo, w.mp2, w.lo2,
                                     c.p, t->x0, t->y0, t->side, w.pa, w.pb, w.psrc, w.adj, w.gamma, c.alpha, lambda,
                                     out);
}

}  // namespace fmm
