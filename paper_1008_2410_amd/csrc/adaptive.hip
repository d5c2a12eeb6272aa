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
template <typename T>
__global__ __launch_bounds__(256) void at_pack_kernel(int n, const int *__restrict__ perm,
                                                       const int *__restrict__ leaf_of, const int4 *__restrict__ cell,
                                                       const double2 *__restrict__ xy, const double *__restrict__ gamma,
                                                       double x0, double y0, double side, double alpha,
                                                       rec_t<T> *__restrict__ rec, double *__restrict__ gamma_sorted)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 c = cell_centre(x0, y0, side, cell[leaf_of[i]]);
    const double2 z = xy[i];
    const double g = gamma[perm[i]];
    rec_t<T> r;
    r.x = (T)(alpha * (z.x - c.x));
    r.y = (T)(alpha * (z.y - c.y));
    r.z = (T)g;
    r.w = (T)0;
    rec[i] = r;
    gamma_sorted[i] = g;
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

// P2M (stage 4) at the leaves of level >= 2, one wavefront per leaf:
//   a_m / w^m = sum_j c_j xi_j^m,  xi_j = (z_j - c)/w,
// lanes over the leaf's particles, then a butterfly over the wavefront per coefficient.
template <int PMAX>
__global__ __launch_bounds__(64) void at_p2m_kernel(const int *__restrict__ cells, const int4 *__restrict__ cell,
                                                     const int2 *__restrict__ range, const double2 *__restrict__ xy,
                                                     const double *__restrict__ gamma, double x0, double y0,
                                                     double side, int p, double2 *__restrict__ mp)
{
    const int lane = threadIdx.x;
    const int k = cells[blockIdx.x];
    const int4 c = cell[k];
    const int2 r = range[k];
    const double w = ldexp(side, -c.x);
    const double rw = 1.0 / w;
    const double2 ctr = cell_centre(x0, y0, side, c);
    // PMAX coefficients throughout (those at m >= p are never stored): no branches on
    // p, so the butterfly below runs step by step over all coefficients at once
    double2 acc[PMAX];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) acc[m] = make_double2(0.0, 0.0);
    for (int j = r.x + lane; j < r.x + r.y; j += 64) {
        const double2 z = xy[j];
        const double2 xi = make_double2((z.x - ctr.x) * rw, (z.y - ctr.y) * rw);
        double2 pw = make_double2(0.0, -gamma[j] * kInv2Pi);
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            acc[m].x += pw.x;
            acc[m].y += pw.y;
            pw = cmul<double>(pw, xi);
        }
    }
    butterfly_step<PMAX>(acc, 32);
    butterfly_step<PMAX>(acc, 16);
    butterfly_step<PMAX>(acc, 8);
    butterfly_step<PMAX>(acc, 4);
    butterfly_step<PMAX>(acc, 2);
    butterfly_step<PMAX>(acc, 1);
    // every lane holds the sums; lane 0 stores them (constant indices: a lane-dependent
    // pick would make the compiler address the array in scratch memory)
    if (lane == 0)
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
template <int PMAX>
__global__ __launch_bounds__(64) void at_m2l_kernel(int first, int ncells, const int4 *__restrict__ cell,
                                                     const int *__restrict__ v_off, const int *__restrict__ v_idx,
                                                     const int *__restrict__ x_off, const int *__restrict__ x_idx,
                                                     const int2 *__restrict__ range, const double2 *__restrict__ xy,
                                                     const double *__restrict__ gamma, double x0, double y0,
                                                     double side, const double *__restrict__ binom, int p,
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
                // -c_j u^(l+1) with c_j = -i Gamma_j/(2 pi):  i (Gamma_j/(2 pi)) u^(l+1)
                const double g = gamma[j] * kInv2Pi;
                double2 ul = u;
#pragma unroll
                for (int l = 0; l < PMAX; ++l) {
                    b[l].x -= g * ul.y;
                    b[l].y += g * ul.x;
                    ul = cmul<double>(ul, u);
                }
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
                                               const rec_t<T> *__restrict__ rec, double x0, double y0, double side,
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
    const rec_t<T> ri = rec[i];
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
            if (lane < len) tile[lane] = rec[base + lane];
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
    const float4 *__restrict__ tile_box_leaf, const rec_t<T> *__restrict__ rec, double x0, double y0, double side,
    double alpha, double cut, double scale, int dense, int64_t n, double2 *__restrict__ near,
    c2<T> *__restrict__ slots)
{
    __shared__ rec_t<T> tile_a[128], tile_b[128];
    const int4 u = work[blockIdx.x];
    if (u.w & kMutualItem) {
        const double step = alpha * ldexp(side, -(u.w >> 9));
        mutual_item<T>(u, tile_a, tile_b, rec, leaf_start, leaf_tile, tile_box_leaf, (T)step,
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
                                                           double *__restrict__ uv_far)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int A = leaf_of[i];
    const int4 c = cell[A];
    const double2 z = xy[i];
    double2 W = make_double2(0.0, 0.0);
    if (c.x >= 2) {
        const double w = ldexp(side, -c.x);
        const double2 ctr = cell_centre(x0, y0, side, c);
        const double2 xi = make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w);
        const double2 *b = lo + (int64_t)A * p;
        double2 acc = b[p - 1];
        for (int l = p - 2; l >= 0; --l) acc = cmac<double>(b[l], acc, xi);
        W = make_double2(acc.x / w, acc.y / w);
    }
    for (int e = w_off[A]; e < w_off[A + 1]; ++e) {
        const int D = w_idx[e];
        const int4 cd = cell[D];
        const double w = ldexp(side, -cd.x);
        const double2 ctr = cell_centre(x0, y0, side, cd);
        const double2 inv = cinv(make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w));
        const double2 *a = mp + (int64_t)D * p;
        double2 acc = a[p - 1];
        for (int m = p - 2; m >= 0; --m) acc = cmac<double>(a[m], acc, inv);
        acc = cmul<double>(acc, inv);
        W.x += acc.x / w;
        W.y += acc.y / w;
    }
    // near field: the target-centric part (mask bit 9) plus the slots of the mutual
    // items (bits d), in order d = 0..8
    const int m = mask[A];
    double2 nr = (m >> 9) & 1 ? near[i] : make_double2(0.0, 0.0);
    double su = 0.0, sv = 0.0;
#pragma unroll
    for (int d = 0; d < 9; ++d)
        if ((m >> d) & 1) {
            const c2<TS> v = slots[d * (int64_t)n + i];
            su += (double)v.x;
            sv += (double)v.y;
        }
    nr.x -= scale * su;
    nr.y += scale * sv;
    const int64_t o = perm[i];
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

inline unsigned blocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

void launch_atree_pack(const AtreeCall &c, const double *gamma, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    if (c.is_double)
        at_pack_kernel<double><<<blocks(n, 256), 256, 0, s>>>(n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, gamma,
                                                              t->x0, t->y0, t->side, c.alpha,
                                                              (double4 *)t->ws.rec, t->ws.gamma);
    else
        at_pack_kernel<float><<<blocks(n, 256), 256, 0, s>>>(n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, gamma,
                                                             t->x0, t->y0, t->side, c.alpha, (float4 *)t->ws.rec,
                                                             t->ws.gamma);
}

void launch_atree_far(const AtreeCall &c, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int deepest = (int)t->sizes[6];
    if (deepest < 2) return;
    const int p = c.p, nb = 2 * p + 1;
    if (t->np2m > 0) {
        if (p <= 16)
            at_p2m_kernel<16><<<(unsigned)t->np2m, 64, 0, s>>>(t->d.p2m_cells, t->d.cell, t->d.range, t->d.xy,
                                                               t->ws.gamma, t->x0, t->y0, t->side, p, t->ws.mp);
        else
            at_p2m_kernel<32><<<(unsigned)t->np2m, 64, 0, s>>>(t->d.p2m_cells, t->d.cell, t->d.range, t->d.xy,
                                                               t->ws.gamma, t->x0, t->y0, t->side, p, t->ws.mp);
    }
    for (int l = deepest - 1; l >= 2; --l) {
        const int cnt = t->inner_off[l + 1] - t->inner_off[l];
        if (cnt == 0) continue;
        at_m2m_kernel<<<blocks((int64_t)cnt * p, 256), 256, 0, s>>>(t->d.inner + t->inner_off[l], cnt, t->d.child,
                                                                    t->ws.binom, nb, p, t->ws.mp);
    }
    // M2L + P2L for every cell of level >= 2 at once, then L2L level by level
    const int first = t->level_off[2], cnt = t->level_off[deepest + 1] - first;
    if (cnt > 0) {
        if (p <= 16)
            at_m2l_kernel<16><<<blocks(cnt, 64), 64, 0, s>>>(first, cnt, t->d.cell, t->d.v_off, t->d.v_idx,
                                                             t->d.x_off, t->d.x_idx, t->d.range, t->d.xy, t->ws.gamma,
                                                             t->x0, t->y0, t->side, t->ws.binom16, p, t->ws.mp,
                                                             t->ws.lo);
        else
            at_m2l_kernel<32><<<blocks(cnt, 64), 64, 0, s>>>(first, cnt, t->d.cell, t->d.v_off, t->d.v_idx,
                                                             t->d.x_off, t->d.x_idx, t->d.range, t->d.xy, t->ws.gamma,
                                                             t->x0, t->y0, t->side, t->ws.binom32, p, t->ws.mp,
                                                             t->ws.lo);
    }
    for (int l = 3; l <= deepest; ++l) {
        const int f = t->level_off[l], nc = t->level_off[l + 1] - f;
        if (nc == 0) continue;
        at_l2l_kernel<<<blocks((int64_t)nc * p, 256), 256, 0, s>>>(f, nc, t->d.cell, t->d.parent, t->ws.binom, nb, p,
                                                                   t->ws.lo);
    }
}

void launch_atree_near(const AtreeCall &c, hipStream_t s)
{
    const fmm_atree *t = c.t;
    if (t->nwork == 0) return;
    const double scale = c.alpha * kInv2Pi;
    // exponent at which 1 - e rounds to 1: FP32 base 2 at 26, FP64 base e at 37.5, one
    // unit of margin for the rounding of the records and the boxes
    const double cut = c.is_double ? 39.0 : 27.0;
    if (c.is_double)
        at_near_kernel<double><<<(unsigned)t->nwork, 64, 0, s>>>(
            t->d.work, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            t->d.leaf_start, t->d.leaf_tile, t->d.tile_box_leaf, (const double4 *)t->ws.rec, t->x0, t->y0, t->side,
            c.alpha, cut, scale, t->dense_leaf, t->n, t->ws.near, (double2 *)t->ws.slots);
    else
        at_near_kernel<float><<<(unsigned)t->nwork, 64, 0, s>>>(
            t->d.work, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            t->d.leaf_start, t->d.leaf_tile, t->d.tile_box_leaf, (const float4 *)t->ws.rec, t->x0, t->y0, t->side,
            c.alpha, cut, scale, t->dense_leaf, t->n, t->ws.near, (float2 *)t->ws.slots);
}

void launch_atree_finalize(const AtreeCall &c, double *uv, double *uv_near, double *uv_far, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    const double scale = c.alpha * kInv2Pi;
    if (c.is_double)
        at_finalize_kernel<double><<<blocks(n, 256), 256, 0, s>>>(
            n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, t->d.w_off, t->d.w_idx, t->ws.mp, t->ws.lo, c.p, t->x0,
            t->y0, t->side, t->ws.near, t->d.mask, (const double2 *)t->ws.slots, scale, uv, uv_near, uv_far);
    else
        at_finalize_kernel<float><<<blocks(n, 256), 256, 0, s>>>(
            n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, t->d.w_off, t->d.w_idx, t->ws.mp, t->ws.lo, c.p, t->x0,
            t->y0, t->side, t->ws.near, t->d.mask, (const float2 *)t->ws.slots, scale, uv, uv_near, uv_far);
}

}  // namespace fmm
