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

__device__ __forceinline__ double2 cpow_int(double2 a, int e)
{
    double2 r = make_double2(1.0, 0.0);
    for (int k = 0; k < e; ++k) r = cmul<double>(r, a);
    return r;
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

// P2M (stage 4) at the leaves of level >= 2, one wavefront per leaf:
//   a_m / w^m = sum_j c_j xi_j^m,  xi_j = (z_j - c)/w.
template <int PMAX>
__global__ __launch_bounds__(64) void at_p2m_kernel(const int *__restrict__ cells, const int4 *__restrict__ cell,
                                                     const int2 *__restrict__ range, const double2 *__restrict__ xy,
                                                     const double *__restrict__ gamma, double x0, double y0,
                                                     double side, int p, double2 *__restrict__ mp)
{
    __shared__ double red[64][2 * PMAX + 1];
    const int lane = threadIdx.x;
    const int k = cells[blockIdx.x];
    const int4 c = cell[k];
    const int2 r = range[k];
    const double w = ldexp(side, -c.x);
    const double2 ctr = cell_centre(x0, y0, side, c);
    double2 acc[PMAX];
#pragma unroll
    for (int m = 0; m < PMAX; ++m) acc[m] = make_double2(0.0, 0.0);
    for (int j = r.x + lane; j < r.x + r.y; j += 64) {
        const double2 z = xy[j];
        const double2 xi = make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w);
        double2 pw = make_double2(0.0, -gamma[j] * kInv2Pi);
#pragma unroll
        for (int m = 0; m < PMAX; ++m)
            if (m < p) {
                acc[m].x += pw.x;
                acc[m].y += pw.y;
                pw = cmul<double>(pw, xi);
            }
    }
#pragma unroll
    for (int m = 0; m < PMAX; ++m) {
        red[lane][2 * m] = acc[m].x;
        red[lane][2 * m + 1] = acc[m].y;
    }
    __syncthreads();
    if (lane < 2 * p) {
        double s = 0.0;
        for (int row = 0; row < 64; ++row) s += red[row][lane];
        ((double *)mp)[(int64_t)k * 2 * p + lane] = s;
    }
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

// Downward pass (stages 6-7) into the cells of one level l >= 2, one thread per
// (cell, l'):  L2L from the parent (when the parent has an expansion),
//   b_k = sum_{j>=k} C(j,k) d^(j-k) 2^-(k+1) b_j(parent);
// M2L from V,  b_l += sum_m (-1)^l C(l+m,m) delta^-(l+m+1) a_m(S), delta = (c - c_S)/w;
// P2L from X,  b_l += -sum_{j in A} c_j zeta_j^-(l+1), zeta_j = (z_j - c)/w.
__global__ __launch_bounds__(256) void at_down_kernel(int first, int ncells, const int4 *__restrict__ cell,
                                                       const int *__restrict__ parent, const int *__restrict__ v_off,
                                                       const int *__restrict__ v_idx, const int *__restrict__ x_off,
                                                       const int *__restrict__ x_idx, const int2 *__restrict__ range,
                                                       const double2 *__restrict__ xy,
                                                       const double *__restrict__ gamma, double x0, double y0,
                                                       double side, const double *__restrict__ binom, int nb, int p,
                                                       const double2 *__restrict__ mp, double2 *__restrict__ lo)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells * p) return;
    const int k = first + t / p, l = t % p;
    const int4 c = cell[k];
    double2 acc = make_double2(0.0, 0.0);
    if (c.x >= 3) {
        const int P = parent[k];
        const double2 d = make_double2(((c.y & 1) - 0.5) * 0.5, ((c.z & 1) - 0.5) * 0.5);
        double2 pw = make_double2(1.0, 0.0);
        for (int j = l; j < p; ++j) {
            const double2 term = cmul<double>(lo[(int64_t)P * p + j], pw);
            acc.x = fma(binom[j * nb + l], term.x, acc.x);
            acc.y = fma(binom[j * nb + l], term.y, acc.y);
            pw = cmul<double>(pw, d);
        }
        const double f = ldexp(1.0, -(l + 1));
        acc.x *= f;
        acc.y *= f;
    }
    const double sg = (l & 1) ? -1.0 : 1.0;
    for (int e = v_off[k]; e < v_off[k + 1]; ++e) {
        const int S = v_idx[e];
        const int4 cs = cell[S];
        const double2 inv = cinv(make_double2((double)(c.y - cs.y), (double)(c.z - cs.z)));
        double2 pw = cpow_int(inv, l + 1);
        for (int m = 0; m < p; ++m) {
            const double2 term = cmul<double>(mp[(int64_t)S * p + m], pw);
            const double f = sg * binom[(l + m) * nb + m];
            acc.x = fma(f, term.x, acc.x);
            acc.y = fma(f, term.y, acc.y);
            pw = cmul<double>(pw, inv);
        }
    }
    if (x_off[k] < x_off[k + 1]) {
        const double w = ldexp(side, -c.x);
        const double2 ctr = cell_centre(x0, y0, side, c);
        for (int e = x_off[k]; e < x_off[k + 1]; ++e) {
            const int2 r = range[x_idx[e]];
            for (int j = r.x; j < r.x + r.y; ++j) {
                const double2 z = xy[j];
                const double2 pw = cpow_int(cinv(make_double2((z.x - ctr.x) / w, (z.y - ctr.y) / w)), l + 1);
                // -c_j pw with c_j = -i Gamma_j/(2 pi):  i (Gamma_j/(2 pi)) pw
                const double g = gamma[j] * kInv2Pi;
                acc.x -= g * pw.y;
                acc.y += g * pw.x;
            }
        }
    }
    lo[(int64_t)k * p + l] = acc;
}

// Near field (stage 9) over U, target-centric as the uniform tree's units: one
// wavefront per unit {leaf A, first, count <= 64, log2 TP}; every source leaf S of
// U(A) in 64-particle tiles staged in LDS, the target moved into S's frame
// (alpha (z_i - c_S) = record_i + alpha (c_A - c_S)).  A source tile whose bounding box
// is at least the cut from the unit's box skips the exponential (1 - e rounds to 1).
template <typename T>
__global__ __launch_bounds__(64) void at_near_kernel(const int4 *__restrict__ units, const int4 *__restrict__ cell,
                                                      const int2 *__restrict__ range, const int *__restrict__ u_off,
                                                      const int *__restrict__ u_idx,
                                                      const int *__restrict__ tile_start,
                                                      const double4 *__restrict__ tile_box,
                                                      const rec_t<T> *__restrict__ rec, double x0, double y0,
                                                      double side, double alpha, double cut, double scale,
                                                      double2 *__restrict__ near)
{
    __shared__ rec_t<T> tile[64];
    const int4 u = units[blockIdx.x];
    const int lane = threadIdx.x;
    const int logtp = u.w;
    const int tp = 1 << logtp;
    const int t = lane & (tp - 1);
    const int k = lane >> logtp;
    const int i = u.y + min(t, u.z - 1);
    const rec_t<T> ri = rec[i];
    const int A = u.x;
    const double2 ca = cell_centre(x0, y0, side, cell[A]);
    const double4 tb = tile_box[tile_start[A] + ((u.y - range[A].x) >> 6)];
    const double a2 = alpha * alpha;
    double au = 0.0, av = 0.0;
    for (int e = u_off[A]; e < u_off[A + 1]; ++e) {
        const int S = u_idx[e];
        const double2 cs = cell_centre(x0, y0, side, cell[S]);
        const int2 r = range[S];
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

// Stages 8 + 10: L2P from the leaf's local expansion (level >= 2),
//   W += (1/w) sum_l b_l xi^l;  M2P from W(leaf),  W += (1/w_D) sum_m a_m zeta^-(m+1);
// (u, v) = near + (Re W, -Im W), scattered to user order.
__global__ __launch_bounds__(256) void at_finalize_kernel(int n, const int *__restrict__ perm,
                                                           const int *__restrict__ leaf_of,
                                                           const int4 *__restrict__ cell,
                                                           const double2 *__restrict__ xy,
                                                           const int *__restrict__ w_off,
                                                           const int *__restrict__ w_idx,
                                                           const double2 *__restrict__ mp,
                                                           const double2 *__restrict__ lo, int p, double x0,
                                                           double y0, double side, const double2 *__restrict__ near,
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
    const double2 nr = near[i];
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
    for (int l = 2; l <= deepest; ++l) {
        const int first = t->level_off[l], cnt = t->level_off[l + 1] - first;
        if (cnt == 0) continue;
        at_down_kernel<<<blocks((int64_t)cnt * p, 256), 256, 0, s>>>(
            first, cnt, t->d.cell, t->d.parent, t->d.v_off, t->d.v_idx, t->d.x_off, t->d.x_idx, t->d.range, t->d.xy,
            t->ws.gamma, t->x0, t->y0, t->side, t->ws.binom, nb, p, t->ws.mp, t->ws.lo);
    }
}

void launch_atree_near(const AtreeCall &c, hipStream_t s)
{
    const fmm_atree *t = c.t;
    if (t->nunits == 0) return;
    const double scale = c.alpha * kInv2Pi;
    // exponent at which 1 - e rounds to 1: FP32 base 2 at 26, FP64 base e at 37.5, one
    // unit of margin for the rounding of the records
    const double cut = c.is_double ? 39.0 : 27.0;
    if (c.is_double)
        at_near_kernel<double><<<(unsigned)t->nunits, 64, 0, s>>>(
            t->d.units, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            (const double4 *)t->ws.rec, t->x0, t->y0, t->side, c.alpha, cut, scale, t->ws.near);
    else
        at_near_kernel<float><<<(unsigned)t->nunits, 64, 0, s>>>(
            t->d.units, t->d.cell, t->d.range, t->d.u_off, t->d.u_idx, t->d.tile_start, t->d.tile_box,
            (const float4 *)t->ws.rec, t->x0, t->y0, t->side, c.alpha, cut, scale, t->ws.near);
}

void launch_atree_finalize(const AtreeCall &c, double *uv, double *uv_near, double *uv_far, hipStream_t s)
{
    const fmm_atree *t = c.t;
    const int n = (int)t->n;
    at_finalize_kernel<<<blocks(n, 256), 256, 0, s>>>(n, t->d.perm, t->d.leaf_of, t->d.cell, t->d.xy, t->d.w_off,
                                                      t->d.w_idx, t->ws.mp, t->ws.lo, c.p, t->x0, t->y0, t->side,
                                                      t->ws.near, uv, uv_near, uv_far);
}

}  // namespace fmm
