// Device helpers shared by the uniform-tree kernels (kernels.hip) and the adaptive-tree
// kernels (adaptive.hip): complex arithmetic on float2 / double2, the near-field
// particle records, the regularised pair kernel of the near field, and its mutual form
// for pairs of dense same-level leaves.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fmm_internal.h"

namespace fmm {

constexpr double kInv2Pi = 0.15915494309189533576888376337251;

// ---------------------------------------------------------------------------------
// Small complex helpers on float2 / double2
// ---------------------------------------------------------------------------------
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> using c2 = typename Vec2<T>::type;

template <typename T> __device__ __forceinline__ c2<T> mk(T x, T y)
{
    c2<T> r;
    r.x = x;
    r.y = y;
    return r;
}

// acc + a * b
template <typename T> __device__ __forceinline__ c2<T> cmac(c2<T> acc, c2<T> a, c2<T> b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

template <typename T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b)
{
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename TO, typename TI> __device__ __forceinline__ c2<TO> cvt(c2<TI> a)
{
    return mk<TO>((TO)a.x, (TO)a.y);
}

// ---------------------------------------------------------------------------------
// Per-particle records for the near field: {X, Y, Gamma, 0} with (X, Y) = alpha (z - c_leaf),
// alpha chosen per call so that the pair exponent needs no extra multiply:
//   FP64: alpha^2 = 1/(2 sigma^2)          -> g = 1 - exp(-s)
//   FP32: alpha^2 = log2(e)/(2 sigma^2)    -> g = 1 - exp2(-s)
// with s = |X_i - X_j|^2 (leaf offset added per neighbour leaf).  Leaf-local origins
// keep FP32 differences accurate at the blob scale.
// ---------------------------------------------------------------------------------
// Workgroups are dealt to the XCDs round-robin; this remaps block b so that XCD x walks
// the contiguous range [x per, (x + 1) per) of logical blocks (grids are launched as a
// multiple of nxcd), which keeps the memory windows each XCD touches few and in its L2.
__device__ __forceinline__ int xcd_block(int nxcd)
{
    const int per = gridDim.x / nxcd;
    return (blockIdx.x % nxcd) * per + blockIdx.x / nxcd;
}
inline unsigned xcd_grid(int64_t work, int per_block, int nxcd)
{
    const int64_t b = (work + per_block - 1) / per_block;
    return (unsigned)((std::max<int64_t>(b, 1) + nxcd - 1) / nxcd * nxcd);
}

template <typename T> struct Rec;
template <> struct Rec<float> { using type = float4; };
template <> struct Rec<double> { using type = double4; };
template <typename T> using rec_t = typename Rec<T>::type;
template <typename R> struct RecScalar;
template <> struct RecScalar<float4> { using type = float; };
template <> struct RecScalar<double4> { using type = double; };

// Where the near-field kernels read a particle's record {X, Y, Gamma, 0} from: the
// particles' coordinates relative to their leaf's centre, kept with the tree and scaled on
// load (the uniform tree: leaf-unit coordinates xi = (z - c_leaf)/w scaled by alpha w; the
// adaptive tree, whose leaves have several widths: z - c_leaf scaled by alpha), and the
// circulations in tree order, gathered per call (only they change between calls).
template <typename T> struct SoaRec {
    const c2<T> *__restrict__ pos;
    const T *__restrict__ gam;
    T scale;
    __device__ __forceinline__ rec_t<T> operator()(int64_t i) const
    {
        const c2<T> p = pos[i];
        rec_t<T> r;
        r.x = p.x * scale;
        r.y = p.y * scale;
        r.z = gam[i];
        r.w = (T)0;
        return r;
    }
};

// g(s) = 1 - exp(-|dz|^2/(2 sigma^2)) in the scaled variable s, and 1/s.
__device__ __forceinline__ float one_minus_exp(float s) { return 1.0f - __builtin_amdgcn_exp2f(-s); }
// FP64 e = exp(-s) and g = 1 - e for s >= 0, g without cancellation: Cody-Waite reduction
// s = k ln2 + r, |r| <= ln2/2 (ln2 as a high part with 21 trailing zero bits, so that k ln2_hi
// is exact, plus the rest), expm1(x) = x p(x) at x = -r with p of degree 10 (the Taylor series
// of expm1(x)/x economized by Chebyshev polynomials on |x| <= 0.3467, in exact rational
// arithmetic, coefficients rounded to double: within 2.3e-17 of p), then e = 2^-k (1 + em1)
// and g = (1 - 2^-k) - 2^-k em1, where 1 - 2^-k is exact.  Within about 2 ulp of both; 2^-k
// underflows to 0 for large s (e = 0, g = 1).  Branch-free, 20 instructions.
__device__ __forceinline__ void exp_pair(double s, double &e, double &g)
{
    constexpr double kInvLn2 = 1.4426950408889634, kLn2Hi = 6.93147180369123816490e-01,
                     kLn2Lo = 1.90821492927058770002e-10;
    const double k = rint(s * kInvLn2);
    const double x = -fma(-k, kLn2Lo, fma(-k, kLn2Hi, s));  // -(s - k ln2)
    double p = 2.5110080609180445e-08;
    p = fma(p, x, 2.7626408708679167e-07);
    p = fma(p, x, 2.7557240802111588e-06);
    p = fma(p, x, 2.4801504223004426e-05);
    p = fma(p, x, 0.000198412698901562);
    p = fma(p, x, 0.0013888888932586684);
    p = fma(p, x, 0.00833333333331956);
    p = fma(p, x, 0.04166666666657286);
    p = fma(p, x, 0.1666666666666668);
    p = fma(p, x, 0.5000000000000006);
    p = fma(p, x, 1.0);
    const double em1 = p * x;  // expm1(-r)
    const double t = ldexp(1.0, -(int)k);
    e = fma(t, em1, t);
    g = fma(-t, em1, 1.0 - t);
}
__device__ __forceinline__ double one_minus_exp(double s)
{
    double e, g;
    exp_pair(s, e, g);
    return g;
}
__device__ __forceinline__ float recip(float s) { return __builtin_amdgcn_rcpf(s); }
// FP64: the hardware reciprocal estimate (relative error below 2^-24, measured) refined by
// one cubic step r + r (d + d^2), d = 1 - s r, which triples the correct bits: within an ulp
// of 1/s (equal to the IEEE quotient on 4M sampled s in [1e-3, 1e6], measured; not
// guaranteed correctly rounded), 4 instructions against 5 for two Newton steps and about 10
// for the division, on a positive normal s (s >= tiny).
__device__ __forceinline__ double recip(double s)
{
    const double r = __builtin_amdgcn_rcp(s);
    const double d = fma(-s, r, 1.0);
    return fma(r, fma(d, d, d), r);
}
// Added to every s: a pair at distance 0 (the particle itself) then gives g = 0 and a
// finite Gamma/s (for |Gamma| < 1e18 in FP32), hence exactly zero, while any s above
// ~1e-13 (FP32) or ~1e-284 (FP64) is unchanged.
template <typename T> __device__ __forceinline__ T tiny();
template <> __device__ __forceinline__ float tiny<float>() { return 1e-20f; }
template <> __device__ __forceinline__ double tiny<double>() { return 1e-300; }

// f = Gamma (1 - e)/s evaluated as q - e q with q = Gamma/s (one fused multiply-add);
// on a far tile e rounds to 0 against 1 and f = q.
__device__ __forceinline__ float exp_neg_scaled(float s) { return __builtin_amdgcn_exp2f(-s); }
__device__ __forceinline__ double exp_neg_scaled(double s) { return exp(-s); }

template <typename T, bool FAR>
__device__ __forceinline__ void p2p_pair(const rec_t<T> &rj, T tx, T ty, T &fu, T &fv)
{
    const T ddx = tx - rj.x;
    const T ddy = ty - rj.y;
    const T s = fma(ddx, ddx, fma(ddy, ddy, tiny<T>()));
    const T q = recip(s) * rj.z;
    T f;
    if (FAR) f = q;
    else if (sizeof(T) == 4) f = fma(-exp_neg_scaled(s), q, q);
    else f = one_minus_exp(s) * q;
    fu = fma(f, ddy, fu);
    fv = fma(f, ddx, fv);
}

template <typename T, int K, bool FAR>
__device__ __forceinline__ void p2p_tile(const rec_t<T> *tile, int len, int k, T tx, T ty, T &fu, T &fv)
{
    if (len == 64) {
#pragma unroll 8
        for (int it = 0; it < 64 / K; ++it) p2p_pair<T, FAR>(tile[k + it * K], tx, ty, fu, fv);
    } else {
        for (int j = k; j < len; j += K) p2p_pair<T, FAR>(tile[j], tx, ty, fu, fv);
    }
}

template <typename T, int K>
__device__ __forceinline__ void p2p_tile_any(const rec_t<T> *tile, int len, int k, T tx, T ty, T &fu, T &fv, bool far)
{
    if (far) p2p_tile<T, K, true>(tile, len, k, tx, ty, fu, fv);
    else p2p_tile<T, K, false>(tile, len, k, tx, ty, fu, fv);
}

// Smallest squared distance between two boxes {xmin, ymin, xmax, ymax}, the first
// shifted by (ox, oy).
__device__ __forceinline__ float box_gap2(float4 a, float ox, float oy, float4 b)
{
    const float gx = fmaxf(0.0f, fmaxf(b.x - (a.z + ox), (a.x + ox) - b.z));
    const float gy = fmaxf(0.0f, fmaxf(b.y - (a.w + oy), (a.y + oy) - b.w));
    return gx * gx + gy * gy;
}

// ---------------------------------------------------------------------------------
// Stage 9, mutual form for pairs of dense leaves.  The kernel of eq. regB-S2DGau is
// odd, K(-z) = -K(z), so one evaluation of g(s)/s serves both particles of a pair.
// One wavefront per item {S, R}: R is S itself or one of its neighbours (+1,0),
// (-1,+1), (0,+1), (+1,+1), so every unordered pair of neighbouring dense leaves is
// one item.  For each pair of 64-particle tiles (b of S, a of R), one tile is held one
// particle per lane ("resident") and the other is staged in LDS and streamed in chunks
// of 16 sources.  Within a chunk, lane l of a 16-lane row meets source (l + j) mod 16
// at step j; the resident sums stay in the lane and each source's sum travels with its
// source: a one-lane rotation within the row per step, fused into the add (a DPP
// operand).  After 16 steps every row holds its partial sums of the chunk's sources;
// two butterfly steps across rows complete them.  Sums for tile b stay in registers
// over the tiles of R; sums for tile a accumulate in its particles' slot in memory.
// Slots: nine per particle, one per neighbour direction d = 3(dy+1) + (dx+1), written
// by exactly one item (the item of S = R writes its own particles' slot 4 from both
// ends, tile b folding in what the earlier tiles wrote).  The near field is the fixed
// order sum of the slots plus the target-centric part for sparse neighbours, so the
// result does not depend on scheduling.
// ---------------------------------------------------------------------------------

// Lane l receives the value of lane 16 (l / 16) + ((l + 1) mod 16): DPP row_ror:15.
__device__ __forceinline__ float row_rot(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x12F, 0xF, 0xF,
                                                                 false));
}
__device__ __forceinline__ double row_rot(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x12F, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x12F, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// 16 steps of one chunk: src points at this lane's start in the chunk's doubled copy
// (src[j] = source (l + j) mod 16).  rgn = -Gamma of the resident particle (zero for an
// idle lane).  On return (cu, cv)[l] = this row's sum for source l mod 16 of the chunk.
template <typename T, bool FAR>
__device__ __forceinline__ void mutual_chunk(const rec_t<T> *src, T rx, T ry, T rgn, T &fu, T &fv, T &cu, T &cv)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const rec_t<T> sj = src[j];
        const T ddx = rx - sj.x;
        const T ddy = ry - sj.y;
        const T ss = fma(ddx, ddx, fma(ddy, ddy, tiny<T>()));
        const T r = recip(ss);
        T h;  // g(s)/s
        if (FAR) h = r;
        else if (sizeof(T) == 4) h = fma(-exp_neg_scaled(ss), r, r);
        else h = one_minus_exp(ss) * r;
        const T wt = h * sj.z;
        fu = fma(wt, ddy, fu);
        fv = fma(wt, ddx, fv);
        const T ws = h * rgn;
        if (j == 0) {
            cu = ws * ddy;
            cv = ws * ddx;
        } else {
            // Not contracted: a multiply and an add that takes the rotation as its DPP
            // operand are two instructions; an FMA needs the rotation as a separate move.
#pragma clang fp contract(off)
            cu = row_rot(cu) + ws * ddy;
            cv = row_rot(cv) + ws * ddx;
        }
    }
    cu = row_rot(cu);
    cv = row_rot(cv);
}

// Records of one tile into LDS, each chunk of 16 stored twice in a row (so that the
// sources of step j are at a constant offset), zero records past the tile's end.
template <typename T, typename Src>
__device__ __forceinline__ rec_t<T> stage_doubled(rec_t<T> *dst, const Src &rec, int first, int len)
{
    const int lane = threadIdx.x;
    rec_t<T> r;
    r.x = r.y = r.z = r.w = (T)0;
    if (lane < len) r = rec(first + lane);
    dst[(lane >> 4) * 32 + (lane & 15)] = r;
    dst[(lane >> 4) * 32 + (lane & 15) + 16] = r;
    return r;
}

// One tile b of S against every tile a of R (a >= b when S = R).  Per block (b, a) the
// tile with more chunks of 16 sits in the lanes and the other is streamed from LDS, so
// that fewer steps are spent; either way both sums come out lane-indexed by particle.
template <typename T, typename Src>
__device__ __forceinline__ void mutual_resident_tile(const int4 it, rec_t<T> *tile_a, rec_t<T> *tile_b, int b,
                                                     int tb, const Src &rec,
                                                     const int *__restrict__ leaf_start,
                                                     const int *__restrict__ tile_start,
                                                     const float4 *__restrict__ tile_box, T step, float cut_leaf2,
                                                     c2<T> *__restrict__ slot_s, c2<T> *__restrict__ slot_r)
{
    const int lane = threadIdx.x;
    const uint32_t S = (uint32_t)it.x, R = (uint32_t)it.y;
    const bool self = S == R;
    const int ds = it.z & 15;
    const int dx = ds % 3 - 1, dy = ds / 3 - 1;  // R - S in leaves
    const T ox = (T)dx * step, oy = (T)dy * step;
    const int s0 = leaf_start[S], s1 = leaf_start[S + 1];
    const int r1 = leaf_start[R + 1];
    const int lenb = min(64, s1 - b);
    const int nchb = (lenb + 15) >> 4;
    __syncthreads();
    const rec_t<T> rb = stage_doubled<T, Src>(tile_b, rec, b, lenb);
    // tile b in the frame of leaf R (resident form); in the streamed form it stays in
    // the frame of S and tile a is moved there
    const T bx = rb.x - ox, by = rb.y - oy;
    const T bgn = lane < lenb ? -rb.z : (T)0;
    const float4 bbox = tile_box[tb];
    T fu = 0, fv = 0;
    if (self && b > s0 && lane < lenb) {  // what the earlier tiles of S wrote for this tile
        const c2<T> o = slot_s[b + lane];
        fu = o.x;
        fv = o.y;
    }
    const bool first_touch = b == s0;  // the first resident tile creates the streamed slots
    int ta = self ? tb : tile_start[R];
    for (int a = self ? b : leaf_start[R]; a < r1; a += 64, ++ta) {
        const int lena = min(64, r1 - a);
        const int ncha = (lena + 15) >> 4;
        const bool diag = self && a == b;
        const bool far = box_gap2(bbox, (float)-dx, (float)-dy, tile_box[ta]) >= cut_leaf2;
        if (diag) {
            // the tile with itself: every ordered pair from the resident end
            __syncthreads();
            for (int c = 0; c < nchb; ++c)
                if (far) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) p2p_pair<T, true>(tile_b[c * 32 + j], bx, by, fu, fv);
                } else {
#pragma unroll
                    for (int j = 0; j < 16; ++j) p2p_pair<T, false>(tile_b[c * 32 + j], bx, by, fu, fv);
                }
            continue;
        }
        c2<T> old;
        old.x = old.y = (T)0;
        if (!first_touch && lane < lena) old = slot_r[a + lane];
        const bool swap = ncha > nchb;  // tile a in the lanes, tile b streamed
        __syncthreads();
        const rec_t<T> ra = stage_doubled<T, Src>(tile_a, rec, a, lena);
        __syncthreads();
        T px, py, pgn;
        const rec_t<T> *src;
        int nch;
        if (swap) {
            px = ra.x + ox;
            py = ra.y + oy;
            pgn = lane < lena ? -ra.z : (T)0;
            src = tile_b;
            nch = nchb;
        } else {
            px = bx;
            py = by;
            pgn = bgn;
            src = tile_a;
            nch = ncha;
        }
        T ru = 0, rv = 0, colu = 0, colv = 0;
        for (int c = 0; c < nch; ++c) {
            T cu, cv;
            const rec_t<T> *sp = src + c * 32 + (lane & 15);
            if (far) mutual_chunk<T, true>(sp, px, py, pgn, ru, rv, cu, cv);
            else mutual_chunk<T, false>(sp, px, py, pgn, ru, rv, cu, cv);
            cu += __shfl_xor(cu, 16);
            cv += __shfl_xor(cv, 16);
            cu += __shfl_xor(cu, 32);
            cv += __shfl_xor(cv, 32);
            if ((lane >> 4) == c) {
                colu = cu;
                colv = cv;
            }
        }
        // sums of tile b and of tile a, lane-indexed
        const T bu = swap ? colu : ru, bv = swap ? colv : rv;
        const T au = swap ? ru : colu, av = swap ? rv : colv;
        fu += bu;
        fv += bv;
        if (lane < lena) {
            c2<T> nw;
            nw.x = old.x + au;
            nw.y = old.y + av;
            slot_r[a + lane] = nw;
        }
    }
    if (lane < lenb) {
        c2<T> nw;
        nw.x = fu;
        nw.y = fv;
        slot_s[b + lane] = nw;
    }
}

template <typename T, typename Src>
__device__ __forceinline__ void mutual_item_src(const int4 it, rec_t<T> *tile_a, rec_t<T> *tile_b, const Src &rec,
                                                const int *__restrict__ leaf_start,
                                                const int *__restrict__ tile_start,
                                                const float4 *__restrict__ tile_box, T step, float cut_leaf2,
                                                int64_t n, c2<T> *__restrict__ slots)
{
    const uint32_t S = (uint32_t)it.x;
    c2<T> *slot_s = slots + (int64_t)(it.z & 15) * n;
    c2<T> *slot_r = slots + (int64_t)(it.z >> 4) * n;
    const int s0 = leaf_start[S], s1 = leaf_start[S + 1];
    for (int b = s0, tb = tile_start[S]; b < s1; b += 64, ++tb)
        mutual_resident_tile<T, Src>(it, tile_a, tile_b, b, tb, rec, leaf_start, tile_start, tile_box, step,
                                     cut_leaf2, slot_s, slot_r);
}


// ---------------------------------------------------------------------------------
// Adjoint near field (shared by the uniform and the adaptive tree)
// ---------------------------------------------------------------------------------
// e = exp(-x) and g = 1 - e in the scaled variable: FP32 base 2 (g by subtraction,
// small x handled by the series below); FP64 base e by the exp_pair above.
__device__ __forceinline__ void exp_pair(float s, float &e, float &g)
{
    e = __builtin_amdgcn_exp2f(-s);
    g = 1.0f - e;
}

// Below this natural exponent the 5-term series of g/s' and (lambda e s' - g)/s'^2 is
// used: its truncation error x^5/720 is under the rounding unit of T there.
template <typename T> __device__ __forceinline__ T series_cut();
template <> __device__ __forceinline__ float series_cut<float>() { return 0.125f; }
template <> __device__ __forceinline__ double series_cut<double>() { return 1e-3; }

// acc: Phi (2); A as its real part and its imaginary part divided by -2 (the factor is
// applied in finalize); B; with SRC also the source-position sums with the adjoint
// charges, At = sum q_j conj(dz')^2 (lambda e s' - g)/s'^2 (2) and Bt = sum q_j e (2).
// conj(dz')^2 = (dx'^2 - dy'^2) - 2i dx' dy' reuses dy'^2 from s'.  SERIES false: the
// pair is known to lie beyond the series cut (its tile's bounding boxes say so), and the
// test is left out.
template <typename T, bool FAR, bool SRC, bool SERIES = true>
__device__ __forceinline__ void p2p_bwd_pair(const rec_t<T> &rj, const c2<T> qj, T tx, T ty, T lambda,
                                             T (&acc)[SRC ? 9 : 5])
{
    T &fpr = acc[0], &fpi = acc[1], &far_r = acc[2], &far_ih = acc[3], &fb = acc[4];
    const T ddx = tx - rj.x;
    const T ddy = ty - rj.y;
    const T dy2 = fma(ddy, ddy, tiny<T>());
    const T s = fma(ddx, ddx, dy2);
    const T r = recip(s);
    if constexpr (FAR) {
        // e rounds to 0 against 1 (g = 1): the terms of the point vortex, Phi: q_j w and
        // A: -Gamma_j w^2 with w = 1/dz' = conj(dz')/s' = cx + i cy.  The A sums take
        // Re(-w^2) = d = cy^2 - cx^2 and Im(-w^2)/-2 = cx cy; the source-position sum takes
        // q_j (d - 2i cx cy).  (Three operations fewer than the general form below.)
        const T cx = r * ddx, cy = -r * ddy;
        fpr = fma(qj.x, cx, fpr);
        fpr = fma(-qj.y, cy, fpr);
        fpi = fma(qj.x, cy, fpi);
        fpi = fma(qj.y, cx, fpi);
        const T d = fma(cy, cy, -cx * cx);
        const T m = cx * cy;
        far_r = fma(rj.z, d, far_r);
        far_ih = fma(rj.z, m, far_ih);
        if constexpr (SRC) {
            const T wi = (T)-2 * m;
            acc[5] = fma(qj.x, d, acc[5]);
            acc[5] = fma(-qj.y, wi, acc[5]);
            acc[6] = fma(qj.x, wi, acc[6]);
            acc[6] = fma(qj.y, d, acc[6]);
        }
        return;
    }
    T e, g;
    exp_pair(s, e, g);
    // g/s': in FP32 as r - e r (one fused multiply-add, as the forward's kernel); in FP64
    // from the accurate g of exp_pair
    T gr;
    if constexpr (sizeof(T) == 4) gr = fma(-e, r, r);
    else gr = g * r;
    T h = (lambda * e - gr) * r;  // lambda e/s' - g/s'^2
    // x = lambda s' is the natural exponent |dz|^2/(2 sigma^2).  For small x, 1 - e
    // cancels; there g/s' and (lambda e s' - g)/s'^2 come from their series
    //   g/s' = lambda (1 - x/2 + x^2/6 - x^3/24 + x^4/120),
    //   (lambda e s' - g)/s'^2 = lambda^2 (-1/2 + x/3 - x^2/8 + x^3/30 - x^4/144).
    // (The test is on s' against the cut divided by lambda, a loop invariant.)
    if (SERIES && s < series_cut<T>() / lambda) {
        const T x = lambda * s;
        gr = lambda * fma(x, fma(x, fma(x, fma(x, (T)(1.0 / 120), (T)(-1.0 / 24)), (T)(1.0 / 6)), (T)-0.5), (T)1);
        h = lambda * lambda *
            fma(x, fma(x, fma(x, fma(x, (T)(-1.0 / 144), (T)(1.0 / 30)), (T)(-1.0 / 8)), (T)(1.0 / 3)), (T)-0.5);
    }
    fb = fma(rj.z, e, fb);  // B: Gamma_j e
    if constexpr (SRC) {
        acc[7] = fma(qj.x, e, acc[7]);
        acc[8] = fma(qj.y, e, acc[8]);
    }
    // Phi: q_j (g/s') conj(dz')
    const T cx = gr * ddx, cy = -gr * ddy;
    fpr = fma(qj.x, cx, fpr);
    fpr = fma(-qj.y, cy, fpr);
    fpi = fma(qj.x, cy, fpi);
    fpi = fma(qj.y, cx, fpi);
    // A: Gamma_j conj(dz')^2 (lambda e s' - g)/s'^2
    const T hg = h * rj.z;
    const T zr = fma((T)-2, dy2, s);  // dx'^2 - dy'^2
    const T zh = ddx * ddy;           // Im conj(dz')^2 / -2
    far_r = fma(hg, zr, far_r);
    far_ih = fma(hg, zh, far_ih);
    if constexpr (SRC) {
        const T wr = h * zr, wi = ((T)-2 * h) * zh;
        acc[5] = fma(qj.x, wr, acc[5]);
        acc[5] = fma(-qj.y, wi, acc[5]);
        acc[6] = fma(qj.x, wi, acc[6]);
        acc[6] = fma(qj.y, wr, acc[6]);
    }
}

template <typename T, int K, bool FAR, bool SRC, bool SERIES = true>
__device__ __forceinline__ void p2p_bwd_tile(const rec_t<T> *tile, const c2<T> *qtile, int len, int k, T tx, T ty,
                                             T lambda, T (&acc)[SRC ? 9 : 5])
{
    if (len == 64) {
#pragma unroll 4
        for (int it = 0; it < 64 / K; ++it)
            p2p_bwd_pair<T, FAR, SRC, SERIES>(tile[k + it * K], qtile[k + it * K], tx, ty, lambda, acc);
    } else {
        for (int j = k; j < len; j += K) p2p_bwd_pair<T, FAR, SRC, SERIES>(tile[j], qtile[j], tx, ty, lambda, acc);
    }
}

// cls 2: every pair of the tile is beyond the exponential's cut (point-vortex terms);
// 1: beyond the series cut (no per-pair test; units of one or two lanes per target,
// which carry nearly all pairs, so the other unrolled variants stay few); 0: the full form.
template <typename T, int K, bool SRC>
__device__ __forceinline__ void p2p_bwd_tile_any(const rec_t<T> *tile, const c2<T> *qtile, int len, int k, T tx, T ty,
                                                 T lambda, T (&acc)[SRC ? 9 : 5], int cls)
{
    if (cls == 2) p2p_bwd_tile<T, K, true, SRC>(tile, qtile, len, k, tx, ty, lambda, acc);
    else if (K <= 2 && cls == 1) p2p_bwd_tile<T, K, false, SRC, false>(tile, qtile, len, k, tx, ty, lambda, acc);
    else p2p_bwd_tile<T, K, false, SRC>(tile, qtile, len, k, tx, ty, lambda, acc);
}

// ---------------------------------------------------------------------------------
// Per-particle gathers of the finalize kernels, written so that a wavefront waits for
// memory a few times rather than once per load.  A load guarded by a lane-dependent
// branch is followed by a wait inside the branch, so nine guarded slot loads cost nine
// memory round trips; a loop over coefficients with a run-time bound waits once per
// coefficient.
// ---------------------------------------------------------------------------------

// Near-field velocity of sorted particle i of n from the mutual form: the target-centric
// part near[i] when bit 9 of the leaf mask m is set, minus/plus scale times the slots
// d = 0..8 whose bits are set, summed in that order.  The slot loads go out together,
// unguarded: a slot the leaf's items did not write is read at the address of the lowest
// one they did (a line this particle reads anyway) and its value discarded by a select,
// so the wavefront waits once.  (Guarding each load by its bit made the compiler wait
// after each.)  su and sv start at +0 and never become -0, so adding +0 for an unset slot
// gives the bits of skipping it.
template <typename TS>
__device__ __forceinline__ double2 near_from_slots(int64_t i, int64_t n, int m, const double2 *__restrict__ near,
                                                   const c2<TS> *__restrict__ slots, double scale)
{
    double2 r = make_double2(0.0, 0.0);
    if ((m >> 9) & 1) r = near[i];
    const int set = m & 0x1FF;
    if (set) {
        const int64_t lowest = (int64_t)__builtin_ctz(set) * n + i;
        c2<TS> v[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) v[d] = slots[(set >> d) & 1 ? (int64_t)d * n + i : lowest];
        double su = 0.0, sv = 0.0;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            const bool on = (set >> d) & 1;
            su += on ? (double)v[d].x : 0.0;
            sv += on ? (double)v[d].y : 0.0;
        }
        r.x -= scale * su;
        r.y += scale * sv;
    }
    return r;
}

// Horner's rule b_{p-1} x^{p-1} + ... + b_0 (p >= 1), in the order l = p-2 .. 0, with the
// coefficients loaded eight at a time ahead of their use (an index below 0 re-reads b_0
// and is not used).
template <typename T>
__device__ __forceinline__ c2<T> horner_prefetch(const c2<T> *__restrict__ b, int p, c2<T> x)
{
    c2<T> acc = b[p - 1];
    for (int l0 = p - 2; l0 >= 0; l0 -= 8) {
        c2<T> c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = b[l0 - k >= 0 ? l0 - k : 0];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (l0 - k >= 0) acc = cmac<T>(c[k], acc, x);
    }
    return acc;
}

// Horner's rule with weighted coefficients, sum_{l=lo}^{p-1} (l + add) b_l x^(l-lo)
// (p > lo), in the order l = p-2 .. lo, the coefficients loaded eight at a time ahead of
// their use: the derivative of the series above with lo = 1, add = 0.
template <typename T>
__device__ __forceinline__ c2<T> horner_weighted_prefetch(const c2<T> *__restrict__ b, int p, c2<T> x, int lo,
                                                          int add)
{
    const c2<T> top = b[p - 1];
    const T wt = (T)(p - 1 + add);
    c2<T> acc = mk<T>(wt * top.x, wt * top.y);
    for (int l0 = p - 2; l0 >= lo; l0 -= 8) {
        c2<T> c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = b[l0 - k >= lo ? l0 - k : lo];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (l0 - k >= lo) {
                const T l = (T)(l0 - k + add);
                acc = cmac<T>(mk<T>(l * c[k].x, l * c[k].y), acc, x);
            }
    }
    return acc;
}

// A velocity row of user row o: the velocity itself, or with a base (the transport
// update of section "Test problem", dx/dt = u, one explicit stage) base + h u.
__device__ __forceinline__ void store_velocity(double *__restrict__ uv, int64_t o, double2 v,
                                               const double *__restrict__ base, double h)
{
    if (base) {
        v.x = fma(h, v.x, base[2 * o]);
        v.y = fma(h, v.y, base[2 * o + 1]);
    }
    uv[2 * o] = v.x;
    uv[2 * o + 1] = v.y;
}

// Second half of a staged finalize: (u, v) of sorted particle i, written in sorted order
// by the finalize kernel, to row perm[i] of the user-order output.  Reading the slot sums
// and writing rows in random order in one kernel took longer (840 us for 2^24 particles)
// than doing each in a kernel of its own (413 + 343 us).
namespace {
__global__ __launch_bounds__(256) void scatter_rows_kernel(int n, const int *__restrict__ perm,
                                                           const double2 *__restrict__ staged,
                                                           double *__restrict__ uv, const double *__restrict__ base,
                                                           double h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    store_velocity(uv, perm[i], staged[i], base, h);
}
}  // namespace

__device__ __forceinline__ void store_adjoint(const AdjointOut &a, int64_t o, double g, double ex, double ey, double sx,
                                              double sy)
{
    if (a.dg) a.dg[o] = a.acc_g ? a.dg[o] + g : g;
    if (a.dxe) {
        a.dxe[2 * o] = ex;
        a.dxe[2 * o + 1] = ey;
    }
    if (a.dxs) {
        a.dxs[2 * o] = sx;
        a.dxs[2 * o + 1] = sy;
    }
    if (a.dxy) {
        double vx = ex + sx, vy = ey + sy;
        if (a.lam) {
            vx += a.lam[2 * o];
            vy += a.lam[2 * o + 1];
        }
        if (a.acc_xy) {
            vx += a.dxy[2 * o];
            vy += a.dxy[2 * o + 1];
        }
        a.dxy[2 * o] = vx;
        a.dxy[2 * o + 1] = vy;
    }
}

}  // namespace fmm
