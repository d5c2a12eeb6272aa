// Device helpers shared by the uniform-tree kernels (kernels.hip) and the adaptive-tree
// kernels (adaptive.hip): complex arithmetic on float2 / double2, the near-field
// particle records, and the regularised pair kernel of the near field.
#pragma once

#include <hip/hip_runtime.h>

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
template <typename T> struct Rec;
template <> struct Rec<float> { using type = float4; };
template <> struct Rec<double> { using type = double4; };
template <typename T> using rec_t = typename Rec<T>::type;

// g(s) = 1 - exp(-|dz|^2/(2 sigma^2)) in the scaled variable s, and 1/s.
__device__ __forceinline__ float one_minus_exp(float s) { return 1.0f - __builtin_amdgcn_exp2f(-s); }
__device__ __forceinline__ double one_minus_exp(double s) { return -expm1(-s); }
__device__ __forceinline__ float recip(float s) { return __builtin_amdgcn_rcpf(s); }
__device__ __forceinline__ double recip(double s) { return 1.0 / s; }
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

}  // namespace fmm
