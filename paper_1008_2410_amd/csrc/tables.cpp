// Radius-scaled translation operators for p-term expansions (host generation, FP64,
// uploaded once per p as FP64 and FP32 copies).
//
// With multipoles scaled as a_m / w^m and locals as b_l w^(l+1) (w = cell width of
// the level), the textbook translations become level independent:
//   M2M (stage 5): A_m = sum_{k<=m} C(m,k) d^(m-k) 2^-k a_k,           d = (c_child - c_parent)/w_parent
//   M2L (stage 6): b_l = sum_m (-1)^l C(l+m,m) delta^-(l+m+1) a_m,     delta = (c_T - c_S)/w
//   L2L (stage 7): b_k = sum_{l>=k} C(l,k) d^(l-k) 2^-(k+1) b_l
// derived from the multipole coefficients of section "Complexity Estimates" and the
// expansion 1/(D + u - v) = sum_{l,m} (-1)^l C(l+m,l) u^l v^m / D^(l+m+1).
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

namespace {

using cd = std::complex<double>;

std::vector<double> binomials(int nmax)
{
    std::vector<double> c((size_t)(nmax + 1) * (nmax + 1), 0.0);
    for (int n = 0; n <= nmax; ++n) {
        c[(size_t)n * (nmax + 1)] = 1.0;
        for (int k = 1; k <= n; ++k)
            c[(size_t)n * (nmax + 1) + k] = c[(size_t)(n - 1) * (nmax + 1) + k - 1] + c[(size_t)(n - 1) * (nmax + 1) + k];
    }
    return c;
}

cd child_offset(int q) { return cd(((q & 1) - 0.5) * 0.5, ((q >> 1) - 0.5) * 0.5); }

template <typename V, typename S>
int upload(V **dst, const std::vector<cd> &src, std::string &err)
{
    std::vector<V> h(src.size());
    for (size_t i = 0; i < src.size(); ++i) {
        h[i].x = (S)src[i].real();
        h[i].y = (S)src[i].imag();
    }
    if (hipMalloc((void **)dst, h.size() * sizeof(V)) != hipSuccess) {
        err = "hipMalloc failed for operator tables";
        return -2;
    }
    if (hipMemcpy(*dst, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMemcpy failed for operator tables";
        return -3;
    }
    return 0;
}

}  // namespace

void free_tables(Tables &tb)
{
    hipFree(tb.m2m_d);
    hipFree(tb.l2l_d);
    hipFree(tb.m2l_d);
    hipFree(tb.m2m_f);
    hipFree(tb.l2l_f);
    hipFree(tb.m2l_f);
    hipFree(tb.mfma_f);
    hipFree(tb.mfma_d);
    hipFree(tb.mfma_entries);
    hipFree(tb.zero_row);
    tb = Tables{};
}

int upload_tables(Tables &tb, int p, std::string &err)
{
    if (tb.p == p) return 0;
    free_tables(tb);
    const int nb = 2 * p;
    const std::vector<double> C = binomials(nb);
    auto binom = [&](int n, int k) { return C[(size_t)n * (nb + 1) + k]; };

    std::vector<cd> m2m((size_t)4 * p * p, 0.0), l2l((size_t)4 * p * p, 0.0), m2l((size_t)49 * p * p, 0.0);
    for (int q = 0; q < 4; ++q) {
        const cd d = child_offset(q);
        for (int m = 0; m < p; ++m)
            for (int k = 0; k <= m; ++k)
                m2m[((size_t)q * p + m) * p + k] = binom(m, k) * std::pow(d, m - k) * std::ldexp(1.0, -k);
        for (int k = 0; k < p; ++k)
            for (int l = k; l < p; ++l)
                l2l[((size_t)q * p + k) * p + l] = binom(l, k) * std::pow(d, l - k) * std::ldexp(1.0, -(k + 1));
    }
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy) {
            if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
            const int o = (dx + 3) * 7 + (dy + 3);
            const cd inv = 1.0 / cd(dx, dy);
            // powers inv^n, n = 1 .. 2p-1, by repeated multiplication
            std::vector<cd> pw(2 * p + 1);
            pw[0] = 1.0;
            for (int n = 1; n <= 2 * p; ++n) pw[n] = pw[n - 1] * inv;
            for (int m = 0; m < p; ++m)
                for (int l = 0; l < p; ++l)
                    m2l[((size_t)o * p + m) * p + l] = ((l & 1) ? -1.0 : 1.0) * binom(l + m, m) * pw[l + m + 1];
        }
    // Real 2p x 2p embedding for the MFMA kernel: y = x R with x, y interleaved (re, im),
    // R[2m][2l] = Re T_lm, R[2m+1][2l] = -Im T_lm, R[2m][2l+1] = Im T_lm, R[2m+1][2l+1] = Re T_lm.
    std::vector<float> mf;
    std::vector<double> md;
    if (p <= 16) {
        mf.assign((size_t)57 * 2 * 32 * 16, 0.0f);
        md.assign((size_t)57 * 4 * 32 * 8, 0.0);
        auto put = [&](int slot, int m, int l, cd v) {
            const int k_re = 2 * m, k_im = 2 * m + 1, n_re = 2 * l, n_im = 2 * l + 1;
            auto at = [&](int k, int n) -> float & { return mf[(((size_t)slot * 2 + k / 16) * 32 + n) * 16 + k % 16]; };
            auto atd = [&](int k, int n) -> double & { return md[(((size_t)slot * 4 + k / 8) * 32 + n) * 8 + k % 8]; };
            at(k_re, n_re) = (float)v.real();
            at(k_im, n_re) = (float)-v.imag();
            at(k_re, n_im) = (float)v.imag();
            at(k_im, n_im) = (float)v.real();
            atd(k_re, n_re) = v.real();
            atd(k_im, n_re) = -v.imag();
            atd(k_re, n_im) = v.imag();
            atd(k_im, n_im) = v.real();
        };
        for (int o = 0; o < 49; ++o)
            for (int m = 0; m < p; ++m)
                for (int l = 0; l < p; ++l) put(o, m, l, m2l[((size_t)o * p + m) * p + l]);
        // L2L: output coefficient k from parent coefficient l (input)
        for (int q = 0; q < 4; ++q)
            for (int k = 0; k < p; ++k)
                for (int l = 0; l < p; ++l) put(49 + q, l, k, l2l[((size_t)q * p + k) * p + l]);
        // M2M: parent coefficient m (output) from child q's coefficient k (input)
        for (int q = 0; q < 4; ++q)
            for (int m = 0; m < p; ++m)
                for (int k = 0; k < p; ++k) put(53 + q, k, m, m2m[((size_t)q * p + m) * p + k]);
    }
    // Entry lists of the MFMA kernel: per parity class (qx, qy) the 27 interaction-list
    // source offsets (dx in [-2-qx, 3-qx], dy in [-2-qy, 3-qy] outside the 3x3 block) and
    // the L2L entry; then the four M2M children.  delta = (c_T - c_S)/w = (-dx, -dy).
    std::vector<int4> ent;
    for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        for (int dy = -2 - qy; dy <= 3 - qy; ++dy)
            for (int dx = -2 - qx; dx <= 3 - qx; ++dx) {
                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
                ent.push_back(make_int4(dx, dy, (3 - dx) * 7 + (3 - dy), 0));
            }
        ent.push_back(make_int4(0, 0, 49 + q, 1));
    }
    for (int q = 0; q < 4; ++q) ent.push_back(make_int4(q, 0, 53 + q, 2));
    int rc = 0;
    if (!rc && p <= 16) {
        if (hipMalloc((void **)&tb.mfma_f, mf.size() * sizeof(float)) != hipSuccess ||
            hipMalloc((void **)&tb.mfma_d, md.size() * sizeof(double)) != hipSuccess) {
            err = "hipMalloc failed for operator tables";
            rc = -2;
        } else if (hipMemcpy(tb.mfma_f, mf.data(), mf.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
                   hipMemcpy(tb.mfma_d, md.data(), md.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            err = "hipMemcpy failed for operator tables";
            rc = -3;
        }
    }
    if (!rc) {
        if (hipMalloc((void **)&tb.mfma_entries, ent.size() * sizeof(int4)) != hipSuccess) {
            err = "hipMalloc failed for operator tables";
            rc = -2;
        } else if (hipMemcpy(tb.mfma_entries, ent.data(), ent.size() * sizeof(int4), hipMemcpyHostToDevice) !=
                   hipSuccess) {
            err = "hipMemcpy failed for operator tables";
            rc = -3;
        }
    }
    if (!rc) {
        if (hipMalloc((void **)&tb.zero_row, 128 * sizeof(double)) != hipSuccess ||
            hipMemset(tb.zero_row, 0, 128 * sizeof(double)) != hipSuccess) {
            err = "allocation of the zero row failed";
            rc = -2;
        }
    }
    if (!rc) rc = upload<double2, double>(&tb.m2m_d, m2m, err);
    if (!rc) rc = upload<double2, double>(&tb.l2l_d, l2l, err);
    if (!rc) rc = upload<double2, double>(&tb.m2l_d, m2l, err);
    if (!rc) rc = upload<float2, float>(&tb.m2m_f, m2m, err);
    if (!rc) rc = upload<float2, float>(&tb.l2l_f, l2l, err);
    if (!rc) rc = upload<float2, float>(&tb.m2l_f, m2l, err);
    if (rc) {
        free_tables(tb);
        return rc;
    }
    tb.p = p;
    return 0;
}

int shared_tables(int device, int p, const Tables **out, std::string &err, bool create)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, Tables> cache;  // node addresses stay valid
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({device, p});
    if (it == cache.end()) {
        if (!create) {
            err = "the expansion tables of p = " + std::to_string(p) + " are not on this device yet";
            return -5;
        }
        Tables tb;
        if (int rc = upload_tables(tb, p, err)) return rc;
        it = cache.emplace(std::make_pair(device, p), tb).first;
    }
    *out = &it->second;
    return 0;
}

}  // namespace fmm
