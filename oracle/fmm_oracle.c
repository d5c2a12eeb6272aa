/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, double-precision CPU implementation of the velocity evaluation of
 * the 2D vortex-particle FMM in M. G. Knepley, "Removing the Barrier to Scalability
 * in Parallel FMM" (arXiv:1008.2410).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no source, header, table or
 * helper with the GPU library; the two are only ever fed the same seeded inputs.
 *
 * Physics (section "Test problem"):
 *   regularised kernel  K_s(z) = (1/(2 pi |z|^2)) (-z_y, z_x) (1 - exp(-|z|^2/(2 s^2)))
 *                       (eq. regB-S2DGau)
 *   velocity            u(z) = sum_j Gamma_j K_s(z - z_j)              (eq. discBiotS2D)
 *   far field           expansions of the singular 1/|z|^2 kernel; the exact kernel
 *                       only on the near field (text after eq. discBiotS2D).
 *
 * Complex form used by the FMM routines.  With the complex charge c_j = -i Gamma_j/(2 pi)
 * (the factor of the multipole coefficients in section "Complexity Estimates") and
 * g(s) = 1 - exp(-s/(2 sigma^2)), the conjugate velocity W = u - i v is
 *     W(z) = sum_j c_j g(|z - z_j|^2) / (z - z_j),
 * which is eq. regB-S2DGau summed per eq. discBiotS2D.  The FMM routines take any
 * complex charges, so the same code evaluates the adjoint field.
 *
 * Entry points (all FP64, row-major (n,2) position arrays, OpenMP over independent
 * outputs only):
 *   orc_root_box      bounding square of a point set
 *   orc_bin           leaf coordinates of points (stages 1-2 of Fig. fmmStages)
 *   orc_direct        O1: exact O(N^2) sum, real form of eq. regB-S2DGau
 *   orc_split_direct  O2: exact kernel on the 3x3 leaf neighbourhood, singular kernel
 *                     elsewhere (the p -> infinity limit of the FMM)
 *   orc_fmm           O3: FMM stages 1-10 with unscaled textbook operators
 *   orc_fmm_jacobian  O4 helper: d(u,v)/d(x,y) of the O3 field at evaluation points
 *                     (sources held fixed)
 *   orc_fmm_src_grad  O5 helper: gradient of a loss through the O3 velocities with
 *                     respect to the source positions (evaluation points held fixed)
 *   orc_direct_grad   O1 gradient: dL/dGamma and dL/dx of a loss through the O1
 *                     velocities, every particle moving as source and target
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - p is the number of terms, m = 0..p-1, for multipole and local expansions.
 *   - Near field = own leaf and the adjacent leaves (max(|di|,|dj|) <= 1), free space
 *     (corner leaves have 4 neighbours, edge leaves 6).
 *   - Interaction list of a cell at level l >= 2 = children of its parent's neighbours
 *     that are not its own neighbours; levels 0 and 1 carry no expansions.
 *   - Binning: i = min(floor((x - x0)/w_L), 2^L - 1); a point on an internal edge goes
 *     to the higher cell; a point outside [x0, x0+S] is an error.
 *   - The pair j = i (s = 0) contributes nothing (the kernel's limit at 0 is 0).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ERANGE (-4)

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------------ */
/* Root cell and binning (stages 1-2)                                              */
/* ------------------------------------------------------------------------------ */

/* Bounding square: x0 = min x, y0 = min y, side = max(range x, range y) * (1 + 2^-20).
 * The factor keeps the largest coordinate strictly inside the top cell. */
void orc_root_box(int64_t n, const double *xy, double *root)
{
    double xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
    for (int64_t i = 1; i < n; ++i) {
        double x = xy[2 * i], y = xy[2 * i + 1];
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    double side = xmax - xmin;
    if (ymax - ymin > side) side = ymax - ymin;
    if (side <= 0.0) side = 1.0;
    root[0] = xmin;
    root[1] = ymin;
    root[2] = side * (1.0 + 1.0 / 1048576.0);
}

/* Leaf coordinate of one scalar coordinate: floor((x - x0)/w) clamped at the top edge. */
static int bin1(double x, double x0, double w, int nside, int32_t *out)
{
    if (!isfinite(x)) return ORC_EINVAL;
    double t = (x - x0) / w;
    if (!(t >= 0.0) || t > (double)nside) return ORC_ERANGE;
    int64_t k = (int64_t)floor(t);
    if (k > nside - 1) k = nside - 1;
    *out = (int32_t)k;
    return ORC_OK;
}

int orc_bin(int64_t n, const double *xy, int depth, const double *root, int32_t *ix, int32_t *iy)
{
    if (depth < 0 || depth > 15) return ORC_EINVAL;
    int nside = 1 << depth;
    double w = root[2] / (double)nside;
    for (int64_t i = 0; i < n; ++i) {
        int rc = bin1(xy[2 * i], root[0], w, nside, &ix[i]);
        if (rc) return rc;
        rc = bin1(xy[2 * i + 1], root[1], w, nside, &iy[i]);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Kernels                                                                         */
/* ------------------------------------------------------------------------------ */

/* f(s) = (1 - exp(-s/(2 sigma^2)))/s for s > 0, written with expm1 for accuracy at
 * small s.  The velocity from one particle is Gamma/(2 pi) * (-dy, dx) * f(s). */
static double reg_f(double s, double sigma)
{
    return -expm1(-s / (2.0 * sigma * sigma)) / s;
}

/* O1.  u_i = sum_{j, s_ij > 0} Gamma_j K_sigma(x_i - x_j), K_sigma of eq. regB-S2DGau. */
void orc_direct(int64_t nt, const double *txy, int64_t ns, const double *sxy, const double *gamma,
                double sigma, double *uv)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double u = 0.0, v = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double dx = txy[2 * i] - sxy[2 * j];
            double dy = txy[2 * i + 1] - sxy[2 * j + 1];
            double s = dx * dx + dy * dy;
            if (s == 0.0) continue;
            double k = gamma[j] * reg_f(s, sigma) / TWO_PI;
            u += -dy * k;
            v += dx * k;
        }
        uv[2 * i] = u;
        uv[2 * i + 1] = v;
    }
}

/* O2.  Same sum, but a source whose leaf is not adjacent to the target's leaf
 * contributes through the singular kernel (1/(2 pi s)) (-dy, dx). */
void orc_split_direct(int64_t nt, const double *txy, const int32_t *tix, const int32_t *tiy,
                      int64_t ns, const double *sxy, const int32_t *six, const int32_t *siy,
                      const double *gamma, double sigma, double *uv)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double u = 0.0, v = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double dx = txy[2 * i] - sxy[2 * j];
            double dy = txy[2 * i + 1] - sxy[2 * j + 1];
            double s = dx * dx + dy * dy;
            if (s == 0.0) continue;
            int near = abs(tix[i] - six[j]) <= 1 && abs(tiy[i] - siy[j]) <= 1;
            double f = near ? reg_f(s, sigma) : 1.0 / s;
            double k = gamma[j] * f / TWO_PI;
            u += -dy * k;
            v += dx * k;
        }
        uv[2 * i] = u;
        uv[2 * i + 1] = v;
    }
}

/* ------------------------------------------------------------------------------ */
/* O3: the FMM (Fig. fmmStages)                                                    */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int depth, p;
    double x0, y0, side;
    /* leaves, row-major cell index c = iy * 2^L + ix */
    int64_t *leaf_start;   /* CSR over leaves, 4^L + 1 entries */
    int64_t *leaf_src;     /* source indices grouped by leaf */
    int64_t **count;       /* count[l][c]: particles in cell c of level l */
    cplx **mpole;          /* mpole[l][c*p + m], l = 2..L */
    cplx **local;          /* local[l][c*p + m], l = 2..L */
    char **needed;         /* needed[l][c]: local expansion required at cell c */
    double *binom;         /* binom[n*(2p+1) + k] = C(n, k), n, k <= 2p */
} otree;

static double cell_w(const otree *t, int l) { return t->side / (double)(1 << l); }

static cplx cell_centre(const otree *t, int l, int cx, int cy)
{
    double w = cell_w(t, l);
    return (t->x0 + (cx + 0.5) * w) + I * (t->y0 + (cy + 0.5) * w);
}

static double C(const otree *t, int n, int k) { return t->binom[n * (2 * t->p + 1) + k]; }

static void otree_free(otree *t)
{
    free(t->leaf_start);
    free(t->leaf_src);
    for (int l = 0; l <= t->depth; ++l) {
        if (t->count) free(t->count[l]);
        if (t->mpole) free(t->mpole[l]);
        if (t->local) free(t->local[l]);
        if (t->needed) free(t->needed[l]);
    }
    free(t->count);
    free(t->mpole);
    free(t->local);
    free(t->needed);
    free(t->binom);
}

/* Stages 1-2: tree, binning, per-level occupancy. */
static int otree_build(otree *t, int64_t ns, const double *sxy, int depth, const double *root, int p)
{
    memset(t, 0, sizeof(*t));
    t->depth = depth;
    t->p = p;
    t->x0 = root[0];
    t->y0 = root[1];
    t->side = root[2];
    int nside = 1 << depth;
    int64_t nleaf = (int64_t)nside * nside;
    int32_t *ix = malloc(sizeof(int32_t) * (ns ? ns : 1));
    int32_t *iy = malloc(sizeof(int32_t) * (ns ? ns : 1));
    t->leaf_start = calloc(nleaf + 1, sizeof(int64_t));
    t->leaf_src = malloc(sizeof(int64_t) * (ns ? ns : 1));
    t->count = calloc(depth + 1, sizeof(int64_t *));
    t->mpole = calloc(depth + 1, sizeof(cplx *));
    t->local = calloc(depth + 1, sizeof(cplx *));
    t->needed = calloc(depth + 1, sizeof(char *));
    int nb = 2 * p + 1;
    t->binom = calloc((size_t)nb * nb, sizeof(double));
    if (!ix || !iy || !t->leaf_start || !t->leaf_src || !t->count || !t->mpole || !t->local ||
        !t->needed || !t->binom) {
        free(ix);
        free(iy);
        return ORC_ENOMEM;
    }
    int rc = orc_bin(ns, sxy, depth, root, ix, iy);
    if (rc) {
        free(ix);
        free(iy);
        return rc;
    }
    /* Pascal's triangle */
    for (int n = 0; n < nb; ++n) {
        t->binom[n * nb] = 1.0;
        for (int k = 1; k <= n; ++k)
            t->binom[n * nb + k] = t->binom[(n - 1) * nb + k - 1] + (k <= n - 1 ? t->binom[(n - 1) * nb + k] : 0.0);
    }
    /* counting sort of sources by leaf (stable: input order kept inside a leaf) */
    for (int64_t j = 0; j < ns; ++j) t->leaf_start[(int64_t)iy[j] * nside + ix[j] + 1]++;
    for (int64_t c = 0; c < nleaf; ++c) t->leaf_start[c + 1] += t->leaf_start[c];
    int64_t *fill = malloc(sizeof(int64_t) * nleaf);
    if (!fill) {
        free(ix);
        free(iy);
        return ORC_ENOMEM;
    }
    memcpy(fill, t->leaf_start, sizeof(int64_t) * nleaf);
    for (int64_t j = 0; j < ns; ++j) t->leaf_src[fill[(int64_t)iy[j] * nside + ix[j]]++] = j;
    free(fill);
    free(ix);
    free(iy);
    /* occupancy per level */
    for (int l = 0; l <= depth; ++l) {
        int64_t ncell = (int64_t)1 << (2 * l);
        t->count[l] = calloc(ncell, sizeof(int64_t));
        t->needed[l] = calloc(ncell, 1);
        if (!t->count[l] || !t->needed[l]) return ORC_ENOMEM;
    }
    for (int64_t c = 0; c < nleaf; ++c) t->count[depth][c] = t->leaf_start[c + 1] - t->leaf_start[c];
    for (int l = depth - 1; l >= 0; --l) {
        int n1 = 1 << l;
        for (int cy = 0; cy < n1; ++cy)
            for (int cx = 0; cx < n1; ++cx) {
                int64_t s = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        s += t->count[l + 1][(int64_t)(2 * cy + b) * (2 * n1) + 2 * cx + a];
                t->count[l][(int64_t)cy * n1 + cx] = s;
            }
    }
    for (int l = 2; l <= depth; ++l) {
        int64_t ncell = (int64_t)1 << (2 * l);
        t->mpole[l] = calloc((size_t)ncell * p, sizeof(cplx));
        t->local[l] = calloc((size_t)ncell * p, sizeof(cplx));
        if (!t->mpole[l] || !t->local[l]) return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* Stage 4, P2M: a_m = sum_{j in leaf} c_j (z_j - z_c)^m, m = 0..p-1. */
static void p2m(otree *t, const double *sxy, const cplx *q)
{
    int L = t->depth, p = t->p, nside = 1 << L;
    int64_t nleaf = (int64_t)nside * nside;
    if (L < 2) return; /* levels 0 and 1 carry no expansions */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < nleaf; ++c) {
        if (t->count[L][c] == 0) continue;
        cplx zc = cell_centre(t, L, (int)(c % nside), (int)(c / nside));
        cplx *a = &t->mpole[L][c * p];
        for (int64_t k = t->leaf_start[c]; k < t->leaf_start[c + 1]; ++k) {
            int64_t j = t->leaf_src[k];
            cplx d = (sxy[2 * j] + I * sxy[2 * j + 1]) - zc;
            cplx pw = 1.0;
            for (int m = 0; m < p; ++m) {
                a[m] += q[j] * pw;
                pw *= d;
            }
        }
    }
}

/* Stage 5, M2M into levels L-1..2:
 * A_m(parent) = sum_children sum_{k<=m} C(m,k) (z_child - z_parent)^(m-k) a_k(child). */
static void m2m(otree *t)
{
    int p = t->p;
    for (int l = t->depth - 1; l >= 2; --l) {
        int n1 = 1 << l;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t c = 0; c < (int64_t)n1 * n1; ++c) {
            if (t->count[l][c] == 0) continue;
            int cx = (int)(c % n1), cy = (int)(c / n1);
            cplx zp = cell_centre(t, l, cx, cy);
            cplx *A = &t->mpole[l][c * p];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    int chx = 2 * cx + a, chy = 2 * cy + b;
                    int64_t ch = (int64_t)chy * (2 * n1) + chx;
                    if (t->count[l + 1][ch] == 0) continue;
                    cplx d = cell_centre(t, l + 1, chx, chy) - zp;
                    const cplx *ac = &t->mpole[l + 1][ch * p];
                    for (int m = 0; m < p; ++m) {
                        cplx s = 0.0;
                        for (int k = 0; k <= m; ++k) s += C(t, m, k) * cpow(d, m - k) * ac[k];
                        A[m] += s;
                    }
                }
        }
    }
}

static int adjacent(int ax, int ay, int bx, int by) { return abs(ax - bx) <= 1 && abs(ay - by) <= 1; }

/* Stages 6-7 for the cells marked as needed.
 * M2L at level l = 2..L for each source S in the interaction list of T:
 *   b_l(T) += sum_{m<p} a_m(S) (-1)^l C(l+m, m) / (z_T - z_S)^(l+m+1),
 * L2L into levels 3..L:
 *   b_k(child) += sum_{l=k}^{p-1} C(l,k) (z_child - z_parent)^(l-k) b_l(parent). */
static void m2l_l2l(otree *t)
{
    int p = t->p;
    for (int l = 2; l <= t->depth; ++l) {
        int n1 = 1 << l;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t c = 0; c < (int64_t)n1 * n1; ++c) {
            if (!t->needed[l][c]) continue;
            int tx = (int)(c % n1), ty = (int)(c / n1);
            cplx zt = cell_centre(t, l, tx, ty);
            cplx *B = &t->local[l][c * p];
            /* interaction list: children of the parent's neighbours that are not neighbours */
            int px = tx >> 1, py = ty >> 1;
            for (int ny = py - 1; ny <= py + 1; ++ny)
                for (int nx = px - 1; nx <= px + 1; ++nx) {
                    if (nx < 0 || ny < 0 || nx >= n1 / 2 || ny >= n1 / 2) continue;
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            int sx = 2 * nx + a, sy = 2 * ny + b;
                            if (adjacent(sx, sy, tx, ty)) continue;
                            int64_t s = (int64_t)sy * n1 + sx;
                            if (t->count[l][s] == 0) continue;
                            cplx D = zt - cell_centre(t, l, sx, sy);
                            const cplx *A = &t->mpole[l][s * p];
                            for (int lo = 0; lo < p; ++lo) {
                                cplx acc = 0.0;
                                double sgn = (lo & 1) ? -1.0 : 1.0;
                                for (int m = 0; m < p; ++m)
                                    acc += A[m] * sgn * C(t, lo + m, m) / cpow(D, lo + m + 1);
                                B[lo] += acc;
                            }
                        }
                }
            if (l >= 3) {
                int64_t pc = (int64_t)py * (n1 / 2) + px;
                cplx d = zt - cell_centre(t, l - 1, px, py);
                const cplx *Bp = &t->local[l - 1][pc * p];
                for (int k = 0; k < p; ++k) {
                    cplx acc = 0.0;
                    for (int lo = k; lo < p; ++lo) acc += C(t, lo, k) * cpow(d, lo - k) * Bp[lo];
                    B[k] += acc;
                }
            }
        }
    }
}

/* Mark the leaves of the evaluation points and all their ancestors. */
static int mark_needed(otree *t, int64_t nt, const double *txy, int32_t *tix, int32_t *tiy)
{
    double root[3] = {t->x0, t->y0, t->side};
    int rc = orc_bin(nt, txy, t->depth, root, tix, tiy);
    if (rc) return rc;
    for (int64_t i = 0; i < nt; ++i) {
        int cx = tix[i], cy = tiy[i];
        for (int l = t->depth; l >= 0; --l) {
            t->needed[l][(int64_t)cy * (1 << l) + cx] = 1;
            cx >>= 1;
            cy >>= 1;
        }
    }
    return ORC_OK;
}

static int fmm_setup(otree *t, int64_t ns, const double *sxy, const cplx *q, int64_t nt, const double *txy,
                     int32_t *tix, int32_t *tiy, int depth, const double *root, int p)
{
    if (ns < 0 || nt < 0 || depth < 0 || depth > 13 || p < 1 || p > 40) return ORC_EINVAL;
    int rc = otree_build(t, ns, sxy, depth, root, p);
    if (!rc) rc = mark_needed(t, nt, txy, tix, tiy);
    if (rc) return rc;
    p2m(t, sxy, q);
    m2m(t);
    m2l_l2l(t);
    return ORC_OK;
}

/* O3.  For each evaluation point z_i (leaf i_leaf):
 *   W_far(z_i)  = sum_{l<p} b_l(leaf) (z_i - z_leaf)^l              (stage 8, L2P)
 *   W_near(z_i) = sum_{j in N(leaf), s > 0} q_j g(s)/(z_i - z_j)     (stage 9, P2P)
 * q: complex charges as interleaved (re, im); W_near, W_far: interleaved (re, im).
 * Stage 10 (the sum) is left to the caller so that each part can be checked. */
int orc_fmm(int64_t ns, const double *sxy, const double *q_ri, int64_t nt, const double *txy,
            double sigma, int depth, const double *root, int p, double *w_near, double *w_far)
{
    if (!(sigma > 0.0)) return ORC_EINVAL;
    const cplx *q = (const cplx *)q_ri;
    otree t;
    int32_t *tix = malloc(sizeof(int32_t) * (nt ? nt : 1));
    int32_t *tiy = malloc(sizeof(int32_t) * (nt ? nt : 1));
    if (!tix || !tiy) {
        free(tix);
        free(tiy);
        return ORC_ENOMEM;
    }
    int rc = fmm_setup(&t, ns, sxy, q, nt, txy, tix, tiy, depth, root, p);
    if (rc) {
        otree_free(&t);
        free(tix);
        free(tiy);
        return rc;
    }
    int L = depth, nside = 1 << L;
    double k2 = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
        cplx z = txy[2 * i] + I * txy[2 * i + 1];
        int cx = tix[i], cy = tiy[i];
        /* L2P */
        cplx wf = 0.0;
        if (L >= 2) {
            cplx d = z - cell_centre(&t, L, cx, cy);
            const cplx *B = &t.local[L][((int64_t)cy * nside + cx) * p];
            cplx pw = 1.0;
            for (int lo = 0; lo < p; ++lo) {
                wf += B[lo] * pw;
                pw *= d;
            }
        }
        /* P2P over the 3x3 neighbourhood */
        cplx wn = 0.0;
        for (int ny = cy - 1; ny <= cy + 1; ++ny)
            for (int nx = cx - 1; nx <= cx + 1; ++nx) {
                if (nx < 0 || ny < 0 || nx >= nside || ny >= nside) continue;
                int64_t c = (int64_t)ny * nside + nx;
                for (int64_t k = t.leaf_start[c]; k < t.leaf_start[c + 1]; ++k) {
                    int64_t j = t.leaf_src[k];
                    cplx dz = z - (sxy[2 * j] + I * sxy[2 * j + 1]);
                    double s = creal(dz) * creal(dz) + cimag(dz) * cimag(dz);
                    if (s == 0.0) continue;
                    double g = -expm1(-s * k2);
                    wn += q[j] * g / dz;
                }
            }
        w_near[2 * i] = creal(wn);
        w_near[2 * i + 1] = cimag(wn);
        w_far[2 * i] = creal(wf);
        w_far[2 * i + 1] = cimag(wf);
    }
    otree_free(&t);
    free(tix);
    free(tiy);
    return ORC_OK;
}

/* h(x) = ((1 + x) e^-x - 1) / x^2, so that f'(s) = kappa^2 h(kappa s) for
 * f(s) = (1 - e^{-kappa s})/s.  Series h = -sum_k (-1)^k (k+1) x^k/(k+2)! below 0.1. */
static double reg_h(double x)
{
    if (x < 0.1) {
        double term = 0.5, sum = 0.0;   /* term = x^k/(k+2)! */
        for (int k = 0; k < 30; ++k) {
            sum += ((k & 1) ? -1.0 : 1.0) * (k + 1) * term;
            term *= x / (k + 3);
        }
        return -sum;
    }
    return ((1.0 + x) * exp(-x) - 1.0) / (x * x);
}

/* The two kernel functions above, for the adaptive oracle (adaptive_oracle.c). */
double orc_reg_f(double s, double sigma) { return reg_f(s, sigma); }
double orc_reg_h(double x) { return reg_h(x); }

/* O4 helper.  Jacobian of the O3 velocity at evaluation points z_i with respect to
 * z_i, sources held fixed, for real circulations gamma.  Per point, J = [du/dx,
 * du/dy, dv/dx, dv/dy], split into the near part (derivative of the real form of
 * eq. regB-S2DGau, including the source at the evaluation point itself, whose
 * kernel is smooth with slope 1/(2 sigma^2)) and the far part (derivative of the
 * local expansion: with W = u - iv analytic, du/dx = Re W', dv/dx = -Im W',
 * du/dy = -Im W', dv/dy = -Re W'). */
int orc_fmm_jacobian(int64_t ns, const double *sxy, const double *gamma, int64_t nt, const double *txy,
                     double sigma, int depth, const double *root, int p, double *j_near, double *j_far)
{
    if (!(sigma > 0.0)) return ORC_EINVAL;
    cplx *q = malloc(sizeof(cplx) * (ns ? ns : 1));
    int32_t *tix = malloc(sizeof(int32_t) * (nt ? nt : 1));
    int32_t *tiy = malloc(sizeof(int32_t) * (nt ? nt : 1));
    if (!q || !tix || !tiy) {
        free(q);
        free(tix);
        free(tiy);
        return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < ns; ++j) q[j] = -I * gamma[j] / TWO_PI;
    otree t;
    int rc = fmm_setup(&t, ns, sxy, q, nt, txy, tix, tiy, depth, root, p);
    if (rc) {
        otree_free(&t);
        free(q);
        free(tix);
        free(tiy);
        return rc;
    }
    int L = depth, nside = 1 << L;
    double kappa = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
        double x = txy[2 * i], y = txy[2 * i + 1];
        int cx = tix[i], cy = tiy[i];
        cplx dw = 0.0;
        if (L >= 2) {
            cplx d = (x + I * y) - cell_centre(&t, L, cx, cy);
            const cplx *B = &t.local[L][((int64_t)cy * nside + cx) * p];
            cplx pw = 1.0;
            for (int lo = 1; lo < p; ++lo) {
                dw += lo * B[lo] * pw;
                pw *= d;
            }
        }
        double uxx = 0, uxy = 0, vxx = 0, vxy = 0;
        for (int ny = cy - 1; ny <= cy + 1; ++ny)
            for (int nx = cx - 1; nx <= cx + 1; ++nx) {
                if (nx < 0 || ny < 0 || nx >= nside || ny >= nside) continue;
                int64_t c = (int64_t)ny * nside + nx;
                for (int64_t k = t.leaf_start[c]; k < t.leaf_start[c + 1]; ++k) {
                    int64_t j = t.leaf_src[k];
                    double dx = x - sxy[2 * j], dy = y - sxy[2 * j + 1];
                    double s = dx * dx + dy * dy;
                    double f = (s == 0.0) ? kappa : reg_f(s, sigma);
                    double fp = kappa * kappa * reg_h(kappa * s);
                    double G = gamma[j] / TWO_PI;
                    /* u = G (-dy) f(s), v = G dx f(s), ds/dx = 2 dx, ds/dy = 2 dy */
                    uxx += G * (-dy) * fp * 2.0 * dx;
                    uxy += G * (-f - dy * fp * 2.0 * dy);
                    vxx += G * (f + dx * fp * 2.0 * dx);
                    vxy += G * dx * fp * 2.0 * dy;
                }
            }
        j_near[4 * i + 0] = uxx;
        j_near[4 * i + 1] = uxy;
        j_near[4 * i + 2] = vxx;
        j_near[4 * i + 3] = vxy;
        j_far[4 * i + 0] = creal(dw);
        j_far[4 * i + 1] = -cimag(dw);
        j_far[4 * i + 2] = -cimag(dw);
        j_far[4 * i + 3] = -creal(dw);
    }
    otree_free(&t);
    free(q);
    free(tix);
    free(tiy);
    return ORC_OK;
}

/* Real-form derivatives of one pair's velocity contribution, (u, v) = G (-dy, dx) f(s),
 * s = dx^2 + dy^2, (dx, dy) = target - source, with respect to the target position:
 * J = [du/dx, du/dy, dv/dx, dv/dy].  f(0) and f'(0) are the kernel's limits. */
static void pair_jacobian(double dx, double dy, double G, double sigma, double *J)
{
    double kappa = 1.0 / (2.0 * sigma * sigma);
    double s = dx * dx + dy * dy;
    double f = (s == 0.0) ? kappa : reg_f(s, sigma);
    double fp = kappa * kappa * reg_h(kappa * s);
    J[0] = G * (-dy) * fp * 2.0 * dx;
    J[1] = G * (-f - dy * fp * 2.0 * dy);
    J[2] = G * (f + dx * fp * 2.0 * dx);
    J[3] = G * dx * fp * 2.0 * dy;
}

/* O5 helper.  Gradient of L through the O3 velocities at the particles with respect to
 * the SOURCE positions, the evaluation points held fixed; g = (dL/du_i, dL/dv_i).
 * Near part: the pair (i, j) term of u_i depends on z_j through z_i - z_j, so its
 * derivative with respect to z_j is minus the pair's Jacobian, summed over the
 * particles i whose 3 x 3 neighbourhood holds j (the pair i = j included: moving the
 * source alone changes it).
 * Far part: the O3 far operator is antisymmetric as a function of both positions,
 * F_ij(z_i, z_j) = -F_ji(z_j, z_i) (symmetric lists, square truncation, exact M2M and
 * L2L), so sum_i q_i dF_ij/dz_j = -Phi'_j, the derivative at z_j of the local expansion
 * of the same FMM run with charges q_i = g_i,u + i g_i,v.  With dL = Re(sum_i q_i dW_i),
 * W = u - iv and c_j = -i Gamma_j/(2 pi):  dL/dx_j = -Re(c_j Phi'_j),
 * dL/dy_j = Im(c_j Phi'_j). */
int orc_fmm_src_grad(int64_t n, const double *xy, const double *gamma, const double *g, double sigma, int depth,
                     const double *root, int p, double *d_near, double *d_far)
{
    if (!(sigma > 0.0)) return ORC_EINVAL;
    cplx *q = malloc(sizeof(cplx) * (n ? n : 1));
    int32_t *tix = malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *tiy = malloc(sizeof(int32_t) * (n ? n : 1));
    if (!q || !tix || !tiy) {
        free(q);
        free(tix);
        free(tiy);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) q[i] = g[2 * i] + I * g[2 * i + 1];
    otree t;
    int rc = fmm_setup(&t, n, xy, q, n, xy, tix, tiy, depth, root, p);
    if (rc) {
        otree_free(&t);
        free(q);
        free(tix);
        free(tiy);
        return rc;
    }
    int L = depth, nside = 1 << L;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < n; ++j) {
        double x = xy[2 * j], y = xy[2 * j + 1];
        int cx = tix[j], cy = tiy[j];
        cplx dphi = 0.0;
        if (L >= 2) {
            cplx d = (x + I * y) - cell_centre(&t, L, cx, cy);
            const cplx *B = &t.local[L][((int64_t)cy * nside + cx) * p];
            cplx pw = 1.0;
            for (int lo = 1; lo < p; ++lo) {
                dphi += lo * B[lo] * pw;
                pw *= d;
            }
        }
        cplx c = -I * gamma[j] / TWO_PI;
        d_far[2 * j] = -creal(c * dphi);
        d_far[2 * j + 1] = cimag(c * dphi);
        double gx = 0.0, gy = 0.0, G = gamma[j] / TWO_PI, J[4];
        for (int ny = cy - 1; ny <= cy + 1; ++ny)
            for (int nx = cx - 1; nx <= cx + 1; ++nx) {
                if (nx < 0 || ny < 0 || nx >= nside || ny >= nside) continue;
                int64_t cell = (int64_t)ny * nside + nx;
                for (int64_t k = t.leaf_start[cell]; k < t.leaf_start[cell + 1]; ++k) {
                    int64_t i = t.leaf_src[k];
                    pair_jacobian(xy[2 * i] - x, xy[2 * i + 1] - y, G, sigma, J);
                    gx -= g[2 * i] * J[0] + g[2 * i + 1] * J[2];
                    gy -= g[2 * i] * J[1] + g[2 * i + 1] * J[3];
                }
            }
        d_near[2 * j] = gx;
        d_near[2 * j + 1] = gy;
    }
    otree_free(&t);
    free(q);
    free(tix);
    free(tiy);
    return ORC_OK;
}

/* O1 gradient.  L through u_i = sum_{j != i, s_ij > 0} Gamma_j K_sigma(x_i - x_j) with
 * every particle moving both as evaluation point and as source; g = (dL/du_i, dL/dv_i).
 * dL/dGamma_j = sum_i g_i . K_sigma(x_i - x_j); each pair (i, j) adds g_i . J_ij to
 * dL/dx_i and subtracts it from dL/dx_j. */
void orc_direct_grad(int64_t n, const double *xy, const double *gamma, double sigma, const double *g,
                     double *dgamma, double *dxy)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n; ++a) {
        double dga = 0.0, ex = 0.0, ey = 0.0, J[4];
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            /* pair (target a, source b): eval derivative of a */
            double dx = xy[2 * a] - xy[2 * b], dy = xy[2 * a + 1] - xy[2 * b + 1];
            double s = dx * dx + dy * dy;
            if (s > 0.0) {
                pair_jacobian(dx, dy, gamma[b] / TWO_PI, sigma, J);
                ex += g[2 * a] * J[0] + g[2 * a + 1] * J[2];
                ey += g[2 * a] * J[1] + g[2 * a + 1] * J[3];
                /* pair (target b, source a): source derivative of a, and dL/dGamma_a */
                pair_jacobian(-dx, -dy, gamma[a] / TWO_PI, sigma, J);
                ex -= g[2 * b] * J[0] + g[2 * b + 1] * J[2];
                ey -= g[2 * b] * J[1] + g[2 * b + 1] * J[3];
                double k = reg_f(s, sigma) / TWO_PI;
                dga += g[2 * b] * (dy * k) + g[2 * b + 1] * (-dx * k);
            }
        }
        dgamma[a] = dga;
        dxy[2 * a] = ex;
        dxy[2 * a + 1] = ey;
    }
}

/* Per-leaf particle counts (row-major leaves) for the pair-count check. */
int orc_leaf_counts(int64_t n, const double *xy, int depth, const double *root, int64_t *counts)
{
    int nside = 1 << depth;
    int32_t *ix = malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *iy = malloc(sizeof(int32_t) * (n ? n : 1));
    if (!ix || !iy) {
        free(ix);
        free(iy);
        return ORC_ENOMEM;
    }
    int rc = orc_bin(n, xy, depth, root, ix, iy);
    if (!rc) {
        memset(counts, 0, sizeof(int64_t) * (size_t)nside * nside);
        for (int64_t i = 0; i < n; ++i) counts[(int64_t)iy[i] * nside + ix[i]]++;
    }
    free(ix);
    free(iy);
    return rc;
}

/* Interaction-list membership for the list-partition check: for target leaf
 * (tx, ty) and source leaf (sx, sy), writes the level at which the source is
 * reached (0 if it is in the near field, -1 if never, -2 if more than once). */
int orc_cover_level(int depth, int tx, int ty, int sx, int sy)
{
    if (adjacent(tx, ty, sx, sy)) return 0;
    int found = -1;
    for (int l = depth; l >= 2; --l) {
        int sh = depth - l;
        int ctx = tx >> sh, cty = ty >> sh, csx = sx >> sh, csy = sy >> sh;
        int in_il = !adjacent(ctx, cty, csx, csy) && adjacent(ctx >> 1, cty >> 1, csx >> 1, csy >> 1);
        if (in_il) {
            if (found != -1) return -2;
            found = l;
        }
    }
    return found;
}
