/*
 * adaptive_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * The velocity evaluation of fmm_oracle.c (O3) on an adaptive quadtree, for uneven
 * particle distributions (the first extension named in the paper's conclusions: with
 * the particles per box held roughly constant, the complexity estimates carry over).
 * The paper fixes no adaptive scheme; this is the adaptive FMM of Carrier, Greengard
 * and Rokhlin (SIAM J. Sci. Stat. Comput. 9, 1988) with its four interaction lists,
 * restated here from their definitions.  Plain FP64, unscaled textbook operators,
 * O(lists) loops; only the test suite loads it, and it shares nothing with the GPU
 * library.
 *
 * Tree (readings listed in the design notes):
 *   - root cell [x0, x0+S]^2; a cell of level l is split into its four quadrants when
 *     it holds more than s_max particles and l < l_max; empty cells are dropped;
 *   - a particle's cell at level l follows the uniform binning of fmm_oracle.c at
 *     level l_max (i = min(floor((x - x0)/w), 2^l_max - 1)), shifted right;
 *   - two cells are adjacent when their closed squares intersect (any levels);
 *   - colleagues of B: the other cells of B's level adjacent to B.
 * Lists (B a cell, A a leaf):
 *   U(A)  leaves adjacent to A, A included                       -> P2P, exact kernel
 *   V(B)  children of the colleagues of B's parent, not adjacent  -> M2L
 *   W(A)  cells D below a colleague of A, D not adjacent to A, D's parent adjacent to A
 *                                                                  -> M2P at A's particles
 *   X(B)  leaves A with B in W(A)                                  -> P2L into B
 * Expansions live on cells of level >= 2 (V is empty above); the far field uses the
 * singular kernel, the near field (U) the regularised one, as in O3.  With every leaf
 * on level l_max the lists are O3's and W, X are empty.
 *
 * O7 (orc_afmm_grad) is the adjoint of O6 in the manner of O4 and O5: circulations by the
 * same evaluation with complex charges, positions by pair Jacobians over U and the
 * derivatives of the far expansions (differentiated L2P and M2P).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

int orc_bin(int64_t n, const double *xy, int depth, const double *root, int32_t *ix, int32_t *iy);
double orc_reg_f(double s, double sigma);
double orc_reg_h(double x);

typedef struct {
    int level, ix, iy, leaf;
    int64_t first, count; /* the cell's sources are src[first .. first + count) */
    int64_t parent;       /* -1 for the root */
    int64_t child[4];     /* -1 for an empty (dropped) quadrant */
} anode;

typedef struct {
    int64_t *off, *idx; /* CSR over cells */
} alist;

typedef struct {
    int lmax, smax;
    double x0, y0, side;
    int64_t n, nnodes;
    anode *nodes;        /* level by level (breadth first) */
    int64_t *src;        /* source indices grouped by cell, recursively */
    int64_t *leaf_of;    /* leaf cell of each source */
    alist coll, U, V, W, X;
} atree;

/* ------------------------------------------------------------------------------ */
/* Growable index lists                                                            */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int64_t *a;
    int64_t n, cap;
} vec;

static int vpush(vec *v, int64_t x)
{
    if (v->n == v->cap) {
        int64_t c = v->cap ? 2 * v->cap : 64;
        int64_t *a = realloc(v->a, sizeof(int64_t) * c);
        if (!a) return ORC_ENOMEM;
        v->a = a;
        v->cap = c;
    }
    v->a[v->n++] = x;
    return ORC_OK;
}

/* CSR builder: items appended in cell order */
typedef struct {
    vec off, idx;
} csr;

static int csr_begin(csr *c) { return vpush(&c->off, c->idx.n); }

static void alist_take(alist *l, csr *c)
{
    l->off = c->off.a;
    l->idx = c->idx.a;
    memset(c, 0, sizeof(*c));
}

static void alist_free(alist *l)
{
    free(l->off);
    free(l->idx);
    l->off = l->idx = NULL;
}

void orc_atree_free(atree *t)
{
    if (!t) return;
    free(t->nodes);
    free(t->src);
    free(t->leaf_of);
    alist_free(&t->coll);
    alist_free(&t->U);
    alist_free(&t->V);
    alist_free(&t->W);
    alist_free(&t->X);
    free(t);
}

/* ------------------------------------------------------------------------------ */
/* Geometry                                                                         */
/* ------------------------------------------------------------------------------ */

/* Closed squares of a and b intersect (in units of the level-l_max cell). */
static int adjacent(const atree *t, const anode *a, const anode *b)
{
    int64_t sa = (int64_t)1 << (t->lmax - a->level), sb = (int64_t)1 << (t->lmax - b->level);
    int64_t ax0 = a->ix * sa, ax1 = ax0 + sa, ay0 = a->iy * sa, ay1 = ay0 + sa;
    int64_t bx0 = b->ix * sb, bx1 = bx0 + sb, by0 = b->iy * sb, by1 = by0 + sb;
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

static cplx centre(const atree *t, const anode *a)
{
    double w = t->side / (double)(1 << a->level);
    return (t->x0 + (a->ix + 0.5) * w) + I * (t->y0 + (a->iy + 0.5) * w);
}

/* ------------------------------------------------------------------------------ */
/* Tree and lists                                                                   */
/* ------------------------------------------------------------------------------ */

static int build_nodes(atree *t, const int32_t *ix, const int32_t *iy)
{
    int64_t cap = 1024;
    t->nodes = malloc(sizeof(anode) * cap);
    int64_t *tmp = malloc(sizeof(int64_t) * (t->n ? t->n : 1));
    if (!t->nodes || !tmp) {
        free(tmp);
        return ORC_ENOMEM;
    }
    anode root = {0, 0, 0, 1, 0, t->n, -1, {-1, -1, -1, -1}};
    t->nodes[0] = root;
    t->nnodes = 1;
    /* cells are appended as they are created, so the array is breadth first */
    for (int64_t k = 0; k < t->nnodes; ++k) {
        anode *b = &t->nodes[k];
        if (b->count <= t->smax || b->level >= t->lmax) continue;
        b->leaf = 0;
        int shift = t->lmax - b->level - 1;
        int64_t cnt[4] = {0, 0, 0, 0};
        for (int64_t j = b->first; j < b->first + b->count; ++j) {
            int64_t s = t->src[j];
            cnt[2 * ((iy[s] >> shift) & 1) + ((ix[s] >> shift) & 1)]++;
        }
        int64_t start[4];
        start[0] = b->first;
        for (int q = 1; q < 4; ++q) start[q] = start[q - 1] + cnt[q - 1];
        int64_t fill[4] = {start[0], start[1], start[2], start[3]};
        for (int64_t j = b->first; j < b->first + b->count; ++j) { /* stable partition */
            int64_t s = t->src[j];
            tmp[fill[2 * ((iy[s] >> shift) & 1) + ((ix[s] >> shift) & 1)]++] = s;
        }
        memcpy(t->src + b->first, tmp + b->first, sizeof(int64_t) * b->count);
        int level = b->level, bx = b->ix, by = b->iy;
        for (int q = 0; q < 4; ++q) {
            if (cnt[q] == 0) continue;
            if (t->nnodes == cap) {
                cap *= 2;
                anode *nn = realloc(t->nodes, sizeof(anode) * cap);
                if (!nn) {
                    free(tmp);
                    return ORC_ENOMEM;
                }
                t->nodes = nn;
            }
            anode c = {level + 1, 2 * bx + (q & 1), 2 * by + (q >> 1), 1, start[q], cnt[q], k, {-1, -1, -1, -1}};
            t->nodes[k].child[q] = t->nnodes;
            t->nodes[t->nnodes++] = c;
        }
    }
    free(tmp);
    for (int64_t k = 0; k < t->nnodes; ++k)
        if (t->nodes[k].leaf)
            for (int64_t j = t->nodes[k].first; j < t->nodes[k].first + t->nodes[k].count; ++j)
                t->leaf_of[t->src[j]] = k;
    return ORC_OK;
}

/* Colleagues: the children of the parent and of the parent's colleagues that are
 * adjacent to the cell (other than the cell itself). */
static int build_colleagues(atree *t)
{
    csr c = {0};
    int rc = ORC_OK;
    for (int64_t k = 0; k < t->nnodes && !rc; ++k) {
        rc = csr_begin(&c);
        const anode *b = &t->nodes[k];
        if (b->parent < 0) continue;
        int64_t P = b->parent;
        /* the parent, then its colleagues (already built: parents precede children) */
        int64_t cand_n = 1 + (c.off.a[P + 1] - c.off.a[P]);
        for (int64_t e = 0; e < cand_n && !rc; ++e) {
            int64_t Q = e == 0 ? P : c.idx.a[c.off.a[P] + e - 1];
            for (int q = 0; q < 4 && !rc; ++q) {
                int64_t ch = t->nodes[Q].child[q];
                if (ch < 0 || ch == k) continue;
                if (adjacent(t, &t->nodes[ch], b)) rc = vpush(&c.idx, ch);
            }
        }
    }
    if (!rc) rc = csr_begin(&c);
    if (rc) {
        free(c.off.a);
        free(c.idx.a);
        return rc;
    }
    alist_take(&t->coll, &c);
    return ORC_OK;
}

#define COLL_BEGIN(t, k) ((t)->coll.off[k])
#define COLL_END(t, k) ((t)->coll.off[(k) + 1])

/* leaves at or below cell c that are adjacent to leaf a */
static int push_adjacent_leaves(const atree *t, int64_t c, int64_t a, vec *out)
{
    if (!adjacent(t, &t->nodes[c], &t->nodes[a])) return ORC_OK;
    if (t->nodes[c].leaf) return vpush(out, c);
    for (int q = 0; q < 4; ++q) {
        int64_t ch = t->nodes[c].child[q];
        if (ch >= 0) {
            int rc = push_adjacent_leaves(t, ch, a, out);
            if (rc) return rc;
        }
    }
    return ORC_OK;
}

/* W: below colleague cell c of leaf a, cells not adjacent to a whose parent is */
static int push_w(const atree *t, int64_t c, int64_t a, vec *out)
{
    for (int q = 0; q < 4; ++q) {
        int64_t d = t->nodes[c].child[q];
        if (d < 0) continue;
        int rc = ORC_OK;
        if (!adjacent(t, &t->nodes[d], &t->nodes[a])) rc = vpush(out, d);
        else if (!t->nodes[d].leaf) rc = push_w(t, d, a, out);
        if (rc) return rc;
    }
    return ORC_OK;
}

static int build_lists(atree *t)
{
    csr u = {0}, v = {0}, w = {0};
    int rc = ORC_OK;
    for (int64_t k = 0; k < t->nnodes && !rc; ++k) {
        const anode *b = &t->nodes[k];
        if ((rc = csr_begin(&u)) || (rc = csr_begin(&v)) || (rc = csr_begin(&w))) break;
        /* V: children of the parent's colleagues, not adjacent */
        if (b->parent >= 0) {
            int64_t P = b->parent;
            for (int64_t e = COLL_BEGIN(t, P); e < COLL_END(t, P) && !rc; ++e) {
                int64_t Q = t->coll.idx[e];
                for (int q = 0; q < 4 && !rc; ++q) {
                    int64_t d = t->nodes[Q].child[q];
                    if (d >= 0 && !adjacent(t, &t->nodes[d], b)) rc = vpush(&v.idx, d);
                }
            }
        }
        if (!b->leaf || rc) continue;
        /* U: the leaf itself, adjacent leaves at or below its colleagues, and coarser
         * adjacent leaves (colleagues of its ancestors) */
        rc = vpush(&u.idx, k);
        for (int64_t e = COLL_BEGIN(t, k); e < COLL_END(t, k) && !rc; ++e)
            rc = push_adjacent_leaves(t, t->coll.idx[e], k, &u.idx);
        for (int64_t A = b->parent; A >= 0 && !rc; A = t->nodes[A].parent)
            for (int64_t e = COLL_BEGIN(t, A); e < COLL_END(t, A) && !rc; ++e) {
                int64_t c = t->coll.idx[e];
                if (t->nodes[c].leaf && adjacent(t, &t->nodes[c], b)) rc = vpush(&u.idx, c);
            }
        /* W */
        for (int64_t e = COLL_BEGIN(t, k); e < COLL_END(t, k) && !rc; ++e) {
            int64_t c = t->coll.idx[e];
            if (!t->nodes[c].leaf) rc = push_w(t, c, k, &w.idx);
        }
    }
    if (!rc && !(rc = csr_begin(&u)) && !(rc = csr_begin(&v))) rc = csr_begin(&w);
    if (rc) {
        free(u.off.a), free(u.idx.a), free(v.off.a), free(v.idx.a), free(w.off.a), free(w.idx.a);
        return rc;
    }
    alist_take(&t->U, &u);
    alist_take(&t->V, &v);
    alist_take(&t->W, &w);
    /* X: the transpose of W */
    int64_t nn = t->nnodes, nw = t->W.off[nn];
    t->X.off = calloc(nn + 1, sizeof(int64_t));
    t->X.idx = malloc(sizeof(int64_t) * (nw ? nw : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (nn ? nn : 1));
    if (!t->X.off || !t->X.idx || !fill) {
        free(fill);
        return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < nw; ++e) t->X.off[t->W.idx[e] + 1]++;
    for (int64_t k = 0; k < nn; ++k) t->X.off[k + 1] += t->X.off[k];
    memcpy(fill, t->X.off, sizeof(int64_t) * nn);
    for (int64_t a = 0; a < nn; ++a)
        for (int64_t e = t->W.off[a]; e < t->W.off[a + 1]; ++e) t->X.idx[fill[t->W.idx[e]]++] = a;
    free(fill);
    return ORC_OK;
}

int orc_atree_build(int64_t n, const double *xy, const double *root, int smax, int lmax, atree **out)
{
    *out = NULL;
    if (n < 1 || smax < 1 || lmax < 0 || lmax > 15 || !(root[2] > 0.0)) return ORC_EINVAL;
    atree *t = calloc(1, sizeof(atree));
    int32_t *ix = malloc(sizeof(int32_t) * n), *iy = malloc(sizeof(int32_t) * n);
    if (!t || !ix || !iy) {
        free(t), free(ix), free(iy);
        return ORC_ENOMEM;
    }
    t->n = n;
    t->lmax = lmax;
    t->smax = smax;
    t->x0 = root[0];
    t->y0 = root[1];
    t->side = root[2];
    t->src = malloc(sizeof(int64_t) * n);
    t->leaf_of = malloc(sizeof(int64_t) * n);
    int rc = (!t->src || !t->leaf_of) ? ORC_ENOMEM : orc_bin(n, xy, lmax, root, ix, iy);
    if (!rc) {
        for (int64_t j = 0; j < n; ++j) t->src[j] = j;
        rc = build_nodes(t, ix, iy);
    }
    free(ix);
    free(iy);
    if (!rc) rc = build_colleagues(t);
    if (!rc) rc = build_lists(t);
    if (rc) {
        orc_atree_free(t);
        return rc;
    }
    *out = t;
    return ORC_OK;
}

/* Sizes: nnodes, leaves, |U|, |V|, |W|, |X| (sums over cells), deepest level, P2P pairs
 * (ordered, the particle with itself excluded). */
void orc_atree_sizes(const atree *t, int64_t *s)
{
    int64_t leaves = 0, deep = 0, pairs = 0;
    for (int64_t k = 0; k < t->nnodes; ++k) {
        const anode *b = &t->nodes[k];
        if (b->level > deep) deep = b->level;
        if (!b->leaf) continue;
        leaves++;
        for (int64_t e = t->U.off[k]; e < t->U.off[k + 1]; ++e) pairs += b->count * t->nodes[t->U.idx[e]].count;
        pairs -= b->count;
    }
    s[0] = t->nnodes;
    s[1] = leaves;
    s[2] = t->U.off[t->nnodes];
    s[3] = t->V.off[t->nnodes];
    s[4] = t->W.off[t->nnodes];
    s[5] = t->X.off[t->nnodes];
    s[6] = deep;
    s[7] = pairs;
}

/* Cells (level, ix, iy, leaf, count, parent) as int64 rows of 6, the leaf of each
 * source, and the four lists (offsets nnodes + 1, indices). */
/* count int64 values; an empty list may have no array at all (memcpy's pointers must not be NULL) */
static void copy_i64(int64_t *dst, const int64_t *src, int64_t count)
{
    if (count > 0) memcpy(dst, src, sizeof(int64_t) * (size_t)count);
}

void orc_atree_export(const atree *t, int64_t *cells, int64_t *leaf_of, int64_t *uo, int64_t *ui, int64_t *vo,
                      int64_t *vi, int64_t *wo, int64_t *wi, int64_t *xo, int64_t *xi)
{
    int64_t nn = t->nnodes;
    for (int64_t k = 0; k < nn; ++k) {
        const anode *b = &t->nodes[k];
        int64_t *r = cells + 6 * k;
        r[0] = b->level, r[1] = b->ix, r[2] = b->iy, r[3] = b->leaf, r[4] = b->count, r[5] = b->parent;
    }
    copy_i64(leaf_of, t->leaf_of, t->n);
    copy_i64(uo, t->U.off, nn + 1);
    copy_i64(vo, t->V.off, nn + 1);
    copy_i64(wo, t->W.off, nn + 1);
    copy_i64(xo, t->X.off, nn + 1);
    copy_i64(ui, t->U.idx, t->U.off[nn]);
    copy_i64(vi, t->V.idx, t->V.off[nn]);
    copy_i64(wi, t->W.idx, t->W.off[nn]);
    copy_i64(xi, t->X.idx, t->X.off[nn]);
}

/* ------------------------------------------------------------------------------ */
/* Evaluation                                                                       */
/* ------------------------------------------------------------------------------ */

/* W_near and W_far at every particle (complex, interleaved), charges q (interleaved).
 *   P2M   a_m(A)  = sum_{j in A} q_j (z_j - z_A)^m                     (leaves, level >= 2)
 *   M2M   a_m(P) += sum_{k<=m} C(m,k) (z_c - z_P)^(m-k) a_k(c)          (cells, level >= 2)
 *   L2L   b_k(B)  = sum_{l>=k} C(l,k) (z_B - z_P)^(l-k) b_l(P)          (parent level >= 2)
 *   M2L   b_l(B) += sum_m a_m(S) (-1)^l C(l+m,m) / (z_B - z_S)^(l+m+1)  (S in V(B))
 *   P2L   b_l(B) += -sum_{j in A} q_j / (z_j - z_B)^(l+1)               (A in X(B))
 *   L2P   W_far  += sum_l b_l(A) (z - z_A)^l                            (A the leaf)
 *   M2P   W_far  += sum_m a_m(D) / (z - z_D)^(m+1)                      (D in W(A))
 *   P2P   W_near += sum_{j in U(A), j != i} q_j g(|z - z_j|^2) / (z - z_j)
 * with g(s) = 1 - exp(-s / (2 sigma^2)). */
/* Multipole and local expansions of every cell of level >= 2 for charges q: the
 * upward pass (P2M, M2M) and the downward pass (L2L, M2L over V, P2L over X) of the
 * evaluation below.  *mp_out, *lo_out: nnodes x p, freed by the caller. */
static int afmm_expansions(const atree *t, const double *xy, const cplx *q, int p, cplx **mp_out, cplx **lo_out)
{
    int64_t nn = t->nnodes;
    cplx *mp = calloc((size_t)nn * p, sizeof(cplx)), *lo = calloc((size_t)nn * p, sizeof(cplx));
    int nb = 2 * p + 1;
    double *binom = calloc((size_t)nb * nb, sizeof(double));
    if (!mp || !lo || !binom) {
        free(mp), free(lo), free(binom);
        return ORC_ENOMEM;
    }
    for (int a = 0; a < nb; ++a) {
        binom[a * nb] = 1.0;
        for (int k = 1; k <= a; ++k) binom[a * nb + k] = binom[(a - 1) * nb + k - 1] + (k < a ? binom[(a - 1) * nb + k] : 0.0);
    }
#define BIN(a, k) binom[(a) * nb + (k)]
    /* upward pass: P2M at leaves, M2M into their ancestors (children follow parents) */
    for (int64_t k = nn - 1; k >= 0; --k) {
        const anode *b = &t->nodes[k];
        if (b->level < 2) continue;
        cplx zc = centre(t, b), *a = mp + k * p;
        if (b->leaf) {
            for (int64_t e = b->first; e < b->first + b->count; ++e) {
                int64_t j = t->src[e];
                cplx d = (xy[2 * j] + I * xy[2 * j + 1]) - zc, pw = 1.0;
                for (int m = 0; m < p; ++m) {
                    a[m] += q[j] * pw;
                    pw *= d;
                }
            }
        } else {
            for (int c = 0; c < 4; ++c) {
                int64_t ch = b->child[c];
                if (ch < 0) continue;
                cplx d = centre(t, &t->nodes[ch]) - zc;
                const cplx *ac = mp + ch * p;
                for (int m = 0; m < p; ++m) {
                    cplx s = 0.0;
                    for (int kk = 0; kk <= m; ++kk) s += BIN(m, kk) * cpow(d, m - kk) * ac[kk];
                    a[m] += s;
                }
            }
        }
    }
    /* downward pass, parents first */
    for (int64_t k = 0; k < nn; ++k) {
        const anode *b = &t->nodes[k];
        if (b->level < 2) continue;
        cplx zb = centre(t, b), *B = lo + k * p;
        if (t->nodes[b->parent].level >= 2) {
            cplx d = zb - centre(t, &t->nodes[b->parent]);
            const cplx *Bp = lo + b->parent * p;
            for (int kk = 0; kk < p; ++kk) {
                cplx s = 0.0;
                for (int l = kk; l < p; ++l) s += BIN(l, kk) * cpow(d, l - kk) * Bp[l];
                B[kk] += s;
            }
        }
        for (int64_t e = t->V.off[k]; e < t->V.off[k + 1]; ++e) {
            int64_t S = t->V.idx[e];
            cplx D = zb - centre(t, &t->nodes[S]);
            const cplx *A = mp + S * p;
            for (int l = 0; l < p; ++l) {
                cplx s = 0.0;
                double sg = (l & 1) ? -1.0 : 1.0;
                for (int m = 0; m < p; ++m) s += A[m] * sg * BIN(l + m, m) / cpow(D, l + m + 1);
                B[l] += s;
            }
        }
        for (int64_t e = t->X.off[k]; e < t->X.off[k + 1]; ++e) {
            const anode *a = &t->nodes[t->X.idx[e]];
            for (int64_t f = a->first; f < a->first + a->count; ++f) {
                int64_t j = t->src[f];
                cplx d = (xy[2 * j] + I * xy[2 * j + 1]) - zb;
                for (int l = 0; l < p; ++l) B[l] -= q[j] / cpow(d, l + 1);
            }
        }
    }
#undef BIN
    free(binom);
    *mp_out = mp;
    *lo_out = lo;
    return ORC_OK;
}

int orc_afmm(int64_t n, const double *xy, const double *q_ri, double sigma, const double *root, int smax,
             int lmax, int p, double *w_near, double *w_far)
{
    if (!(sigma > 0.0) || p < 1 || p > 40) return ORC_EINVAL;
    atree *t;
    int rc = orc_atree_build(n, xy, root, smax, lmax, &t);
    if (rc) return rc;
    const cplx *q = (const cplx *)q_ri;
    cplx *mp, *lo;
    if ((rc = afmm_expansions(t, xy, q, p, &mp, &lo))) {
        orc_atree_free(t);
        return rc;
    }
    /* evaluation at the particles */
    double k2 = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t A = t->leaf_of[i];
        const anode *a = &t->nodes[A];
        cplx z = xy[2 * i] + I * xy[2 * i + 1];
        cplx wf = 0.0, wn = 0.0;
        if (a->level >= 2) {
            cplx d = z - centre(t, a), pw = 1.0;
            const cplx *B = lo + A * p;
            for (int l = 0; l < p; ++l) {
                wf += B[l] * pw;
                pw *= d;
            }
        }
        for (int64_t e = t->W.off[A]; e < t->W.off[A + 1]; ++e) {
            int64_t D = t->W.idx[e];
            cplx d = z - centre(t, &t->nodes[D]);
            const cplx *M = mp + D * p;
            for (int m = 0; m < p; ++m) wf += M[m] / cpow(d, m + 1);
        }
        for (int64_t e = t->U.off[A]; e < t->U.off[A + 1]; ++e) {
            const anode *s = &t->nodes[t->U.idx[e]];
            for (int64_t f = s->first; f < s->first + s->count; ++f) {
                int64_t j = t->src[f];
                cplx dz = z - (xy[2 * j] + I * xy[2 * j + 1]);
                double ss = creal(dz) * creal(dz) + cimag(dz) * cimag(dz);
                if (ss == 0.0) continue;
                wn += q[j] * (-expm1(-ss * k2)) / dz;
            }
        }
        w_near[2 * i] = creal(wn);
        w_near[2 * i + 1] = cimag(wn);
        w_far[2 * i] = creal(wf);
        w_far[2 * i + 1] = cimag(wf);
    }
    free(mp);
    free(lo);
    orc_atree_free(t);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* O7: the adjoint of O6                                                            */
/* ------------------------------------------------------------------------------ */

/* Far field of the expansions (lo, mp) at z in leaf A, and its derivative d/dz:
 *   L2P   sum_l b_l (z - z_A)^l,           derivative sum_{l>=1} l b_l (z - z_A)^(l-1)
 *   M2P   sum_m a_m / (z - z_D)^(m+1),     derivative -sum_m (m+1) a_m / (z - z_D)^(m+2)  (D in W(A)) */
static void far_at(const atree *t, int64_t A, cplx z, const cplx *lo, const cplx *mp, int p, cplx *w, cplx *dw)
{
    const anode *a = &t->nodes[A];
    cplx f = 0.0, df = 0.0;
    if (a->level >= 2) {
        cplx d = z - centre(t, a), pw = 1.0;
        const cplx *B = lo + A * p;
        for (int l = 0; l < p; ++l) {
            f += B[l] * pw;
            if (l + 1 < p) df += (l + 1) * B[l + 1] * pw;
            pw *= d;
        }
    }
    for (int64_t e = t->W.off[A]; e < t->W.off[A + 1]; ++e) {
        int64_t D = t->W.idx[e];
        cplx d = z - centre(t, &t->nodes[D]);
        const cplx *M = mp + D * p;
        for (int m = 0; m < p; ++m) {
            f += M[m] / cpow(d, m + 1);
            df -= (m + 1) * M[m] / cpow(d, m + 2);
        }
    }
    *w = f;
    *dw = df;
}

/* Real-form derivatives of one pair's velocity contribution, (u, v) = G (-dy, dx) f(s),
 * s = dx^2 + dy^2, (dx, dy) = target - source, with respect to the target position:
 * J = [du/dx, du/dy, dv/dx, dv/dy]; at s = 0 (a particle with itself) the smooth limit
 * f(0) = 1/(2 sigma^2). */
static void pair_jac(double dx, double dy, double G, double sigma, double *J)
{
    double kappa = 1.0 / (2.0 * sigma * sigma);
    double s = dx * dx + dy * dy;
    double f = (s == 0.0) ? kappa : orc_reg_f(s, sigma);
    double fp = kappa * kappa * orc_reg_h(kappa * s);
    J[0] = G * (-dy) * fp * 2.0 * dx;
    J[1] = G * (-f - dy * fp * 2.0 * dy);
    J[2] = G * (f + dx * fp * 2.0 * dx);
    J[3] = G * dx * fp * 2.0 * dy;
}

/* Gradient of a loss L(u) through the O6 velocities at the particles, g = (dL/du_i,
 * dL/dv_i), q_i = g_i,u + i g_i,v, c_j = -i Gamma_j / (2 pi):
 *   dgamma  dL/dGamma_j = -Im(Phi_j) / (2 pi), Phi = the same adaptive FMM with charges
 *           q (its operator is antisymmetric: the near kernel is odd over symmetric U
 *           lists, M2L runs over symmetric V lists and M2P over W is the transpose of P2L
 *           over X at equal truncation);
 *   dx_eval the evaluation points moving, the sources fixed: J_i^T g_i with J the
 *           Jacobian of (u, v): the pair Jacobians over U (the particle with itself
 *           included) plus the derivative W' of the far field of the charges c;
 *   dx_src  the sources moving, the evaluation points fixed: minus the pair Jacobians
 *           against the particles whose U holds the source (U is symmetric), and, the far
 *           operator being antisymmetric in both positions, -Re(c_j Phi'_j), Im(c_j Phi'_j)
 *           with Phi' the derivative of the far field of the charges q.
 * Each particle moving both as evaluation point and as source, with the tree held fixed,
 * has gradient dx_eval + dx_src. */
int orc_afmm_grad(int64_t n, const double *xy, const double *gamma, const double *g, double sigma,
                  const double *root, int smax, int lmax, int p, double *dgamma, double *dx_eval, double *dx_src)
{
    if (!(sigma > 0.0) || p < 1 || p > 40) return ORC_EINVAL;
    atree *t;
    int rc = orc_atree_build(n, xy, root, smax, lmax, &t);
    if (rc) return rc;
    cplx *c = malloc(sizeof(cplx) * (n ? n : 1)), *q = malloc(sizeof(cplx) * (n ? n : 1));
    cplx *mpc = NULL, *loc = NULL, *mpq = NULL, *loq = NULL;
    if (!c || !q) rc = ORC_ENOMEM;
    if (!rc) {
        for (int64_t j = 0; j < n; ++j) {
            c[j] = -I * gamma[j] / TWO_PI;
            q[j] = g[2 * j] + I * g[2 * j + 1];
        }
        rc = afmm_expansions(t, xy, c, p, &mpc, &loc);
    }
    if (!rc) rc = afmm_expansions(t, xy, q, p, &mpq, &loq);
    if (rc) {
        free(c), free(q), free(mpc), free(loc), free(mpq), free(loq);
        orc_atree_free(t);
        return rc;
    }
    double k2 = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t A = t->leaf_of[i];
        double x = xy[2 * i], y = xy[2 * i + 1];
        cplx z = x + I * y, wc, dwc, phi, dphi;
        far_at(t, A, z, loc, mpc, p, &wc, &dwc);
        far_at(t, A, z, loq, mpq, p, &phi, &dphi);
        cplx phin = 0.0;
        double J[4] = {0, 0, 0, 0}, Jp[4], sx = 0.0, sy = 0.0;
        for (int64_t e = t->U.off[A]; e < t->U.off[A + 1]; ++e) {
            const anode *s = &t->nodes[t->U.idx[e]];
            for (int64_t f = s->first; f < s->first + s->count; ++f) {
                int64_t j = t->src[f];
                double dx = x - xy[2 * j], dy = y - xy[2 * j + 1], ss = dx * dx + dy * dy;
                if (ss > 0.0) phin += q[j] * (-expm1(-ss * k2)) / (dx + I * dy);
                /* i as evaluation point, j as source */
                pair_jac(dx, dy, gamma[j] / TWO_PI, sigma, Jp);
                for (int k = 0; k < 4; ++k) J[k] += Jp[k];
                /* i as source, j as evaluation point */
                pair_jac(-dx, -dy, gamma[i] / TWO_PI, sigma, Jp);
                sx -= g[2 * j] * Jp[0] + g[2 * j + 1] * Jp[2];
                sy -= g[2 * j] * Jp[1] + g[2 * j + 1] * Jp[3];
            }
        }
        /* far part of the Jacobian: W = u - iv analytic, du/dx = Re W', du/dy = -Im W',
         * dv/dx = -Im W', dv/dy = -Re W' */
        J[0] += creal(dwc);
        J[1] += -cimag(dwc);
        J[2] += -cimag(dwc);
        J[3] += -creal(dwc);
        dgamma[i] = -cimag(phin + phi) / TWO_PI;
        dx_eval[2 * i] = J[0] * g[2 * i] + J[2] * g[2 * i + 1];
        dx_eval[2 * i + 1] = J[1] * g[2 * i] + J[3] * g[2 * i + 1];
        dx_src[2 * i] = sx - creal(c[i] * dphi);
        dx_src[2 * i + 1] = sy + cimag(c[i] * dphi);
    }
    free(c), free(q), free(mpc), free(loc), free(mpq), free(loq);
    orc_atree_free(t);
    return ORC_OK;
}
