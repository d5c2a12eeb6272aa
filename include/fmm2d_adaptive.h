/*
 * fmm2d_adaptive.h -- C ABI of the adaptive-tree variant of the velocity evaluation
 * (libfmm2d.so, gfx950), for uneven particle distributions.
 *
 * The paper's conclusions note that an uneven distribution puts more work in the
 * direct (near-field) sum for the same N, and that with the particles per box held
 * roughly constant the complexity estimates of section "Complexity Estimates" carry
 * over unchanged.  The paper fixes no adaptive scheme; this variant caps the particles
 * per leaf with an adaptive quadtree and evaluates it with the four interaction lists
 * of the adaptive FMM of Carrier, Greengard and Rokhlin (SIAM J. Sci. Stat. Comput. 9,
 * 1988):
 *   tree   the root cell (the bounding square of the particles, or root_box) is split
 *          into its four quadrants while it holds more than max_leaf particles and its
 *          level is below max_depth, recursively; empty cells are dropped.  Particles
 *          are binned as by fmm_build_tree at depth max_depth.
 *   U(A)   leaves adjacent to leaf A (closed squares intersect), A included: the exact
 *          regularised kernel of eq. regB-S2DGau, pair by pair (near field)
 *   V(B)   children of the colleagues (same-level adjacent cells) of B's parent that are
 *          not adjacent to B: multipole-to-local translation (M2L)
 *   W(A)   cells D below a colleague of leaf A, not adjacent to A, whose parent is:
 *          D's multipole expansion evaluated at A's particles (M2P)
 *   X(B)   leaves A with B in W(A): A's particles into B's local expansion (P2L)
 * with P2M at the leaves, M2M and L2L along the tree, and L2P at the leaves, all on
 * cells of level >= 2 and with the singular kernel (the far-field substitution after
 * eq. discBiotS2D), as in fmm2d.h.  With every leaf on level max_depth the lists are
 * those of the uniform tree of depth max_depth and the result equals fmm_velocity's up
 * to rounding.
 *
 * Accuracy: far-field pairs are at least one leaf width apart, so the leaves must stay
 * wider than the blob core (width >= ~8 sigma for FP64 accuracy, ~6 sigma for the
 * mixed form): max_depth plays the role of the uniform tree's depth.
 *
 * The conventions of fmm2d.h apply (device pointers unless "host", (n, 2) row-major
 * FP64 positions and velocities, void* streams, FMM_* status codes with
 * fmm_last_error(), one host thread per handle, inputs never modified).
 */
#ifndef FMM2D_ADAPTIVE_H
#define FMM2D_ADAPTIVE_H

#include <stdint.h>

#include "fmm2d.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_atree fmm_atree;

/* Sizes reported by fmm_atree_info, in this order. */
enum {
    FMM_AT_CELLS = 0,     /* non-empty cells of the tree, the root included */
    FMM_AT_LEAVES = 1,    /* leaves */
    FMM_AT_U = 2,         /* sum over leaves of |U| */
    FMM_AT_V = 3,         /* sum over cells of |V| */
    FMM_AT_W = 4,         /* sum over leaves of |W| */
    FMM_AT_X = 5,         /* sum over cells of |X| (= |W|) */
    FMM_AT_DEEPEST = 6,   /* deepest level of a leaf */
    FMM_AT_PAIRS = 7,     /* ordered near-field pairs: sum over leaves A of n_A sum_{S in U(A)} n_S, minus N */
    FMM_AT_COUNT = 8
};

/* Builds the adaptive tree of n particles xy (device, (n, 2)) on the current device:
 * keys on the finest grid, a stable sort, the cells level by level, the U, V, W, X
 * lists and the near-field plan, all in device kernels on `stream` (which is
 * synchronised to read back sizes).  max_leaf >= 1, 0 <= max_depth <= 15,
 * 1 <= n < 2^31.  root_box (host, {x0, y0, side}) or NULL for the bounding square with
 * side (1 + 2^-20) max(range x, range y).  Returns FMM_EINVAL for bad arguments or a
 * non-finite position, FMM_ERANGE (naming the particle) for a particle outside root_box,
 * FMM_ENOMEM / FMM_EDEVICE on allocation or runtime failures.  *out owns its device
 * memory until fmm_atree_destroy.  The device is synchronised at the end, and the
 * temporaries' memory goes back from the stream-ordered pool to the device. */
int fmm_atree_build(const double *xy, int64_t n, int max_leaf, int max_depth, const double *root_box, void *stream,
                    fmm_atree **out);

/* The same tree built on the host (positions copied down once, the arrays uploaded):
 * the reference that the device build is checked against.  Arguments and results as
 * fmm_atree_build; the two trees are identical array for array. */
int fmm_atree_build_host(const double *xy, int64_t n, int max_leaf, int max_depth, const double *root_box,
                         void *stream, fmm_atree **out);

/* Stages 1-3 again for particles that have moved (the time-stepped form): a new tree
 * for xy built as fmm_atree_build with the max_leaf and max_depth of `prev`, which takes
 * over prev's evaluation workspace (the per-particle arrays as they are, the expansion
 * arrays grown when the new tree has more cells); prev is then destroyed.
 *   prev   tree of the same n on the current device; destroyed on success (after a device
 *          synchronisation), unchanged on error.
 *   xy, n, root_box, stream, out   as fmm_atree_build; n must equal prev's (FMM_EINVAL).
 * FMM_ESTATE for a NULL prev or one in use by another call. */
int fmm_atree_rebuild(fmm_atree *prev, const double *xy, int64_t n, const double *root_box, void *stream,
                      fmm_atree **out);

/* Set an option of the tree.  Two keys of fmm2d.h apply here:
 *  FMM_OPT_NEAR_OCCUPANCY: 1..8 keeps at most that many forward near-field wavefronts per
 *    SIMD resident (by reserving LDS) while the far field runs beside them on side_stream,
 *    0 = no cap, -1 (default) = chosen per call from the tree's predicted far/near time
 *    ratio (mixed precision; no cap in FP64).  A call whose side_stream is main_stream runs
 *    serialised and uncapped.  Results do not depend on it.
 *  FMM_OPT_VALIDATE: 1 checks the circulations (and dL/du of an adjoint call) for NaN and
 *    infinities first, FMM_EINVAL naming the lowest particle index (synchronises
 *    main_stream); 0 (default) no check.
 * fmm_atree_rebuild keeps both.  FMM_EINVAL for another key or a value out of range,
 * FMM_ESTATE for a NULL tree. */
int fmm_atree_set_option(fmm_atree *tree, int key, int64_t value);

/* Host: sizes[FMM_AT_COUNT] (see the enum), root_box[3] (may be NULL). */
/* As fmm_share_workspace (fmm2d.h) for two adaptive trees of the same n on one device
 * (their cell counts may differ: the expansion arrays grow to the larger). */
int fmm_atree_share_workspace(fmm_atree *tree, fmm_atree *from);

int fmm_atree_info(const fmm_atree *tree, int64_t *sizes, double *root_box);

/* Host arrays of n entries, user order: level, ix and iy of each particle's leaf
 * (cell coordinates on the leaf's level).  Any of the three may be NULL. */
int fmm_atree_leaves(const fmm_atree *tree, int32_t *level, int32_t *ix, int32_t *iy);

/* Velocities (u, v) of every particle (device, (n, 2), user order) from circulations
 * gamma (device, n, user order), blob core sigma > 0, p terms (1..32) and precision
 * FMM_FP64 or FMM_MIXED (near-field pairs in FP32 on leaf-relative records, every
 * expansion in FP64).  The far field (P2M, M2M, M2L, P2L, L2L) runs on side_stream (NULL:
 * a stream owned by the tree) concurrently with the near field on main_stream; the call
 * is ordered after prior work on main_stream and its results are complete in stream
 * order on main_stream. */
int fmm_atree_velocity(fmm_atree *tree, const double *gamma, double sigma, int p, int precision,
                       void *main_stream, void *side_stream, double *uv);

/* As fmm_atree_velocity, with the near-field (U) and far-field (V, W, X and the tree
 * translations) parts in separate outputs. */
int fmm_atree_velocity_parts(fmm_atree *tree, const double *gamma, double sigma, int p, int precision,
                             void *main_stream, void *side_stream, double *uv_near, double *uv_far);

/* Adjoint of fmm_atree_velocity for a loss L(u): given dl_duv = dL/du (device, (n, 2)
 * FP64, user order) returns, each optional (NULL skips it; all NULL is a no-op):
 *   dl_dgamma  device, n:      dL/dGamma;
 *   dl_dxeval  device, (n, 2): dL/dx with the particles moving as evaluation points only;
 *   dl_dxsrc   device, (n, 2): dL/dx with the particles moving as sources only;
 *   dl_dxy     device, (n, 2): dl_dxeval + dl_dxsrc, the gradient of a particle moving as a
 *              whole (the tree held fixed: the derivative of the discrete method away from
 *              cell boundaries).  As for the uniform
 * tree (fmm_velocity_backward), the adaptive operator is antisymmetric (odd near kernel
 * over symmetric U lists, M2L over symmetric V lists, M2P over W the transpose of P2L over
 * X), so the circulation gradient is one more evaluation with the complex charges
 * q = dL/du + i dL/dv, and the position gradients combine the near-field sums over U
 * with the derivatives of the far fields of the charges c and q.  Arguments, precision
 * and streams as fmm_atree_velocity; the first call on a tree also makes its adjoint
 * work list (synchronising main_stream). */
int fmm_atree_velocity_backward(fmm_atree *tree, const double *gamma, double sigma, int p, int precision,
                                const double *dl_duv, void *main_stream, void *side_stream, double *dl_dgamma,
                                double *dl_dxeval, double *dl_dxsrc, double *dl_dxy);

/* One explicit stage of the particle transport (section "Test problem", dx/dt = u) over
 * the adaptive tree: x_out = x_base + h u, as fmm_transport_step (fmm2d.h) does for the
 * uniform tree; arguments and errors as there. */
int fmm_atree_transport_step(fmm_atree *tree, const double *gamma, double sigma, int p, int precision,
                             void *main_stream, void *side_stream, const double *x_base, double h, double *x_out);

/* Adjoint of fmm_atree_transport_step with respect to the tree's particles, with the
 * flags FMM_ACC_GAMMA, FMM_ACC_X and FMM_IDENTITY of fmm2d.h, as fmm_transport_vjp does
 * for the uniform tree. */
int fmm_atree_transport_vjp(fmm_atree *tree, const double *gamma, double sigma, int p, int precision,
                            const double *lam, double h, int flags, void *main_stream, void *side_stream,
                            double *dl_dgamma, double *dl_dx);

/* Frees the tree and its device memory (after the device work using it is done; the
 * device is synchronised and the memory goes back from the stream-ordered pool to the
 * device); NULL is ignored. */
void fmm_atree_destroy(fmm_atree *tree);

#ifdef __cplusplus
}
#endif

#endif
