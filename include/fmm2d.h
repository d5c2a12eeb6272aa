/*
 * fmm2d.h -- C ABI of the MI355X (gfx950) evaluation phase of the 2D vortex-particle
 * fast multipole method of M. G. Knepley, "Removing the Barrier to Scalability in
 * Parallel FMM" (arXiv:1008.2410).
 *
 * Problem (section "Test problem"): N vortex particles at z_j = x_j + i y_j carry
 * circulations Gamma_j and Gaussian blobs of core sigma (eqs. omega, zeta).  The
 * velocity at each particle is
 *     u(z_i) = sum_{j != i} Gamma_j K_sigma(z_i - z_j)                 (eq. discBiotS2D)
 *     K_sigma(z) = (1/(2 pi |z|^2)) (-z_y, z_x) (1 - exp(-|z|^2/(2 sigma^2)))
 *                                                                      (eq. regB-S2DGau)
 * evaluated by the FMM on a uniform quadtree: the exact kernel on each leaf's 3x3
 * leaf neighbourhood (near field, stage 9 of Fig. fmmStages) and p-term expansions
 * of the singular 1/|z|^2 kernel elsewhere (far field, stages 4-8; the substitution
 * is stated after eq. discBiotS2D).  Stage 10 sums the two.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers (HIP global memory on the current
 *    device) owned by the caller, unless a comment says "host".  Positions are
 *    (n, 2) row-major FP64 (x0, y0, x1, y1, ...); velocities likewise (u, v).
 *  - Streams are hipStream_t passed as void*; NULL means the null stream.  Work is
 *    enqueued asynchronously; no call synchronises the host unless stated.
 *  - Every entry point returns FMM_OK or a negative status and never aborts.  On
 *    failure fmm_last_error() returns a message (thread-local) and the outputs are
 *    unspecified but never partly scattered: the user-order outputs are written by
 *    the last kernel of a call.
 *  - A tree handle may be used by one host thread at a time; a concurrent call on
 *    the same handle returns FMM_ESTATE.  Different handles are independent.
 *  - Calls on one tree share its device workspace: consecutive calls must be ordered
 *    on the device (the same main stream, or synchronised in between).
 *  - Inputs are never modified.
 */
#ifndef FMM2D_H
#define FMM2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_tree fmm_tree;

enum {
    FMM_OK = 0,
    FMM_EINVAL = -1,  /* bad argument: null pointer, n < 1, depth or p out of range, bad sigma */
    FMM_ENOMEM = -2,  /* device or host allocation failed */
    FMM_EDEVICE = -3, /* a HIP runtime call or kernel launch failed */
    FMM_ERANGE = -4,  /* a particle lies outside the root cell */
    FMM_ESTATE = -5   /* handle busy in another thread, or invalid handle */
};

/* Arithmetic of fmm_velocity / fmm_velocity_backward. */
enum {
    FMM_FP64 = 0,  /* every stage in FP64 */
    FMM_MIXED = 1  /* P2P, P2M, fine-level M2M/M2L/L2L and L2P in FP32 on radius-scaled
                      coefficients; coarse-level M2M/M2L/L2L and the near+far sum in FP64 */
};

/* Options for fmm_set_option. */
enum {
    FMM_OPT_SCHEDULE = 1,     /* 0: far field on a second stream, concurrent with P2P;
                                 1: everything serialised on the main stream;
                                 2 (default): per call from the tree's predicted far/near time
                                 ratio: serialised in the mixed form when the far field is
                                 predicted more than 2.5 times the near field (where overlapping
                                 measured slower on one GPU), concurrent otherwise and in FP64 */
    FMM_OPT_COARSE_LEVEL = 2, /* L_c: levels <= L_c of the up/down sweeps run in FP64 on the far-
                                 field stream (default 3, range 1..depth); those of them with at
                                 most 256 cells (levels <= 4) in one single-workgroup kernel, the
                                 others as wide launches */
    FMM_OPT_TIMING = 3,       /* 1: record HIP events around each stage of every call for
                                 fmm_get_timings (default 0) */
                              /* keys 4 and 5 (a persistent near-field grid, a cap on the far-field
                                 grids) were measured slower than the default and are withdrawn:
                                 FMM_EINVAL */
    FMM_OPT_NEAR_MUTUAL = 6,  /* 1 (default): pairs of neighbouring dense leaves are evaluated once
                                 for both particles (the kernel is odd), the rest from the target
                                 end; 0: every pair from the target end.  Results agree to rounding. */
    FMM_OPT_DENSE_LEAF = 7,   /* particles that make a leaf dense for FMM_OPT_NEAR_MUTUAL (default 32) */
    FMM_OPT_NEAR_OCCUPANCY = 8, /* 1..8: in a concurrent call the forward near-field kernel keeps at
                                  most this many wavefronts per SIMD resident (by reserving LDS),
                                  leaving room for the far field beside it; 0 = no cap; -1 (default)
                                  = per call from the tree (mixed: 3 for leaves of more than 2500
                                  near-field pairs per particle with at least 64K near-field work
                                  entries, else by the predicted far/near time ratio 6, 5, 4 or
                                  none; FP64: 2 or none) */
    FMM_OPT_VALIDATE = 9      /* 1: every evaluation first checks the circulations (and an adjoint
                                 call its dL/du) for NaN and infinities on the device and returns
                                 FMM_EINVAL, naming the lowest particle index, before any other
                                 work; the check synchronises main_stream.  0 (default): no check
                                 (a non-finite input then gives non-finite outputs) */
};

/* Stage indices of fmm_get_timings. */
enum {
    FMM_T_PACK = 0,     /* a0: gather circulations into Morton order */
    FMM_T_FAR = 1,      /* stages 4-7: P2M, M2M, M2L, L2L (side stream) */
    FMM_T_P2P = 2,      /* stage 9: near-field direct sum (main stream) */
    FMM_T_FINAL = 3,    /* stages 8 + 10: L2P, near+far sum, scatter to user order */
    FMM_T_TOTAL = 4,    /* whole call, first to last kernel */
    FMM_T_COUNT = 5
};

/*
 * Stages 1-3 of Fig. fmmStages: tree construction, particle binning, interaction
 * lists.  Builds a uniform quadtree of depth L (4^L leaves, section "Complexity
 * Estimates") over n particles and keeps everything later calls need.
 *   xy        device, (n, 2) FP64 positions in user order; read once.
 *   n         1 <= n < 2^31.
 *   depth     1 <= depth <= 12.
 *   root_box  host, {x0, y0, side} of the root cell, or NULL for the bounding square
 *             x0 = min x, y0 = min y, side = max(range x, range y) * (1 + 2^-20).
 *   stream    stream on which xy is valid.
 *   out       receives the handle; free it with fmm_destroy_tree.
 * Leaf of a particle: (min(floor((x - x0)/w), 2^L - 1), same for y), w = side/2^L;
 * a particle outside [x0, x0 + side]^2 gives FMM_ERANGE, a non-finite one FMM_EINVAL
 * (the message names the lowest offending index).
 * The build runs on the device (binning, a stable radix sort by leaf and sub-leaf
 * Morton key, leaf offsets, cell lists, work lists) and synchronises `stream`; then, the
 * device synchronised, its temporaries' memory goes back from the stream-ordered pool to
 * the device.  The tree owns its device buffers, and workspace for each (p, precision)
 * is allocated on first use and kept until fmm_destroy_tree.
 */
int fmm_build_tree(const double *xy, int64_t n, int depth, const double *root_box, void *stream,
                   fmm_tree **out);

/* The same tree built on the host (positions copied down once, the arrays uploaded):
 * the reference that the device build is checked against.  Arguments and results as
 * fmm_build_tree; the two trees are identical array for array. */
int fmm_build_tree_host(const double *xy, int64_t n, int depth, const double *root_box, void *stream,
                        fmm_tree **out);

/* Stages 1-3 again for particles that have moved (section "Test problem": the particles
 * are carried by the flow, so every time step needs a tree for the new positions).
 * Builds a new tree for xy as fmm_build_tree does, with the depth and the FMM_OPT_*
 * options of `prev`, and hands prev's evaluation workspace to it; prev is then destroyed.
 * A time-stepping loop that rebuilds this way allocates the workspace once instead of
 * once per tree.  The rebuild holds one tree's arrays at a time: it synchronises the
 * device, its temporaries use the workspace's per-call region (so no call on a tree
 * sharing that workspace may run meanwhile), and prev's arrays are released as soon as
 * the positions have passed their checks, before the new tree's are allocated.
 *   prev      tree of the same n on the current device, or one left without arrays by a
 *             failed rebuild; destroyed on success.  On an error found before the build
 *             starts (NULL or busy prev, other n or device) or by the position checks
 *             (FMM_ERANGE, FMM_EINVAL) prev is unchanged.  On a later error (FMM_ENOMEM,
 *             FMM_EDEVICE) prev keeps its workspace and options but has no arrays: every
 *             call on it but fmm_rebuild_tree and fmm_destroy_tree then returns FMM_ESTATE.
 *   xy, n, root_box, stream, out   as fmm_build_tree; n must equal prev's (FMM_EINVAL).
 * FMM_ESTATE for a NULL prev or one in use by another call. */
int fmm_rebuild_tree(fmm_tree *prev, const double *xy, int64_t n, const double *root_box, void *stream,
                     fmm_tree **out);

/* Let `tree` use the evaluation workspace of `from` (its own is freed) until either is
 * destroyed or rebuilt; the memory is freed with the last tree using it.  For trees that
 * are evaluated one after the other, such as the two trees of each step of a
 * time-stepping adjoint (the positions and the midpoint of the step), this halves the
 * memory of the workspace (the per-particle arrays and the expansions).  A call on either
 * tree first clears the multipoles when the other tree made the previous call.  Calls on
 * the two trees must be ordered on the device (the same main stream).  FMM_EINVAL unless
 * both have the same n, depth and device; FMM_ESTATE for a NULL or busy handle.
 * Synchronises the device. */
int fmm_share_workspace(fmm_tree *tree, fmm_tree *from);

/* Host-side facts about a tree (any pointer may be NULL):
 *   n, depth, root_box[3] (host);
 *   p2p_pairs       ordered near-field pairs sum_T n_T sum_{S in N(T)} n_S - n, the pair
 *                   count of the direct-work formula of section "Complexity Estimates";
 *   m2l_pairs       (target, source) cell pairs of the interaction lists, levels 2..L,
 *                   with both cells non-empty;
 *   nonempty_leaves, max_leaf  occupancy of the leaf level. */
int fmm_tree_info(const fmm_tree *tree, int64_t *n, int *depth, double *root_box, int64_t *p2p_pairs,
                  int64_t *m2l_pairs, int64_t *nonempty_leaves, int64_t *max_leaf);

/* Non-empty cells per level: nonempty[l] for l = 0 .. min(depth, max_levels - 1)
 * (host array of max_levels entries; entries past depth are set to 0). */
int fmm_tree_levels(const fmm_tree *tree, int64_t *nonempty, int max_levels);

/* Sorted order of the tree.  perm: device, n int64, perm[k] = user index of the k-th
 * particle; particles are grouped by leaf in leaf-Morton order and, inside a leaf,
 * ordered by the Morton index of their cell in a 64 x 64 grid over the leaf (ties by
 * user index).  leaf: device, n int32 or NULL, leaf[k] = Morton index of that
 * particle's leaf (x in the even bits). */
int fmm_tree_permutation(const fmm_tree *tree, int64_t *perm, int32_t *leaf, void *stream);

/*
 * Stages 4-10: velocity of every particle.
 *   gamma       device, n FP64 circulations (user order).
 *   sigma       blob core, finite, > 0.
 *   p           expansion terms, 1 <= p <= 32 (coefficients m = 0..p-1).
 *   precision   FMM_FP64 or FMM_MIXED.
 *   main_stream P2P, pack and the final sum run here; the call is ordered after prior
 *               work on it, and later work on it sees the result.
 *   side_stream far-field stream (NULL: the tree's own non-blocking stream); the
 *               library forks it from main_stream and joins it back with events.
 *   uv          device, (n, 2) FP64 velocities (u, v) in user order.
 */
int fmm_velocity(fmm_tree *tree, const double *gamma, double sigma, int p, int precision, void *main_stream,
                 void *side_stream, double *uv);

/*
 * fmm_velocity for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same stages and kernels,
 * the same results bit for bit, with every per-call array (records, near-field sums and
 * slots, multipoles and locals of all levels) in the library's static device workspace of
 * 128 MiB, a file-scope array each device holds from the library's first use until the
 * process ends.  The call allocates nothing and creates no event: FMM_OPT_TIMING is not
 * applied (FMM_OPT_VALIDATE is, and synchronises main_stream).
 *   Preconditions: the tree (built by fmm_build_tree) and the expansion tables of p on the
 *   device, which any earlier allocating evaluation with this p makes (FMM_ESTATE if not).
 *   Size limit: an evaluation needs about n (104 bytes mixed, 192 bytes FP64 with the mutual
 *   near field; 32 / 48 without it) + 22 p 4^depth (mixed) or 43 p 4^depth (FP64) bytes;
 *   beyond 128 MiB the call returns FMM_EINVAL, naming both sizes, before any work.
 *   Sharing: all calls of the process on one device use the same workspace; calls that
 *   overlap on one device race and must be ordered (one stream, or synchronised), as
 *   calls on one tree must be.  The multipoles are cleared by each call.
 * Arguments as fmm_velocity.
 */
int fmm_velocity_noalloc(fmm_tree *tree, const double *gamma, double sigma, int p, int precision,
                         void *main_stream, void *side_stream, double *uv);

/* As fmm_velocity, but the near field (stage 9) and far field (stage 8) velocities are
 * written separately, each (n, 2) FP64 in user order, so that each stage can be checked. */
int fmm_velocity_parts(fmm_tree *tree, const double *gamma, double sigma, int p, int precision,
                       void *main_stream, void *side_stream, double *uv_near, double *uv_far);

/*
 * Adjoint of fmm_velocity for a loss L(u): given dL/du (device, (n, 2) FP64, user
 * order) returns (each output device memory in user order, written in full)
 *   dl_dgamma  device, n FP64:  dL/dGamma_j = -Im((A q)_j)/(2 pi), q_i = dL/du_i + i dL/dv_i,
 *              where A is the FMM operator (W = u - iv = A c, c_j = -i Gamma_j/(2 pi)),
 *              exactly antisymmetric for square truncation, so A^T q = -A q is one
 *              more FMM pass with complex charges q;
 *   dl_dxeval  device, (n, 2) FP64: derivative with respect to the evaluation
 *              positions with the sources held fixed: near part from the derivative of
 *              eq. regB-S2DGau (the particle's own blob included, slope 1/(4 pi sigma^2)),
 *              far part from the derivative of the local expansion;
 *   dl_dxsrc   device, (n, 2) FP64: derivative with respect to the source positions with
 *              the evaluation points held fixed: near part minus the pair derivatives
 *              seen from the sources (own blob included, with the opposite sign), far part
 *              -Re(c_j Phi'_j), Im(c_j Phi'_j), Phi' the derivative of the q-field's local
 *              expansion;
 *   dl_dxy     device, (n, 2) FP64: dl_dxeval + dl_dxsrc, the derivative for particles
 *              moving as a whole (source and evaluation point, the tree's cells held fixed).
 * Any output may be NULL to skip it.  Other arguments as fmm_velocity.  The paper has no
 * backward pass; this is the transpose of the discrete operator defined by stages 4-10.
 */
int fmm_velocity_backward(fmm_tree *tree, const double *gamma, double sigma, int p, int precision,
                          const double *dl_duv, void *main_stream, void *side_stream, double *dl_dgamma,
                          double *dl_dxeval, double *dl_dxsrc, double *dl_dxy);

/*
 * One explicit stage of the particle transport of section "Test problem" (the particles
 * move with the velocity they induce, dx/dt = u, circulations carried unchanged):
 *   x_out = x_base + h u,   u = the velocity of every particle of the tree (stages 4-10),
 * written in user order by the last kernel of the call; x_base (device, (n, 2) FP64, user
 * order) may be the tree's own positions or any other array, and x_out may equal x_base.
 * Midpoint RK2 is two calls: x_half = x + (dt/2) u(x) over a tree of x, then
 * x_next = x + dt u(x_half) over a tree of x_half.  Other arguments as fmm_velocity;
 * FMM_EINVAL for a NULL array or a non-finite h.
 */
int fmm_transport_step(fmm_tree *tree, const double *gamma, double sigma, int p, int precision,
                       void *main_stream, void *side_stream, const double *x_base, double h, double *x_out);

/* Flags of fmm_transport_vjp. */
enum {
    FMM_ACC_GAMMA = 1, /* dl_dgamma is added to instead of written */
    FMM_ACC_X = 2,     /* dl_dx is added to instead of written */
    FMM_IDENTITY = 4   /* dl_dx includes lam itself: the stage's x_base is the tree's positions */
};

/*
 * Adjoint of fmm_transport_step with respect to the tree's particles: given
 * lam = dL/dx_out (device, (n, 2) FP64, user order),
 *   dl_dgamma  (n)     h dL/dGamma through u (as fmm_velocity_backward with dL/du = h lam);
 *   dl_dx      (n, 2)  h (dl_dxeval + dl_dxsrc) for dL/du = h lam, plus lam with
 *                      FMM_IDENTITY (the derivative through x_base = x);
 * each written, or added to with FMM_ACC_GAMMA / FMM_ACC_X (a NULL output is skipped).
 * The backward step of midpoint RK2 from per-step checkpoints is two calls with no other
 * arithmetic: lam_half = vjp(tree of x_half, lam, h = dt, flags FMM_ACC_GAMMA) and
 * lam = vjp(tree of x, lam_half, h = dt/2, flags FMM_ACC_GAMMA | FMM_ACC_X | FMM_IDENTITY),
 * since x_next = x + dt u(x_half) and x_half = x + (dt/2) u(x).  FMM_EINVAL for a NULL lam,
 * a non-finite h or an unknown flag; other arguments as fmm_velocity.
 */
int fmm_transport_vjp(fmm_tree *tree, const double *gamma, double sigma, int p, int precision, const double *lam,
                      double h, int flags, void *main_stream, void *side_stream, double *dl_dgamma, double *dl_dx);

/* The near-field plan (stage 9) in force (any pointer may be NULL):
 *   mutual_items  wavefront items of the mutual form (0 when it is off or finds no
 *                 pair of dense leaves);
 *   mutual_pairs  ordered pairs (i != j) those items evaluate, each unordered pair once
 *                 for both particles;
 *   target_units  work units of the target-centric form, which covers the other pairs. */
int fmm_near_plan_info(const fmm_tree *tree, int64_t *mutual_items, int64_t *mutual_pairs, int64_t *target_units);

/* Set an FMM_OPT_* option on a tree.  FMM_EINVAL for an unknown key or bad value. */
int fmm_set_option(fmm_tree *tree, int key, int64_t value);

/* Per-stage device time (milliseconds, from HIP events on the stream each stage runs
 * on) summed over the calls made since the last fmm_get_timings with FMM_OPT_TIMING
 * on.  ms: host, FMM_T_COUNT doubles; calls: host, receives the number of calls.
 * Synchronises the recorded events; resets the sums. */
int fmm_get_timings(fmm_tree *tree, double *ms, int64_t *calls);

/* Event times of the most recent call made with FMM_OPT_TIMING on and not yet summed by
 * fmm_get_timings (that call is kept for it), in milliseconds after the call's first event:
 *   ms[0] stage-in start (0), ms[1] pack end (main stream), ms[2] far-field chain start and
 *   ms[3] its end (side stream, or the main stream when serialised), ms[4] P2P start and
 *   ms[5] its end (main stream), ms[6] final stage start, ms[7] its end.
 * A far chain running concurrently with P2P (the two-stream schedule of section
 * "Concurrency", no edge between stages 4-8 and 9 in Fig. fmmStages) shows ms[2] < ms[5]
 * and ms[4] < ms[3].  ms: host, count doubles (entries past 7 are set to 0).  Synchronises
 * the recorded events.  FMM_ESTATE when no such call is pending. */
int fmm_get_timeline(fmm_tree *tree, double *ms, int count);

/* Free a tree and its device memory (synchronises the device first); the memory goes
 * back from the stream-ordered pool to the device.  NULL is a no-op. */
void fmm_destroy_tree(fmm_tree *tree);

/* Message for the last failed call on this host thread ("" if none). */
const char *fmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FMM2D_H */
