"""CPU oracle for the 2D vortex-particle FMM evaluation -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does: it must not
route through the oracle or fall back to the CPU.

The arithmetic lives in ``fmm_oracle.c`` (plain FP64 C, OpenMP over independent
outputs), written from Knepley, "Removing the Barrier to Scalability in Parallel
FMM" (arXiv:1008.2410).  This wrapper only marshals numpy arrays and, for the
adjoint (O4), combines oracle outputs per the chain rule.

Levels (see the C file's header for the readings of points the paper leaves open):
  direct        O1  exact O(N^2) regularised Biot-Savart sum (eqs. regB-S2DGau,
                    discBiotS2D)
  split_direct  O2  exact kernel on the 3x3 leaf neighbourhood, singular kernel
                    elsewhere (the far-field substitution after eq. discBiotS2D)
  fmm           O3  FMM stages 1-10 (Fig. fmmStages), unscaled textbook operators
  fmm_grad      O4  gradient of L(u) through O3: dL/dGamma and dL/dx_eval
  fmm_src_grad  O5  gradient of L(u) through O3 with respect to the source positions
  direct_grad       gradient of L(u) through O1, every particle moving as source and
                    evaluation point
  afmm          O6  O3 on an adaptive quadtree (cells split above s_max particles, down
                    to l_max) with the U, V, W, X lists of the adaptive FMM
                    (``adaptive_oracle.c``)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("fmm_oracle.c", "adaptive_oracle.c")]
# ORACLE_SANITIZE=1 selects a build with AddressSanitizer and UndefinedBehaviorSanitizer
# (the process must preload gcc's libasan; tests/test_sanitizers.py runs the oracle's pins so)
SANITIZE = os.environ.get("ORACLE_SANITIZE", "") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]
_lib = None

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ERANGE = 0, -1, -2, -4


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc into liboracle.so (in place), or with
    ORACLE_SANITIZE=1 into liboracle_san.so with the sanitizers."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in _SRCS):
        opt = SANITIZE_FLAGS if SANITIZE else ["-O2"]
        cmd = ["gcc", *opt, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", *_SRCS, "-o", _SO + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        Ci = ctypes.c_int
        lib.orc_root_box.argtypes = [I64, P, P]
        lib.orc_root_box.restype = None
        lib.orc_bin.argtypes = [I64, P, Ci, P, P, P]
        lib.orc_direct.argtypes = [I64, P, I64, P, P, D, P]
        lib.orc_direct.restype = None
        lib.orc_split_direct.argtypes = [I64, P, P, P, I64, P, P, P, P, D, P]
        lib.orc_split_direct.restype = None
        lib.orc_fmm.argtypes = [I64, P, P, I64, P, D, Ci, P, Ci, P, P]
        lib.orc_fmm_jacobian.argtypes = [I64, P, P, I64, P, D, Ci, P, Ci, P, P]
        lib.orc_fmm_src_grad.argtypes = [I64, P, P, P, D, Ci, P, Ci, P, P]
        lib.orc_direct_grad.argtypes = [I64, P, P, D, P, P, P]
        lib.orc_direct_grad.restype = None
        lib.orc_leaf_counts.argtypes = [I64, P, Ci, P, P]
        lib.orc_cover_level.argtypes = [Ci, Ci, Ci, Ci, Ci]
        lib.orc_atree_build.argtypes = [I64, P, P, Ci, Ci, ctypes.POINTER(ctypes.c_void_p)]
        lib.orc_atree_free.argtypes = [P]
        lib.orc_atree_free.restype = None
        lib.orc_atree_sizes.argtypes = [P, P]
        lib.orc_atree_sizes.restype = None
        lib.orc_atree_export.argtypes = [P] * 11
        lib.orc_atree_export.restype = None
        lib.orc_afmm.argtypes = [I64, P, P, D, P, Ci, Ci, Ci, P, P]
        lib.orc_afmm_grad.argtypes = [I64, P, P, P, D, P, Ci, Ci, Ci, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(rc: int, what: str):
    if rc != ORC_OK:
        raise OracleError(f"{what} failed with status {rc}")


def root_box(xy) -> tuple:
    xy = _f64(xy, (-1, 2))
    out = np.zeros(3)
    _load().orc_root_box(xy.shape[0], _ptr(xy), _ptr(out))
    return tuple(float(v) for v in out)


def resolve_root(xy, root) -> tuple:
    return root_box(xy) if root is None else tuple(float(v) for v in root)


def bin_leaves(xy, depth: int, root=None):
    """Leaf coordinates (ix, iy) of each point (stage 2)."""
    xy = _f64(xy, (-1, 2))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    ix = np.zeros(xy.shape[0], dtype=np.int32)
    iy = np.zeros(xy.shape[0], dtype=np.int32)
    _check(_load().orc_bin(xy.shape[0], _ptr(xy), depth, _ptr(r), _ptr(ix), _ptr(iy)), "orc_bin")
    return ix, iy


def leaf_counts(xy, depth: int, root=None) -> np.ndarray:
    """Particles per leaf, shape (2^L, 2^L) indexed [iy, ix]."""
    xy = _f64(xy, (-1, 2))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    c = np.zeros((1 << depth) * (1 << depth), dtype=np.int64)
    _check(_load().orc_leaf_counts(xy.shape[0], _ptr(xy), depth, _ptr(r), _ptr(c)), "orc_leaf_counts")
    return c.reshape(1 << depth, 1 << depth)


def cover_level(depth: int, t: tuple, s: tuple) -> int:
    return int(_load().orc_cover_level(depth, t[0], t[1], s[0], s[1]))


def direct(xy, gamma, sigma: float, targets=None) -> np.ndarray:
    """O1: velocities (N_t, 2) at ``targets`` (default: the particles themselves)."""
    xy = _f64(xy, (-1, 2))
    g = _f64(gamma, (-1,))
    t = xy if targets is None else _f64(targets, (-1, 2))
    uv = np.zeros((t.shape[0], 2))
    _load().orc_direct(t.shape[0], _ptr(t), xy.shape[0], _ptr(xy), _ptr(g), float(sigma), _ptr(uv))
    return uv


def split_direct(xy, gamma, sigma: float, depth: int, root=None, targets=None) -> np.ndarray:
    """O2: exact kernel for sources in the target leaf's 3x3 neighbourhood, singular kernel
    (1/|z|^2 form) for all other sources."""
    xy = _f64(xy, (-1, 2))
    g = _f64(gamma, (-1,))
    r = resolve_root(xy, root)
    t = xy if targets is None else _f64(targets, (-1, 2))
    six, siy = bin_leaves(xy, depth, r)
    tix, tiy = bin_leaves(t, depth, r)
    uv = np.zeros((t.shape[0], 2))
    _load().orc_split_direct(t.shape[0], _ptr(t), _ptr(tix), _ptr(tiy), xy.shape[0], _ptr(xy),
                             _ptr(six), _ptr(siy), _ptr(g), float(sigma), _ptr(uv))
    return uv


def charges(gamma) -> np.ndarray:
    """Complex charges c_j = -i Gamma_j / (2 pi) (the factor of the multipole coefficients)."""
    return (-1j / (2.0 * math.pi)) * np.asarray(gamma, dtype=np.float64)


def fmm(xy, q, sigma: float, depth: int, p: int, root=None, targets=None):
    """O3 with complex charges q: returns (W_near, W_far), complex arrays of the conjugate
    velocity W = u - i v at the targets (default: the particles)."""
    xy = _f64(xy, (-1, 2))
    qc = np.ascontiguousarray(q, dtype=np.complex128)
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    t = xy if targets is None else _f64(targets, (-1, 2))
    wn = np.zeros(t.shape[0], dtype=np.complex128)
    wf = np.zeros(t.shape[0], dtype=np.complex128)
    _check(_load().orc_fmm(xy.shape[0], _ptr(xy), _ptr(qc), t.shape[0], _ptr(t), float(sigma), depth,
                           _ptr(r), p, _ptr(wn), _ptr(wf)), "orc_fmm")
    return wn, wf


def w_to_uv(w: np.ndarray) -> np.ndarray:
    """Stage 10 output convention: (u, v) = (Re W, -Im W)."""
    return np.stack([w.real, -w.imag], axis=1)


def fmm_velocity(xy, gamma, sigma: float, depth: int, p: int, root=None, targets=None,
                 parts: bool = False):
    """O3 velocities (N_t, 2): stage 10 sums the near and far parts."""
    wn, wf = fmm(xy, charges(gamma), sigma, depth, p, root, targets)
    if parts:
        return w_to_uv(wn), w_to_uv(wf)
    return w_to_uv(wn + wf)


def fmm_jacobian(xy, gamma, sigma: float, depth: int, p: int, root=None, targets=None):
    """d(u, v)/d(x, y) of the O3 field at the targets with the sources fixed, as
    (J_near, J_far), each (N_t, 2, 2) with J[i] = [[du/dx, du/dy], [dv/dx, dv/dy]]."""
    xy = _f64(xy, (-1, 2))
    g = _f64(gamma, (-1,))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    t = xy if targets is None else _f64(targets, (-1, 2))
    jn = np.zeros((t.shape[0], 4))
    jf = np.zeros((t.shape[0], 4))
    _check(_load().orc_fmm_jacobian(xy.shape[0], _ptr(xy), _ptr(g), t.shape[0], _ptr(t), float(sigma),
                                    depth, _ptr(r), p, _ptr(jn), _ptr(jf)), "orc_fmm_jacobian")
    return jn.reshape(-1, 2, 2), jf.reshape(-1, 2, 2)


def fmm_grad(xy, gamma, sigma: float, depth: int, p: int, dl_duv, root=None):
    """O4: gradient of a loss L(u) through the O3 velocities at the particles.

    dl_duv (N, 2) holds dL/du_i, dL/dv_i.  With q_i = dL/du_i + i dL/dv_i, the FMM
    operator A (W = A c) is antisymmetric (A_ij = -A_ji: symmetric neighbour and
    interaction lists, square truncation l, m < p, exact M2M/L2L), so the transpose
    pass is the same FMM run with charges q, and
        dL/dGamma_j = Re( sum_i q_i A_ij (-i/2pi) ) = -Im( (A q)_j ) / (2 pi).
    dL/dx_eval_i = J_i^T dL/duv_i with J the Jacobian of (u, v) at the evaluation
    point (sources held fixed).
    Returns (dL/dGamma (N,), dL/dx_eval (N, 2))."""
    g = np.asarray(dl_duv, dtype=np.float64).reshape(-1, 2)
    q = g[:, 0] + 1j * g[:, 1]
    wn, wf = fmm(xy, q, sigma, depth, p, root)
    dgamma = -(wn + wf).imag / (2.0 * math.pi)
    jn, jf = fmm_jacobian(xy, gamma, sigma, depth, p, root)
    jac = jn + jf
    dx = np.einsum("nij,ni->nj", jac, g)
    return dgamma, dx


def fmm_src_grad(xy, gamma, sigma: float, depth: int, p: int, dl_duv, root=None):
    """O5: gradient of L(u) through the O3 velocities at the particles with respect to
    the source positions, evaluation points held fixed, as (near part, far part), each
    (N, 2).  Near: minus the pair Jacobians summed over the particles whose
    neighbourhood holds the source.  Far: -Re(c_j Phi'_j), Im(c_j Phi'_j) with Phi' the
    derivative of the local expansion of the FMM run with charges q = dL/du + i dL/dv
    (the far operator is antisymmetric)."""
    xy = _f64(xy, (-1, 2))
    gm = _f64(gamma, (-1,))
    g = _f64(dl_duv, (-1, 2))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    dn = np.zeros_like(xy)
    df = np.zeros_like(xy)
    _check(_load().orc_fmm_src_grad(xy.shape[0], _ptr(xy), _ptr(gm), _ptr(g), float(sigma), depth, _ptr(r), p,
                                    _ptr(dn), _ptr(df)), "orc_fmm_src_grad")
    return dn, df


def fmm_grad_full(xy, gamma, sigma: float, depth: int, p: int, dl_duv, root=None):
    """O4 + O5: (dL/dGamma (N,), dL/dx_eval (N, 2), dL/dx_src (N, 2)).  The gradient
    with respect to the particle positions, each particle moving as evaluation point and
    as source (the tree's cells held fixed), is dL/dx_eval + dL/dx_src."""
    dgamma, dx_eval = fmm_grad(xy, gamma, sigma, depth, p, dl_duv, root)
    dn, df = fmm_src_grad(xy, gamma, sigma, depth, p, dl_duv, root)
    return dgamma, dx_eval, dn + df


def direct_grad(xy, gamma, sigma: float, dl_duv):
    """Gradient of L(u) through the O1 velocities: (dL/dGamma (N,), dL/dx (N, 2)), each
    particle moving both as evaluation point and as source."""
    xy = _f64(xy, (-1, 2))
    gm = _f64(gamma, (-1,))
    g = _f64(dl_duv, (-1, 2))
    dg = np.zeros(xy.shape[0])
    dx = np.zeros_like(xy)
    _load().orc_direct_grad(xy.shape[0], _ptr(xy), _ptr(gm), float(sigma), _ptr(g), _ptr(dg), _ptr(dx))
    return dg, dx


def pair_count(counts: np.ndarray) -> int:
    """Ordered near-field pairs (j != i) summed over targets: sum_T n_T sum_{S in N(T)} n_S - N."""
    c = np.asarray(counts, dtype=np.int64)
    pad = np.pad(c, 1)
    n1 = c.shape[0]
    nb = sum(pad[1 + a:1 + a + n1, 1 + b:1 + b + n1] for a in (-1, 0, 1) for b in (-1, 0, 1))
    return int((c * nb).sum() - c.sum())


# --- O6: the adaptive tree -------------------------------------------------------------

ATREE_SIZE_KEYS = ("cells", "leaves", "u", "v", "w", "x", "deepest", "p2p_pairs")


def adaptive_tree(xy, smax: int, lmax: int, root=None) -> dict:
    """The adaptive tree of O6 and its lists: ``cells`` (K, 6) int64 rows (level, ix, iy,
    leaf, count, parent), ``leaf_of`` (N,), the lists ``U``, ``V``, ``W``, ``X`` as
    (offsets (K+1,), indices), and the sizes of ``ATREE_SIZE_KEYS``."""
    xy = _f64(xy, (-1, 2))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    lib = _load()
    h = ctypes.c_void_p()
    _check(lib.orc_atree_build(xy.shape[0], _ptr(xy), _ptr(r), int(smax), int(lmax), ctypes.byref(h)),
           "orc_atree_build")
    try:
        s = np.zeros(8, dtype=np.int64)
        lib.orc_atree_sizes(h, _ptr(s))
        k = int(s[0])
        cells = np.zeros((k, 6), dtype=np.int64)
        leaf_of = np.zeros(xy.shape[0], dtype=np.int64)
        offs = [np.zeros(k + 1, dtype=np.int64) for _ in range(4)]
        idxs = [np.zeros(max(int(s[2 + i]), 1), dtype=np.int64) for i in range(4)]
        lib.orc_atree_export(h, _ptr(cells), _ptr(leaf_of), _ptr(offs[0]), _ptr(idxs[0]), _ptr(offs[1]),
                             _ptr(idxs[1]), _ptr(offs[2]), _ptr(idxs[2]), _ptr(offs[3]), _ptr(idxs[3]))
    finally:
        lib.orc_atree_free(h)
    out = {"cells": cells, "leaf_of": leaf_of, "root": tuple(float(v) for v in r),
           "sizes": {key: int(v) for key, v in zip(ATREE_SIZE_KEYS, s)}}
    for name, o, ix in zip("UVWX", offs, idxs):
        out[name] = (o, ix[:int(o[-1])])
    return out


def afmm(xy, q, sigma: float, smax: int, lmax: int, p: int, root=None):
    """O6 with complex charges q at the particles: (W_near, W_far), complex."""
    xy = _f64(xy, (-1, 2))
    qc = np.ascontiguousarray(q, dtype=np.complex128)
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    wn = np.zeros(xy.shape[0], dtype=np.complex128)
    wf = np.zeros(xy.shape[0], dtype=np.complex128)
    _check(_load().orc_afmm(xy.shape[0], _ptr(xy), _ptr(qc), float(sigma), _ptr(r), int(smax), int(lmax), int(p),
                            _ptr(wn), _ptr(wf)), "orc_afmm")
    return wn, wf


def afmm_velocity(xy, gamma, sigma: float, smax: int, lmax: int, p: int, root=None, parts: bool = False):
    """O6 velocities (N, 2) at the particles (near + far, or both parts)."""
    wn, wf = afmm(xy, charges(gamma), sigma, smax, lmax, p, root)
    if parts:
        return w_to_uv(wn), w_to_uv(wf)
    return w_to_uv(wn + wf)


def afmm_grad(xy, gamma, sigma: float, smax: int, lmax: int, p: int, dl_duv, root=None):
    """O7: gradient of a loss L(u) through the O6 velocities at the particles, as O4 + O5
    for the uniform tree: (dL/dGamma (N,), dL/dx_eval (N, 2), dL/dx_src (N, 2)); the
    particles moving as evaluation points and as sources (tree held fixed) have gradient
    dL/dx_eval + dL/dx_src."""
    xy = _f64(xy, (-1, 2))
    gm = _f64(gamma, (-1,))
    g = _f64(dl_duv, (-1, 2))
    r = np.asarray(resolve_root(xy, root), dtype=np.float64)
    dg = np.zeros(xy.shape[0])
    dxe = np.zeros_like(xy)
    dxs = np.zeros_like(xy)
    _check(_load().orc_afmm_grad(xy.shape[0], _ptr(xy), _ptr(gm), _ptr(g), float(sigma), _ptr(r), int(smax),
                                 int(lmax), int(p), _ptr(dg), _ptr(dxe), _ptr(dxs)), "orc_afmm_grad")
    return dg, dxe, dxs
