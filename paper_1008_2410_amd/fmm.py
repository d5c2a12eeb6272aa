"""Python binding of the gfx950 FMM library: torch tensors in, torch tensors out.

Every step of the evaluation runs in the HIP kernels of libfmm2d.so; this module
only checks tensor shapes and devices, allocates outputs with torch and passes
pointers and the current HIP stream to the C ABI (include/fmm2d.h).  There is no
CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

PRECISIONS = {"fp64": L.FMM_FP64, "mixed": L.FMM_MIXED}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_device_f64(x: torch.Tensor, name: str, shape: tuple, device) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if tuple(x.shape) != shape:
        raise ValueError(f"{name} must have shape {shape}, got {tuple(x.shape)}")
    if device is not None and x.device != device:
        raise ValueError(f"{name} is on {x.device}, tree on {device}")
    return x.detach().contiguous()


def _check_out(out: torch.Tensor, n: int, device) -> torch.Tensor:
    """An output tensor the library writes through directly: float64, shape (n, 2),
    contiguous, on the tree's device (a copy would leave the caller's tensor unwritten)."""
    if not isinstance(out, torch.Tensor):
        raise ValueError("out must be a tensor")
    if out.dtype != torch.float64:
        raise ValueError(f"out must be float64, got {out.dtype}")
    if tuple(out.shape) != (n, 2):
        raise ValueError(f"out must have shape {(n, 2)}, got {tuple(out.shape)}")
    if out.device != device:
        raise ValueError(f"out is on {out.device}, tree on {device}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    return out


def _precision(precision) -> int:
    if isinstance(precision, str):
        return PRECISIONS[precision]
    return int(precision)


class _Adjoint:
    """Adjoint and transport calls shared by Tree and ATree (the C entry points differ only
    by the prefix fmm_ / fmm_atree_)."""

    _prefix = "fmm_"

    def _abi(self, name: str):
        return getattr(L.load(), self._prefix + name)

    def share_workspace(self, other) -> None:
        """Use the evaluation workspace of `other` (a tree of the same kind, n and depth)
        from now on; for trees evaluated one after the other."""
        if type(other) is not type(self):
            raise ValueError("both trees must be of the same kind")
        with torch.cuda.device(self.device):
            L.check(self._abi("share_workspace")(self.handle, other.handle), self._prefix + "share_workspace")

    def velocity_backward(self, gamma: torch.Tensor, sigma: float, p: int, precision, dl_duv: torch.Tensor,
                          need_gamma: bool = True, need_x: bool = True, need_src: bool = False,
                          need_xy: bool = False):
        """Adjoint of velocity for a loss with gradient dl_duv: (dL/dGamma (n,) or None,
        dL/dx_eval (n, 2) or None), then dL/dx_src (n, 2) with need_src, then with need_xy
        dL/dx_eval + dL/dx_src (n, 2), the gradient of particles moving as a whole, summed by
        the library."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        d = _as_device_f64(dl_duv, "dl_duv", (self.n, 2), self.device)

        def new(flag, shape):
            return torch.empty(shape, dtype=torch.float64, device=self.device) if flag else None

        dg, dx = new(need_gamma, (self.n,)), new(need_x, (self.n, 2))
        ds, dxy = new(need_src, (self.n, 2)), new(need_xy, (self.n, 2))
        with torch.cuda.device(self.device):
            L.check(self._abi("velocity_backward")(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                                   _ptr(d), _stream_ptr(), None, _ptr(dg), _ptr(dx), _ptr(ds),
                                                   _ptr(dxy)), self._prefix + "velocity_backward")
        return (dg, dx) + ((ds,) if need_src else ()) + ((dxy,) if need_xy else ())

    def transport_step(self, gamma: torch.Tensor, sigma: float, p: int, precision, x_base: torch.Tensor, h: float,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """x_base + h u, u the velocity of the tree's particles (one explicit transport stage)."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        xb = _as_device_f64(x_base, "x_base", (self.n, 2), self.device)
        xo = _check_out(out, self.n, self.device) if out is not None else torch.empty_like(xb)
        with torch.cuda.device(self.device):
            L.check(self._abi("transport_step")(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                                _stream_ptr(), None, _ptr(xb), float(h), _ptr(xo)),
                    self._prefix + "transport_step")
        return xo

    def transport_vjp(self, gamma: torch.Tensor, sigma: float, p: int, precision, lam: torch.Tensor, h: float,
                      flags: int, dl_dgamma: torch.Tensor | None, dl_dx: torch.Tensor | None):
        """Adjoint of transport_step with respect to the tree's particles (fmm_transport_vjp):
        writes, or with the FMM_ACC_* flags adds to, dl_dgamma (n,) and dl_dx (n, 2) in place."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        lm = _as_device_f64(lam, "lam", (self.n, 2), self.device)
        if dl_dgamma is not None:
            if dl_dgamma.dtype != torch.float64 or tuple(dl_dgamma.shape) != (self.n,) or \
                    dl_dgamma.device != self.device or not dl_dgamma.is_contiguous():
                raise ValueError("dl_dgamma must be a contiguous float64 (n,) tensor on the tree's device")
        if dl_dx is not None:
            _check_out(dl_dx, self.n, self.device)
        with torch.cuda.device(self.device):
            L.check(self._abi("transport_vjp")(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                               _ptr(lm), float(h), int(flags), _stream_ptr(), None, _ptr(dl_dgamma),
                                               _ptr(dl_dx)), self._prefix + "transport_vjp")


class Tree(_Adjoint):
    """Uniform quadtree over n particles (stages 1-3): Morton-sorted particles, leaf
    offsets, per-level occupancy and near-field work units, resident on the device.
    builder: "device" (the GPU build) or "host" (the reference build; same tree)."""

    def __init__(self, xy: torch.Tensor, depth: int, root_box=None, stream=None, builder: str = "device"):
        if not isinstance(xy, torch.Tensor) or xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be an (n, 2) tensor")
        self.device = xy.device
        xy = _as_device_f64(xy, "xy", tuple(xy.shape), None)
        self.n = int(xy.shape[0])
        self.depth = int(depth)
        lib = L.load()
        handle = ctypes.c_void_p()
        rb = (ctypes.c_double * 3)(*[float(v) for v in root_box]) if root_box is not None else None
        if builder not in ("device", "host"):
            raise ValueError("builder must be 'device' or 'host'")
        fn = lib.fmm_build_tree if builder == "device" else lib.fmm_build_tree_host
        with torch.cuda.device(self.device):
            L.check(fn(_ptr(xy), self.n, self.depth, rb, _stream_ptr(stream), ctypes.byref(handle)),
                    "fmm_build_tree" if builder == "device" else "fmm_build_tree_host")
        self._h = handle

    def rebuild(self, xy: torch.Tensor, root_box=None, stream=None) -> "Tree":
        """Rebuild in place for new positions of the same n particles (fmm_rebuild_tree):
        same depth and options, the evaluation workspace kept.  Returns self."""
        if not isinstance(xy, torch.Tensor) or xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be an (n, 2) tensor")
        if xy.device != self.device:
            raise ValueError("xy must be on the tree's device")
        xy = _as_device_f64(xy, "xy", (self.n, 2), None)
        rb = (ctypes.c_double * 3)(*[float(v) for v in root_box]) if root_box is not None else None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_rebuild_tree(self.handle, _ptr(xy), self.n, rb, _stream_ptr(stream),
                                              ctypes.byref(handle)), "fmm_rebuild_tree")
        self._h = handle
        return self

    # -- lifetime -----------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().fmm_destroy_tree(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("tree has been closed")
        return self._h

    # -- facts --------------------------------------------------------------------
    def info(self) -> dict:
        n = ctypes.c_int64()
        depth = ctypes.c_int()
        root = (ctypes.c_double * 3)()
        pairs = ctypes.c_int64()
        m2l = ctypes.c_int64()
        ne = ctypes.c_int64()
        mx = ctypes.c_int64()
        L.check(L.load().fmm_tree_info(self.handle, ctypes.byref(n), ctypes.byref(depth), root, ctypes.byref(pairs),
                                       ctypes.byref(m2l), ctypes.byref(ne), ctypes.byref(mx)), "fmm_tree_info")
        return {"n": n.value, "depth": depth.value, "root_box": tuple(root), "p2p_pairs": pairs.value,
                "m2l_pairs": m2l.value, "nonempty_leaves": ne.value, "max_leaf": mx.value}

    def levels(self) -> list:
        """Non-empty cells per level, levels 0 .. depth."""
        buf = (ctypes.c_int64 * (self.depth + 1))()
        L.check(L.load().fmm_tree_levels(self.handle, buf, self.depth + 1), "fmm_tree_levels")
        return list(buf)

    def permutation(self):
        """(perm, leaf): perm[k] = user index of the k-th particle in Morton order, leaf[k] its leaf."""
        perm = torch.empty(self.n, dtype=torch.int64, device=self.device)
        leaf = torch.empty(self.n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_tree_permutation(self.handle, _ptr(perm), _ptr(leaf), _stream_ptr()),
                    "fmm_tree_permutation")
        return perm, leaf

    def near_plan(self) -> dict:
        """Near-field plan: mutual items, ordered pairs they evaluate, target-centric units."""
        v = [ctypes.c_int64() for _ in range(3)]
        L.check(L.load().fmm_near_plan_info(self.handle, *[ctypes.byref(x) for x in v]), "fmm_near_plan_info")
        return {"mutual_items": v[0].value, "mutual_pairs": v[1].value, "target_units": v[2].value}

    def set_option(self, key: int, value: int):
        L.check(L.load().fmm_set_option(self.handle, int(key), int(value)), "fmm_set_option")

    def timings(self) -> dict:
        """Per-stage device milliseconds summed over calls since the last read (FMM_OPT_TIMING on)."""
        ms = (ctypes.c_double * L.FMM_T_COUNT)()
        calls = ctypes.c_int64()
        L.check(L.load().fmm_get_timings(self.handle, ms, ctypes.byref(calls)), "fmm_get_timings")
        names = ["pack", "far", "p2p", "final", "total"]
        return {"calls": calls.value, **{k: ms[i] for i, k in enumerate(names)}}

    def timeline(self) -> dict:
        """Event times (ms after the call's first event) of the last call made with
        FMM_OPT_TIMING on and not yet read by timings()."""
        ms = (ctypes.c_double * 8)()
        L.check(L.load().fmm_get_timeline(self.handle, ms, 8), "fmm_get_timeline")
        names = ["start", "pack_end", "far_start", "far_end", "p2p_start", "p2p_end", "final_start", "final_end"]
        return {k: ms[i] for i, k in enumerate(names)}

    # -- evaluation ---------------------------------------------------------------
    def velocity(self, gamma: torch.Tensor, sigma: float, p: int, precision="mixed", out=None,
                 side_stream=None) -> torch.Tensor:
        """(n, 2) float64 velocities in user order (stages 4-10)."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        uv = _check_out(out, self.n, self.device) if out is not None else \
            torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_velocity(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                          _stream_ptr(), _stream_ptr(side_stream) if side_stream else None,
                                          _ptr(uv)), "fmm_velocity")
        return uv

    def velocity_parts(self, gamma: torch.Tensor, sigma: float, p: int, precision="mixed"):
        """(near, far) velocities, each (n, 2) float64 in user order."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        near = torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        far = torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_velocity_parts(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                                _stream_ptr(), None, _ptr(near), _ptr(far)), "fmm_velocity_parts")
        return near, far



class ATree(_Adjoint):
    """Adaptive quadtree over n particles for uneven distributions (include/fmm2d_adaptive.h):
    cells split while they hold more than max_leaf particles, down to max_depth, and the
    U, V, W, X lists of the adaptive FMM, resident on the device.
    builder: "device" (the GPU build) or "host" (the reference build; same tree)."""

    _prefix = "fmm_atree_"

    def __init__(self, xy: torch.Tensor, max_leaf: int, max_depth: int, root_box=None, stream=None,
                 builder: str = "device"):
        if not isinstance(xy, torch.Tensor) or xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be an (n, 2) tensor")
        self.device = xy.device
        xy = _as_device_f64(xy, "xy", tuple(xy.shape), None)
        self.n = int(xy.shape[0])
        self.max_leaf, self.max_depth = int(max_leaf), int(max_depth)
        handle = ctypes.c_void_p()
        rb = (ctypes.c_double * 3)(*[float(v) for v in root_box]) if root_box is not None else None
        if builder not in ("device", "host"):
            raise ValueError("builder must be 'device' or 'host'")
        name = "fmm_atree_build" if builder == "device" else "fmm_atree_build_host"
        with torch.cuda.device(self.device):
            L.check(getattr(L.load(), name)(_ptr(xy), self.n, self.max_leaf, self.max_depth, rb, _stream_ptr(stream),
                                            ctypes.byref(handle)), name)
        self._h = handle

    def rebuild(self, xy: torch.Tensor, root_box=None, stream=None) -> "ATree":
        """Rebuild on the device for new positions of the same n particles (fmm_atree_rebuild):
        same max_leaf and max_depth, the evaluation workspace kept.  Returns self."""
        if not isinstance(xy, torch.Tensor) or xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be an (n, 2) tensor")
        if xy.device != self.device:
            raise ValueError("xy must be on the tree's device")
        xy = _as_device_f64(xy, "xy", (self.n, 2), None)
        rb = (ctypes.c_double * 3)(*[float(v) for v in root_box]) if root_box is not None else None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_atree_rebuild(self.handle, _ptr(xy), self.n, rb, _stream_ptr(stream),
                                               ctypes.byref(handle)), "fmm_atree_rebuild")
        self._h = handle
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().fmm_atree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("tree is closed")
        return self._h

    def set_option(self, key: int, value: int):
        """fmm_atree_set_option: FMM_OPT_NEAR_OCCUPANCY (-1 automatic, 0 no cap, 1..8)."""
        L.check(L.load().fmm_atree_set_option(self.handle, int(key), int(value)), "fmm_atree_set_option")

    def info(self) -> dict:
        """Sizes of the tree and its lists (keys of _lib.FMM_AT_KEYS) and the root cell."""
        sizes = (ctypes.c_int64 * 8)()
        root = (ctypes.c_double * 3)()
        L.check(L.load().fmm_atree_info(self.handle, sizes, root), "fmm_atree_info")
        out = {k: int(v) for k, v in zip(L.FMM_AT_KEYS, sizes)}
        out["root_box"] = tuple(root)
        return out

    def leaves(self):
        """(level, ix, iy) of each particle's leaf, numpy int32 arrays in user order."""
        import numpy as np
        lv, ix, iy = (np.zeros(self.n, dtype=np.int32) for _ in range(3))
        L.check(L.load().fmm_atree_leaves(self.handle, lv.ctypes.data_as(ctypes.c_void_p),
                                          ix.ctypes.data_as(ctypes.c_void_p), iy.ctypes.data_as(ctypes.c_void_p)),
                "fmm_atree_leaves")
        return lv, ix, iy

    def velocity(self, gamma: torch.Tensor, sigma: float, p: int, precision="mixed", out=None,
                 serial: bool = False) -> torch.Tensor:
        """(n, 2) float64 velocities in user order.  serial: the far field on the current
        stream after the near field instead of beside it (for timing the stages alone)."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        uv = _check_out(out, self.n, self.device) if out is not None else \
            torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            s = _stream_ptr()
            L.check(L.load().fmm_atree_velocity(self.handle, _ptr(g), float(sigma), int(p), _precision(precision),
                                                s, s if serial else None, _ptr(uv)), "fmm_atree_velocity")
        return uv

    def velocity_parts(self, gamma: torch.Tensor, sigma: float, p: int, precision="mixed"):
        """(near, far) velocities, each (n, 2) float64 in user order."""
        g = _as_device_f64(gamma, "gamma", (self.n,), self.device)
        near = torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        far = torch.empty((self.n, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.load().fmm_atree_velocity_parts(self.handle, _ptr(g), float(sigma), int(p),
                                                      _precision(precision), _stream_ptr(), None, _ptr(near),
                                                      _ptr(far)), "fmm_atree_velocity_parts")
        return near, far



class VelocityFn(torch.autograd.Function):
    """u = FMM velocity of the particles of `tree` (a Tree or an ATree) with circulations gamma.

    Backward returns dL/dGamma and dL/dxy, the derivative with respect to the particle
    positions, each particle moving both as evaluation point and as source
    (dL/dx_eval + dL/dx_src); the tree's cells are held fixed."""

    @staticmethod
    def forward(ctx, xy, gamma, tree, sigma: float, p: int, precision="mixed"):
        uv = tree.velocity(gamma, sigma, p, precision)
        ctx.save_for_backward(gamma)
        ctx.tree, ctx.sigma, ctx.p, ctx.precision = tree, sigma, p, precision
        return uv

    @staticmethod
    def backward(ctx, grad_uv):
        (gamma,) = ctx.saved_tensors
        need_x, need_g = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_g):
            return None, None, None, None, None, None
        res = ctx.tree.velocity_backward(gamma.detach(), ctx.sigma, ctx.p, ctx.precision, grad_uv.contiguous(),
                                         need_gamma=need_g, need_x=False, need_xy=need_x)
        return (res[2] if need_x else None), res[0], None, None, None, None


def velocity(xy: torch.Tensor, gamma: torch.Tensor, sigma: float, depth: int, p: int, precision="mixed",
             root_box=None, tree=None) -> torch.Tensor:
    """Differentiable velocities of particles at xy over `tree` (a Tree or an ATree built for
    xy); builds a uniform tree of the given depth unless one is given."""
    if tree is None:
        tree = Tree(xy, depth, root_box)
    return VelocityFn.apply(xy, gamma, tree, sigma, p, precision)
