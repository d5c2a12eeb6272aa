"""Time-stepped transport of the vortex particles and its adjoint.

Section "Test problem": the particles move with the flow they induce and carry their
circulations unchanged, dx/dt = u(x) with u from eq. discBiotS2D.  The paper does not
fix a time integrator; this module uses the explicit midpoint rule (RK2),

    x_{n+1/2} = x_n + (dt/2) u(x_n),     x_{n+1} = x_n + dt u(x_{n+1/2}),

with every velocity an FMM evaluation (stages 4-10) over a tree rebuilt for the
current positions (stages 1-3), as the positions change (Tree.rebuild: the evaluation
workspace of the tree is kept from one rebuild to the next).  With adaptive=(max_leaf,
max_depth) every evaluation uses the adaptive tree (ATree, rebuilt on the device for the
current positions the same way) instead of the uniform tree of the given depth.

Each stage is one fmm_transport_step call (the velocity and the update x_base + h u in
the library's kernels).  The gradient of a loss L(x_N) with respect to x_0 and Gamma is
the discrete adjoint of those steps, run backwards with per-step checkpoints (only x_n is
kept per step; the midpoint of step n is recomputed in its backward step):

    lambda_half = dt J_half^T lambda_{n+1}                 (x_{n+1} = x_n + dt u(x_half))
    lambda_n    = lambda_{n+1} + lambda_half + (dt/2) J_n^T lambda_half
                                                           (x_half = x_n + (dt/2) u(x_n))
    dL/dGamma  += the Gamma parts of the same two products

with J the Jacobian of the velocities with respect to the particles moving as sources and
evaluation points.  Each line is one fmm_transport_vjp call, the accumulation and the
identity term done by the library (flags FMM_ACC_GAMMA, FMM_ACC_X, FMM_IDENTITY), so no
arithmetic of the method runs outside it.  Trees are treated as fixed within each
evaluation (the leaf of a particle does not change under an infinitesimal move), which is
the derivative of the discrete method away from leaf boundaries.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from .fmm import ATree, Tree


@dataclass
class RK2Stats:
    """Timing of a run (seconds, host clock around synchronised device work) and the peak
    of device memory in use (all allocations on the device, sampled while trees are alive)."""
    tree_build: float = 0.0
    velocity: float = 0.0
    backward: float = 0.0
    evals: int = 0
    vjps: int = 0
    peak_bytes: int = 0
    torch_reserved_bytes: int = 0   # the part held by torch's caching allocator (inputs, checkpoints)
    per_step: list = field(default_factory=list)


def _sample_memory(device, stats: RK2Stats):
    free, total = torch.cuda.mem_get_info(device)
    if total - free > stats.peak_bytes:
        stats.peak_bytes = total - free
        stats.torch_reserved_bytes = torch.cuda.memory_reserved(device)


def _tree_for(tree, xy, depth, root_box, adaptive):
    """A tree for the positions xy: `tree` rebuilt in place (its workspace kept), or a new
    uniform or adaptive tree when it is None."""
    if tree is not None:
        return tree.rebuild(xy, root_box)
    return ATree(xy, adaptive[0], adaptive[1], root_box) if adaptive is not None else Tree(xy, depth, root_box)


def _rebuilt(tree, xy, depth, root_box, stats: RK2Stats, adaptive=None):
    """`tree` rebuilt for xy (a new tree when it is None), timed as a tree build."""
    t0 = time.perf_counter()
    tree = _tree_for(tree, xy, depth, root_box, adaptive)
    torch.cuda.synchronize(xy.device)
    stats.tree_build += time.perf_counter() - t0
    return tree


def _stage(tree, x_base, h, gamma, sigma, p, precision, stats: RK2Stats, out=None):
    """x_base + h u over `tree` (one fmm_transport_step, into `out` when given), timed as a
    velocity evaluation."""
    t0 = time.perf_counter()
    out = tree.transport_step(gamma, sigma, p, precision, x_base, h, out)
    torch.cuda.synchronize(x_base.device)
    stats.velocity += time.perf_counter() - t0
    stats.evals += 1
    _sample_memory(x_base.device, stats)
    return out


def rk2_forward(xy0: torch.Tensor, gamma: torch.Tensor, sigma: float, depth: int, p: int, dt: float, steps: int,
                precision="mixed", root_box=None, stats: RK2Stats | None = None, adaptive=None):
    """Advance the particles `steps` midpoint-RK2 steps.  Returns (x_N, checkpoints) with
    checkpoints[n] = x_n, n = 0..steps-1 (device tensors)."""
    stats = stats if stats is not None else RK2Stats()
    x = xy0.detach().contiguous()
    g = gamma.detach().contiguous()
    checkpoints = []
    tree = None
    try:
        for _ in range(steps):
            checkpoints.append(x)
            tree = _rebuilt(tree, x, depth, root_box, stats, adaptive)
            xm = _stage(tree, x, 0.5 * dt, g, sigma, p, precision, stats)
            tree = _rebuilt(tree, xm, depth, root_box, stats, adaptive)
            x = _stage(tree, x, dt, g, sigma, p, precision, stats)
    finally:
        if tree is not None:
            tree.close()
    return x, checkpoints


def rk2_backward(checkpoints, gamma: torch.Tensor, sigma: float, depth: int, p: int, dt: float,
                 dl_dxN: torch.Tensor, precision="mixed", root_box=None, stats: RK2Stats | None = None,
                 adaptive=None):
    """Discrete adjoint of rk2_forward: (dL/dx_0, dL/dGamma) from dL/dx_N."""
    from ._lib import FMM_ACC_GAMMA, FMM_ACC_X, FMM_IDENTITY
    stats = stats if stats is not None else RK2Stats()
    g = gamma.detach().contiguous()
    lam = dl_dxN.detach().contiguous().clone()   # lambda_n, updated in place by the library
    lam_half = torch.empty_like(lam)
    dgamma = torch.empty_like(g)
    tree0 = treem = None
    try:
        for k, x in enumerate(reversed(checkpoints)):
            t0 = time.perf_counter()
            tree0 = _rebuilt(tree0, x, depth, root_box, stats, adaptive)
            # the midpoint is only read by the build of its tree (which keeps its own sorted
            # copy), so it lives in lam_half until the first product overwrites it
            xm = _stage(tree0, x, 0.5 * dt, g, sigma, p, precision, stats, out=lam_half)
            first = treem is None
            treem = _rebuilt(treem, xm, depth, root_box, stats, adaptive)
            if first:
                treem.share_workspace(tree0)  # the two trees are used one after the other
            t1 = time.perf_counter()
            acc_g = FMM_ACC_GAMMA if k > 0 else 0
            treem.transport_vjp(g, sigma, p, precision, lam, dt, acc_g, dgamma, lam_half)
            tree0.transport_vjp(g, sigma, p, precision, lam_half, 0.5 * dt, FMM_ACC_GAMMA | FMM_ACC_X | FMM_IDENTITY,
                                dgamma, lam)
            torch.cuda.synchronize(x.device)
            _sample_memory(x.device, stats)
            stats.backward += time.perf_counter() - t1
            stats.vjps += 2
            stats.per_step.append(time.perf_counter() - t0)
    finally:
        for tr in (treem, tree0):
            if tr is not None:
                tr.close()
    return lam, dgamma


class RK2Transport(torch.autograd.Function):
    """x_N = RK2 transport of x_0 with circulations gamma; differentiable in both."""

    @staticmethod
    def forward(ctx, xy0, gamma, sigma: float, depth: int, p: int, dt: float, steps: int, precision="mixed",
                root_box=None, adaptive=None):
        xN, checkpoints = rk2_forward(xy0, gamma, sigma, depth, p, dt, steps, precision, root_box, adaptive=adaptive)
        ctx.save_for_backward(gamma, *checkpoints)
        ctx.args = (sigma, depth, p, dt, precision, root_box, adaptive)
        return xN

    @staticmethod
    def backward(ctx, grad_xN):
        gamma, *checkpoints = ctx.saved_tensors
        sigma, depth, p, dt, precision, root_box, adaptive = ctx.args
        dx0, dg = rk2_backward(checkpoints, gamma, sigma, depth, p, dt, grad_xN, precision, root_box,
                               adaptive=adaptive)
        return dx0, dg, None, None, None, None, None, None, None, None


def transport(xy0: torch.Tensor, gamma: torch.Tensor, sigma: float, depth: int, p: int, dt: float, steps: int,
              precision="mixed", root_box=None, adaptive=None) -> torch.Tensor:
    """Differentiable midpoint-RK2 transport of the particles (see the module docstring)."""
    return RK2Transport.apply(xy0, gamma, sigma, depth, p, dt, steps, precision, root_box, adaptive)
