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

The gradient of a loss L(x_N) with respect to x_0 and Gamma is the discrete adjoint of
those steps, run backwards with per-step checkpoints (only x_n is kept per step; the
two velocities of step n are recomputed in its backward step):

    mu      = dt lambda_{n+1}                  (cotangent of u(x_{n+1/2}))
    lambda' = VJP_x u(x_{n+1/2}) [mu]           (every particle moving as source and target)
    nu      = (dt/2) lambda'                    (cotangent of u(x_n))
    lambda_n = lambda_{n+1} + lambda' + VJP_x u(x_n) [nu]
    dL/dGamma += VJP_Gamma u(x_{n+1/2}) [mu] + VJP_Gamma u(x_n) [nu]

with each VJP one fmm_velocity_backward call (dL/dx_eval + dL/dx_src, dL/dGamma).
Trees are treated as fixed within each evaluation (the leaf of a particle does not
change under an infinitesimal move), which is the derivative of the discrete method
away from leaf boundaries.
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
    per_step: list = field(default_factory=list)


def _sample_memory(device, stats: RK2Stats):
    free, total = torch.cuda.mem_get_info(device)
    stats.peak_bytes = max(stats.peak_bytes, total - free)


def _tree_for(tree, xy, depth, root_box, adaptive):
    """A tree for the positions xy: `tree` rebuilt in place (its workspace kept), or a new
    uniform or adaptive tree when it is None."""
    if tree is not None:
        return tree.rebuild(xy, root_box)
    return ATree(xy, adaptive[0], adaptive[1], root_box) if adaptive is not None else Tree(xy, depth, root_box)


def _velocity(tree, xy, gamma, sigma, depth, p, precision, root_box, stats: RK2Stats, adaptive=None):
    """u(xy) over `tree` rebuilt for xy (a new tree when it is None); returns (tree, u)."""
    t0 = time.perf_counter()
    tree = _tree_for(tree, xy, depth, root_box, adaptive)
    torch.cuda.synchronize(xy.device)
    t1 = time.perf_counter()
    uv = tree.velocity(gamma, sigma, p, precision)
    torch.cuda.synchronize(xy.device)
    t2 = time.perf_counter()
    stats.tree_build += t1 - t0
    stats.velocity += t2 - t1
    stats.evals += 1
    _sample_memory(xy.device, stats)
    return tree, uv


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
            tree, u0 = _velocity(tree, x, g, sigma, depth, p, precision, root_box, stats, adaptive)
            xm = x + (0.5 * dt) * u0
            tree, um = _velocity(tree, xm, g, sigma, depth, p, precision, root_box, stats, adaptive)
            x = x + dt * um
    finally:
        if tree is not None:
            tree.close()
    return x, checkpoints


def rk2_backward(checkpoints, gamma: torch.Tensor, sigma: float, depth: int, p: int, dt: float,
                 dl_dxN: torch.Tensor, precision="mixed", root_box=None, stats: RK2Stats | None = None,
                 adaptive=None):
    """Discrete adjoint of rk2_forward: (dL/dx_0, dL/dGamma) from dL/dx_N."""
    stats = stats if stats is not None else RK2Stats()
    g = gamma.detach().contiguous()
    lam = dl_dxN.detach().contiguous().clone()
    dgamma = torch.zeros_like(g)
    tree0 = treem = None
    try:
        for x in reversed(checkpoints):
            t0 = time.perf_counter()
            tree0, u0 = _velocity(tree0, x, g, sigma, depth, p, precision, root_box, stats, adaptive)
            xm = x + (0.5 * dt) * u0
            treem, _ = _velocity(treem, xm, g, sigma, depth, p, precision, root_box, stats, adaptive)
            t1 = time.perf_counter()
            mu = dt * lam
            dgm, dxm, dsm = treem.velocity_backward(g, sigma, p, precision, mu, need_src=True)
            torch.cuda.synchronize(x.device)
            _sample_memory(x.device, stats)
            lam_mid = dxm + dsm
            nu = (0.5 * dt) * lam_mid
            dg0, dx0, ds0 = tree0.velocity_backward(g, sigma, p, precision, nu, need_src=True)
            lam = lam + lam_mid + dx0 + ds0
            dgamma += dgm + dg0
            torch.cuda.synchronize(x.device)
            stats.backward += time.perf_counter() - t1
            stats.vjps += 2
            stats.per_step.append(time.perf_counter() - t0)
    finally:
        for tr in (tree0, treem):
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
