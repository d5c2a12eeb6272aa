"""GPU parity of the adjoint (fmm_velocity_backward) against the CPU oracle's O4 and O5.

Bars: FP64 form within 1e-9 (vector rel-L2) of the oracle gradient; mixed form
within 1e-4; both against central finite differences of the FP64 forward where the
forward API can evaluate them (circulations, and positions with every particle
moving as source and evaluation point; the split into evaluation-position and
source-position parts is checked against the oracle, whose parts are pinned by
finite differences in the oracle tests).
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_1008_2410_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _grads(fmm_mod, w, dl_duv, precision, tree=None):
    tree = tree or fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    dg, dx = tree.velocity_backward(_t(w.gamma), w.sigma, w.p, precision, _t(dl_duv))
    return dg.cpu().numpy(), dx.cpu().numpy()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-4)])
@pytest.mark.parametrize("n,depth,p", [(4096, 4, 10), (3000, 5, 12), (700, 1, 6), (5000, 3, 16)])
def test_backward_matches_oracle(fmm_mod, oracle_mod, precision, tol, n, depth, p):
    w = W.uniform_lamb_oseen(n=n, seed=n + depth, depth=depth, p=p)
    ustar = W.smooth_target_field(w.xy, seed=7)
    uv = oracle_mod.fmm_velocity(w.xy, w.gamma, w.sigma, w.depth, w.p, w.root_box)
    dl = uv - ustar
    dg_ref, dx_ref, ds_ref = oracle_mod.fmm_grad_full(w.xy, w.gamma, w.sigma, w.depth, w.p, dl, w.root_box)
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    dg, dx, ds = (a.cpu().numpy() for a in tree.velocity_backward(_t(w.gamma), w.sigma, w.p, precision, _t(dl),
                                                                  need_src=True))
    assert rel_l2(dg, dg_ref) < tol
    assert rel_l2(dx, dx_ref) < tol
    assert rel_l2(ds, ds_ref) < tol
    # the default call (no source-position output) gives the same bits for the rest
    dg2, dx2 = _grads(fmm_mod, w, dl, precision, tree=tree)
    assert np.array_equal(dg, dg2) and np.array_equal(dx, dx2)


def test_position_gradient_central_differences_on_gpu(fmm_mod):
    """Every particle moving as source and evaluation point: dL/dx_eval + dL/dx_src against
    central differences of L through the GPU FP64 forward (tree rebuilt at each point, the
    moved particle's leaf unchanged)."""
    w = W.uniform_lamb_oseen(n=3000, seed=78, depth=4, p=14)
    ustar = W.smooth_target_field(w.xy, seed=9)
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    uv = tree.velocity(_t(w.gamma), w.sigma, w.p, "fp64").cpu().numpy()
    _, dx, ds = tree.velocity_backward(_t(w.gamma), w.sigma, w.p, "fp64", _t(uv - ustar), need_src=True)
    tot = (dx + ds).cpu().numpy()

    def loss(xy):
        t = fmm_mod.Tree(_t(xy), w.depth, w.root_box)
        u = t.velocity(_t(w.gamma), w.sigma, w.p, "fp64").cpu().numpy()
        return 0.5 * ((u - ustar) ** 2).sum()

    h = 1e-6
    checked = 0
    for k in np.random.Generator(np.random.PCG64(4)).permutation(w.n):
        frac = (w.xy[k] * 16) % 1.0
        if np.any(frac < 0.01) or np.any(frac > 0.99):
            continue
        for comp in (0, 1):
            a, b = w.xy.copy(), w.xy.copy()
            a[k, comp] += h
            b[k, comp] -= h
            fd = (loss(a) - loss(b)) / (2 * h)
            assert abs(fd - tot[k, comp]) <= 1e-5 * abs(fd) + 1e-9, (k, comp, fd, tot[k, comp])
        checked += 1
        if checked == 4:
            break
    assert checked == 4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lone_particle_has_no_net_position_gradient(fmm_mod, precision):
    """The blob's own slope enters dL/dx_eval and, with the opposite sign, dL/dx_src."""
    w = W.Workload("one", np.array([[0.3, 0.4]]), np.array([1.3]), 0.05, 3, 10, (0, 0, 1), "fp64")
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    _, dx, ds = tree.velocity_backward(_t(w.gamma), w.sigma, w.p, precision, _t(np.array([[0.7, -0.2]])),
                                       need_src=True)
    dx, ds = dx.cpu().numpy(), ds.cpu().numpy()
    assert np.abs(dx).max() > 1.0
    assert np.abs(dx + ds).max() <= (1e-12 if precision == "fp64" else 1e-6) * np.abs(dx).max()


def test_gamma_gradient_central_differences_on_gpu(fmm_mod):
    """u is linear in Gamma: central differences of L(Gamma) with the GPU FP64 forward equal
    dL/dGamma to roundoff."""
    w = W.uniform_lamb_oseen(n=6000, seed=77, depth=5, p=12)
    ustar = W.smooth_target_field(w.xy, seed=8)
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    g = _t(w.gamma)
    uv = tree.velocity(g, w.sigma, w.p, "fp64").cpu().numpy()
    dg, _ = _grads(fmm_mod, w, uv - ustar, "fp64", tree=tree)
    for k in np.random.Generator(np.random.PCG64(3)).choice(w.n, 8, replace=False):
        h = 1e-3  # L is exactly quadratic in Gamma: any step is exact up to roundoff
        vals = []
        for sgn in (1, -1):
            gg = w.gamma.copy()
            gg[k] += sgn * h
            u = tree.velocity(_t(gg), w.sigma, w.p, "fp64").cpu().numpy()
            vals.append(0.5 * ((u - ustar) ** 2).sum())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dg[k]) <= 1e-7 * abs(dg[k]) + 1e-14, (k, fd, dg[k])


def test_uniform_target_field_mixed(fmm_mod, oracle_mod):
    """2^20 uniform particles, depth 8, p = 12, FP32 forward, L = 0.5 sum |u - u*|^2:
    the mixed gradient within 1e-4 of the FP64 oracle gradient, over all particles and
    at the 64 seeded coordinates (32 circulations, 32 positions)."""
    w = W.uniform_target_field()
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    uv = tree.velocity(_t(w.gamma), w.sigma, w.p, "mixed").cpu().numpy()
    dl = uv - w.extra["u_target"]
    dg, dx = _grads(fmm_mod, w, dl, "mixed", tree=tree)
    dg_ref, dx_ref = oracle_mod.fmm_grad(w.xy, w.gamma, w.sigma, w.depth, w.p, dl, w.root_box)
    assert rel_l2(dg, dg_ref) < 1e-4
    assert rel_l2(dx, dx_ref) < 1e-4
    gi = w.extra["fd_gamma_idx"]
    xi = w.extra["fd_x_idx"]
    xc = w.extra["fd_x_comp"]
    assert rel_l2(dg[gi], dg_ref[gi]) < 1e-4
    assert rel_l2(dx[xi, xc], dx_ref[xi, xc]) < 1e-4


def test_autograd_function(fmm_mod, oracle_mod):
    import torch
    w = W.uniform_lamb_oseen(n=3000, seed=5, depth=4, p=10)
    ustar = _t(W.smooth_target_field(w.xy, seed=2))
    xy = _t(w.xy).requires_grad_(True)
    g = _t(w.gamma).requires_grad_(True)
    uv = fmm_mod.velocity(xy, g, w.sigma, w.depth, w.p, "fp64", root_box=w.root_box)
    loss = 0.5 * ((uv - ustar) ** 2).sum()
    loss.backward()
    dl = (uv - ustar).detach().cpu().numpy()
    dg_ref, dx_ref, ds_ref = oracle_mod.fmm_grad_full(w.xy, w.gamma, w.sigma, w.depth, w.p, dl, w.root_box)
    assert rel_l2(g.grad.cpu().numpy(), dg_ref) < 1e-9
    assert rel_l2(xy.grad.cpu().numpy(), dx_ref + ds_ref) < 1e-9


def test_backward_deterministic(fmm_mod):
    w = W.uniform_lamb_oseen(n=20000, seed=6, depth=6, p=12)
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    dl = np.random.Generator(np.random.PCG64(0)).standard_normal((w.n, 2))
    for precision in ("fp64", "mixed"):
        a = _grads(fmm_mod, w, dl, precision, tree=tree)
        b = _grads(fmm_mod, w, dl, precision, tree=tree)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_uniform_target_field_central_differences_fp64(fmm_mod):
    """The differentiation configuration at full size (2^20 uniform particles, depth 8,
    p = 12, L = 0.5 sum |u - u*|^2): the FP64 gradient at the 64 seeded coordinates against
    central differences of the FP64 forward, the difference of the losses summed per
    particle, 0.5 (u+ - u-).(u+ + u- - 2 u*), so that unchanged particles add no rounding.
    32 circulations with step 1e-6 (L is quadratic in Gamma: exact up to rounding).  32
    positions, each particle moving as evaluation point and as source (tree rebuilt for the
    moved particle; coordinates within 0.03 leaf widths of a leaf edge, where the method
    is discontinuous, skipped), with steps 1e-4 and 5e-5 combined by Richardson extrapolation
    ((4 D(h/2) - D(h))/3 cancels the h^2 term, up to 1e-5 of the derivative at 1e-4 where two
    particles are much closer than the blob core): a moved source changes the far field of all
    2^20 particles, and below ~1e-5 the rounding of those changes, summed over the field,
    exceeds 1e-6 of the derivative (a step of 1e-6 gives errors up to 8e-6)."""
    import torch
    w = W.uniform_target_field()
    xy, g = _t(w.xy), _t(w.gamma)
    ustar = _t(w.extra["u_target"])
    tree = fmm_mod.Tree(xy, w.depth, w.root_box)
    uv = tree.velocity(g, w.sigma, w.p, "fp64")
    dg, dx, ds = (a.cpu().numpy() for a in tree.velocity_backward(g, w.sigma, w.p, "fp64", uv - ustar,
                                                                    need_src=True))
    dxt = dx + ds

    def central(up, um, h):
        return float((0.5 * (up - um) * (up + um - 2 * ustar)).sum()) / (2 * h)

    h = 1e-6
    worst_g = 0.0
    for k in w.extra["fd_gamma_idx"]:
        gp, gm = g.clone(), g.clone()
        gp[k] += h
        gm[k] -= h
        fd = central(tree.velocity(gp, w.sigma, w.p, "fp64"), tree.velocity(gm, w.sigma, w.p, "fp64"), h)
        worst_g = max(worst_g, abs(fd - dg[k]) / abs(dg[k]))
    hx = 1e-4
    root = w.root_box
    lw = root[2] / 2 ** w.depth
    fds, ads = [], []
    moved = fmm_mod.Tree(xy, w.depth, root)
    for k, c in zip(w.extra["fd_x_idx"], w.extra["fd_x_comp"]):
        frac = ((w.xy[k, c] - root[c]) / lw) % 1.0
        if frac < 0.03 or frac > 0.97:
            continue
        d = []
        for step in (hx, hx / 2):
            us = []
            for sgn in (1, -1):
                x2 = xy.clone()
                x2[k, c] += sgn * step
                us.append(moved.rebuild(x2, root).velocity(g, w.sigma, w.p, "fp64"))
            d.append(central(us[0], us[1], step))
        fds.append((4 * d[1] - d[0]) / 3)
        ads.append(dxt[k, c])
    fds, ads = np.array(fds), np.array(ads)
    scale = np.median(np.abs(ads))
    worst_x = np.max(np.abs(fds - ads) / (np.abs(ads) + 0.1 * scale))
    print(f"[2^20 target field] FD vs FP64 adjoint: worst relative difference Gamma {worst_g:.2e}; positions "
          f"rel-L2 {rel_l2(fds, ads):.2e}, worst {worst_x:.2e} against |dL/dx| + 0.1 median ({len(fds)} coordinates)",
          flush=True)
    assert worst_g < 1e-7
    assert rel_l2(fds, ads) < 1e-6
    assert worst_x < 1e-5
    assert len(fds) >= 26
    moved.close()
    tree.close()
    torch.cuda.synchronize()


def test_user_order_above_cache_size(fmm_mod):
    """Above 2^24 particles the velocities and the three adjoint outputs reach user order
    through the staging windows.  Renumbering the particles (a random permutation of the
    user order; the tree, hence every sum, is the same) must permute every output the same
    way: a wrong staging slot would move values between particles.  Every particle sits in
    a cell of its own on the 2^15 x 2^15 grid of sub-leaf keys (depth 9, 64 x 64 per leaf),
    so the tree order does not depend on the numbering and the outputs must agree bit for
    bit, in both precisions."""
    import torch
    n = (1 << 24) + 4097
    r = np.random.Generator(np.random.PCG64(31))
    cells = np.unique(r.integers(0, 1 << 30, size=n + n // 8))
    cells = r.permutation(cells)[:n]
    assert len(cells) == n
    ij = np.stack([cells >> 15, cells & 0x7FFF], axis=1).astype(np.float64)
    xy = (ij + 0.25 + 0.5 * r.random((n, 2))) / 32768.0
    g = r.standard_normal(n) / n
    dl = r.standard_normal((n, 2))
    order = r.permutation(n)
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    sigma, p = 0.5 / 512, 8
    out = {}
    for key, perm in (("a", np.arange(n)), ("b", order)):
        tree = fmm_mod.Tree(_t(xy[perm]), 9, (0.0, 0.0, 1.0))
        res = []
        for precision in ("mixed", "fp64"):
            gt, dlt = _t(g[perm]), _t(dl[perm])
            res.append(tree.velocity(gt, sigma, p, precision).cpu().numpy())
            res += [v.cpu().numpy() for v in tree.velocity_backward(gt, sigma, p, precision, dlt, need_src=True)]
        out[key] = res
        del tree
        torch.cuda.empty_cache()
    names = ["uv", "dgamma", "dxeval", "dxsrc"] * 2
    for name, a, b in zip(names, out["a"], out["b"]):
        assert np.array_equal(a, b[inv]), name
