"""GPU parity of the midpoint-RK2 transport and its discrete adjoint.

The oracle side advances the same particles with the same rule, each velocity an O3
evaluation over a tree rebuilt for the current positions (bounding square), and its
gradient chains the oracle's O4 + O5 vector-Jacobian products through the steps.
Bars: FP64 positions within 1e-12 (rel-L2) and gradients within 1e-9 of the oracle's;
mixed within 1e-6 and 1e-4; the FP64 gradient also against central differences of the
GPU transport.
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_1008_2410_amd import workloads as W

pytestmark = pytest.mark.gpu

DT, STEPS = 2e-3, 3


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _oracle_rk2(oracle_mod, xy, g, sigma, depth, p):
    xs = [xy]
    x = xy
    for _ in range(STEPS):
        u0 = oracle_mod.fmm_velocity(x, g, sigma, depth, p, None)
        xm = x + 0.5 * DT * u0
        um = oracle_mod.fmm_velocity(xm, g, sigma, depth, p, None)
        x = x + DT * um
        xs.append(x)
    return xs


def _oracle_rk2_grad(oracle_mod, xs, g, sigma, depth, p, dl_dxN):
    lam = dl_dxN.copy()
    dg = np.zeros_like(g)
    for x in reversed(xs[:-1]):
        u0 = oracle_mod.fmm_velocity(x, g, sigma, depth, p, None)
        xm = x + 0.5 * DT * u0
        mu = DT * lam
        dgm, dxm, dsm = oracle_mod.fmm_grad_full(xm, g, sigma, depth, p, mu, None)
        lam_mid = dxm + dsm
        dg0, dx0, ds0 = oracle_mod.fmm_grad_full(x, g, sigma, depth, p, 0.5 * DT * lam_mid, None)
        lam = lam + lam_mid + dx0 + ds0
        dg += dgm + dg0
    return lam, dg


@pytest.fixture(scope="module")
def patches():
    return W.gaussian_patches(n=3000, n_patches=4, depth=4, p=12, sigma=0.01, seed=21, precision="fp64")


@pytest.mark.parametrize("precision,tol_x,tol_g", [("fp64", 1e-12, 1e-9), ("mixed", 1e-6, 1e-4)])
def test_rk2_matches_oracle(fmm_mod, oracle_mod, patches, precision, tol_x, tol_g):
    from paper_1008_2410_amd import rk2
    w = patches
    xs = _oracle_rk2(oracle_mod, w.xy, w.gamma, w.sigma, w.depth, w.p)
    target = W.smooth_target_field(w.xy, seed=5)
    dl = xs[-1] - target  # L = 0.5 |x_N - target|^2
    lam_ref, dg_ref = _oracle_rk2_grad(oracle_mod, xs, w.gamma, w.sigma, w.depth, w.p, dl)
    xN, ck = rk2.rk2_forward(_t(w.xy), _t(w.gamma), w.sigma, w.depth, w.p, DT, STEPS, precision)
    assert rel_l2(xN.cpu().numpy() - w.xy, xs[-1] - w.xy) < tol_x
    lam, dg = rk2.rk2_backward(ck, _t(w.gamma), w.sigma, w.depth, w.p, DT, _t(dl), precision)
    assert rel_l2(lam.cpu().numpy(), lam_ref) < tol_g
    assert rel_l2(dg.cpu().numpy(), dg_ref) < tol_g


def test_rk2_gradient_central_differences(fmm_mod, patches):
    """dL/dGamma and dL/dx_0 of the FP64 transport against central differences of it
    (particles away from leaf edges and from the bounding square's extremes)."""
    import torch
    from paper_1008_2410_amd import rk2
    w = patches
    target = W.smooth_target_field(w.xy, seed=6)
    g0 = _t(w.gamma)

    def loss(xy, g):
        xN, _ = rk2.rk2_forward(_t(xy), _t(g), w.sigma, w.depth, w.p, DT, STEPS, "fp64")
        return 0.5 * ((xN.cpu().numpy() - target) ** 2).sum()

    xy0 = _t(w.xy).requires_grad_(True)
    gg = g0.clone().requires_grad_(True)
    xN = rk2.transport(xy0, gg, w.sigma, w.depth, w.p, DT, STEPS, "fp64")
    (0.5 * ((xN - _t(target)) ** 2).sum()).backward()
    dx, dg = xy0.grad.cpu().numpy(), gg.grad.cpu().numpy()
    lo, hi = w.xy.min(axis=0), w.xy.max(axis=0)
    side = (hi - lo).max()
    h = 1e-6
    checked = 0
    for k in np.random.Generator(np.random.PCG64(8)).permutation(w.n):
        frac = ((w.xy[k] - lo) / side * 16) % 1.0
        if np.any(frac < 0.02) or np.any(frac > 0.98):
            continue
        comp = checked % 2
        a, b = w.xy.copy(), w.xy.copy()
        a[k, comp] += h
        b[k, comp] -= h
        fd = (loss(a, w.gamma) - loss(b, w.gamma)) / (2 * h)
        assert abs(fd - dx[k, comp]) <= 1e-5 * abs(fd) + 1e-9, (k, comp, fd, dx[k, comp])
        a, b = w.gamma.copy(), w.gamma.copy()
        a[k] += h
        b[k] -= h
        fd = (loss(w.xy, a) - loss(w.xy, b)) / (2 * h)
        assert abs(fd - dg[k]) <= 1e-5 * abs(fd) + 1e-9, (k, fd, dg[k])
        checked += 1
        if checked == 4:
            break
    assert checked == 4
    torch.cuda.synchronize()


def _oracle_rk2_adaptive(oracle_mod, xy, g, sigma, smax, lmax, p):
    xs = [xy]
    x = xy
    for _ in range(STEPS):
        u0 = oracle_mod.afmm_velocity(x, g, sigma, smax, lmax, p)
        xm = x + 0.5 * DT * u0
        um = oracle_mod.afmm_velocity(xm, g, sigma, smax, lmax, p)
        x = x + DT * um
        xs.append(x)
    return xs


def _oracle_rk2_adaptive_grad(oracle_mod, xs, g, sigma, smax, lmax, p, dl_dxN):
    lam = dl_dxN.copy()
    dg = np.zeros_like(g)
    for x in reversed(xs[:-1]):
        u0 = oracle_mod.afmm_velocity(x, g, sigma, smax, lmax, p)
        xm = x + 0.5 * DT * u0
        dgm, dxm, dsm = oracle_mod.afmm_grad(xm, g, sigma, smax, lmax, p, DT * lam)
        lam_mid = dxm + dsm
        dg0, dx0, ds0 = oracle_mod.afmm_grad(x, g, sigma, smax, lmax, p, 0.5 * DT * lam_mid)
        lam = lam + lam_mid + dx0 + ds0
        dg += dgm + dg0
    return lam, dg


@pytest.mark.parametrize("precision,tol_x,tol_g", [("fp64", 1e-12, 1e-9), ("mixed", 1e-6, 1e-4)])
def test_rk2_adaptive_matches_oracle(fmm_mod, oracle_mod, precision, tol_x, tol_g):
    """The transport and its adjoint with an adaptive tree (leaves of at most 20 particles,
    depth <= 9) built for every evaluation, against the same steps over O6 and O7."""
    from paper_1008_2410_amd import rk2
    r = np.random.Generator(np.random.PCG64(31))
    xy = np.concatenate([r.random((400, 2)), 0.3 + 0.02 * r.random((600, 2)),
                         0.7 + 0.005 * r.standard_normal((300, 2))])
    g = r.standard_normal(len(xy)) / len(xy)
    sigma, smax, lmax, p = 0.002, 20, 9, 12
    xs = _oracle_rk2_adaptive(oracle_mod, xy, g, sigma, smax, lmax, p)
    target = W.smooth_target_field(xy, seed=5)
    dl = xs[-1] - target
    lam_ref, dg_ref = _oracle_rk2_adaptive_grad(oracle_mod, xs, g, sigma, smax, lmax, p, dl)
    xN, ck = rk2.rk2_forward(_t(xy), _t(g), sigma, 0, p, DT, STEPS, precision, adaptive=(smax, lmax))
    assert rel_l2(xN.cpu().numpy() - xy, xs[-1] - xy) < tol_x
    lam, dg = rk2.rk2_backward(ck, _t(g), sigma, 0, p, DT, _t(dl), precision, adaptive=(smax, lmax))
    assert rel_l2(lam.cpu().numpy(), lam_ref) < tol_g
    assert rel_l2(dg.cpu().numpy(), dg_ref) < tol_g


def test_transport_full_size(fmm_mod, oracle_mod):
    """The time-stepped configuration at full size (2^25 particles in 16 patches, depth 11,
    p = 16, dt = 1e-3, 5 steps): the first velocity (mixed) within 1e-5 of O3 on a
    4096-particle sample; the linear impulse sum_i Gamma_i x_i kept by the FP64 steps to
    rounding (each velocity has sum_i Gamma_i u_i = 0: the operator is antisymmetric); the
    FP64 gradient in Gamma along Gamma itself against a central difference of the FP64
    transport."""
    import torch
    from paper_1008_2410_amd import rk2
    w = W.transport_patches()
    dt, steps = w.extra["dt"], w.extra["steps"]
    idx = w.extra["sample"]
    xy, g = _t(w.xy), _t(w.gamma)
    tree = fmm_mod.Tree(xy, w.depth, None)
    u0 = tree.velocity(g, w.sigma, w.p, "mixed").cpu().numpy()[idx]
    tree.close()
    ref = oracle_mod.fmm_velocity(w.xy, w.gamma, w.sigma, w.depth, w.p, None, targets=w.xy[idx])
    err = rel_l2(u0, ref)
    print(f"[transport 2^25] first velocity mixed rel-L2 vs O3 on 4096: {err:.3e}", flush=True)
    assert err < 1e-5
    target = _t(W.smooth_target_field(w.xy, seed=55))

    def run(gm):
        xN, ck = rk2.rk2_forward(xy, gm, w.sigma, w.depth, w.p, dt, steps, "fp64")
        return xN, ck, 0.5 * float(((xN - target) ** 2).sum())

    xN, ck, _ = run(g)
    dx = xN - xy
    drift = float((g[:, None] * dx).sum(0).abs().max())  # change of sum_i Gamma_i x_i
    scale = float((g.abs()[:, None] * dx.abs()).sum())
    print(f"[transport 2^25] linear impulse drift {drift:.3e} (scale {scale:.3e})", flush=True)
    assert drift < 1e-10 * scale
    _, dg = rk2.rk2_backward(ck, g, w.sigma, w.depth, w.p, dt, xN - target, "fp64")
    eps = 1e-5
    fd = (run(g * (1 + eps))[2] - run(g * (1 - eps))[2]) / (2 * eps)
    ad = float((dg * g).sum())
    print(f"[transport 2^25] dL/deps along Gamma: adjoint {ad:.10e}, central difference {fd:.10e}", flush=True)
    assert abs(ad - fd) <= 1e-6 * abs(fd)
    torch.cuda.synchronize()
