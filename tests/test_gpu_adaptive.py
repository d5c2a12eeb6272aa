"""GPU parity of the adaptive-tree evaluation (include/fmm2d_adaptive.h) against the
oracle O6.

Structure (integers, bit-exact): the eight sizes of fmm_atree_info (cells, leaves, list
lengths, deepest level, near-field pairs) and the leaf (level, ix, iy) of every
particle equal the oracle's.  The device build equals the host reference build: same
sizes and leaves, and every evaluation (forward and parts, both precisions) bit for bit,
which reads every array of the tree.  The adjoint (fmm_atree_velocity_backward) against
the oracle's O7: FP64 within 1e-9 and mixed within 1e-4 (vector rel-L2), the bars of the
uniform tree's adjoint.  Values: FP64 within 1e-12 (rel-L2) of O6 and mixed within
1e-5 (FP32 records relative to the leaf centre lose accuracy in wide leaves: 2.4e-6 with
the whole set in one leaf), the near and far parts separately (the two sides use
different operator forms: scaled tables and Horner on the GPU, unscaled powers in the
oracle).  With equal leaf
counts the tree is the uniform one and the result equals fmm_velocity's.  At 2^20
particles, sampled particles against the direct sum O1 (p = 20, the far kernel exact at
the leaf widths used).
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_1008_2410_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _clustered(seed=1):
    r = np.random.Generator(np.random.PCG64(seed))
    xy = np.concatenate([r.random((500, 2)), 0.3 + 0.02 * r.random((900, 2)),
                         0.71 + 0.005 * r.standard_normal((300, 2)), [[0.999, 0.001], [0.0, 0.0]]])
    return xy, r.standard_normal(len(xy))


def _cases():
    xy, g = _clustered()
    for smax, lmax in ((20, 9), (5, 7), (1, 5), (60, 12), (300, 8), (3, 0), (2, 15)):
        yield f"clustered-{smax}-{lmax}", xy, g, smax, lmax, 0.002
    w = W.gaussian_patches(n=60000, depth=5, p=12, sigma=0.004, seed=11, precision="fp64")
    yield "patches-64-9", w.xy, w.gamma, 64, 9, 0.0005
    yield "patches-32-11", w.xy, w.gamma, 32, 11, 0.0002


CASES = list(_cases())


def _oracle_structure(oracle_mod, xy, smax, lmax):
    t = oracle_mod.adaptive_tree(xy, smax, lmax)
    cells, lo = t["cells"], t["leaf_of"]
    return t["sizes"], (cells[lo, 0], cells[lo, 1], cells[lo, 2])


@pytest.mark.parametrize("name,xy,g,smax,lmax,sigma", CASES, ids=[c[0] for c in CASES])
def test_structure_matches_oracle(fmm_mod, oracle_mod, name, xy, g, smax, lmax, sigma):
    tree = fmm_mod.ATree(_t(xy), smax, lmax)
    sizes, leaves = _oracle_structure(oracle_mod, xy, smax, lmax)
    info = tree.info()
    assert {k: info[k] for k in sizes} == sizes
    assert info["root_box"] == oracle_mod.root_box(xy)
    for got, ref in zip(tree.leaves(), leaves):
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("name,xy,g,smax,lmax,sigma", CASES, ids=[c[0] for c in CASES])
def test_velocity_matches_oracle(fmm_mod, oracle_mod, name, xy, g, smax, lmax, sigma):
    p = 14
    rn, rf = oracle_mod.afmm_velocity(xy, g, sigma, smax, lmax, p, parts=True)
    tree = fmm_mod.ATree(_t(xy), smax, lmax)
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        near, far = (a.cpu().numpy() for a in tree.velocity_parts(_t(g), sigma, p, precision))
        assert rel_l2(near, rn) < tol, (precision, rel_l2(near, rn))
        if np.any(rf != 0):
            assert rel_l2(far, rf) < 1e-12, (precision, rel_l2(far, rf))  # FP64 expansions in both forms
        else:
            assert np.all(far == 0)
        full = tree.velocity(_t(g), sigma, p, precision).cpu().numpy()
        assert rel_l2(full, rn + rf) < tol
        again = tree.velocity(_t(g), sigma, p, precision).cpu().numpy()
        assert np.array_equal(full, again)


def _same_atree(td, th, g, sigma, p):
    assert td.info() == th.info()
    for a, b in zip(td.leaves(), th.leaves()):
        assert np.array_equal(a, b)
    for precision in ("fp64", "mixed"):
        assert np.array_equal(td.velocity(g, sigma, p, precision).cpu().numpy(),
                              th.velocity(g, sigma, p, precision).cpu().numpy()), precision
        a = td.velocity_parts(g, sigma, p, precision)
        b = th.velocity_parts(g, sigma, p, precision)
        assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b)), precision


@pytest.mark.parametrize("name,xy,g,smax,lmax,sigma", CASES, ids=[c[0] for c in CASES])
def test_device_build_equals_host_build(fmm_mod, name, xy, g, smax, lmax, sigma):
    x = _t(xy)
    td = fmm_mod.ATree(x, smax, lmax, builder="device")
    th = fmm_mod.ATree(x, smax, lmax, builder="host")
    _same_atree(td, th, _t(g), sigma, 12)


def test_device_build_equals_host_build_clustered_large(fmm_mod):
    """2^18 particles of the clustered workload (background and Gaussian clusters), leaves
    capped at 32 and 128 down to depth 15: deep, uneven trees with many W/X entries."""
    w = W.clustered_background(n=1 << 18)
    x = _t(w.xy)
    for smax in (32, 128):
        td = fmm_mod.ATree(x, smax, 15, builder="device")
        th = fmm_mod.ATree(x, smax, 15, builder="host")
        info = td.info()
        assert info["deepest"] >= 12 and info["w"] > 0
        _same_atree(td, th, _t(w.gamma), w.sigma, 16)
        td.close()
        th.close()


@pytest.mark.parametrize("name,xy,g,smax,lmax,sigma", CASES, ids=[c[0] for c in CASES])
def test_backward_matches_oracle(fmm_mod, oracle_mod, name, xy, g, smax, lmax, sigma):
    p = 12
    dl = np.random.Generator(np.random.PCG64(9)).standard_normal((len(xy), 2))
    ref = oracle_mod.afmm_grad(xy, g, sigma, smax, lmax, p, dl)
    for builder in ("device", "host"):
        tree = fmm_mod.ATree(_t(xy), smax, lmax, builder=builder)
        for precision, tol in (("fp64", 1e-9), ("mixed", 1e-4)):
            got = [a.cpu().numpy() for a in tree.velocity_backward(_t(g), sigma, p, precision, _t(dl), need_src=True)]
            errs = [rel_l2(a, b) for a, b in zip(got, ref)]
            print(f"[adaptive adjoint {name} {builder} {precision}] rel-L2 vs O7: dgamma {errs[0]:.2e} "
                  f"dx_eval {errs[1]:.2e} dx_src {errs[2]:.2e}", flush=True)
            for what, err in zip(("dgamma", "dx_eval", "dx_src"), errs):
                assert err < tol, (builder, precision, what, err)
            # the same call without the source output gives the same other two
            dg, dx = tree.velocity_backward(_t(g), sigma, p, precision, _t(dl))
            assert np.array_equal(dg.cpu().numpy(), got[0]) and np.array_equal(dx.cpu().numpy(), got[1])
        tree.close()


def test_autograd_through_the_adaptive_tree(fmm_mod, oracle_mod):
    """fmm.velocity over an ATree: torch autograd gives dL/dGamma and dL/dxy (every particle
    moving as evaluation point and as source) equal to O7's."""
    xy, g = _clustered(2)
    dl = np.random.Generator(np.random.PCG64(12)).standard_normal((len(xy), 2))
    sigma, p = 0.002, 12
    dg_ref, dxe_ref, dxs_ref = oracle_mod.afmm_grad(xy, g, sigma, 20, 9, p, dl)
    x = _t(xy).requires_grad_(True)
    gg = _t(g).requires_grad_(True)
    tree = fmm_mod.ATree(_t(xy), 20, 9)
    uv = fmm_mod.velocity(x, gg, sigma, 0, p, "fp64", tree=tree)
    (uv * _t(dl)).sum().backward()
    assert rel_l2(gg.grad.cpu().numpy(), dg_ref) < 1e-9
    assert rel_l2(x.grad.cpu().numpy(), dxe_ref + dxs_ref) < 1e-9


def test_rebuild_equals_fresh_tree(fmm_mod):
    """A rebuilt tree (new positions, the old tree's workspace) gives what a tree built
    afresh gives, bit for bit, forward and adjoint: to a uniform cloud (fewer cells), to a
    tight cluster (more cells: the expansion arrays grow) and back."""
    xy, g = _clustered(3)
    n = len(xy)
    r = np.random.Generator(np.random.PCG64(41))
    x_uni = r.random((n, 2))
    x_tight = 0.5 + 0.004 * r.standard_normal((n, 2))
    dl = _t(r.standard_normal((n, 2)))
    gt = _t(g)
    sigma, p = 0.0005, 12
    tree = fmm_mod.ATree(_t(xy), 8, 12)
    for precision in ("fp64", "mixed"):  # fill the workspace, the adjoint's arrays included
        tree.velocity(gt, sigma, p, precision)
        tree.velocity_backward(gt, sigma, p, precision, dl, need_src=True)
    for x in (x_uni, x_tight, xy):
        tree.rebuild(_t(x))
        fresh = fmm_mod.ATree(_t(x), 8, 12)
        _same_atree(tree, fresh, gt, sigma, p)
        for precision in ("fp64", "mixed"):
            a = tree.velocity_backward(gt, sigma, p, precision, dl, need_src=True)
            b = fresh.velocity_backward(gt, sigma, p, precision, dl, need_src=True)
            assert all(np.array_equal(u.cpu().numpy(), v.cpu().numpy()) for u, v in zip(a, b)), precision
        fresh.close()
    tree.close()


def test_rebuild_errors_leave_the_tree(fmm_mod):
    import ctypes

    from paper_1008_2410_amd import _lib
    xy, g = _clustered(5)
    n = len(xy)
    tree = fmm_mod.ATree(_t(xy), 16, 8, (0.0, 0.0, 1.0))
    before = tree.velocity(_t(g), 0.002, 10, "fp64").cpu().numpy()
    out = ctypes.c_void_p()
    other = _t(np.random.Generator(np.random.PCG64(6)).random((n + 1, 2)))
    rc = _lib.load().fmm_atree_rebuild(tree.handle, ctypes.c_void_p(other.data_ptr()), n + 1, None, None,
                                       ctypes.byref(out))
    assert rc == _lib.FMM_EINVAL and not out.value
    bad = xy.copy()
    bad[11] = (1.5, 0.5)
    with pytest.raises(_lib.FmmError) as e:
        tree.rebuild(_t(bad), (0.0, 0.0, 1.0))
    assert e.value.status == _lib.FMM_ERANGE and "particle 11" in str(e.value)
    assert np.array_equal(tree.velocity(_t(g), 0.002, 10, "fp64").cpu().numpy(), before)
    tree.close()


def test_near_occupancy_cap_leaves_results_unchanged(fmm_mod):
    """FMM_OPT_NEAR_OCCUPANCY only limits how many near-field wavefronts share the chip with
    the far field: every cap, the automatic choice and the serialised call give the same
    bits, in both precisions, on a rebuilt tree too; values outside [-1, 8] and other keys
    are rejected."""
    from paper_1008_2410_amd import _lib
    name, xy, g, smax, lmax, sigma = CASES[-2]
    gt = _t(g)
    tree = fmm_mod.ATree(_t(xy), smax, lmax)
    for rebuilt in (False, True):
        if rebuilt:
            tree.set_option(_lib.FMM_OPT_NEAR_OCCUPANCY, 3)
            tree.rebuild(_t(xy[::-1].copy()))
            gt = _t(g[::-1].copy())
        for precision in ("mixed", "fp64"):
            ref = tree.velocity(gt, sigma, 12, precision, serial=True).cpu().numpy()
            for occ in (0, 1, 5, 8, -1):
                tree.set_option(_lib.FMM_OPT_NEAR_OCCUPANCY, occ)
                got = tree.velocity(gt, sigma, 12, precision).cpu().numpy()
                assert np.array_equal(got, ref), (rebuilt, precision, occ)
    for key, value in ((_lib.FMM_OPT_NEAR_OCCUPANCY, 9), (_lib.FMM_OPT_NEAR_OCCUPANCY, -2),
                       (_lib.FMM_OPT_SCHEDULE, 0)):
        with pytest.raises(_lib.FmmError) as e:
            tree.set_option(key, value)
        assert e.value.status == _lib.FMM_EINVAL
    tree.close()


def test_equal_leaf_counts_match_the_uniform_tree(fmm_mod, oracle_mod):
    r = np.random.Generator(np.random.PCG64(8))
    h = 1.0 / 64
    g1 = (np.arange(64) + 0.5) * h
    xy = np.stack(np.meshgrid(g1, g1, indexing="xy"), -1).reshape(-1, 2) + (r.random((4096, 2)) - 0.5) * 0.3 * h
    g = r.standard_normal(4096)
    root = (0.0, 0.0, 1.0)
    at = fmm_mod.ATree(_t(xy), 15, 4, root)
    info = at.info()
    assert info["leaves"] == 256 and info["w"] == 0 and info["deepest"] == 4
    ut = fmm_mod.Tree(_t(xy), 4, root)
    assert info["p2p_pairs"] == ut.info()["p2p_pairs"]
    for precision, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        a = at.velocity(_t(g), 0.01, 12, precision).cpu().numpy()
        u = ut.velocity(_t(g), 0.01, 12, precision).cpu().numpy()
        assert rel_l2(a, u) < tol, precision


def test_small_and_degenerate(fmm_mod, oracle_mod):
    for xy in (np.array([[0.3, 0.4]]), np.array([[0.3, 0.4], [0.3, 0.4]]), np.array([[0.1, 0.1], [0.9, 0.8]])):
        g = np.arange(1.0, len(xy) + 1.0)
        for smax, lmax in ((1, 0), (1, 6), (4, 3)):
            tree = fmm_mod.ATree(_t(xy), smax, lmax)
            u = tree.velocity(_t(g), 0.05, 8, "fp64").cpu().numpy()
            ref = oracle_mod.afmm_velocity(xy, g, 0.05, smax, lmax, 8)
            assert np.allclose(u, ref, rtol=1e-12, atol=1e-14), (xy, smax, lmax)


def test_large_sampled_against_direct_sum(fmm_mod, oracle_mod):
    """2^20 particles in Gaussian patches (the workload's sigma), leaves capped at 64 down to
    depth 10 (leaf width >= 8 sigma): 2000 sampled particles against O1."""
    w = W.gaussian_patches(n=1 << 20, depth=10, p=20)
    tree = fmm_mod.ATree(_t(w.xy), 64, 10)
    info = tree.info()
    assert info["w"] > 0 and info["deepest"] == 10
    side = info["root_box"][2]
    assert side / 2 ** 10 >= 8 * w.sigma  # exp(-d^2/(2 sigma^2)) < 2e-14 beyond one leaf
    idx = np.random.Generator(np.random.PCG64(4)).choice(w.n, 2000, replace=False)
    ref = oracle_mod.direct(w.xy, w.gamma, w.sigma, targets=w.xy[idx])
    for precision, tol in (("fp64", 1e-8), ("mixed", 2e-5)):
        u = tree.velocity(_t(w.gamma), w.sigma, 20, precision).cpu().numpy()
        err = rel_l2(u[idx], ref)
        print(f"[adaptive 2^20 {precision}] rel-L2 vs direct on 2000 particles: {err:.3e}", flush=True)
        assert err < tol


def test_linear_impulse_fp64(fmm_mod):
    """sum_i Gamma_i u_i = 0 to roundoff for the FP64 adaptive evaluation (antisymmetric
    operator: odd near kernel over symmetric U, M2L over symmetric V, M2P/P2L transposes)."""
    xy, g = _clustered(4)
    for smax, lmax in ((20, 9), (1, 5), (60, 12)):
        u = fmm_mod.ATree(_t(xy), smax, lmax).velocity(_t(g), 0.001, 12, "fp64").cpu().numpy()
        imp = (g[:, None] * u).sum(axis=0)
        assert np.all(np.abs(imp) < 1e-13 * (np.abs(g)[:, None] * np.abs(u)).sum()), (smax, lmax, imp)


@pytest.mark.parametrize("builder", ["device", "host"])
def test_errors(fmm_mod, builder):
    from paper_1008_2410_amd import _lib
    xy = np.array([[0.5, 0.5], [0.2, 0.3], [1.5, 0.2], [0.1, 0.1], [1.2, 0.1]])
    with pytest.raises(_lib.FmmError) as e:
        fmm_mod.ATree(_t(xy), 4, 3, (0.0, 0.0, 1.0), builder=builder)
    assert e.value.status == _lib.FMM_ERANGE and "particle 2" in str(e.value)
    xy[1, 0] = np.nan
    for root in (None, (0.0, 0.0, 1.0)):
        with pytest.raises(_lib.FmmError) as e:
            fmm_mod.ATree(_t(xy), 4, 3, root, builder=builder)
        assert e.value.status == _lib.FMM_EINVAL
    tree = fmm_mod.ATree(_t(np.array([[0.1, 0.2], [0.3, 0.4]])), 1, 3, builder=builder)
    for bad in ((0.0, 8, "fp64"), (0.1, 0, "fp64"), (0.1, 33, "fp64"), (0.1, 8, 7)):
        with pytest.raises(_lib.FmmError) as e:
            tree.velocity(_t(np.ones(2)), *bad)
        assert e.value.status == _lib.FMM_EINVAL
