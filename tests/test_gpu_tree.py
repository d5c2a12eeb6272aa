"""The device tree build (stages 1-3 on the GPU) against the host reference build.

Both builds must give the same tree array for array, so the checks are bit-exact: the
permutation and leaf of every particle, the statistics of fmm_tree_info, the
near-field plan, and every output of the evaluation (forward, parts, adjoint), which
reads every other array of the tree.  The host build itself is checked against the
oracle's binning and pair counts in test_gpu_forward.py.
"""
import numpy as np
import pytest

from paper_1008_2410_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _cases():
    r = np.random.Generator(np.random.PCG64(12))
    yield "uniform", W.uniform_lamb_oseen()
    yield "patches", W.gaussian_patches(n=60000, depth=5, p=12, sigma=0.004, seed=11, precision="fp64")
    yield "clump", W.Workload("clump", 0.5 + 0.01 * r.random((300, 2)), r.standard_normal(300), 0.003, 5, 8,
                              (0, 0, 1), "fp64")
    yield "sparse12", W.Workload("sparse12", r.random((1000, 2)), r.standard_normal(1000), 0.001, 12, 6, None,
                                 "fp64")
    yield "one", W.Workload("one", np.array([[0.3, 0.7]]), np.array([1.0]), 0.1, 3, 5, (0, 0, 1), "fp64")
    yield "edges", W.Workload("edges", np.array([[1.0, 1.0], [0.5, 0.5], [0.25, 0.75], [0.0, 1.0], [0.5, 0.5],
                                                 [0.1, 0.9]]), np.array([1.0, -2.0, 0.5, 0.25, 1.5, -1.0]), 0.05,
                              3, 6, (0, 0, 1), "fp64")
    yield "depth1", W.Workload("depth1", r.random((400, 2)), r.standard_normal(400), 0.05, 1, 4, None, "fp64")


CASES = list(_cases())


@pytest.mark.parametrize("name,w", CASES, ids=[c[0] for c in CASES])
def test_device_build_equals_host_build(fmm_mod, name, w):
    xy = _t(w.xy)
    td = fmm_mod.Tree(xy, w.depth, w.root_box, builder="device")
    th = fmm_mod.Tree(xy, w.depth, w.root_box, builder="host")
    assert td.info() == th.info()
    assert td.near_plan() == th.near_plan()
    pd, ld = td.permutation()
    ph, lh = th.permutation()
    assert np.array_equal(pd.cpu().numpy(), ph.cpu().numpy())
    assert np.array_equal(ld.cpu().numpy(), lh.cpu().numpy())
    g = _t(w.gamma)
    dl = _t(np.random.Generator(np.random.PCG64(3)).standard_normal((w.n, 2)))
    for precision in ("fp64", "mixed"):
        assert np.array_equal(td.velocity(g, w.sigma, w.p, precision).cpu().numpy(),
                              th.velocity(g, w.sigma, w.p, precision).cpu().numpy()), precision
        a = td.velocity_parts(g, w.sigma, w.p, precision)
        b = th.velocity_parts(g, w.sigma, w.p, precision)
        assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b)), precision
        a = td.velocity_backward(g, w.sigma, w.p, precision, dl, need_src=True)
        b = th.velocity_backward(g, w.sigma, w.p, precision, dl, need_src=True)
        assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b)), precision


def test_device_build_large_lattice(fmm_mod):
    """2^20 particles, depth 8: the multi-tile radix sort and scans at size."""
    w = W.lattice_lamb_oseen()
    xy = _t(w.xy)
    td = fmm_mod.Tree(xy, w.depth, w.root_box, builder="device")
    th = fmm_mod.Tree(xy, w.depth, w.root_box, builder="host")
    assert td.info() == th.info()
    assert np.array_equal(td.permutation()[0].cpu().numpy(), th.permutation()[0].cpu().numpy())
    g = _t(w.gamma)
    assert np.array_equal(td.velocity(g, w.sigma, w.p, "mixed").cpu().numpy(),
                          th.velocity(g, w.sigma, w.p, "mixed").cpu().numpy())


def test_device_build_option_rebuilds_plan(fmm_mod):
    """Changing the dense threshold rebuilds the plan on the device: same as the host tree's."""
    w = CASES[1][1]
    xy = _t(w.xy)
    td = fmm_mod.Tree(xy, w.depth, w.root_box, builder="device")
    th = fmm_mod.Tree(xy, w.depth, w.root_box, builder="host")
    g = _t(w.gamma)
    for dense in (1, 100):
        td.set_option(7, dense)
        th.set_option(7, dense)
        assert td.near_plan() == th.near_plan()
        assert np.array_equal(td.velocity(g, w.sigma, w.p, "mixed").cpu().numpy(),
                              th.velocity(g, w.sigma, w.p, "mixed").cpu().numpy())


def test_device_build_errors(fmm_mod):
    from paper_1008_2410_amd import _lib
    xy = np.array([[0.5, 0.5], [0.2, 0.3], [1.5, 0.2], [0.1, 0.1]])
    with pytest.raises(_lib.FmmError) as e:
        fmm_mod.Tree(_t(xy), 3, (0.0, 0.0, 1.0))
    assert e.value.status == _lib.FMM_ERANGE
    assert "particle 2" in str(e.value)
    xy[1, 0] = np.nan
    with pytest.raises(_lib.FmmError) as e:
        fmm_mod.Tree(_t(xy), 3, None)
    assert e.value.status == _lib.FMM_EINVAL


def _same_tree_outputs(ta, tb, g, sigma, p, dl):
    """Bit-exact equality of two trees' facts and of every evaluation they give."""
    assert ta.info() == tb.info()
    assert ta.near_plan() == tb.near_plan()
    assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(ta.permutation(), tb.permutation()))
    for precision in ("mixed", "fp64"):
        assert np.array_equal(ta.velocity(g, sigma, p, precision).cpu().numpy(),
                              tb.velocity(g, sigma, p, precision).cpu().numpy()), precision
        a = ta.velocity_parts(g, sigma, p, precision)
        b = tb.velocity_parts(g, sigma, p, precision)
        assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b)), precision
        a = ta.velocity_backward(g, sigma, p, precision, dl, need_src=True)
        b = tb.velocity_backward(g, sigma, p, precision, dl, need_src=True)
        assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b)), precision


def test_rebuild_equals_fresh_tree(fmm_mod):
    """A rebuilt tree (new positions, the old tree's workspace) gives what a tree built
    afresh for those positions gives, bit for bit: from a uniform cloud to Gaussian
    patches in the same root box (most cells fall empty, and their multipoles must not
    keep the old values), and back; the options of the old tree carry over."""
    w = W.gaussian_patches(n=60000, depth=5, p=12, sigma=0.004, seed=11, precision="fp64")
    r = np.random.Generator(np.random.PCG64(21))
    lo = min(0.0, float(w.xy.min())) - 1e-3
    box = (lo, lo, max(1.0, float(w.xy.max())) + 1e-3 - lo)  # holds both clouds
    x_uni = _t(r.random((w.n, 2)))
    x_pat = _t(w.xy)
    g = _t(w.gamma)
    dl = _t(r.standard_normal((w.n, 2)))
    tree = fmm_mod.Tree(x_uni, w.depth, box)
    tree.set_option(7, 48)  # dense leaf threshold
    tree.set_option(2, 2)   # coarse level
    # fill the workspace (both precisions, the adjoint's arrays too) with this tree's values
    for precision in ("fp64", "mixed"):
        tree.velocity(g, w.sigma, w.p, precision)
        tree.velocity_backward(g, w.sigma, w.p, precision, dl, need_src=True)
    for x in (x_pat, x_uni):
        tree.rebuild(x, box)
        fresh = fmm_mod.Tree(x, w.depth, box)
        fresh.set_option(7, 48)
        fresh.set_option(2, 2)
        _same_tree_outputs(tree, fresh, g, w.sigma, w.p, dl)
        fresh.close()
    # bounding-square rebuild (root box from the new positions)
    tree.rebuild(x_pat)
    fresh = fmm_mod.Tree(x_pat, w.depth)
    fresh.set_option(7, 48)
    fresh.set_option(2, 2)
    _same_tree_outputs(tree, fresh, g, w.sigma, w.p, dl)
    tree.close()


def test_rebuild_errors_leave_the_tree(fmm_mod):
    """A rebuild that fails (other n, a particle outside the root box, a closed tree)
    leaves the old tree as it was."""
    import ctypes

    from paper_1008_2410_amd import _lib
    r = np.random.Generator(np.random.PCG64(22))
    n = 2000
    xy = _t(r.random((n, 2)))
    g = _t(r.standard_normal(n))
    tree = fmm_mod.Tree(xy, 4, (0.0, 0.0, 1.0))
    before = tree.velocity(g, 0.01, 8, "fp64").cpu().numpy()
    lib = _lib.load()
    out = ctypes.c_void_p()
    other = _t(r.random((n + 1, 2)))
    rc = lib.fmm_rebuild_tree(tree.handle, ctypes.c_void_p(other.data_ptr()), n + 1, None, None, ctypes.byref(out))
    assert rc == _lib.FMM_EINVAL and not out.value
    with pytest.raises(ValueError):
        tree.rebuild(other)
    bad = r.random((n, 2))
    bad[7] = (1.5, 0.5)
    with pytest.raises(_lib.FmmError) as e:
        tree.rebuild(_t(bad), (0.0, 0.0, 1.0))
    assert e.value.status == _lib.FMM_ERANGE and "particle 7" in str(e.value)
    assert np.array_equal(tree.velocity(g, 0.01, 8, "fp64").cpu().numpy(), before)
    rc = lib.fmm_rebuild_tree(None, ctypes.c_void_p(xy.data_ptr()), n, None, None, ctypes.byref(out))
    assert rc == _lib.FMM_ESTATE
    tree.close()


def _pool_bytes(attr):
    """An attribute of the device's default stream-ordered pool (the library's arrays)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), 0) == 0
    v = ctypes.c_uint64()
    assert hip.hipMemPoolGetAttribute(pool, ctypes.c_int(attr), ctypes.byref(v)) == 0
    return hip, pool, v.value


def test_rebuild_holds_one_tree(fmm_mod):
    """A rebuild with a workspace releases the old tree's arrays before it allocates the
    new ones and keeps its temporaries in the workspace's per-call region: the library's
    device memory never grows by more than a small part of one tree's arrays while the
    tree is rebuilt (building the new tree beside the old one, with temporaries from the
    pool, would add about twice a tree's arrays).  Outputs after the rebuild as from a
    fresh tree (bit for bit)."""
    import ctypes
    used_cur, used_high = 7, 8   # hipMemPoolAttrUsedMemCurrent, hipMemPoolAttrUsedMemHigh
    r = np.random.Generator(np.random.PCG64(31))
    n, depth, p, sigma = 1 << 18, 7, 12, 0.002
    x0 = _t(r.random((n, 2)))
    x1 = _t(np.clip(r.random((n, 2)) ** 1.5, 0.0, 1.0))
    g = _t(r.standard_normal(n))
    dl = _t(r.standard_normal((n, 2)))
    box = (0.0, 0.0, 1.0)
    tree = fmm_mod.Tree(x0, depth, box)
    tree.velocity(g, sigma, p, "mixed")
    tree.velocity_backward(g, sigma, p, "mixed", dl, need_src=True)
    import torch
    torch.cuda.synchronize()
    hip, pool, before = _pool_bytes(used_cur)
    other = fmm_mod.Tree(x1, depth, box)
    torch.cuda.synchronize()
    tree_bytes = _pool_bytes(used_cur)[2] - before
    other.close()
    torch.cuda.synchronize()
    assert tree_bytes > 20 * n   # the sorted positions, permutations and staging alone
    zero = ctypes.c_uint64(0)
    if hip.hipMemPoolSetAttribute(pool, ctypes.c_int(used_high), ctypes.byref(zero)) != 0:
        pytest.skip("the pool's high-water mark cannot be reset on this runtime")
    before = _pool_bytes(used_cur)[2]
    assert _pool_bytes(used_high)[2] <= before + (1 << 20)
    tree.rebuild(x1, box)
    torch.cuda.synchronize()
    growth = _pool_bytes(used_high)[2] - before
    assert growth < 0.25 * tree_bytes, (growth, tree_bytes)
    fresh = fmm_mod.Tree(x1, depth, box)
    _same_tree_outputs(tree, fresh, g, sigma, p, dl)
    fresh.close()
    tree.close()


def test_rebuild_without_workspace(fmm_mod):
    """A rebuild before any evaluation (no workspace yet, so the build's temporaries come
    from the pool) gives the tree a fresh build gives, bit for bit; so does a second
    rebuild after an evaluation (temporaries in the workspace's per-call region)."""
    r = np.random.Generator(np.random.PCG64(41))
    n, depth, p, sigma = 30000, 5, 10, 0.004
    box = (0.0, 0.0, 1.0)
    x0, x1, x2 = (_t(r.random((n, 2))) for _ in range(3))
    g = _t(r.standard_normal(n))
    dl = _t(r.standard_normal((n, 2)))
    tree = fmm_mod.Tree(x0, depth, box)
    tree.rebuild(x1, box)
    fresh = fmm_mod.Tree(x1, depth, box)
    _same_tree_outputs(tree, fresh, g, sigma, p, dl)
    fresh.close()
    tree.rebuild(x2, box)
    fresh = fmm_mod.Tree(x2, depth, box)
    _same_tree_outputs(tree, fresh, g, sigma, p, dl)
    fresh.close()
    tree.close()
