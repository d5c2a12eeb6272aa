"""GPU parity of the mutual near-field form.

Pairs of neighbouring dense leaves are evaluated once for both particles (the
regularized kernel is odd) and summed through per-direction slots; the rest of
stage 9 runs from the target end.  Bars: the near field (stage 9) against the
oracle's, FP64 rel-L2 <= 1e-10 and mixed <= 1e-5; against the target-centric form
FP64 <= 1e-13 and mixed <= 2e-6 (the two forms round differently); repeated
calls bit-identical.
"""
import numpy as np
import pytest

from conftest import rel_l2
from paper_1008_2410_amd import workloads as W

pytestmark = pytest.mark.gpu

OPT_NEAR_MUTUAL, OPT_DENSE_LEAF = 6, 7


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _parts(tree, w, precision):
    near, far = tree.velocity_parts(_t(w.gamma), w.sigma, w.p, precision)
    return near.cpu().numpy(), far.cpu().numpy()


@pytest.fixture(scope="module")
def patches():
    # 60000 particles in Gaussian patches, depth 5: leaves from 1 to several hundred
    # particles; sigma = 0.004 gives both tile classes (with and without the exponential).
    return W.gaussian_patches(n=60000, depth=5, p=12, sigma=0.004, seed=11, precision="fp64")


@pytest.mark.parametrize("dense", [1, 24, 32, 100])
@pytest.mark.parametrize("precision,tol,tol_tc", [("fp64", 1e-10, 1e-13), ("mixed", 1e-5, 2e-6)])
def test_mutual_near_field(fmm_mod, oracle_mod, patches, dense, precision, tol, tol_tc):
    w = patches
    counts = oracle_mod.leaf_counts(w.xy, w.depth, oracle_mod.root_box(w.xy))
    occupied = counts[counts > 0]
    assert dense == 1 or (occupied.min() < dense <= occupied.max())  # both forms are exercised
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    tree.set_option(OPT_DENSE_LEAF, dense)
    near, far = _parts(tree, w, precision)
    on, of = oracle_mod.fmm_velocity(w.xy, w.gamma, w.sigma, w.depth, w.p, w.root_box, parts=True)
    assert rel_l2(near, on) < tol
    full = tree.velocity(_t(w.gamma), w.sigma, w.p, precision).cpu().numpy()
    assert rel_l2(full, on + of) < tol
    again = tree.velocity(_t(w.gamma), w.sigma, w.p, precision).cpu().numpy()
    assert np.array_equal(full, again)
    tree.set_option(OPT_NEAR_MUTUAL, 0)
    near_tc, far_tc = _parts(tree, w, precision)
    assert rel_l2(near, near_tc) < tol_tc
    assert np.array_equal(far, far_tc)


def test_mutual_ragged_tiles(fmm_mod, oracle_mod):
    """Leaves holding 1, 15, 16, 17, 33, 63, 64, 65, 127, 128, 129 and 200 particles next
    to each other (depth 3), every dense threshold form, FP64 against the oracle."""
    r = np.random.Generator(np.random.PCG64(5))
    sizes = {(2, 2): 200, (3, 2): 129, (4, 2): 128, (2, 3): 127, (3, 3): 65, (4, 3): 64,
             (2, 4): 63, (3, 4): 33, (4, 4): 17, (5, 4): 16, (5, 3): 15, (5, 2): 1, (1, 1): 70}
    xy = np.concatenate([(np.array(c) + r.random((m, 2))) / 8.0 for c, m in sizes.items()])
    g = r.standard_normal(len(xy))
    w = W.Workload("ragged", xy, g, 0.01, 3, 10, (0.0, 0.0, 1.0), "fp64")
    on = oracle_mod.fmm_velocity(xy, g, w.sigma, w.depth, w.p, w.root_box, parts=True)[0]
    tree = fmm_mod.Tree(_t(xy), w.depth, w.root_box)
    for dense in (1, 16, 17, 64, 65, 1 << 30):
        tree.set_option(OPT_DENSE_LEAF, dense)
        plan = tree.near_plan()
        if dense == 1:  # every pair of occupied neighbouring leaves is a mutual pair
            assert plan["mutual_pairs"] == tree.info()["p2p_pairs"]
        if dense == 1 << 30:
            assert plan["mutual_items"] == 0 and plan["mutual_pairs"] == 0
        for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
            near, _ = _parts(tree, w, precision)
            assert rel_l2(near, on) < tol, (dense, precision)


def test_mutual_option_errors(fmm_mod):
    from paper_1008_2410_amd import _lib
    w = W.uniform_lamb_oseen(n=500, depth=3)
    tree = fmm_mod.Tree(_t(w.xy), w.depth, w.root_box)
    for key, bad in ((OPT_NEAR_MUTUAL, 2), (OPT_DENSE_LEAF, 0)):
        with pytest.raises(_lib.FmmError):
            tree.set_option(key, bad)
