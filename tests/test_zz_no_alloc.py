"""fmm_velocity_noalloc (the evaluation for callers that cannot allocate, in the
library's static device workspace) against fmm_velocity, through the C ABI: the same bits
on two calls in a row, the second on a smaller input, in both precisions; the size limit
and the missing-table precondition give their documented errors."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _call(lib, name, tree, g, sigma, p, precision, out):
    import torch
    from paper_1008_2410_amd import _lib
    fn = getattr(lib, name)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(tree.handle, ctypes.c_void_p(g.data_ptr()), float(sigma), int(p), int(precision), s, None,
              ctypes.c_void_p(out.data_ptr())), _lib


def test_noalloc_matches_velocity(fmm_mod):
    import torch
    from paper_1008_2410_amd import _lib, workloads as W
    lib = _lib.load()
    cases = [W.gaussian_patches(n=300_000, n_patches=4, depth=7, p=16, sigma=0.002, seed=71, n_sample=8),
             W.uniform_lamb_oseen(n=40_000, seed=72, depth=6, p=12)]
    prepared = {}
    for w in cases:
        for precision in (_lib.FMM_MIXED, _lib.FMM_FP64):
            if (w.p, precision) not in prepared:  # the tables of p, made by an allocating call on another tree
                other = fmm_mod.Tree(_t(w.xy[:1000]), 3, w.root_box)
                other.velocity(_t(w.gamma[:1000]), w.sigma, w.p, precision)
                other.close()
                prepared[(w.p, precision)] = True
    trees = [fmm_mod.Tree(_t(w.xy), w.depth, w.root_box) for w in cases]
    gam = [_t(w.gamma) for w in cases]
    outs = [torch.full((w.n, 2), float("nan"), dtype=torch.float64, device="cuda") for w in cases]
    refs = [torch.empty((w.n, 2), dtype=torch.float64, device="cuda") for w in cases]
    # a first call loads the library's code objects and the static workspace on the device
    # (the HIP runtime does that on first use); the memory check covers the calls after it
    rc, _ = _call(lib, "fmm_velocity_noalloc", trees[1], gam[1], cases[1].sigma, cases[1].p, _lib.FMM_MIXED, outs[1])
    assert rc == _lib.FMM_OK, lib.fmm_last_error()
    for precision in (_lib.FMM_MIXED, _lib.FMM_FP64):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for k, w in enumerate(cases):  # larger input first, then the smaller one
            rc, _ = _call(lib, "fmm_velocity_noalloc", trees[k], gam[k], w.sigma, w.p, precision, outs[k])
            assert rc == _lib.FMM_OK, lib.fmm_last_error()
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0  # no device memory taken by the two calls
        for k, w in enumerate(cases):
            rc, _ = _call(lib, "fmm_velocity", trees[k], gam[k], w.sigma, w.p, precision, refs[k])
            assert rc == _lib.FMM_OK, lib.fmm_last_error()
            assert torch.equal(outs[k], refs[k]), (k, precision)
        # and once more after the allocating calls: the static workspace keeps no state
        rc, _ = _call(lib, "fmm_velocity_noalloc", trees[1], gam[1], cases[1].sigma, cases[1].p, precision, outs[1])
        assert rc == _lib.FMM_OK and torch.equal(outs[1], refs[1])
    for t in trees:
        t.close()


def test_noalloc_limits(fmm_mod):
    import torch
    from paper_1008_2410_amd import _lib
    lib = _lib.load()
    r = np.random.Generator(np.random.PCG64(73))
    n = 1_500_000   # mixed with the mutual near field: about 104 bytes per particle, above 128 MiB
    xy = r.random((n, 2))
    g = _t(r.standard_normal(n) / n)
    tree = fmm_mod.Tree(_t(xy[:2000]), 4, (0.0, 0.0, 1.0))
    tree.velocity(g[:2000], 1e-3, 9, "mixed")
    tree.close()
    tree = fmm_mod.Tree(_t(xy), 8, (0.0, 0.0, 1.0))
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    rc, _ = _call(lib, "fmm_velocity_noalloc", tree, g, 1e-3, 9, _lib.FMM_MIXED, out)
    assert rc == _lib.FMM_EINVAL and b"static workspace" in lib.fmm_last_error()
    rc, _ = _call(lib, "fmm_velocity_noalloc", tree, g, 1e-3, 29, _lib.FMM_MIXED, out)  # tables of p = 29 absent
    assert rc in (_lib.FMM_ESTATE, _lib.FMM_EINVAL)
    tree.close()
