"""Pins of the adaptive-tree oracle (O6) to things other than itself.

* The four lists against a brute-force restatement of their definitions (every cell
  against every cell, in Python, from the cells' levels and coordinates alone).
* Exactly-once coverage: for every ordered pair of leaves (T, S), S reaches T by
  exactly one route: S in U(T); an ancestor-or-self of S in V of an ancestor-or-self
  of T; an ancestor-or-self of S in W(T); or S in X of an ancestor-or-self of T.
* Special cases: one leaf (s_max >= N) is the direct sum O1; a lattice with equal
  leaf counts splits into the uniform tree, where O6 equals O3 and W, X are empty.
* Accuracy: with sigma small enough that the far kernel is exact, O6 matches O1
  within the truncation error of p terms on clustered points with non-empty W, X.

The adjoint O7 against differences of O6 itself and against independent gradients:
* circulations: the loss sum_i g_i . u_i is linear in Gamma, so a central difference with
  step 1 is exact to rounding;
* positions: central differences of O6 with one particle moved (the tree unchanged),
  where a particle with Gamma = 0 isolates the evaluation-point part, one with g = 0 the
  source part;
* one leaf: the O1 gradient (direct sum); equal leaf counts: O4 + O5 of the uniform tree.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from conftest import rel_l2


def _clustered(seed=1):
    r = np.random.Generator(np.random.PCG64(seed))
    xy = np.concatenate([r.random((500, 2)), 0.3 + 0.02 * r.random((900, 2)),
                         0.71 + 0.005 * r.standard_normal((300, 2)), [[0.999, 0.001], [0.0, 0.0]]])
    return xy, r.standard_normal(len(xy))


def _box(c, lmax):
    level, ix, iy = int(c[0]), int(c[1]), int(c[2])
    s = 1 << (lmax - level)
    return ix * s, (ix + 1) * s, iy * s, (iy + 1) * s


def _adj(a, b, lmax):
    ax0, ax1, ay0, ay1 = _box(a, lmax)
    bx0, bx1, by0, by1 = _box(b, lmax)
    return ax0 <= bx1 and bx0 <= ax1 and ay0 <= by1 and by0 <= ay1


def _sets(t, name):
    off, idx = t[name]
    return [set(idx[off[k]:off[k + 1]].tolist()) for k in range(len(off) - 1)]


def _ancestors(cells, k):
    out = []
    while k >= 0:
        out.append(k)
        k = int(cells[k, 5])
    return out


@pytest.mark.parametrize("smax,lmax", [(20, 9), (5, 7), (60, 12), (1, 5)])
def test_lists_match_definitions(smax, lmax):
    xy, _ = _clustered()
    t = O.adaptive_tree(xy, smax, lmax)
    cells = t["cells"]
    K = len(cells)
    leaf = cells[:, 3].astype(bool)
    level = cells[:, 0]
    # the split rule
    for k in range(K):
        assert (not leaf[k]) == (cells[k, 4] > smax and level[k] < lmax)
        if cells[k, 5] >= 0:
            assert level[cells[k, 5]] == level[k] - 1
    counts = np.bincount(t["leaf_of"], minlength=K)
    assert np.array_equal(counts[leaf], cells[leaf, 4]) and counts[~leaf].sum() == 0
    adj = np.array([[_adj(cells[a], cells[b], lmax) for b in range(K)] for a in range(K)])
    desc = [set() for _ in range(K)]  # proper descendants
    for k in range(K):
        for a in _ancestors(cells, int(cells[k, 5])):
            desc[a].add(k)
    coll = [{b for b in range(K) if b != a and level[b] == level[a] and adj[a, b]} for a in range(K)]
    U, V, W, X = (_sets(t, n) for n in "UVWX")
    for a in range(K):
        par = int(cells[a, 5])
        v_ref = set()
        if par >= 0:
            v_ref = {d for c in coll[par] for d in range(K) if cells[d, 5] == c and not adj[a, d]}
        assert V[a] == v_ref
        if leaf[a]:
            assert U[a] == {b for b in range(K) if leaf[b] and adj[a, b]}
            w_ref = {d for c in coll[a] for d in desc[c]
                     if not adj[a, d] and adj[a, int(cells[d, 5])]}
            assert W[a] == w_ref
        else:
            assert not U[a] and not W[a]
        assert X[a] == {b for b in range(K) if leaf[b] and a in W[b]}


@pytest.mark.parametrize("smax,lmax", [(20, 9), (5, 7), (1, 5), (300, 8)])
def test_every_pair_of_leaves_covered_once(smax, lmax):
    xy, _ = _clustered(3)
    t = O.adaptive_tree(xy, smax, lmax)
    cells = t["cells"]
    K = len(cells)
    U, V, W, X = (_sets(t, n) for n in "UVWX")
    leaves = [k for k in range(K) if cells[k, 3]]
    anc = {k: _ancestors(cells, k) for k in range(K)}
    assert t["sizes"]["w"] > 0 or smax >= 300  # the adaptive routes are exercised
    for T, S in itertools.product(leaves, leaves):
        routes = int(S in U[T])
        routes += sum(1 for a in anc[T] for b in anc[S] if b in V[a])
        routes += sum(1 for b in anc[S] if b in W[T])
        routes += sum(1 for a in anc[T] if S in X[a])
        assert routes == 1, (T, S, routes)


def test_single_leaf_is_the_direct_sum():
    xy, g = _clustered(5)
    t = O.adaptive_tree(xy, len(xy), 6)
    assert t["sizes"]["cells"] == 1 and t["sizes"]["p2p_pairs"] == len(xy) * (len(xy) - 1)
    un, uf = O.afmm_velocity(xy, g, 0.003, len(xy), 6, 8, parts=True)
    assert np.all(uf == 0.0)
    assert rel_l2(un, O.direct(xy, g, 0.003)) < 1e-13


def test_equal_leaf_counts_give_the_uniform_tree():
    r = np.random.Generator(np.random.PCG64(8))
    L, m = 4, 16  # a jittered 64 x 64 lattice: 16 particles in every depth-4 leaf
    h = 1.0 / 64
    g1 = (np.arange(64) + 0.5) * h
    xy = np.stack(np.meshgrid(g1, g1, indexing="xy"), -1).reshape(-1, 2) + (r.random((4096, 2)) - 0.5) * 0.3 * h
    g = r.standard_normal(4096)
    root = (0.0, 0.0, 1.0)
    t = O.adaptive_tree(xy, m - 1, L, root)
    s = t["sizes"]
    assert s["leaves"] == 4 ** L and s["w"] == 0 and s["x"] == 0 and s["deepest"] == L
    assert s["p2p_pairs"] == _uniform_pairs(xy, L, root)
    an, af = O.afmm_velocity(xy, g, 0.01, m - 1, L, 12, root, parts=True)
    un, uf = O.fmm_velocity(xy, g, 0.01, L, 12, root, parts=True)
    assert rel_l2(an, un) < 1e-14
    assert rel_l2(af, uf) < 1e-13


def _uniform_pairs(xy, L, root):
    c = O.leaf_counts(xy, L, root)
    pad = np.pad(c, 1)
    nb = sum(pad[1 + dy:1 + dy + c.shape[0], 1 + dx:1 + dx + c.shape[1]] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return int(np.sum(c * nb) - c.sum())


@pytest.mark.parametrize("smax,lmax,p,tol", [(20, 9, 20, 1e-8), (8, 8, 12, 1e-5), (40, 10, 30, 1e-11)])
def test_matches_direct_sum_within_truncation(smax, lmax, p, tol):
    xy, g = _clustered(2)
    t = O.adaptive_tree(xy, smax, lmax)
    assert t["sizes"]["w"] > 0 and t["sizes"]["x"] > 0
    # the far kernel differs from the regularised one by exp(-d^2/(2 sigma^2)), d >= the
    # narrowest leaf: below 1e-300 here
    sigma = 1e-6
    u = O.afmm_velocity(xy, g, sigma, smax, lmax, p)
    assert rel_l2(u, O.direct(xy, g, sigma)) < tol


@pytest.mark.parametrize("smax,lmax", [(20, 9), (5, 7), (1, 5)])
def test_linear_impulse(smax, lmax):
    """sum_i Gamma_i u_i = 0 to roundoff: the near kernel is odd over symmetric U lists, M2L
    is antisymmetric over symmetric V lists with square truncation, and M2P over W is the
    exact transpose of P2L over X (same p, exact M2M and L2L chains)."""
    xy, g = _clustered(4)
    u = O.afmm_velocity(xy, g, 0.001, smax, lmax, 12)
    imp = (g[:, None] * u).sum(axis=0)
    scale = (np.abs(g)[:, None] * np.abs(u)).sum()
    assert np.all(np.abs(imp) < 1e-13 * scale), (imp, scale)


def _adjoint_case(seed):
    xy, gamma = _clustered(seed)
    r = np.random.Generator(np.random.PCG64(seed + 100))
    dl = r.standard_normal((len(xy), 2))
    return xy, gamma, dl


@pytest.mark.parametrize("smax,lmax", [(8, 7), (30, 10)])
def test_adjoint_circulation_exact_difference(smax, lmax):
    xy, gamma, dl = _adjoint_case(5)
    sigma, p = 0.002, 12
    root = O.root_box(xy)
    dg, _, _ = O.afmm_grad(xy, gamma, sigma, smax, lmax, p, dl, root)

    def loss(gm):
        return float(np.sum(dl * O.afmm_velocity(xy, gm, sigma, smax, lmax, p, root)))

    scale = np.abs(dg).max()
    for j in np.random.Generator(np.random.PCG64(7)).choice(len(xy), 12, replace=False):
        e = np.zeros(len(xy))
        e[j] = 1.0
        fd = 0.5 * (loss(gamma + e) - loss(gamma - e))
        assert abs(dg[j] - fd) <= 1e-11 * scale, (j, dg[j], fd)


def test_adjoint_positions_central_differences():
    xy, gamma, dl = _adjoint_case(6)
    n = len(xy)
    sigma, p, smax, lmax = 0.002, 14, 10, 8
    zero_g = np.arange(0, n, 5)        # no source role: the evaluation part alone
    zero_dl = np.arange(2, n, 7)       # no evaluation role: the source part alone
    gamma = gamma.copy()
    dl = dl.copy()
    gamma[zero_g] = 0.0
    dl[zero_dl] = 0.0
    root = O.root_box(xy)
    dg, dxe, dxs = O.afmm_grad(xy, gamma, sigma, smax, lmax, p, dl, root)
    assert np.all(dxs[zero_g] == 0.0) and np.all(dxe[zero_dl] == 0.0)
    # particles away from the lines of the finest grid keep their cells when moved by h
    w = root[2] / 2 ** lmax
    frac = np.stack([(xy[:, 0] - root[0]) / w, (xy[:, 1] - root[1]) / w], 1) % 1.0
    inside = np.all((frac > 1e-3) & (frac < 1 - 1e-3), axis=1)
    h = 1e-7

    def loss(x):
        return float(np.sum(dl * O.afmm_velocity(x, gamma, sigma, smax, lmax, p, root)))

    picks = [k for k in list(zero_g[:6]) + list(zero_dl[:6]) + list(range(1, n, 97))[:10] if inside[k]]
    assert len(picks) >= 15
    got, want = [], []
    for k in picks:
        for d in range(2):
            xp, xm = xy.copy(), xy.copy()
            xp[k, d] += h
            xm[k, d] -= h
            got.append((loss(xp) - loss(xm)) / (2 * h))
            want.append(dxe[k, d] + dxs[k, d])
    assert rel_l2(np.array(got), np.array(want)) < 1e-6


def test_adjoint_single_leaf_is_the_direct_gradient():
    xy, gamma, dl = _adjoint_case(7)
    dg, dxe, dxs = O.afmm_grad(xy, gamma, 0.01, len(xy), 6, 10, dl)
    rg, rx = O.direct_grad(xy, gamma, 0.01, dl)
    assert rel_l2(dg, rg) < 1e-13
    assert rel_l2(dxe + dxs, rx) < 1e-13


def test_adjoint_equal_leaf_counts_give_the_uniform_adjoint():
    r = np.random.Generator(np.random.PCG64(8))
    h = 1.0 / 64
    g1 = (np.arange(64) + 0.5) * h
    xy = np.stack(np.meshgrid(g1, g1, indexing="xy"), -1).reshape(-1, 2) + (r.random((4096, 2)) - 0.5) * 0.3 * h
    g = r.standard_normal(4096)
    dl = r.standard_normal((4096, 2))
    root = (0.0, 0.0, 1.0)
    dg, dxe, dxs = O.afmm_grad(xy, g, 0.01, 15, 4, 12, dl, root)
    ug, uxe, uxs = O.fmm_grad_full(xy, g, 0.01, 4, 12, dl, root)
    assert rel_l2(dg, ug) < 1e-12
    assert rel_l2(dxe, uxe) < 1e-12
    assert rel_l2(dxs, uxs) < 1e-12
