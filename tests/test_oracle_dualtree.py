"""Pins the level-wise dual-tree oracle: Theorem 2's guarantee against the FP64
exhaustive sum, exact coverage of all (query, reference) pairs by the resolved
node pairs, translation and permutation invariance of the decisions, and a
planted mistake that the guarantee test must catch."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle.dualtree as DT
from oracle.dualtree import BASE, SPLIT, dualtree
from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import mixture

HS = [1e-3, 1e-2, 0.03, 0.1, 0.3, 1.0, 10.0]


def _max_rel(res_G, xq, xr, w, hs):
    G = gauss_sum_exhaustive(xq, xr, w, hs)
    return (np.abs(res_G - G) / G).max(axis=1)


@pytest.mark.parametrize("D,n,method", [(1, 1200, "dito"), (2, 1500, "dito"), (3, 1500, "dito"),
                                        (5, 1000, "dito"), (2, 1200, "dfdo"), (3, 1200, "dfd")])
def test_theorem2_monochromatic(D, n, method):
    x, w, _ = mixture((11, D), n, D, 4, (0.02, 0.1), weights=(0.5, 1.5))
    res = DT.dualtree(x, x, w, HS, 0.01, leaf_size=32, method=method)
    rel = _max_rel(res.G, x, x, w, HS)
    assert np.all(rel <= 0.01), rel


@pytest.mark.parametrize("D,n", [(2, 1200), (3, 1200), (8, 800)])
def test_theorem2_sphere_rect_bounds(D, n):
    """Theorem 2 with the sphere-rectangle node bounds, which never resolve
    fewer pairs than the box bounds' traversal of the same input."""
    x, w, _ = mixture((13, D), n, D, 4, (0.02, 0.1), weights=(0.5, 1.5))
    hs = [0.01, 0.05, 0.2, 1.0]
    res = DT.dualtree(x, x, w, hs, 0.01, leaf_size=32, node_bounds="sphere_rect")
    rel = _max_rel(res.G, x, x, w, hs)
    assert np.all(rel <= 0.01), rel
    box = DT.dualtree(x, x, w, hs, 0.01, leaf_size=32)
    assert res.counts.sum() <= box.counts.sum()


@pytest.mark.parametrize("D,method", [(2, "dito"), (3, "dito"), (3, "dfto")])
def test_theorem2_far_first_pair_order(D, method):
    """A best-first walk of each query node's reference list (decreasing
    dmin^2) keeps Theorem 2 and covers the same work as the tree order up to
    a few percent: the order of the walk within a level hardly matters."""
    x, w, _ = mixture((17, D), 1500, D, 4, (0.02, 0.1), weights=(0.5, 1.5))
    hs = [1e-3, 0.01, 0.05, 0.2, 1.0]
    res = DT.dualtree(x, x, w, hs, 0.01, leaf_size=32, method=method, pair_order="far_first", trace=True)
    rel = _max_rel(res.G, x, x, w, hs)
    assert np.all(rel <= 0.01), rel
    tree = DT.dualtree(x, x, w, hs, 0.01, leaf_size=32, method=method)
    assert abs(res.counts[:, BASE].sum() - tree.counts[:, BASE].sum()) <= 0.1 * tree.counts[:, BASE].sum()
    # the walk order is the stated one: within every (h, level, Q), in the
    # order the trace records the decisions, dmin^2 does not increase and
    # equal distances come by increasing R
    from oracle.bounds import box_dist2
    qt, rt = res.qtree, res.rtree
    last = {}
    for hk, lvl, Q, R, code, p in res.trace:
        d2 = box_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R])[0]
        key = (hk, lvl, Q)
        if key in last:
            pd2, pR = last[key]
            assert d2 < pd2 or (d2 == pd2 and R > pR), (key, pd2, pR, d2, R)
        last[key] = (d2, R)


@pytest.mark.parametrize("D,method,M", [(1, "dito", None), (2, "dito", None), (3, "dito", None),
                                         (2, "dfto", None), (3, "dfdo", None), (2, "dito", 600)])
def test_theorem2_depth_first_paper_mode(D, method, M):
    """Paper mode (the recursion of Figures 1 and 7 in its printed order)
    keeps Theorem 2 and resolves every (query, reference) point pair exactly
    once."""
    r, w, q = mixture((19, D), 1500, D, 4, (0.02, 0.1), weights=(0.5, 1.5), m_queries=M)
    q = r if M is None else q
    # (far queries of the bichromatic case underflow at h = 1e-3: G = 0 there)
    hs = [1e-3, 0.01, 0.05, 0.2, 1.0] if M is None else [0.01, 0.05, 0.2, 1.0]
    res = DT.dualtree(q, r, w, hs, 0.01, leaf_size=32, method=method, traversal="depth_first", trace=True)
    rel = _max_rel(res.G, q, r, w, hs)
    assert np.all(rel <= 0.01), rel
    qt, rt = res.qtree, res.rtree
    for k in range(len(hs)):
        cover = np.zeros((q.shape[0], r.shape[0]), dtype=np.int64)
        for hk, depth, Q, R, code, p in res.trace:
            if hk == k and code != SPLIT:
                cover[np.ix_(qt.perm[qt.begin[Q]:qt.end[Q]], rt.perm[rt.begin[R]:rt.end[R]])] += 1
        assert np.all(cover == 1), k


def test_depth_first_rejects_frontier_only_options():
    x, w, _ = mixture((3, 2), 200, 2, 2, 0.1)
    for kw in (dict(record_feasible=True), dict(pair_order="far_first"), dict(replay={})):
        with pytest.raises(ValueError):
            DT.dualtree(x, x, w, [0.1], 0.01, traversal="depth_first", **kw)
    with pytest.raises(ValueError):
        DT.dualtree(x, x, w, [0.1], 0.01, traversal="breadth")


@pytest.mark.parametrize("D", [2, 3])
def test_theorem2_bichromatic(D):
    r, w, q = mixture((12, D), 1500, D, 4, (0.02, 0.1), weights=(0.5, 1.5), m_queries=700)
    hs = [0.01, 0.05, 0.2, 1.0]
    res = DT.dualtree(q, r, w, hs, 0.01, leaf_size=32)
    rel = _max_rel(res.G, q, r, w, hs)
    assert np.all(rel <= 0.01), rel


def test_resolved_pairs_cover_every_point_pair_once():
    r, w, q = mixture((13, 2), 900, 2, 3, 0.08, m_queries=500)
    hs = [0.005, 0.05, 0.5]
    res = DT.dualtree(q, r, w, hs, 0.01, leaf_size=16, trace=True)
    qt, rt = res.qtree, res.rtree
    for k in range(len(hs)):
        cover = np.zeros((500, 900), dtype=np.int64)
        for hk, lvl, Q, R, code, p in res.trace:
            if hk == k and code != SPLIT:
                qp = qt.perm[qt.begin[Q]:qt.end[Q]]
                rp = rt.perm[rt.begin[R]:rt.end[R]]
                cover[np.ix_(qp, rp)] += 1
        assert np.all(cover == 1)


def test_translation_invariance_on_dyadic_grid():
    rng = np.random.default_rng(3)
    x = np.round(rng.uniform(0, 1, (800, 2)) * 2 ** 20) / 2 ** 20
    w = np.full(800, 1.0 / 1024)
    hs = [0.01, 0.1]
    a = DT.dualtree(x, x, w, hs, 0.01, leaf_size=16, trace=True)
    y = x + 0.125                                       # every subtraction stays exact
    b = DT.dualtree(y, y, w, hs, 0.01, leaf_size=16, trace=True)
    assert a.trace == b.trace
    assert np.allclose(a.G, b.G, rtol=1e-12)


def test_permutation_invariance():
    x, _, _ = mixture((14, 3), 1024, 3, 4, (0.02, 0.1))
    w = np.full(1024, 1.0 / 1024)                       # exact node sums in any order
    hs = [0.02, 0.2]
    a = DT.dualtree(x, x, w, hs, 0.01, leaf_size=16)
    sh = np.random.default_rng(5).permutation(1024)
    xs = x[sh]
    b = DT.dualtree(xs, xs, w[sh], hs, 0.01, leaf_size=16)
    assert np.array_equal(a.counts, b.counts)
    assert np.allclose(a.G[:, sh], b.G, rtol=1e-12)


def test_planted_token_sign_error_is_caught(monkeypatch):
    # section 5 prints the token both as W_R(W E/(eps G) - 1) and as its
    # negative; taking the wrong sign turns every withdrawal into a deposit and
    # prunes far too much: the guarantee test must notice
    x, w, _ = mixture((15, 2), 1200, 2, 4, (0.02, 0.1), weights=(0.5, 1.5))
    real = DT.need
    monkeypatch.setattr(DT, "need", lambda *a: -real(*a))
    res = DT.dualtree(x, x, w, HS, 0.01, leaf_size=32)
    assert _max_rel(res.G, x, x, w, HS).max() > 0.01


@settings(max_examples=15, deadline=None)
@given(seed=st.integers(0, 10 ** 6), D=st.integers(1, 4), n=st.integers(2, 400),
       logh=st.floats(-3, 1), leaf=st.integers(1, 40))
def test_theorem2_property(seed, D, n, logh, leaf):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, D)) * rng.uniform(0.01, 1, D)
    w = rng.uniform(0.5, 1.5, n)
    h = 10.0 ** logh
    res = DT.dualtree(x, x, w, [h], 0.01, leaf_size=leaf)
    assert _max_rel(res.G, x, x, w, [h]).max() <= 0.01
