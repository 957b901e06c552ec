"""Degenerate inputs on the GPU dual-tree path, each checked against the oracle
as in the main parity test (tree and decisions bit-exact, values to rounding,
Theorem 2 against the FP64 exhaustive sum):

* one reference and one query; one point, monochromatic (G = w);
* every point at the same place (boxes of zero extent, splits decided by the
  point index alone);
* points on a coarse lattice (many equal coordinates);
* a tree that is a single leaf (leaf size above N), and leaves of one point;
* a dimension of zero extent (points on a plane in three dimensions);
* one query against many references;
* bandwidths far below and far above the point spacing (every pair a base
  case; every pair pruned by finite difference at the root);
* the largest dimension the library accepts (D = 64);
* a query inside a sparsely filled leaf box whose every term lies below the
  float range (the base tiles' underflow rescue);
* the most bandwidths one call accepts (4096).
"""
import numpy as np
import pytest

import oracle.dualtree as DT
from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu

TOL_ROUND = 1e-4


def _rng(seed):
    return np.random.default_rng(seed)


def _case(name):
    """(queries, refs, weights, bandwidths, leaf, monochromatic)."""
    if name == "one_ref_one_query":
        r = np.array([[0.2, 0.4]])
        q = np.array([[0.25, 0.3]])
        return q, r, np.array([1.5]), np.array([0.1, 1.0]), 16, False
    if name == "one_point_mono":
        r = np.array([[0.3, 0.1, 0.7]])
        return r, r, np.array([2.0]), np.array([1e-3, 0.1, 10.0]), 16, True
    if name == "all_points_equal":
        r = np.tile(np.array([[0.5, 0.25, 0.75]]), (300, 1))
        w = _rng(1).uniform(0.5, 1.5, 300)
        return r, r, w, np.array([1e-3, 0.1, 1.0]), 16, True
    if name == "coarse_lattice":
        r = _rng(2).integers(0, 3, (800, 2)) * 0.5
        w = _rng(3).uniform(0.5, 1.5, 800)
        return r, r, w, np.array([0.05, 0.3, 2.0]), 16, True
    if name == "single_leaf_tree":
        r, w, _ = mixture((4, 2), 100, 2, 2, (0.05, 0.1))
        return r, r, w, np.array([0.01, 0.1, 1.0]), 128, True
    if name == "one_point_leaves":
        r, w, _ = mixture((5, 2), 300, 2, 3, (0.02, 0.1))
        return r, r, w, np.array([0.01, 0.05, 0.3]), 1, True
    if name == "flat_dimension":
        r, w, _ = mixture((6, 3), 1200, 3, 4, (0.02, 0.1))
        r[:, 1] = 0.5
        return r, r, w, np.array([0.01, 0.05, 0.3, 1.0]), 32, True
    if name == "one_query":
        r, w, _ = mixture((7, 2), 2000, 2, 4, (0.02, 0.1))
        q = np.array([[0.45, 0.55]])
        return q, r, w, np.array([0.05, 0.3, 2.0]), 32, False
    if name == "max_dimension":
        r, w, q = mixture((9, 64), 600, 64, 3, (0.02, 0.1), m_queries=200)
        return q, r, w, np.array([0.3, 1.0, 4.0]), 32, False
    if name == "extreme_bandwidths":
        r, w, _ = mixture((8, 2), 1500, 2, 4, (0.02, 0.1))
        return r, r, w, np.array([1e-6, 1e4]), 32, True
    if name == "sparse_box_underflow":
        # two tight clusters at opposite corners of [0,1]^8, one leaf; a query at
        # the centre lies inside the leaf's box (box distance 0) but at squared
        # distance 2 from every point: at h = 0.1 and 0.07 every term is e^-100
        # and e^-204, below the float range unless the shift comes from the
        # points themselves
        rng = _rng(10)
        r = np.concatenate([rng.normal(0.0, 0.01, (100, 8)), rng.normal(1.0, 0.01, (100, 8))])
        q = np.concatenate([np.full((1, 8), 0.5), rng.normal(0.0, 0.01, (2, 8)), rng.normal(0.6, 0.05, (5, 8))])
        w = rng.uniform(0.5, 1.5, 200)
        return q, r, w, np.array([0.07, 0.1, 0.3]), 256, False
    raise KeyError(name)


CASES = ["one_ref_one_query", "one_point_mono", "all_points_equal", "coarse_lattice", "single_leaf_tree",
         "one_point_leaves", "flat_dimension", "one_query", "extreme_bandwidths", "max_dimension",
         "sparse_box_underflow"]


@pytest.mark.parametrize("method", ["dito", "dfto"])
@pytest.mark.parametrize("name", CASES)
def test_degenerate_parity(name, method):
    banner("degenerate", name, method)
    q, r, w, hs, leaf, mono = _case(name)
    D = r.shape[1]
    c = ctx()
    qq = r if mono else q
    G = c.gauss_sum(qq, r, w, hs, 0.01, method=method, leaf_size=leaf, keep_trace=1)
    ref = DT.dualtree(qq, r, w, hs, 0.01, leaf_size=leaf, method=method, trace=True)
    for which, t in ((0, ref.rtree), (1, ref.qtree)):
        gt = c.get_tree(which, D)
        assert np.array_equal(gt["perm"], t.perm)
        assert np.array_equal(gt["begin"], t.begin) and np.array_equal(gt["count"], t.count)
        assert np.array_equal(gt["left"], t.left)
        for k in ("lo", "hi", "ctr", "rinf"):
            assert np.array_equal(gt[k], getattr(t, k)), k
    got = c.get_trace().astype(np.int64)
    want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.array_equal(key(got), key(want))
    assert np.array_equal(c.pair_counts(len(hs)), ref.counts)
    exact = gauss_sum_exhaustive(qq, r, w, hs)
    assert np.all(exact > 0)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01
    if name == "one_point_mono":
        np.testing.assert_allclose(G, np.full((len(hs), 1), 2.0), rtol=1e-6)
    if name == "all_points_equal":
        np.testing.assert_allclose(G, np.full((len(hs), 300), w.sum()), rtol=1e-6)


def test_most_bandwidths_per_call():
    """4096 bandwidths in one call (the most accepted).  Bandwidths never
    interact in the traversal, so the decisions and values of each sampled
    bandwidth equal the oracle's run on that bandwidth alone."""
    banner("degenerate", "4096 bandwidths")
    r, w, _ = mixture((10, 2), 500, 2, 3, (0.02, 0.1))
    hs = np.logspace(-3, 1, 4096)
    c = ctx()
    G = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32, keep_trace=1)
    assert G.shape == (4096, 500)
    tr = c.get_trace().astype(np.int64)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    for k in (0, 1, 7, 8, 1000, 2047, 2048, 3001, 4094, 4095):
        ref = DT.dualtree(r, r, w, hs[k:k + 1], 0.01, leaf_size=32, trace=True)
        want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
        want[:, 0] = k
        got = tr[tr[:, 0] == k]
        assert got.shape == want.shape, (k, got.shape, want.shape)
        assert np.array_equal(key(got), key(want)), k
        exact = gauss_sum_exhaustive(r, r, w, hs[k:k + 1])[0]
        assert (np.abs(G[k] - ref.G[0]) / exact).max() <= TOL_ROUND, k
        assert (np.abs(G[k] - exact) / exact).max() <= 0.01, k
