"""Pins the kd-tree (section 6, Figure 5) by brute force on its defining properties."""
import math

import numpy as np
import pytest

from oracle.kdtree import attach_moments, build_kdtree
from oracle import series as S
from paper_1206_6857_amd.datagen import mixture


@pytest.mark.parametrize("D,n,leaf", [(1, 300, 8), (2, 1000, 16), (3, 777, 20), (5, 513, 64), (2, 40, 64)])
def test_tree_properties(D, n, leaf):
    x, w, _ = mixture((5, D), n, D, 3, (0.02, 0.2), weights=(0.5, 1.5))
    t = build_kdtree(x, w, leaf)
    assert sorted(t.perm.tolist()) == list(range(n))
    assert t.begin[0] == 0 and t.end[0] == n
    for i in range(t.n_nodes):
        pts = t.perm[t.begin[i]:t.end[i]]
        xs = x[pts]
        assert np.array_equal(t.lo[i], xs.min(0)) and np.array_equal(t.hi[i], xs.max(0))
        assert np.array_equal(t.ctr[i], 0.5 * (t.lo[i] + t.hi[i]))
        assert t.rinf[i] == np.abs(xs - t.ctr[i]).max()
        assert abs(t.W[i] - math.fsum(w[pts])) <= 1e-13 * t.W[i]
        assert t.wmin[i] == w[pts].min()
        if t.left[i] < 0:
            assert t.count[i] <= leaf
            assert np.all(np.diff(pts) > 0)           # leaf points in index order
        else:
            assert t.count[i] > leaf
            l, r = t.left[i], t.left[i] + 1
            assert t.depth[l] == t.depth[r] == t.depth[i] + 1
            assert t.begin[l] == t.begin[i] and t.end[l] == t.begin[r] and t.end[r] == t.end[i]
            # left child: the smallest multiple of leaf_size that is >= half
            assert t.count[l] % leaf == 0
            assert 2 * t.count[l] >= t.count[i] > 2 * (t.count[l] - leaf)
            ext = t.hi[i] - t.lo[i]
            d = int(np.argmax(ext))
            key = lambda j: (x[j, d], j)
            lpts = sorted(t.perm[t.begin[l]:t.end[l]].tolist(), key=key)
            rpts = sorted(t.perm[t.begin[r]:t.end[r]].tolist(), key=key)
            assert key(lpts[-1]) < key(rpts[0])      # split by (x_d, index)
    assert np.all(np.diff(t.depth) >= 0)                # breadth-first numbering
    leaves = t.count[t.left < 0]
    if n > leaf:
        assert np.sum(leaves != leaf) <= 1              # all leaves but one are full


def test_tree_geometry_is_permutation_invariant():
    x, w, _ = mixture((6, 2), 700, 2, 3, 0.1)
    t1 = build_kdtree(x, w, 16)
    rng = np.random.default_rng(0)
    sh = rng.permutation(700)
    t2 = build_kdtree(x[sh], w[sh], 16)
    assert np.array_equal(t1.left, t2.left) and np.array_equal(t1.begin, t2.begin)
    assert np.array_equal(t1.lo, t2.lo) and np.array_equal(t1.hi, t2.hi)
    for i in range(t1.n_nodes):
        a = set(t1.perm[t1.begin[i]:t1.end[i]].tolist())
        b = set(sh[t2.perm[t2.begin[i]:t2.end[i]]].tolist())
        assert a == b


def test_tree_moments_match_direct_moments():
    x, w, _ = mixture((7, 2), 300, 2, 2, 0.1, weights=(0.5, 1.5))
    t = build_kdtree(x, w, 16)
    M = attach_moments(t, 6)
    for i in (0, 1, 2, t.n_nodes - 1):
        pts = t.perm[t.begin[i]:t.end[i]]
        want = S.raw_moments(x[pts], w[pts], t.ctr[i], 6)
        assert np.allclose(M[i], want, rtol=1e-11, atol=1e-16)
