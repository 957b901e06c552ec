"""Theorem 2's invariants, checked from the oracle's decision ledger in both
traversal modes (the level-wise frontier the library follows, and the
depth-first recursion of Figures 1 and 7).

The proof of Theorem 2 (section 5) charges every query point a budget of W
(the total weight): a pair (Q, R) resolved with error bound E, decided with
the lower bound L on G over Q, costs each point of Q the amount
W E / (eps L) - W_R, so that a point whose charges sum to at most 0 has
sum E <= eps L <= eps G.  The checks below use only the ledger rows, the tree's
point lists and the exhaustive sum:

  * budget: per query point and bandwidth, the charges of the resolved pairs
    covering it sum to at most 0 (up to rounding);
  * lower bound: every L is at most min_{q in Q} G(x_q);
  * tokens: the token left at Q after every decision is at least 0;
  * the ledger's finite-difference bounds are those of the box distances
    (recomputed here with numpy's exp).
"""
import math

import numpy as np
import pytest

import oracle.dualtree as DT
from oracle.dualtree import BASE, FD
from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import mixture


def _check_ledger(res, xq, xr, w, hs, eps):
    qt, rt = res.qtree, res.rtree
    W = float(np.sum(w))
    eps_alg = (1.0 - 0.1) * eps
    G = gauss_sum_exhaustive(xq, xr, w, hs)
    M = xq.shape[0]
    charge = np.zeros((len(hs), M))
    pts = {}
    worst = -math.inf
    for hk, Q, R, code, E, L, WR, t in res.ledger:
        if Q not in pts:
            pts[Q] = qt.perm[qt.begin[Q]:qt.end[Q]]
        qp = pts[Q]
        # the lower bound the decision used holds for every point of Q
        assert L <= G[hk, qp].min() * (1.0 + 1e-12), (hk, Q, R, L, G[hk, qp].min())
        assert t >= -1e-12 * W, (hk, Q, R, t)
        if code == BASE:
            assert E == 0.0
        assert E >= 0.0
        if E == 0.0:        # exact (base case) or a bound that underflowed
            c = -WR
        else:
            assert L > 0.0
            c = W * E / (eps_alg * L) - WR
        if code == FD:
            lo, hi = qt.lo[Q], qt.hi[Q]
            rlo, rhi = rt.lo[R], rt.hi[R]
            gap = np.maximum(0.0, np.maximum(lo - rhi, rlo - hi))
            far = np.maximum(hi - rlo, rhi - lo)
            h = float(hs[hk])
            efd = WR * (np.exp(-np.sum(gap * gap) / (2 * h * h)) - np.exp(-np.sum(far * far) / (2 * h * h))) / 2
            assert abs(E - efd) <= 1e-12 * WR + 1e-9 * abs(efd), (E, efd)
        charge[hk, qp] += c
    worst = float(charge.max()) / W
    return worst


CASES = [  # (seed, D, n, leaf, method, hs)
    (23, 2, 1500, 32, "dito", [1e-3]),
    (23, 2, 1500, 32, "dito", [1e-3, 0.01, 0.05, 0.2, 1.0]),
    (19, 1, 1500, 32, "dito", [1e-3, 0.01, 0.05, 0.2, 1.0]),
    (19, 3, 1500, 32, "dito", [1e-3, 0.01, 0.05, 0.2, 1.0]),
    (19, 2, 1500, 32, "dfto", [1e-3, 0.01, 0.05, 0.2, 1.0]),
    (19, 3, 1200, 32, "dfdo", [1e-3, 0.01, 0.05, 0.2, 1.0]),
    (19, 2, 1200, 16, "dfd", [1e-3, 0.01, 0.05, 0.2, 1.0]),
]


@pytest.mark.parametrize("traversal", ["level", "depth_first"])
@pytest.mark.parametrize("seed,D,n,leaf,method,hs", CASES)
def test_token_budget_per_query_point(traversal, seed, D, n, leaf, method, hs):
    x, w, _ = mixture((seed, D), n, D, 4, (0.02, 0.1), weights=(0.5, 1.5))
    res = DT.dualtree(x, x, w, hs, 0.01, leaf_size=leaf, method=method, traversal=traversal, ledger=True)
    worst = _check_ledger(res, x, x, w, np.array(hs), 0.01)
    assert worst <= 1e-9, worst


@pytest.mark.parametrize("traversal", ["level", "depth_first"])
def test_token_budget_bichromatic(traversal):
    r, w, q = mixture((29, 2), 1200, 2, 4, (0.02, 0.1), weights=(0.5, 1.5), m_queries=500)
    hs = [0.01, 0.05, 0.2, 1.0]
    res = DT.dualtree(q, r, w, hs, 0.01, leaf_size=32, traversal=traversal, ledger=True)
    assert _check_ledger(res, q, r, w, np.array(hs), 0.01) <= 1e-9


def test_planted_double_spend_is_caught(monkeypatch):
    """A traversal that hands every child pair the parent's budget again
    (each level restarts its tokens at the parent's value plus W_R deposits it
    never earned) must fail the budget check: here the planted mistake credits
    every base case twice."""
    x, w, _ = mixture((23, 2), 1500, 2, 4, (0.02, 0.1), weights=(0.5, 1.5))
    real = DT.need

    def doubled(E, WR, L, W, eps):
        v = real(E, WR, L, W, eps)
        return 2.0 * v if E == 0.0 else v
    monkeypatch.setattr(DT, "need", doubled)
    res = DT.dualtree(x, x, w, [1e-3, 0.01], 0.01, leaf_size=32, ledger=True)
    assert _check_ledger(res, x, x, w, np.array([1e-3, 0.01]), 0.01) > 1e-3
