"""Pins the O(p^D) (DFTO) part of the oracle against facts that do not come
from its own code:

* the tensor index sets: size p^D, every component below p, closed under
  taking smaller indices, a prefix of every larger order, equal to the graded
  set in one dimension;
* Cramer's inequality, checked with numpy's physicists' Hermite polynomials,
  which the oracle does not use;
* the product form: for one reference point, the truncated tensor far-field and
  local series equal the product of D one-dimensional truncated series written
  out with numpy's Hermite polynomials;
* exact H2H and L2L in the tensor family, convergence to the exact sum;
* the derived bounds hold on random node pairs and are not vacuous;
* Theorem 2 for the whole DFTO traversal.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite as npherm

from oracle import bounds as B
from oracle import series as S
from oracle.dualtree import dualtree
from oracle.exhaustive import gauss_sum_exhaustive
from oracle.multiindex import (MAX_TERMS, index_set, multi_indices, plimit_for, plimit_tensor, set_size,
                               tensor_indices)


def _h(n, t):
    """h_n(t) = H_n(t) e^{-t^2} from numpy's physicists' Hermite series."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npherm.hermval(t, c) * np.exp(-t * t)


@pytest.mark.parametrize("D,p", [(1, 5), (2, 4), (3, 3), (4, 2), (5, 3)])
def test_tensor_sets(D, p):
    s = tensor_indices(D, p)
    assert len(s) == p ** D == set_size(D, p, "tensor") == len(set(s))
    assert all(max(a) < p for a in s)
    ss = set(s)
    for a in s:
        for d in range(D):
            if a[d]:
                b = a[:d] + (a[d] - 1,) + a[d + 1:]
                assert b in ss
    assert tensor_indices(D, p + 1)[: p ** D] == s
    # ordered by the largest component
    assert [max(a) for a in s] == sorted(max(a) for a in s)


def test_tensor_equals_graded_in_one_dimension():
    for p in range(1, 11):
        assert tensor_indices(1, p) == multi_indices(1, p)


def test_tensor_order_limits():
    for D in range(1, 12):
        P = plimit_tensor(D)
        assert 1 <= P <= plimit_for(D)
        assert P == 1 or P ** D <= MAX_TERMS
        assert P == plimit_for(D) or (P + 1) ** D > MAX_TERMS


def test_cramer_inequality():
    t = np.linspace(-12, 12, 4001)
    worst = 0.0
    for n in range(0, 31):
        lhs = np.abs(_h(n, t))
        rhs = 2.0 ** (n / 2) * math.sqrt(math.factorial(n)) * np.exp(-t * t / 2)
        worst = max(worst, float((lhs / rhs).max()))
    assert worst <= B.KC
    assert worst > 0.999  # reached at n = 0, t = 0: the inequality is tight


def test_tensor_parts_are_the_series():
    rng = np.random.default_rng(5)
    for _ in range(200):
        rho = float(rng.uniform(0, 3))
        p = int(rng.integers(1, 9))
        a, b = B.tensor_parts(rho, p)
        assert a == pytest.approx(sum(rho ** n / math.sqrt(math.factorial(n)) for n in range(p)), rel=1e-14)
        term = rho ** p / math.sqrt(math.factorial(p))
        full = 0.0
        for n in range(p, p + 400):
            full += term
            term *= rho / math.sqrt(n + 1)
        if rho / math.sqrt(p + 1) < 1:
            assert full <= b * (1 + 1e-12)
        else:
            assert b == math.inf


@pytest.mark.parametrize("D,p", [(2, 3), (3, 4), (2, 6)])
def test_tensor_series_factorise(D, p):
    rng = np.random.default_rng(D * 10 + p)
    h = 0.7
    s = 1.0 / math.sqrt(2 * h * h)
    xr = rng.uniform(-0.3, 0.3, (1, D))
    cR = np.zeros(D)
    xq = rng.uniform(0.2, 1.5, (4, D))
    cQ = xq.mean(0)
    # far field: prod_d sum_{n<p} (sr_d)^n / n! h_n(t_d)
    A = S.hermite_moments(xr, [1.0], cR, p, h, "tensor")
    got = S.eval_hermite(A, p, cR, xq, h, "tensor")
    want = np.ones(len(xq))
    for d in range(D):
        sr = (xr[0, d] - cR[d]) * s
        t = (xq[:, d] - cR[d]) * s
        want *= sum(sr ** n / math.factorial(n) * _h(n, t) for n in range(p))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
    # local: prod_d sum_{n<p} (u_d)^n / n! h_n(v_d), u = (x_q - x_Q) s, v = (x_r - x_Q) s
    B_ = S.direct_local(xr, [1.0], p, cQ, h, "tensor")
    got = S.eval_local(B_, p, cQ, xq, h, "tensor")
    want = np.ones(len(xq))
    for d in range(D):
        v = (xr[0, d] - cQ[d]) * s
        u = (xq[:, d] - cQ[d]) * s
        want *= sum(u ** n / math.factorial(n) * _h(n, np.array([v]))[0] for n in range(p))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_tensor_h2h_l2l_exact_and_convergence():
    rng = np.random.default_rng(11)
    D, p, h = 3, 4, 0.8
    xr = rng.uniform(-0.2, 0.2, (30, D))
    w = rng.uniform(0.5, 1.5, 30)
    c1, c0 = np.array([0.05, -0.02, 0.03]), np.zeros(D)
    M1 = S.raw_moments(xr, w, c1, p, "tensor")
    np.testing.assert_allclose(S.h2h(M1, c1, c0, D, p, "tensor"), S.raw_moments(xr, w, c0, p, "tensor"),
                               rtol=1e-12, atol=1e-14)
    Bp = S.direct_local(xr + 2.0, w, p, c0, h, "tensor")
    cc = np.array([0.1, 0.05, -0.08])
    xq = cc + rng.uniform(-0.05, 0.05, (6, D))
    np.testing.assert_allclose(S.eval_local(S.l2l(Bp, p, c0, cc, h, "tensor"), p, cc, xq, h, "tensor"),
                               S.eval_local(Bp, p, c0, xq, h, "tensor"), rtol=1e-12)
    # a high order reproduces the exact sum
    xq = rng.uniform(0.5, 1.0, (5, D))
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    A = S.hermite_moments(xr, w, c0, 9, h, "tensor")
    np.testing.assert_allclose(S.eval_hermite(A, 9, c0, xq, h, "tensor"), exact, rtol=1e-9)


def _node(rng, n, D, centre, rad):
    pts = centre + rng.uniform(-1, 1, (n, D)) * rad
    lo, hi = pts.min(0), pts.max(0)
    ctr = 0.5 * (lo + hi)
    return pts, lo, hi, ctr, float(np.abs(pts - ctr).max())


def test_tensor_bounds_hold_on_random_pairs():
    rng = np.random.default_rng(200)
    worst = {"DH": 0.0, "DL": 0.0, "H2L": 0.0}
    for _ in range(120):
        D = int(rng.choice([1, 2, 3, 4]))
        h = float(10 ** rng.uniform(-1.3, 0))
        sep = float(rng.uniform(0, 4)) * h
        c = rng.uniform(0, 1, D)
        direc = rng.normal(size=D)
        direc /= np.linalg.norm(direc)
        xr, lor, hir, cr, rr = _node(rng, int(rng.integers(5, 40)), D, c + sep * direc,
                                     float(rng.uniform(0.05, 1.2)) * h)
        xq, loq, hiq, cq, rq = _node(rng, int(rng.integers(5, 30)), D, c, float(rng.uniform(0.05, 1.2)) * h)
        w = rng.uniform(0.5, 1.5, xr.shape[0])
        exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
        dmin2, _ = B.box_dist2(loq, hiq, lor, hir)
        g = math.exp(-dmin2 / (4 * h * h))
        WR = float(w.sum())
        tol = 1e-12 * WR
        for p in range(1, plimit_tensor(D) + 1):
            A = S.hermite_moments(xr, w, cr, p, h, "tensor")
            errs = {
                "DH": (np.abs(S.eval_hermite(A, p, cr, xq, h, "tensor") - exact).max(),
                       B.e_dh_tensor(WR, g, D, p, rr / h)),
                "DL": (np.abs(S.eval_local(S.direct_local(xr, w, p, cq, h, "tensor"), p, cq, xq, h, "tensor")
                              - exact).max(), B.e_dl_tensor(WR, g, D, p, rq / h)),
                "H2L": (np.abs(S.eval_local(S.h2l(A, p, cr, cq, h, "tensor"), p, cq, xq, h, "tensor")
                               - exact).max(), B.e_h2l_tensor(WR, g, D, p, rq / h, rr / h)),
            }
            for k, (err, bound) in errs.items():
                assert err <= bound + tol, (k, D, p, err, bound)
                if err > 1e3 * tol and bound < math.inf:
                    worst[k] = max(worst[k], err / bound)
    for k, v in worst.items():
        assert v > 0.01, (k, v)


def test_tensor_bound_special_values():
    # a point node has no truncation error; an oversized node has no bound
    assert B.e_dh_tensor(3.0, 0.5, 3, 2, 0.0) == 0.0
    assert B.e_dh_tensor(3.0, 0.5, 3, 2, 2.0) == math.inf     # 2/sqrt(3) >= 1
    assert B.e_h2l_tensor(3.0, 0.5, 3, 2, 0.1, 1.3) == math.inf
    # grows with the weight and the Gaussian factor, shrinks with the order
    assert B.e_dh_tensor(2.0, 1.0, 2, 3, 0.4) == pytest.approx(2 * B.e_dh_tensor(1.0, 1.0, 2, 3, 0.4))
    assert B.e_dh_tensor(1.0, 1.0, 2, 4, 0.4) < B.e_dh_tensor(1.0, 1.0, 2, 3, 0.4)


def test_tensor_costs():
    assert B.term_cost(3, 4, "tensor") == 3 * 4 ** 3
    assert B.h2l_cost(3, 4, "tensor") == 3 * 4 ** 6
    assert B.term_cost(3, 4) == 3 ** 5 and B.h2l_cost(3, 4) == 3 ** 9


@pytest.mark.parametrize("D,N,seed", [(1, 1200, 1), (2, 2000, 2), (3, 2000, 3)])
def test_dfto_theorem2(D, N, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(c, 0.05, (N // 4, D)) for c in rng.uniform(0, 1, (4, D))])
    w = rng.uniform(0.5, 1.5, len(x))
    hs = np.array([0.005, 0.02, 0.08, 0.3, 1.0])
    eps = 0.01
    r = dualtree(x, x, w, hs, eps, leaf_size=32, method="dfto")
    exact = gauss_sum_exhaustive(x, x, w, hs)
    assert (np.abs(r.G - exact) / exact).max() <= eps
    counts = r.counts.sum(0)
    assert counts[1] + counts[2] + counts[3] > 0  # series prunes happen
    assert r.family == "tensor" and r.plimit == plimit_tensor(D)


def test_dfto_needs_box_bounds():
    x = np.random.default_rng(0).random((50, 2))
    with pytest.raises(ValueError):
        dualtree(x, x, np.ones(50), [0.1], 0.01, method="dfto", node_bounds="sphere_rect")


def test_index_set_rejects_unknown_family():
    with pytest.raises(ValueError):
        index_set(2, 3, "other")
