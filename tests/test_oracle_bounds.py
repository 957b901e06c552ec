"""Pins the truncation-error bounds (Lemmas 4-6), the finite-difference error
(section 5) and the box distance bounds on random node pairs: the true error of
each approximation never exceeds its bound, and the bounds are not vacuous."""
import itertools
import math

import numpy as np
import pytest

from oracle import bounds as B
from oracle import series as S
from oracle.exhaustive import gauss_sum_exhaustive
from oracle.multiindex import plimit_for


def _node(rng, n, D, centre, rad):
    pts = centre + rng.uniform(-1, 1, (n, D)) * rad
    lo, hi = pts.min(0), pts.max(0)
    ctr = 0.5 * (lo + hi)
    rinf = float(np.abs(pts - ctr).max())
    return pts, lo, hi, ctr, rinf


def _random_pairs(seed, count):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        D = int(rng.choice([1, 2, 3, 5]))
        h = float(10 ** rng.uniform(-1.3, 0))
        rad_q = float(rng.uniform(0.05, 1.2)) * h
        rad_r = float(rng.uniform(0.05, 1.2)) * h
        sep = float(rng.uniform(0, 4)) * h
        cq = rng.uniform(0, 1, D)
        direction = rng.normal(size=D)
        direction /= np.linalg.norm(direction)
        xr, lor, hir, cr, rr = _node(rng, int(rng.integers(5, 40)), D, cq + sep * direction, rad_r)
        xq, loq, hiq, cq_, rq = _node(rng, int(rng.integers(5, 30)), D, cq, rad_q)
        w = rng.uniform(0.5, 1.5, xr.shape[0])
        yield D, h, (xq, loq, hiq, cq_, rq), (xr, lor, hir, cr, rr), w


def _pair_errors(D, h, Q, R, w, pmax):
    xq, loq, hiq, cq, rq = Q
    xr, lor, hir, cr, rr = R
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    dmin2, _ = B.box_dist2(loq, hiq, lor, hir)
    g = math.exp(-dmin2 / (4 * h * h))
    W_R = float(w.sum())
    out = []
    for p in range(1, pmax + 1):
        A = S.hermite_moments(xr, w, cr, p, h)
        dh = np.abs(S.eval_hermite(A, p, cr, xq, h) - exact).max()
        dl = np.abs(S.eval_local(S.direct_local(xr, w, p, cq, h), p, cq, xq, h) - exact).max()
        hl = np.abs(S.eval_local(S.h2l(A, p, cr, cq, h), p, cq, xq, h) - exact).max()
        out.append((p, dh, B.e_dh(W_R, g, D, p, rr / h),
                    dl, B.e_dl(W_R, g, D, p, rq / h),
                    hl, B.e_h2l(W_R, g, D, p, rq / h, rr / h)))
    return out


def test_lemmas_4_5_6_hold_on_random_pairs():
    worst = {"DH": 0.0, "DL": 0.0, "H2L": 0.0}
    for D, h, Q, R, w in _random_pairs(100, 120):
        pmax = min(plimit_for(D), 6) if D > 1 else 8
        for p, dh, edh, dl, edl, hl, ehl in _pair_errors(D, h, Q, R, w, pmax):
            tol = 1e-12 * float(w.sum())  # rounding of the series themselves
            assert dh <= edh + tol, (D, p, dh, edh)
            assert dl <= edl + tol, (D, p, dl, edl)
            assert hl <= ehl + tol, (D, p, hl, ehl)
            if dh > 1e3 * tol:
                worst["DH"] = max(worst["DH"], dh / edh)
            if dl > 1e3 * tol:
                worst["DL"] = max(worst["DL"], dl / edl)
            if hl > 1e3 * tol:
                worst["H2L"] = max(worst["H2L"], hl / ehl)
    # the bounds are informative, not vacuous
    for k, v in worst.items():
        assert v > 0.02, (k, v)


def test_dropping_the_weight_factor_is_caught():
    # a planted mistake in the bound (W_R omitted) must violate Lemma 4 somewhere
    violated = False
    for D, h, Q, R, w in _random_pairs(200, 60):
        for p, dh, edh, *_ in _pair_errors(D, h, Q, R, w, 3):
            if dh > edh / float(w.sum()) * 1.0000001:
                violated = True
    assert violated


def test_finite_difference_error_bound():
    # every kernel value of the pair lies in [K(dmax), K(dmin)] (section 5)
    for D, h, Q, R, w in _random_pairs(300, 80):
        xq, loq, hiq, _, _ = Q
        xr, lor, hir, _, _ = R
        dmin2, dmax2 = B.box_dist2(loq, hiq, lor, hir)
        kmin, kmax = math.exp(-dmin2 / (2 * h * h)), math.exp(-dmax2 / (2 * h * h))
        W_R = float(w.sum())
        exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
        approx = 0.5 * W_R * (kmin + kmax)
        assert np.abs(exact - approx).max() <= B.e_fd(W_R, kmin, kmax) * (1 + 1e-12) + 1e-300


@pytest.mark.parametrize("D", [1, 2, 3])
def test_box_distance_bounds_brute_force(D):
    rng = np.random.default_rng(40 + D)
    for _ in range(40):
        lo1 = rng.uniform(0, 1, D); hi1 = lo1 + rng.uniform(0, 0.5, D)
        lo2 = rng.uniform(0, 1, D); hi2 = lo2 + rng.uniform(0, 0.5, D)
        dmin2, dmax2 = B.box_dist2(lo1, hi1, lo2, hi2)
        k = 7
        g1 = np.array(list(itertools.product(*[np.linspace(lo1[d], hi1[d], k) for d in range(D)])))
        g2 = np.array(list(itertools.product(*[np.linspace(lo2[d], hi2[d], k) for d in range(D)])))
        d2 = ((g1[:, None, :] - g2[None, :, :]) ** 2).sum(-1)
        assert d2.min() >= dmin2 * (1 - 1e-12) - 1e-15
        assert d2.max() <= dmax2 * (1 + 1e-12)
        assert abs(d2.max() - dmax2) <= 1e-12 * max(1.0, dmax2)  # attained at corners
        cell = (np.maximum(hi1 - lo1, hi2 - lo2) / (k - 1))
        assert math.sqrt(d2.min()) - math.sqrt(dmin2) <= np.linalg.norm(cell) + 1e-12


@pytest.mark.parametrize("D", [2, 3, 8])
def test_sphere_rect_bounds_brute_force(D):
    """On node pairs of a real tree: the sphere-rectangle bounds enclose the
    true closest and farthest point pairs (brute force over the points), and
    are never looser than the box bounds."""
    from oracle.kdtree import build_kdtree
    from paper_1206_6857_amd.datagen import mixture
    x, w, _ = mixture((45, D), 700, D, 3, (0.02, 0.2))
    t = build_kdtree(x, w, 24)
    rng = np.random.default_rng(46 + D)
    tighter_min = tighter_max = 0
    for _ in range(60):
        a, b = rng.integers(0, t.n_nodes, 2)
        pa, pb = x[t.perm[t.begin[a]:t.end[a]]], x[t.perm[t.begin[b]:t.end[b]]]
        d2 = ((pa[:, None, :] - pb[None, :, :]) ** 2).sum(-1)
        smin, smax = B.sphere_rect_dist2(t.lo[a], t.hi[a], t.lo[b], t.hi[b], t.ctr[a], t.ctr[b],
                                         t.rad[a], t.rad[b])
        bmin, bmax = B.box_dist2(t.lo[a], t.hi[a], t.lo[b], t.hi[b])
        assert d2.min() >= smin * (1 - 1e-12) - 1e-15
        assert d2.max() <= smax * (1 + 1e-12)
        assert smin >= bmin and smax <= bmax
        tighter_min += smin > bmin
        tighter_max += smax < bmax
    assert tighter_max > 0   # the ball bound is not always the box bound


def test_node_radius_is_the_largest_distance_to_the_centre():
    from oracle.kdtree import build_kdtree
    from paper_1206_6857_amd.datagen import mixture
    x, w, _ = mixture((47, 3), 500, 3, 3, (0.02, 0.2))
    t = build_kdtree(x, w, 16)
    for i in range(t.n_nodes):
        xs = x[t.perm[t.begin[i]:t.end[i]]]
        want = max(math.sqrt(math.fsum((v - c) ** 2 for v, c in zip(row, t.ctr[i]))) for row in xs)
        assert abs(t.rad[i] - want) <= 1e-15 * max(1.0, want)
        assert t.rad[i] <= math.sqrt(3) * t.rinf[i] * (1 + 1e-15) and t.rad[i] >= t.rinf[i]


def test_best_method_orders_and_ties():
    # Figure 6: first minimum in the order DH, DL, H2L, DIRECT
    name, p, E = B.best_method(2, 8, 1e9, 1.0, 1.0, 0.1, 0.1, 2, 2)
    assert name == "DH" and p == 1          # all four costs are 8 -> DH first
    name, p, E = B.best_method(2, 8, 1e9, 1.0, 1.0, 0.1, 0.1, 5, 2)
    assert name == "DL" and p == 1          # c_DL = c_H2L = 8 < 20 -> DL before H2L
    name, p, E = B.best_method(2, 8, 0.0, 1.0, 1.0, 0.1, 0.1, 100, 10)
    assert name == "DIRECT"
    name, p, E = B.best_method(3, 6, 1e9, 1.0, 1.0, 0.1, 0.1, 1000, 1000)
    assert name == "H2L" and p == 1         # 27 < 1000*9
