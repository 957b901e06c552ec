"""Pins the expansions and translation operators against closed forms, a
library routine and exact identities (sections 1-3)."""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite as nph

from oracle.exhaustive import gauss_sum_exhaustive
from oracle.hermite import hermite_fn_table, hermite_poly_table
from oracle.multiindex import multi_indices
from oracle import series as S


def test_hermite_polys_match_numpy_hermval():
    t = np.linspace(-6, 6, 101)
    tab = hermite_poly_table(t, 20)
    for n in range(21):
        c = np.zeros(n + 1)
        c[n] = 1.0
        ref = nph.hermval(t, c)
        assert np.allclose(tab[n], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_hermite_rodrigues_low_orders():
    t = np.linspace(-3, 3, 13)
    tab = hermite_poly_table(t, 3)
    assert np.allclose(tab[0], 1.0)
    assert np.allclose(tab[1], 2 * t)
    assert np.allclose(tab[2], 4 * t ** 2 - 2)
    assert np.allclose(tab[3], 8 * t ** 3 - 12 * t)


def test_hermite_function_inequality_constant_one():
    # |h_n(t)| <= 2^{n/2} sqrt(n!) e^{-t^2/2}: the inequality used in Lemma 4's proof
    t = np.linspace(-12, 12, 4001)
    tab = hermite_fn_table(t, 30)
    for n in range(31):
        lhs = np.abs(tab[n]) * np.exp(t * t / 2)
        assert lhs.max() <= math.sqrt(2.0 ** n * math.factorial(n)) * (1 + 1e-9)


def test_generating_function_1d_converges():
    # exp(-(t-s)^2) = sum_n s^n/n! h_n(t) (the identity behind section 1's expansions)
    t = np.linspace(-3, 3, 31)
    for s in (-0.9, 0.3, 0.8):
        exact = np.exp(-(t - s) ** 2)
        tab = hermite_fn_table(t, 60)
        errs = []
        for p in (2, 6, 12, 24, 40):
            approx = sum(s ** n / math.factorial(n) * tab[n] for n in range(p))
            errs.append(np.abs(approx - exact).max())
        assert all(errs[i + 1] < errs[i] or errs[i + 1] < 1e-13 for i in range(len(errs) - 1))
        assert errs[-1] < 1e-12


def _cloud(rng, n, D, ctr, rad):
    return ctr + rng.uniform(-rad, rad, size=(n, D))


@pytest.mark.parametrize("D", [1, 2, 3])
def test_direct_hermite_converges_to_exhaustive(D):
    rng = np.random.default_rng(10 + D)
    h = 0.3
    xr = _cloud(rng, 40, D, 0.2, 0.15)
    w = rng.uniform(0.5, 1.5, 40)
    xq = _cloud(rng, 25, D, 0.9, 0.2)
    ctr = 0.5 * (xr.min(0) + xr.max(0))
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    errs = []
    for p in (1, 3, 6, 10, 16):
        A = S.hermite_moments(xr, w, ctr, p, h)
        errs.append(np.abs(S.eval_hermite(A, p, ctr, xq, h) - exact).max() / exact.max())
    assert errs[-1] < 1e-9 and errs[-1] < errs[0] * 1e-4


def test_monopole_order_one():
    rng = np.random.default_rng(3)
    h = 0.2
    xr = _cloud(rng, 30, 2, 0.0, 0.1)
    w = rng.uniform(0.5, 1.5, 30)
    ctr = np.array([0.01, -0.02])
    xq = _cloud(rng, 10, 2, 0.5, 0.3)
    A = S.hermite_moments(xr, w, ctr, 1, h)
    got = S.eval_hermite(A, 1, ctr, xq, h)
    want = w.sum() * np.exp(-((xq - ctr) ** 2).sum(1) / (2 * h * h))
    assert np.allclose(got, want, rtol=1e-13)


def test_worked_example_coefficients_d2_p2():
    # section 2: the O(D^p) expansion at p=2 stores sum w, sum w x1~, sum w x2~
    rng = np.random.default_rng(4)
    h = 0.25
    xr = rng.uniform(0, 1, (17, 2))
    w = rng.uniform(0.5, 1.5, 17)
    ctr = np.array([0.5, 0.5])
    A = S.hermite_moments(xr, w, ctr, 2, h)
    xt = (xr - ctr) / math.sqrt(2 * h * h)
    assert np.allclose(A, [w.sum(), (w * xt[:, 0]).sum(), (w * xt[:, 1]).sum()], rtol=1e-14)


@pytest.mark.parametrize("D,p", [(2, 8), (3, 6), (5, 4)])
def test_raw_moments_scale_to_hermite_moments(D, p):
    rng = np.random.default_rng(5)
    xr = rng.uniform(0, 0.1, (50, D))
    w = rng.uniform(0.5, 1.5, 50)
    ctr = 0.5 * (xr.min(0) + xr.max(0))
    for h in (0.01, 0.3):
        a = S.scale_moments(S.raw_moments(xr, w, ctr, p), D, p, h)
        b = S.hermite_moments(xr, w, ctr, p, h)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())


@pytest.mark.parametrize("D,p", [(2, 8), (3, 6), (5, 4)])
def test_h2h_is_exact(D, p):
    # Lemma 2 on truncated moments is an exact identity
    rng = np.random.default_rng(6)
    xr = rng.uniform(0, 0.2, (40, D))
    w = rng.uniform(0.5, 1.5, 40)
    c_child = xr.mean(0)
    c_parent = c_child + rng.uniform(-0.1, 0.1, D)
    M_child = S.raw_moments(xr, w, c_child, p)
    got = S.h2h(M_child, c_child, c_parent, D, p)
    want = S.raw_moments(xr, w, c_parent, p)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
    h = 0.07
    gs = S.h2h_scaled(S.scale_moments(M_child, D, p, h), c_child, c_parent, D, p, h)
    assert np.allclose(gs, S.scale_moments(want, D, p, h), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("D,p", [(2, 8), (3, 6)])
def test_l2l_is_exact(D, p):
    # Lemma 3: re-centring a truncated Taylor polynomial is exact
    rng = np.random.default_rng(7)
    h = 0.2
    B = rng.normal(size=len(multi_indices(D, p)))
    cp = rng.uniform(0, 1, D)
    cc = cp + rng.uniform(-0.05, 0.05, D)
    xq = cc + rng.uniform(-0.05, 0.05, (20, D))
    Cc = S.l2l(B, p, cp, cc, h)
    assert np.allclose(S.eval_local(Cc, p, cc, xq, h), S.eval_local(B, p, cp, xq, h), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_direct_local_converges_to_exhaustive(D):
    rng = np.random.default_rng(20 + D)
    h = 0.3
    xr = _cloud(rng, 30, D, 0.9, 0.2)
    w = rng.uniform(0.5, 1.5, 30)
    xq = _cloud(rng, 20, D, 0.1, 0.1)
    cq = 0.5 * (xq.min(0) + xq.max(0))
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    errs = []
    for p in (1, 4, 8, 14):
        B = S.direct_local(xr, w, p, cq, h)
        errs.append(np.abs(S.eval_local(B, p, cq, xq, h) - exact).max() / exact.max())
    assert errs[-1] < 1e-8 and errs[-1] < errs[0] * 1e-4


@pytest.mark.parametrize("D", [1, 2])
def test_h2l_converges_to_exhaustive(D):
    # Lemma 1: the translated series converges to the far-field sum
    rng = np.random.default_rng(30 + D)
    h = 0.4
    xr = _cloud(rng, 30, D, 0.0, 0.08)
    w = rng.uniform(0.5, 1.5, 30)
    xq = _cloud(rng, 20, D, 0.6, 0.08)
    cr = 0.5 * (xr.min(0) + xr.max(0))
    cq = 0.5 * (xq.min(0) + xq.max(0))
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    errs = []
    for p in (1, 3, 6, 10, 14):
        A = S.hermite_moments(xr, w, cr, p, h)
        B = S.h2l(A, p, cr, cq, h)
        errs.append(np.abs(S.eval_local(B, p, cq, xq, h) - exact).max() / exact.max())
    assert errs[-1] < 1e-8 and errs[-1] < errs[0] * 1e-4


def test_h2l_sign_error_is_caught(monkeypatch):
    # a planted mistake: drop the (-1)^|beta| factor of Lemma 1 -> the series no
    # longer converges to the exhaustive sum
    rng = np.random.default_rng(41)
    h = 0.4
    xr = _cloud(rng, 30, 2, 0.0, 0.08)
    w = rng.uniform(0.5, 1.5, 30)
    xq = _cloud(rng, 20, 2, 0.6, 0.08)
    cr = 0.5 * (xr.min(0) + xr.max(0))
    cq = 0.5 * (xq.min(0) + xq.max(0))
    exact = gauss_sum_exhaustive(xq, xr, w, [h])[0]
    A = S.hermite_moments(xr, w, cr, 10, h)
    B = S.h2l(A, 10, cr, cq, h)
    mis = multi_indices(2, 10)
    bad = np.array([b * (-1) ** sum(a) for a, b in zip(mis, B)])
    good_err = np.abs(S.eval_local(B, 10, cq, xq, h) - exact).max() / exact.max()
    bad_err = np.abs(S.eval_local(bad, 10, cq, xq, h) - exact).max() / exact.max()
    assert good_err < 1e-6 < bad_err
