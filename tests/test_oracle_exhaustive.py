"""Pins the plain FP64 definition (section 1) against brute force and closed forms."""
import math

import mpmath
import numpy as np

from oracle.exhaustive import gauss_sum_exhaustive


def test_matches_fsum_and_mpmath_on_tiny_inputs():
    rng = np.random.default_rng(1)
    xq = rng.uniform(0, 1, (7, 3))
    xr = rng.uniform(0, 1, (11, 3))
    w = rng.uniform(0.5, 1.5, 11)
    hs = [0.05, 0.3, 2.0]
    G = gauss_sum_exhaustive(xq, xr, w, hs)
    mpmath.mp.dps = 50
    for k, h in enumerate(hs):
        for i in range(7):
            terms = [w[j] * math.exp(-sum((xq[i, d] - xr[j, d]) ** 2 for d in range(3)) / (2 * h * h))
                     for j in range(11)]
            assert abs(G[k, i] - math.fsum(terms)) <= 1e-14 * math.fsum(terms)
            exact = mpmath.fsum(mpmath.mpf(w[j]) * mpmath.e ** (
                -mpmath.fsum((mpmath.mpf(xq[i, d]) - mpmath.mpf(xr[j, d])) ** 2 for d in range(3))
                / (2 * mpmath.mpf(h) ** 2)) for j in range(11))
            assert abs(mpmath.mpf(G[k, i]) - exact) / exact < 1e-14


def test_single_reference_closed_form():
    xq = np.array([[0.1, 0.2], [0.9, -0.4]])
    xr = np.array([[0.3, 0.3]])
    for h in (0.1, 1.0):
        G = gauss_sum_exhaustive(xq, xr, [2.5], [h])[0]
        want = 2.5 * np.exp(-((xq - xr) ** 2).sum(1) / (2 * h * h))
        assert np.allclose(G, want, rtol=1e-15)


def test_coincident_points_sum_to_total_weight():
    x0 = np.array([[0.4, 0.7, 0.1]])
    xr = np.repeat(x0, 9, axis=0)
    w = np.arange(1, 10, dtype=float)
    G = gauss_sum_exhaustive(x0, xr, w, [1e-3, 1.0])
    assert np.all(G == w.sum())


def test_large_and_small_bandwidth_limits():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (50, 2))
    w = rng.uniform(0.5, 1.5, 50)
    Gbig = gauss_sum_exhaustive(x, x, w, [1e6])[0]
    assert np.allclose(Gbig, w.sum(), rtol=1e-12)
    Gsmall = gauss_sum_exhaustive(x, x, w, [1e-6])[0]   # distinct points: only the self term
    assert np.allclose(Gsmall, w, rtol=1e-15)
