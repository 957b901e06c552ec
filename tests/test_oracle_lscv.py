"""Pins the LSCV oracle: its double-sum closed form against brute-force
numerical integration and explicit leave-one-out loops, and its minimiser
against the normal-reference bandwidth on a large Gaussian sample."""
import math

import numpy as np

from oracle.lscv import lscv, lscv_brute


def test_closed_form_matches_brute_force_1d():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, 40)
    grid = np.linspace(-9, 9, 6001)
    for h in (0.1, 0.3, 1.0):
        want = lscv_brute(x, h, grid)
        got = lscv(x[:, None], [h])[0]
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (h, got, want)


def test_two_dimensional_normalisation_by_explicit_loops():
    # the D-dependent normalisations (2 pi s^2)^(-D/2) at D = 2, by explicit
    # loops over point pairs with 2-D Gaussian densities
    rng = np.random.default_rng(2)
    x = rng.normal(0, 1, (25, 2))
    h = 0.4
    N = len(x)
    phi2 = lambda u, s: math.exp(-float(u @ u) / (2 * s * s)) / (2 * math.pi * s * s)
    integral = sum(phi2(x[i] - x[j], math.sqrt(2) * h) for i in range(N) for j in range(N)) / N ** 2
    loo = sum(phi2(x[i] - x[j], h) for i in range(N) for j in range(N) if j != i) / (N - 1)
    want = integral - 2 * loo / N
    assert abs(lscv(x, [h])[0] - want) <= 1e-12 * abs(want)


def test_minimiser_near_normal_reference_bandwidth():
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (1500, 1))
    hs = np.exp(np.linspace(np.log(0.05), np.log(1.5), 40))
    h_best = hs[np.argmin(lscv(x, hs))]
    h_ref = 1.06 * x.std() * len(x) ** (-0.2)      # normal-reference rule
    assert 0.6 * h_ref <= h_best <= 1.6 * h_ref, (h_best, h_ref)
