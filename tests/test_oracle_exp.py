"""Pins the oracle's own exponential against the platform exp and 50-digit mpmath."""
import math

import mpmath
import numpy as np

from oracle.exp64 import exp64


def _ulp_diff(a, b):
    return abs(a - b) / math.ulp(b)


def test_exp64_matches_libm_within_2ulp():
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-700, 0, 20000), rng.uniform(-1, 1, 5000),
                         -np.logspace(-12, 2.8, 2000)])
    worst = max(_ulp_diff(exp64(x), math.exp(x)) for x in xs)
    assert worst <= 2.0, worst


def test_exp64_against_mpmath():
    mpmath.mp.dps = 50
    rng = np.random.default_rng(2)
    for x in list(rng.uniform(-690, 5, 300)) + [0.0, -0.5, -math.log(2), -1e-300]:
        exact = mpmath.e ** mpmath.mpf(float(x))
        got = exp64(x)
        assert abs(mpmath.mpf(got) - exact) / exact < 5e-16


def test_exp64_special_values():
    assert exp64(0.0) == 1.0
    assert exp64(-1000.0) == 0.0
    assert exp64(-700.5) == 0.0
    assert 0.0 < exp64(-699.9) < 1e-300
