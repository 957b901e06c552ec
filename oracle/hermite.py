"""Hermite functions (section 1, note 2).

h_n(t) = exp(-t^2) H_n(t), where H_n is the physicists' Hermite polynomial
defined by the Rodrigues formula H_n(t) = (-1)^n exp(t^2) d^n/dt^n exp(-t^2).
The polynomials satisfy the textbook three-term recurrence
    H_0 = 1,  H_1 = 2t,  H_{n+1} = 2t H_n - 2n H_{n-1},
which is how they are evaluated here.  The multivariate function is the product
h_alpha(t) = prod_d h_{alpha_d}(t_d).

Pinned by tests/test_oracle_series.py against numpy.polynomial.hermite.hermval
(an independent implementation of the same polynomials) and against the
explicit low-order forms obtained from the Rodrigues formula.
"""

import numpy as np


def hermite_poly_table(t, nmax):
    """H_0..H_nmax at t (array-like); returns array of shape (nmax+1,) + t.shape."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty((nmax + 1,) + t.shape, dtype=np.float64)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = 2.0 * t
    for n in range(1, nmax):
        out[n + 1] = 2.0 * t * out[n] - 2.0 * n * out[n - 1]
    return out


def hermite_fn_table(t, nmax):
    """h_0..h_nmax at t: h_n(t) = exp(-t^2) H_n(t)."""
    t = np.asarray(t, dtype=np.float64)
    return hermite_poly_table(t, nmax) * np.exp(-t * t)


def hermite_multi(alpha, t):
    """h_alpha(t) = prod_d h_{alpha_d}(t_d) for one point t of length D."""
    t = np.asarray(t, dtype=np.float64)
    val = 1.0
    for d, a in enumerate(alpha):
        val *= hermite_fn_table(t[d], a)[a]
    return float(val)
