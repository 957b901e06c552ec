"""The plain definition (section 1):

    G_h(x_q) = sum_{r=1}^{N} w_r exp(-|x_q - x_r|^2 / (2 h^2))

in double precision, with the squared distance in difference form
sum_d (x_qd - x_rd)^2 and the platform exp.  With positive terms the relative
rounding error is ~1e-15, so this is the truth the error tolerance is judged
against.  The self term of a monochromatic sum is included (the definition has
no exclusion).

Pinned by tests/test_oracle_exhaustive.py against math.fsum / 50-digit mpmath
brute force on tiny inputs and against closed forms (one reference point,
coincident points, h -> infinity, h -> 0).
"""

import numpy as np


def gauss_sum_exhaustive(xq, xr, w, hs, block=256):
    """Returns G of shape (len(hs), M) in query order."""
    xq = np.atleast_2d(np.asarray(xq, dtype=np.float64))
    xr = np.atleast_2d(np.asarray(xr, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64)
    hs = np.atleast_1d(np.asarray(hs, dtype=np.float64))
    M, D = xq.shape
    out = np.zeros((len(hs), M))
    for b in range(0, M, block):
        q = xq[b:b + block]
        d2 = np.zeros((q.shape[0], xr.shape[0]))
        for d in range(D):
            diff = q[:, d:d + 1] - xr[None, :, d]
            d2 += diff * diff
        for k, h in enumerate(hs):
            out[k, b:b + block] = np.exp(-d2 / (2.0 * h * h)) @ w
    return out


def gauss_sum_exhaustive_rows(xq_rows, xr, w, hs):
    """Same definition for a few query rows; used for sampled checks at large N."""
    return gauss_sum_exhaustive(xq_rows, xr, w, hs, block=64)
