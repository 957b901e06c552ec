"""Least-squares cross-validation score of a Gaussian kernel density
estimate, by its plain definition.  TEST INFRASTRUCTURE ONLY.

The paper's experiments sweep bandwidths around the one that minimises the
standard least-squares cross-validation score (section 7, after Silverman
1986); the multi-bandwidth sum is its inner loop.  For points x_1..x_N in
D dimensions and the estimate f_h(x) = (1/N) sum_j phi_h(x - x_j), with
phi_h(u) = (2 pi h^2)^(-D/2) exp(-|u|^2 / 2h^2):

    LSCV(h) = integral f_h(x)^2 dx - (2/N) sum_i f_{h,-i}(x_i),
    f_{h,-i}(x_i) = 1/(N-1) sum_{j != i} phi_h(x_i - x_j).

The product of two Gaussians of variance h^2 integrates to a Gaussian of
variance 2 h^2, so the first term is a double sum:

    integral f_h^2 = (1/N^2) sum_i sum_j phi_{sqrt(2) h}(x_i - x_j).

In terms of G_h(x_q) = sum_r exp(-|x_q - x_r|^2 / 2h^2) over the points
themselves (unit weights, self term included):

    LSCV(h) = (4 pi h^2)^(-D/2) / N^2 * sum_i G_{sqrt2 h}(x_i)
              - 2 (2 pi h^2)^(-D/2) / (N (N-1)) * sum_i (G_h(x_i) - 1).
"""

import math

import numpy as np

from .exhaustive import gauss_sum_exhaustive


def lscv(x, hs):
    """LSCV(h) for every h, FP64, from exhaustive sums."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, D = x.shape
    hs = np.atleast_1d(np.asarray(hs, dtype=np.float64))
    w = np.ones(N)
    out = np.zeros(len(hs))
    G2 = gauss_sum_exhaustive(x, x, w, math.sqrt(2.0) * hs)
    G1 = gauss_sum_exhaustive(x, x, w, hs)
    for k, h in enumerate(hs):
        a = (4.0 * math.pi * h * h) ** (-D / 2.0) / (N * N)
        b = 2.0 * (2.0 * math.pi * h * h) ** (-D / 2.0) / (N * (N - 1.0))
        out[k] = a * math.fsum(G2[k]) - b * math.fsum(G1[k] - 1.0)
    return out


def lscv_brute(x, h, grid):
    """Brute force on a 1-D sample: the integral by the trapezoid rule on
    `grid`, the leave-one-out term by explicit loops."""
    x = np.asarray(x, dtype=np.float64).ravel()
    N = len(x)
    phi = lambda u: math.exp(-u * u / (2 * h * h)) / math.sqrt(2 * math.pi * h * h)
    f = np.array([sum(phi(g - xj) for xj in x) / N for g in grid])
    integral = float(np.trapezoid(f * f, grid))
    loo = 0.0
    for i in range(N):
        loo += sum(phi(x[i] - x[j]) for j in range(N) if j != i) / (N - 1)
    return integral - 2.0 * loo / N
