"""Hermite (far-field) and Taylor (local) expansions of the Gaussian kernel and
their translation operators (sections 1-3).

Notation: s = 1/sqrt(2 h^2) scales every displacement.  For a reference node R
with centre x_R and a query node Q with centre x_Q:

  Hermite moments (Lemma 1)   A_alpha = sum_{r in R} w_r/alpha! ((x_r-x_R) s)^alpha
  far-field value (sec. 1)     G_R(x_q) ~ sum_{|alpha|<p} A_alpha h_alpha((x_q-x_R) s)
  local coefficients (sec. 1)  B_beta = sum_{r in R} w_r/beta! h_beta((x_r-x_Q) s)
  local value                   G_R(x_q) ~ sum_{|beta|<p} B_beta ((x_q-x_Q) s)^beta
  H2L (Lemma 1)   B_beta = (-1)^{|beta|}/beta! sum_{|alpha|<p} A_alpha h_{alpha+beta}((x_Q-x_R) s)
  H2H (Lemma 2)   A_gamma = sum_{alpha<=gamma} A'_alpha ((x_R'-x_R) s)^{gamma-alpha}/(gamma-alpha)!
  L2L (Lemma 3)   C_alpha = sum_{beta>=alpha} beta!/(alpha!(beta-alpha)!) B_beta ((x_Q-x_Q') s)^{beta-alpha}

The paper's Lemma 1 prints the H2L sign as (-1)^beta; it is read as
(-1)^{|beta|}, the form used in Lemmas 5 and 6, which is what the derivative
identity d/dt h_n = -h_{n+1} gives.

Because the moments depend on h only through s^{|alpha|}, the tree stores
h-independent "raw" moments M_alpha = sum_r w_r (x_r-x_R)^alpha/alpha! and
scales them per bandwidth: A_alpha = M_alpha s^{|alpha|}.  H2H holds for raw
moments with s = 1.  "Order p" means the multi-indices with |alpha| < p
(family "graded", the O(D^p) expansions), or with alpha_d < p in every
dimension (family "tensor", the O(p^D) expansions of the DFTO variant): every
formula above holds for both sets, which are closed under taking smaller
indices, and L2L re-expands a local series exactly in either.

Pinned by tests/test_oracle_series.py: the generating-function identity of
section 1 (truncation error -> 0 as p grows, exact 1-D reduction), H2H and L2L
exactness on truncated series (Lemmas 2-3), H2L convergence to the direct
Hermite value, the order-1 monopole, and the worked D=2, p=2 example of
section 2.
"""

import math

import numpy as np

from .hermite import hermite_fn_table
from .multiindex import index_set, mi_degree, mi_factorial


def _scale(h):
    return 1.0 / math.sqrt(2.0 * h * h)


def _monomials(diff, mis):
    """diff: (n, D) -> (n, len(mis)) with diff^alpha per row."""
    diff = np.atleast_2d(np.asarray(diff, dtype=np.float64))
    n, D = diff.shape
    out = np.ones((n, len(mis)), dtype=np.float64)
    for i, a in enumerate(mis):
        for d in range(D):
            if a[d]:
                out[:, i] = out[:, i] * diff[:, d] ** a[d]
    return out


def _hermite_products(t, mis):
    """t: (n, D) -> (n, len(mis)) with h_alpha(t) per row."""
    t = np.atleast_2d(np.asarray(t, dtype=np.float64))
    n, D = t.shape
    nmax = max(mi_degree(a) for a in mis) if mis else 0
    tabs = [hermite_fn_table(t[:, d], nmax) for d in range(D)]  # (nmax+1, n)
    out = np.ones((n, len(mis)), dtype=np.float64)
    for i, a in enumerate(mis):
        for d in range(D):
            out[:, i] = out[:, i] * tabs[d][a[d]]
    return out


def raw_moments(points, w, ctr, p, family="graded"):
    """M_alpha = sum_r w_r (x_r - ctr)^alpha / alpha!, |alpha| < p (Figure 5,
    buildLeaf), h-independent form of Lemma 1's A_alpha."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    D = points.shape[1]
    mis = index_set(D, p, family)
    mono = _monomials(points - np.asarray(ctr, dtype=np.float64), mis)
    w = np.asarray(w, dtype=np.float64)
    return np.array([np.sum(w * mono[:, i]) / mi_factorial(a) for i, a in enumerate(mis)])


def scale_moments(M, D, p, h, family="graded"):
    """A_alpha = M_alpha (2h^2)^{-|alpha|/2} for the first C(D+p-1,D) entries."""
    s = _scale(h)
    mis = index_set(D, p, family)
    return np.array([M[i] * s ** mi_degree(a) for i, a in enumerate(mis)])


def hermite_moments(points, w, ctr, p, h, family="graded"):
    """A_alpha straight from Lemma 1's definition (used to pin scale_moments)."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    D = points.shape[1]
    mis = index_set(D, p, family)
    mono = _monomials((points - np.asarray(ctr, dtype=np.float64)) * _scale(h), mis)
    w = np.asarray(w, dtype=np.float64)
    return np.array([np.sum(w * mono[:, i]) / mi_factorial(a) for i, a in enumerate(mis)])


def h2h(M_child, ctr_child, ctr_parent, D, p, family="graded"):
    """Lemma 2 on raw moments: M_gamma = sum_{alpha<=gamma} M'_alpha
    (x_R'-x_R)^{gamma-alpha}/(gamma-alpha)!, |gamma| < p (Figure 5, buildInternal)."""
    mis = index_set(D, p, family)
    shift = np.asarray(ctr_child, dtype=np.float64) - np.asarray(ctr_parent, dtype=np.float64)
    out = np.zeros(len(mis))
    for gi, g in enumerate(mis):
        acc = 0.0
        for ai, a in enumerate(mis):
            if all(a[d] <= g[d] for d in range(D)):
                diff = tuple(g[d] - a[d] for d in range(D))
                mono = 1.0
                for d in range(D):
                    mono *= shift[d] ** diff[d]
                acc += M_child[ai] * mono / mi_factorial(diff)
        out[gi] = acc
    return out


def h2h_scaled(A_child, ctr_child, ctr_parent, D, p, h, family="graded"):
    """Lemma 2 exactly as stated, on scaled moments A (pins h2h)."""
    mis = index_set(D, p, family)
    shift = (np.asarray(ctr_child, dtype=np.float64) - np.asarray(ctr_parent, dtype=np.float64)) * _scale(h)
    out = np.zeros(len(mis))
    for gi, g in enumerate(mis):
        for ai, a in enumerate(mis):
            if all(a[d] <= g[d] for d in range(D)):
                diff = tuple(g[d] - a[d] for d in range(D))
                mono = 1.0
                for d in range(D):
                    mono *= shift[d] ** diff[d]
                out[gi] += A_child[ai] * mono / mi_factorial(diff)
    return out


def eval_hermite(A, p, ctr_R, xq, h, family="graded"):
    """Direct Hermite evaluation (EVALM/DIRECTM, section 6):
    sum_{|alpha|<p} A_alpha h_alpha((x_q - x_R) s) for every row of xq."""
    xq = np.atleast_2d(np.asarray(xq, dtype=np.float64))
    D = xq.shape[1]
    mis = index_set(D, p, family)
    hv = _hermite_products((xq - np.asarray(ctr_R, dtype=np.float64)) * _scale(h), mis)
    return hv @ np.asarray(A[: len(mis)], dtype=np.float64)


def direct_local(points, w, p, ctr_Q, h, family="graded"):
    """Direct local accumulation (DIRECTL, section 6):
    B_beta = sum_r w_r/beta! h_beta((x_r - x_Q) s), |beta| < p."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    D = points.shape[1]
    mis = index_set(D, p, family)
    hv = _hermite_products((points - np.asarray(ctr_Q, dtype=np.float64)) * _scale(h), mis)
    w = np.asarray(w, dtype=np.float64)
    return np.array([np.sum(w * hv[:, i]) / mi_factorial(b) for i, b in enumerate(mis)])


def h2l(A, p, ctr_R, ctr_Q, h, family="graded"):
    """Lemma 1: B_beta = (-1)^{|beta|}/beta! sum_{|alpha|<p} A_alpha
    h_{alpha+beta}((x_Q - x_R) s), for |beta| < p."""
    ctr_R = np.asarray(ctr_R, dtype=np.float64)
    D = ctr_R.shape[0]
    mis = index_set(D, p, family)
    t = (np.asarray(ctr_Q, dtype=np.float64) - ctr_R) * _scale(h)
    tabs = [hermite_fn_table(t[d], 2 * p) for d in range(D)]
    out = np.zeros(len(mis))
    for bi, b in enumerate(mis):
        acc = 0.0
        for ai, a in enumerate(mis):
            hv = 1.0
            for d in range(D):
                hv *= tabs[d][a[d] + b[d]]
            acc += A[ai] * hv
        out[bi] = (-1.0) ** mi_degree(b) / mi_factorial(b) * acc
    return out


def l2l(B, p, ctr_parent, ctr_child, h, family="graded"):
    """Lemma 3: C_alpha = sum_{beta>=alpha, |beta|<p} beta!/(alpha!(beta-alpha)!)
    B_beta ((x_Q - x_Q') s)^{beta-alpha}, Q the child, Q' the parent."""
    ctr_parent = np.asarray(ctr_parent, dtype=np.float64)
    D = ctr_parent.shape[0]
    mis = index_set(D, p, family)
    u = (np.asarray(ctr_child, dtype=np.float64) - ctr_parent) * _scale(h)
    out = np.zeros(len(mis))
    for ai, a in enumerate(mis):
        acc = 0.0
        for bi, b in enumerate(mis):
            if all(b[d] >= a[d] for d in range(D)):
                diff = tuple(b[d] - a[d] for d in range(D))
                mono = 1.0
                for d in range(D):
                    mono *= u[d] ** diff[d]
                coef = mi_factorial(b) / (mi_factorial(a) * mi_factorial(diff))
                acc += coef * B[bi] * mono
        out[ai] = acc
    return out


def eval_local(B, p, ctr_Q, xq, h, family="graded"):
    """Local evaluation (EVALL, section 6): sum_{|beta|<p} B_beta ((x_q-x_Q) s)^beta."""
    xq = np.atleast_2d(np.asarray(xq, dtype=np.float64))
    D = xq.shape[1]
    mis = index_set(D, p, family)
    mono = _monomials((xq - np.asarray(ctr_Q, dtype=np.float64)) * _scale(h), mis)
    return mono @ np.asarray(B[: len(mis)], dtype=np.float64)
