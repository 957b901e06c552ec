"""Seeded synthetic inputs shaped like the paper's kernel-density workloads.

This module holds only random-number plumbing (NumPy PCG64 streams) and no part
of the summation method, so tests and the benchmark can feed identical inputs
to the library and to an independent checker.

The paper's datasets (astronomy, simulation, pharmaceutical, ... scaled to the
unit hypercube, section 7) are not available; Gaussian mixtures with the stated
dimensions, cluster counts, cluster spreads and size skew stand in for them.

Recipe for every workload (stream 0 = references, 1 = queries, 2 = mixture
parameters shared by both):
  1. component means ~ U[0,1]^D;
  2. per-component sigma (fixed or uniform in a range);
  3. component sizes (equal, or proportional to k^-1.5 with largest-remainder
     rounding);
  4. points = mean + sigma * N(0, I_D), no clipping;
  5. shuffle, so the input is not cluster-sorted;
  6. weights (1/N, or uniform in [0.5, 1.5]).
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    D: int
    refs: np.ndarray
    weights: np.ndarray
    queries: np.ndarray          # the same object as refs when monochromatic
    bandwidths: np.ndarray
    eps: float
    monochromatic: bool
    meta: dict = field(default_factory=dict)


def power_law_sizes(n, k, exponent):
    """Component sizes proportional to i^-exponent, i = 1..k, summing to n
    (largest-remainder rounding)."""
    raw = np.arange(1, k + 1, dtype=np.float64) ** (-exponent)
    share = raw / raw.sum() * n
    base = np.floor(share).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return base


def equal_sizes(n, k):
    base = np.full(k, n // k, dtype=np.int64)
    base[: n - int(base.sum())] += 1
    return base


def _mixture_params(seed_key, D, k, sigma):
    rng = np.random.default_rng(list(seed_key) + [2])
    means = rng.random((k, D))
    if np.isscalar(sigma):
        sig = np.full(k, float(sigma))
    else:
        sig = rng.uniform(sigma[0], sigma[1], size=k)
    return means, sig


def _draw(seed_key, stream, means, sig, sizes):
    rng = np.random.default_rng(list(seed_key) + [stream])
    D = means.shape[1]
    parts = [means[i] + sig[i] * rng.standard_normal((int(sizes[i]), D)) for i in range(len(sizes))]
    pts = np.concatenate(parts, axis=0)
    pts = pts[rng.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts, dtype=np.float64), rng


def mixture(seed_key, n, D, k, sigma, sizes="equal", weights="uniform_n", stream=0, m_queries=None):
    """Reference (and optionally query) draws from one Gaussian mixture.

    sigma: a float, or (lo, hi) for per-component U(lo, hi).
    sizes: "equal" or ("power", exponent).
    weights: "uniform_n" (1/N each) or (lo, hi) for U(lo, hi).
    Returns (refs, weights, queries_or_None)."""
    means, sig = _mixture_params(seed_key, D, k, sigma)
    def size_vec(m):
        return equal_sizes(m, k) if sizes == "equal" else power_law_sizes(m, k, sizes[1])
    refs, rng = _draw(seed_key, stream, means, sig, size_vec(n))
    if weights == "uniform_n":
        w = np.full(n, 1.0 / n)
    else:
        w = rng.uniform(weights[0], weights[1], size=n)
    q = None
    if m_queries is not None:
        q, _ = _draw(seed_key, 1, means, sig, size_vec(m_queries))
    return refs, np.ascontiguousarray(w), q


def _mixture_draw(seed_key, *a, **k):
    return mixture(seed_key, *a, **k)


def logspace_bandwidths(lo_exp, hi_exp, n):
    return np.array([10.0 ** (lo_exp + (hi_exp - lo_exp) * i / (n - 1)) for i in range(n)]) if n > 1 \
        else np.array([10.0 ** lo_exp])


def workload(cfg, scale=1.0, D=None, draw=0):
    """The five workloads (by index 0..4), optionally with N and M scaled down.
    draw > 0 gives another independent draw of the same workload (its points
    and weights; the bandwidths and eps are the same).

    0: D=2, N=M=10,000 monochromatic, 4 components sigma=0.05, w=1/N, h=0.1.
    1: D=3, N=M=100,000 monochromatic, 8 components sigma~U(0.01,0.1), w=1/N,
       10 bandwidths log-spaced 1e-3..1.
    2: D=5, N=M=500,000 monochromatic, 64 components with sizes ~ k^-1.5,
       sigma~U(0.005,0.05), w~U(0.5,1.5), 32 bandwidths log-spaced 1e-3..1.
    3: D=16 bichromatic, N=200,000 refs, M=50,000 queries, 16 components
       sigma=0.1, w~U(0.5,1.5), 16 bandwidths 0.05*40^(k/15).
    4: N=M=1,000,000 for D in {2,3,5,8}, 64 bandwidths log-spaced 1e-3..1; D=2,
       3, 5 follow workloads 0, 1, 2, D=8 follows workload 3's mixture.
    eps = 0.01 for all."""
    def n_of(base):
        return max(2, int(round(base * scale)))

    def mixture(seed_key, *a, **k):
        return _mixture_draw(tuple(seed_key) + ((draw,) if draw else ()), *a, **k)
    if cfg == 0:
        N = n_of(10_000)
        r, w, _ = mixture((0, 2), N, 2, 4, 0.05)
        return Workload("d2_n%d_mono_1h" % N, 2, r, w, r, np.array([0.1]), 0.01, True)
    if cfg == 1:
        N = n_of(100_000)
        r, w, _ = mixture((1, 3), N, 3, 8, (0.01, 0.1))
        return Workload("d3_n%d_mono_10h" % N, 3, r, w, r, logspace_bandwidths(-3, 0, 10), 0.01, True)
    if cfg == 2:
        N = n_of(500_000)
        r, w, _ = mixture((2, 5), N, 5, 64, (0.005, 0.05), sizes=("power", 1.5), weights=(0.5, 1.5))
        return Workload("d5_n%d_mono_32h" % N, 5, r, w, r, logspace_bandwidths(-3, 0, 32), 0.01, True)
    if cfg == 3:
        N, M = n_of(200_000), n_of(50_000)
        r, w, q = mixture((3, 16), N, 16, 16, 0.1, weights=(0.5, 1.5), m_queries=M)
        hs = np.array([0.05 * 40.0 ** (k / 15.0) for k in range(16)])
        return Workload("d16_n%d_m%d_bichro_16h" % (N, M), 16, r, w, q, hs, 0.01, False)
    if cfg == 4:
        D = D or 2
        N = n_of(1_000_000)
        hs = logspace_bandwidths(-3, 0, 64)
        if D == 2:
            r, w, _ = mixture((4, 2), N, 2, 4, 0.05)
        elif D == 3:
            r, w, _ = mixture((4, 3), N, 3, 8, (0.01, 0.1))
        elif D == 5:
            r, w, _ = mixture((4, 5), N, 5, 64, (0.005, 0.05), sizes=("power", 1.5), weights=(0.5, 1.5))
        else:
            r, w, _ = mixture((4, D), N, D, 16, 0.1, weights=(0.5, 1.5))
        return Workload("d%d_n%d_mono_64h" % (D, N), D, r, w, r, hs, 0.01, True)
    raise ValueError(cfg)
