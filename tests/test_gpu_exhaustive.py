"""Parity of the plain GPU exhaustive path against the FP64 oracle, and the
C ABI's argument errors."""
import numpy as np
import pytest

from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu

# Rounding budget of the float32 path: the exponent a = d^2/(2h^2) carries a
# relative error of about (2D+2) 2^-24 from the split-coordinate difference and
# the D-term sum, so a term's relative error is ~a (2D+2) 2^-24 plus one ulp of
# exp2; float partial sums of <= 256 terms add <= 256 2^-24 in the worst case.
# For the queries of these mixtures a <= ~200 on the dominant terms, giving the
# bound below: half of the 1e-3 share of eps reserved for rounding.  The median
# check catches systematic errors that a max-only bound would hide.
TOL = 5e-4
TOL_MEDIAN = 1e-6


@pytest.mark.parametrize("D,M,N,nh", [(1, 300, 517, 3), (2, 1000, 1000, 1), (3, 777, 2049, 10),
                                      (5, 513, 700, 17), (8, 129, 300, 4), (16, 260, 1100, 16),
                                      (7, 33, 65, 2), (3, 1, 1, 1), (64, 100, 300, 3)])
def test_exhaustive_matches_oracle(D, M, N, nh):
    banner("exhaustive", D, M, N, nh)
    r, w, q = mixture((50, D), N, D, 3, (0.02, 0.2), weights=(0.5, 1.5), m_queries=M)
    hs = np.logspace(-2, 0.5, nh)
    G = ctx().gauss_sum(q, r, w, hs, 0.01, method="exhaustive")
    want = gauss_sum_exhaustive(q, r, w, hs)
    # where the FP64 reference underflows (true G below ~1e-300) the GPU may still
    # resolve a tiny value; both are then zero to within double range
    ok = want > 1e-290
    assert np.all(G[~ok] < 1e-290)
    rel = np.abs(G[ok] - want[ok]) / want[ok]
    assert rel.max() <= TOL, rel.max()
    assert np.median(rel) <= TOL_MEDIAN, np.median(rel)


def test_exhaustive_monochromatic_torch_device():
    import torch
    banner("exhaustive torch device")
    r, w, _ = mixture((51, 3), 3000, 3, 4, (0.01, 0.1))
    hs = np.array([1e-3, 1e-2, 0.1, 1.0])
    rt = torch.from_numpy(r).cuda()
    G = ctx().gauss_sum(rt, rt, torch.from_numpy(w).cuda(), torch.from_numpy(hs).cuda(), 0.01,
                        method="exhaustive").cpu().numpy()
    want = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G - want) / want).max() <= TOL


@pytest.mark.parametrize("bad", ["nan", "inf", "w0", "wneg", "h0", "eps0", "eps1", "D0"])
def test_invalid_arguments(bad):
    import paper_1206_6857_amd as g
    banner("invalid", bad)
    r = np.random.default_rng(0).uniform(0, 1, (50, 2))
    w = np.ones(50)
    hs = np.array([0.1])
    eps = 0.01
    kw = {}
    if bad == "nan":
        r[3, 1] = np.nan
    elif bad == "inf":
        r[7, 0] = np.inf
    elif bad == "w0":
        w[4] = 0.0
    elif bad == "wneg":
        w[9] = -1.0
    elif bad == "h0":
        hs = np.array([0.1, 0.0])
    elif bad == "eps0":
        eps = 0.0
    elif bad == "eps1":
        eps = 1.0
    elif bad == "D0":
        r = np.zeros((50, 0))
    with pytest.raises(g.GaussSumError) as e:
        ctx().gauss_sum(r, r, w, hs, eps, **kw)
    assert e.value.status == -1
    # the context stays usable
    ok = ctx().gauss_sum(np.ones((3, 2)), np.ones((3, 2)), np.ones(3), [1.0], 0.01, method="exhaustive")
    assert np.allclose(ok, 3.0)
