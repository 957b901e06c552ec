"""Least-squares cross-validation scores (gs_lscv) against the FP64 oracle:
every score within its reported bound of the exact score, and the same
minimising bandwidth wherever the bounds separate it from the others."""
import numpy as np
import pytest

from oracle.lscv import lscv
from paper_1206_6857_amd import _lib
from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("D,N,method", [(2, 3000, "dualtree"), (3, 2500, "dualtree"), (2, 2000, "exhaustive")])
def test_lscv_within_bound_of_oracle(D, N, method):
    banner("lscv", D, N, method)
    x, _, _ = mixture((71, D), N, D, 5, (0.02, 0.1))
    hs = np.logspace(-3, 0, 13)
    got, bound = ctx().lscv(x, hs, eps=0.01, method=method)
    want = lscv(x, hs)
    assert np.all(bound > 0)
    assert np.all(np.abs(got - want) <= bound + 1e-12 * np.abs(want)), np.abs(got - want) / bound
    k = int(np.argmin(want))
    others = np.delete(np.arange(len(hs)), k)
    if np.all(want[others] - want[k] > 2 * (bound[others] + bound[k])):
        assert int(np.argmin(got)) == k


@pytest.mark.parametrize("name", ["two_points", "one_dimension_one_bandwidth", "most_bandwidths"])
def test_lscv_edge_cases(name):
    """The fewest points the score is defined for (N = 2), a single bandwidth
    in one dimension, and the most bandwidths gs_lscv accepts (2048)."""
    banner("lscv edge", name)
    if name == "two_points":
        x = np.array([[0.1, 0.2], [0.15, 0.3]])
        hs = np.array([0.01, 0.1, 1.0])
    elif name == "one_dimension_one_bandwidth":
        x, _, _ = mixture((72, 1), 1500, 1, 3, (0.02, 0.1))
        hs = np.array([0.02])
    else:
        x, _, _ = mixture((73, 2), 200, 2, 3, (0.02, 0.1))
        hs = np.logspace(-3, 1, 2048)
    got, bound = ctx().lscv(x, hs, eps=0.01)
    want = lscv(x, hs)
    assert got.shape == want.shape == bound.shape
    assert np.all(bound > 0)
    assert np.all(np.abs(got - want) <= bound + 1e-12 * np.abs(want)), np.abs(got - want) / bound


def test_lscv_rejects_bad_arguments():
    import paper_1206_6857_amd as g
    c = ctx()
    x = np.random.default_rng(0).random((1, 2))
    with pytest.raises(g.GaussSumError) as e:
        c.lscv(x, [0.1])
    assert e.value.status == _lib.GS_EINVAL
    x = np.random.default_rng(0).random((10, 2))
    with pytest.raises(g.GaussSumError):
        c.lscv(x, [0.1, -1.0])
