"""The library's multi-index enumeration (host table, no GPU) is bit-exact with the oracle's."""
import os

import numpy as np
import pytest

from oracle.multiindex import multi_indices
from paper_1206_6857_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")


@pytest.mark.parametrize("D,p", [(1, 10), (2, 8), (3, 6), (4, 5), (5, 4), (6, 2), (8, 3), (16, 1), (64, 1)])
def test_multi_indices_bit_exact(D, p):
    import paper_1206_6857_amd as g
    got = g.gs_multi_indices(D, p)
    want = np.array(multi_indices(D, p), dtype=np.int32).reshape(-1, D)
    assert got.shape == want.shape and np.array_equal(got, want)


def test_multi_indices_rejects_bad_args():
    import paper_1206_6857_amd as g
    for D, p in [(0, 2), (65, 1), (2, 0), (2, 11)]:
        with pytest.raises(g.GaussSumError):
            g.gs_multi_indices(D, p)


@pytest.mark.parametrize("D,p", [(1, 10), (2, 8), (3, 6), (4, 4), (5, 3), (6, 2), (8, 2), (16, 1), (64, 1)])
def test_tensor_indices_bit_exact(D, p):
    import paper_1206_6857_amd as g
    from oracle.multiindex import tensor_indices
    got = g.gs_tensor_indices(D, p)
    want = np.array(tensor_indices(D, p), dtype=np.int32).reshape(-1, D)
    assert got.shape == want.shape and np.array_equal(got, want)


def test_tensor_indices_rejects_bad_args():
    import paper_1206_6857_amd as g
    for D, p in [(0, 2), (65, 1), (2, 0), (2, 11), (3, 7), (9, 2)]:
        with pytest.raises(g.GaussSumError):
            g.gs_tensor_indices(D, p)
