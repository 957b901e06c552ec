"""The Python binding refuses arrays whose sizes disagree before it passes any
pointer to the library: the C ABI takes plain pointers and sizes and reads or
writes exactly what the sizes say, so a mismatch would run past a caller's
buffer.  The checks run before the first library call, so no GPU is needed
(the context is made without gs_create)."""
import numpy as np
import pytest

import paper_1206_6857_amd as g


@pytest.fixture
def c():
    obj = object.__new__(g.Context)
    obj._h = None
    obj.device = 0
    return obj


def test_refs_of_another_dimension(c):
    with pytest.raises(ValueError, match="same dimension"):
        c.gauss_sum(np.zeros((5, 2)), np.zeros((7, 3)), np.ones(7), [0.1], 0.01)


def test_weights_of_another_length(c):
    with pytest.raises(ValueError, match="weights"):
        c.gauss_sum(np.zeros((5, 2)), np.zeros((7, 2)), np.ones(6), [0.1], 0.01)
    with pytest.raises(ValueError, match="weights"):
        c.gauss_sum(np.zeros((5, 2)), np.zeros((7, 2)), np.ones(8), [0.1], 0.01)


@pytest.mark.parametrize("shape", [(2, 4), (1, 5), (10,), (2, 5, 1)])
def test_output_of_another_shape(c, shape):
    with pytest.raises(ValueError, match="out must have shape"):
        c.gauss_sum(np.zeros((5, 2)), np.zeros((7, 2)), np.ones(7), [0.1, 0.2], 0.01, out=np.zeros(shape))


def test_points_must_be_two_dimensional(c):
    with pytest.raises(ValueError):
        c.gauss_sum(np.zeros(5), np.zeros(5), np.ones(5), [0.1], 0.01)
    with pytest.raises(ValueError):
        c.lscv(np.zeros(5), [0.1])


def test_policy_arrays_of_another_width(c):
    with pytest.raises(ValueError, match="records"):
        c.policy_gradient(np.zeros((10, 23), dtype=np.float32))
    with pytest.raises(ValueError, match="records"):
        c.policy_train(np.zeros((10, 25), dtype=np.float32), steps=1)
    with pytest.raises(ValueError, match="features"):
        c.policy_predict(np.zeros((10, 15), dtype=np.float32))
    with pytest.raises(ValueError, match="features"):
        c.policy_predict(np.zeros(16, dtype=np.float32))
