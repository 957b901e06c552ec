"""The FP64 operations every pruning decision is made of, on the device, bit
for bit against the host: division and square root must be correctly rounded
(IEEE-754, as numpy's are), and the library's own exp must equal the oracle's
independent exp of the same definition.  The decide kernels are compiled
without contraction, so with these three matching, the decisions made from
them match the oracle's."""
import numpy as np
import pytest

from oracle.exp64 import exp64
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu


def _inputs(n):
    rng = np.random.default_rng(19)
    x = np.concatenate([
        rng.uniform(-60.0, 0.0, n),                       # the range of -d^2 / 2h^2 that matters
        rng.uniform(-700.0, 709.0, n // 4),
        -np.exp(rng.uniform(-40, 6, n // 4)),              # tiny to large negative magnitudes
        (np.arange(-200, 200) + 0.5) / 1.4426950408889634,  # reduction boundaries
        [0.0, -0.0, -700.0, np.nextafter(-700.0, 0.0), np.nextafter(-700.0, -1.0), -745.0, 709.0,
         -1e-300, 5e-324],
    ])
    y = np.concatenate([np.exp(rng.uniform(-30, 30, x.size - 3)), [1.0, 5e-324, 1.7976931348623157e308]])
    # quotients in and below the subnormal range (x tiny, y >= 1), and square roots
    # of subnormal y, swept over the subnormal binades
    m = 4000
    xs = np.concatenate([10.0 ** rng.uniform(-323.5, -300.0, m), -(10.0 ** rng.uniform(-323.5, -300.0, m // 4))])
    ys = np.concatenate([10.0 ** rng.uniform(0.0, 10.0, m), 10.0 ** rng.uniform(0.0, 3.0, m // 4)])
    ysub = np.concatenate([np.ldexp(rng.uniform(1.0, 2.0, 60), -k) for k in range(1023, 1075)] +
                          [np.array([5e-324, 1e-323, 2.2250738585072009e-308, 2.2250738585072014e-308])])
    xsub = rng.uniform(-1.0, 1.0, ysub.size)
    return np.concatenate([x, xs, xsub]), np.concatenate([y, ys, ysub])


def test_decision_arithmetic_is_bit_exact():
    banner("decision arithmetic")
    x, y = _inputs(20001)
    e, q, s = ctx().decision_arith(x, y)
    want_e = np.array([exp64(v) for v in x])
    assert np.array_equal(e.view(np.int64), want_e.view(np.int64)), np.nonzero(e != want_e)[0][:5]
    with np.errstate(all="ignore"):
        want_q, want_s = x / y, np.sqrt(y)
    # the inputs do reach the subnormal range
    tiny = np.abs(want_q) < 2.2250738585072014e-308
    assert np.count_nonzero(tiny & (want_q != 0.0)) > 1000
    assert np.count_nonzero(y < 2.2250738585072014e-308) > 1000
    assert np.array_equal(q.view(np.int64), want_q.view(np.int64)), np.nonzero(q != want_q)[0][:5]
    assert np.array_equal(s.view(np.int64), want_s.view(np.int64)), np.nonzero(s != want_s)[0][:5]
