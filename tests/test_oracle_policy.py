"""Pins the policy network reference (oracle.mlp) and the training records
(oracle.policy) by means independent of their own formulas: central finite
differences for the gradient, the closed form of Adam's first step, a
hand-checked cost-to-go on a tiny trace, and the replay of the oracle's own
rule decisions through its certification path."""
import math

import numpy as np
import pytest

import oracle.dualtree as DT
from oracle import mlp
from oracle.policy import CostModel, cost_to_go, records
from paper_1206_6857_amd.datagen import mixture


def _batch(seed, n=37):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, mlp.N_PARAMS)
    X = rng.normal(0, 1, (n, 16))
    T = rng.normal(0, 1, (n, 4))
    Mk = (rng.random((n, 4)) < 0.6).astype(float)
    return theta, X, T, Mk


def test_gradient_matches_central_differences():
    theta, X, T, Mk = _batch(1)
    g = mlp.gradient(theta, X, T, Mk)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T, Mk) - mlp.loss(tm, X, T, Mk)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_masked_outputs_get_no_gradient():
    theta, X, T, _ = _batch(3)
    Mk = np.zeros((X.shape[0], 4))
    Mk[:, 2] = 1.0
    g = mlp.unpack(mlp.gradient(theta, X, T, Mk))
    assert np.all(g["W3"][[0, 1, 3]] == 0.0) and np.all(g["b3"][[0, 1, 3]] == 0.0)
    assert np.any(g["W3"][2] != 0.0)


def test_adam_first_step_closed_form():
    # first step: m^ = g, v^ = g^2, so theta moves by lr g / (|g| + eps)
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, _, _ = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, 0.01)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss_on_a_learnable_target():
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (256, 16))
    T = np.stack([X[:, 0] * 2 - X[:, 1], np.abs(X[:, 2]), X[:, 3] ** 2, X[:, 4]], axis=1)
    Mk = np.ones_like(T)
    theta = rng.normal(0, 0.1, mlp.N_PARAMS)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, T, Mk)
    for step in range(1, 301):
        theta, m, v = mlp.adam_step(theta, m, v, mlp.gradient(theta, X, T, Mk), step, 3e-3)
    assert mlp.loss(theta, X, T, Mk) < 0.1 * l0


class _Tree:
    def __init__(self, count, left):
        self.count = np.array(count)
        self.left = np.array(left)


def test_cost_to_go_by_hand():
    # query tree: root 0 -> leaves 1, 2; reference tree: root 0 -> leaves 1, 2
    qt = _Tree([4, 2, 2], [1, -1, -1])
    rt = _Tree([6, 3, 3], [1, -1, -1])
    cm = CostModel(pair=1.0, dh=0.5, dl=0.25, h2l=0.125, base=0.01)
    trace = [(0, 0, 0, 0, DT.SPLIT, 0),
             (0, 1, 1, 1, DT.BASE, 0), (0, 1, 1, 2, DT.FD, 0),
             (0, 1, 2, 1, DT.DH, 2), (0, 1, 2, 2, DT.DL, 1)]
    c = cost_to_go(trace, qt, rt, 1, cm)
    # D=1: C(p, 1) = p terms
    want_leaves = [1 + 2 * 3 * 0.01, 1.0, 1 + 2 * 2 * 0.5, 1 + 3 * 1 * 0.25]
    assert np.allclose(c[1:], want_leaves)
    assert math.isclose(c[0], 1.0 + sum(want_leaves))


def test_replay_of_own_rule_decisions_reproduces_the_run():
    r, w, _ = mixture((21, 2), 700, 2, 4, (0.02, 0.1))
    hs = np.array([0.01, 0.05, 0.3])
    a = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True, record_feasible=True)
    rep = {tuple(t[:4]): (t[4], t[5]) for t in a.trace}
    b = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True, replay=rep)
    assert a.trace == b.trace
    assert np.array_equal(a.G, b.G)
    # every replayed series choice was at its smallest admitted order
    for t in a.trace:
        if t[4] in (DT.DH, DT.DL, DT.H2L):
            assert a.feasible[tuple(t[:4])][DT.NAME[t[4]]] == t[5]


def test_replay_rejects_an_order_the_bound_does_not_admit():
    r, w, _ = mixture((22, 2), 700, 2, 4, (0.02, 0.1))
    hs = np.array([0.05, 0.3])
    a = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True)
    rep = {tuple(t[:4]): (t[4], t[5]) for t in a.trace}
    series = [k for k, v in rep.items() if v[0] in (DT.DH, DT.DL, DT.H2L) and v[1] > 1]
    assert series
    k = series[0]
    rep[k] = (rep[k][0], rep[k][1] - 1)      # one order too low
    with pytest.raises(DT.CertificationError):
        DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, replay=rep)


def test_replay_of_other_admitted_choices_keeps_theorem_2():
    """Direct instead of every series choice (always admitted): different
    pair lists, same guarantee."""
    from oracle.exhaustive import gauss_sum_exhaustive
    r, w, _ = mixture((23, 3), 800, 3, 4, (0.02, 0.1))
    hs = np.array([0.02, 0.1, 0.5])
    a = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True)

    class Direct(dict):
        def __missing__(self, key):
            return (DT.SPLIT, 0)
    b = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True, replay=Direct())
    assert b.counts[:, 1:4].sum() == 0 and a.counts[:, 1:4].sum() > 0
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(b.G - exact) / exact).max() <= 0.01


def test_records_shapes_and_masks():
    r, w, _ = mixture((24, 2), 600, 2, 4, (0.02, 0.1))
    hs = np.array([0.02, 0.2])
    a = DT.dualtree(r, r, w, hs, 0.01, leaf_size=16, trace=True, record_feasible=True)
    cm = CostModel(0.5, 2e-3, 2e-3, 1e-3, 3e-4)
    keys, F, T, Mk = records(a.trace, a.feasible, a.qtree, a.rtree, hs, 2, cm)
    assert len(keys) == len(a.feasible) > 0
    assert np.all(np.isfinite(T[Mk > 0]))
    codes = {tuple(t[:4]): t[4] for t in a.trace}
    for n, k in enumerate(keys):
        assert (Mk[n, 3] == 1.0) == (codes[k] in (DT.BASE, DT.SPLIT))
        assert Mk[n, :3].sum() == len(a.feasible[k])


def test_forward_on_a_hand_computed_network():
    """A sparse network whose output is worked out by hand below.  A dropped
    bias, a missing or misplaced ReLU, or a transposed weight matrix each
    changes at least one of the four outputs.

      x = (1, -2, 0.5, 0, ...)
      layer 1: a1_0 = 2*1 + 1*(-2) + 0.5 = 0.5   -> h1_0 = 0.5
               a1_1 = 1*(-2) - 1        = -3    -> h1_1 = 0     (ReLU)
               a1_2 = 4*0.5             = 2     -> h1_2 = 2
               a1_3 = -1 (bias only)            -> h1_3 = 0
      layer 2: a2_0 = h1_0 - h1_2 + 3   = 1.5   -> h2_0 = 1.5
               a2_1 = 5 h1_1 + 0.25     = 0.25  -> h2_1 = 0.25
               a2_2 = -h1_2 + 1         = -1    -> h2_2 = 0     (ReLU)
      output:  y_0 = 2 h2_0 + 0.1              = 3.1
               y_1 = -h2_0 + 4 h2_1            = -0.5
               y_2 = 7 h2_2 - 0.5              = -0.5
               y_3 = h2_0 + h2_1 + h2_2 + 1    = 2.75
    """
    P = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    P["W1"][0, 0], P["W1"][0, 1], P["b1"][0] = 2.0, 1.0, 0.5
    P["W1"][1, 1], P["b1"][1] = 1.0, -1.0
    P["W1"][2, 2] = 4.0
    P["b1"][3] = -1.0
    P["W2"][0, 0], P["W2"][0, 2], P["b2"][0] = 1.0, -1.0, 3.0
    P["W2"][1, 1], P["b2"][1] = 5.0, 0.25
    P["W2"][2, 2], P["b2"][2] = -1.0, 1.0
    P["W3"][0, 0], P["b3"][0] = 2.0, 0.1
    P["W3"][1, 0], P["W3"][1, 1] = -1.0, 4.0
    P["W3"][2, 2], P["b3"][2] = 7.0, -0.5
    P["W3"][3, :3], P["b3"][3] = 1.0, 1.0
    x = np.zeros((1, 16))
    x[0, :3] = (1.0, -2.0, 0.5)
    y, _ = mlp.forward(mlp.pack(P), x)
    assert np.allclose(y[0], [3.1, -0.5, -0.5, 2.75], rtol=0, atol=1e-15), y


def test_pair_features_of_a_hand_built_pair():
    """Two boxes in D = 2 whose distances are worked out by hand:
    Q = [0,1] x [0,2] (8 points, a leaf, rinf 1), R = [3,4] x [0,1]
    (32 points, internal, rinf 0.5), h = 0.5.  The closest points are 2 apart
    along the first axis (dmin = 2); the farthest are 4 apart along the first
    and 2 along the second (dmax = sqrt(20) = 2 sqrt(5))."""
    from types import SimpleNamespace

    from oracle.policy import pair_features
    qt = SimpleNamespace(lo=[np.array([0.0, 0.0])], hi=[np.array([1.0, 2.0])], count=[8], rinf=[1.0],
                         left=[-1])
    rt = SimpleNamespace(lo=[np.array([3.0, 0.0])], hi=[np.array([4.0, 1.0])], count=[32], rinf=[0.5],
                         left=[5])
    f = pair_features(qt, rt, 0, 0, 0.5, 2)
    want = np.zeros(16)
    want[:10] = [3.0,                              # log2 8
                 5.0,                              # log2 32
                 math.log2(5.0),                   # log2(1 + 2/0.5)
                 math.log2(1.0 + 4.0 * math.sqrt(5.0)),  # log2(1 + 2 sqrt5 / 0.5)
                 -1.0,                             # log2 0.5
                 math.log2(3.0),                   # log2(1 + 1/0.5)
                 1.0,                              # log2(1 + 0.5/0.5)
                 1.0, 0.0,                         # Q is a leaf, R is not
                 2.0 / 16.0]
    assert np.allclose(f, want, rtol=0, atol=1e-14), f - want
