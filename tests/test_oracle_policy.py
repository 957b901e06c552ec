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
