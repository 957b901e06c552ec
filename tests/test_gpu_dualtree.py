"""Parity of the GPU dual-tree path with the oracle.

* Tree: every integer and box field bit-exact with the oracle's kd-tree.
* Decisions: the trace (h, level, Q, R, code, p) of every decided node pair is
  identical to the oracle's level-wise traversal (integer work, bit-exact).
* Values: G~ differs from the oracle's G~ only by rounding (same pair lists),
  and every query meets Theorem 2's |G~ - G| <= eps G against the FP64
  exhaustive sum.
"""
import numpy as np
import pytest

import oracle.dualtree as DT
from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu

# Rounding of the GPU value path against the oracle's identical pair lists:
# float32 base tiles (exponent error ~a (D+2) 2^-24, a = d^2/2h^2 <= ~100 on
# the terms that matter), double-precision series.  1e-4 relative to G is a
# tenth of the 1e-3 share of eps reserved for rounding.
TOL_ROUND = 1e-4

CASES = [
    # (name, D, N, M (None: monochromatic), hs, leaf, method[, plimit])
    ("d1", 1, 900, None, [1e-3, 1e-2, 0.05, 0.3, 2.0], 16, "dito"),
    ("d2", 2, 1500, None, [1e-3, 1e-2, 0.03, 0.1, 0.3, 1.0, 10.0], 32, "dito"),
    ("d3", 3, 1500, None, [1e-3, 1e-2, 0.05, 0.2, 1.0], 32, "dito"),
    ("d5", 5, 1000, None, [1e-2, 0.1, 0.5, 3.0], 32, "dito"),
    ("d2_dfdo", 2, 1200, None, [1e-2, 0.1, 1.0], 32, "dfdo"),
    ("d3_dfd", 3, 1200, None, [1e-2, 0.1, 1.0], 32, "dfd"),
    ("d2_bi", 2, 1300, 700, [0.01, 0.05, 0.2, 1.0], 32, "dito"),
    ("d3_bi", 3, 1100, 500, [0.02, 0.1, 0.5], 16, "dito"),
    ("d16_bi", 16, 900, 300, [0.05, 0.3, 2.0], 64, "dito"),
    ("d2_leaf64_ragged", 2, 1001, None, [0.02, 0.2], 64, "dito"),
    ("d2_plimit5_generic", 2, 1200, None, [0.03, 0.1, 0.3], 32, "dito", 5),
    ("d4_table", 4, 1000, None, [0.05, 0.2, 1.0], 32, "dito"),
    # one series method at a time (bestMethod restricted by fmm_mask), so that
    # each expansion kernel carries every series prune of the run
    ("d2_h2l_only", 2, 1500, None, [0.03, 0.1, 0.3, 1.0], 32, "dito", 0, 4),
    ("d3_h2l_only", 3, 1500, None, [0.05, 0.2, 1.0], 32, "dito", 0, 4),
    ("d3_dl_only", 3, 1500, None, [0.05, 0.2, 1.0], 32, "dito", 0, 2),
    ("d3_dh_only", 3, 1500, None, [0.05, 0.2, 1.0], 32, "dito", 0, 1),
    # O(p^D) expansions (tensor index sets, generic kernels) and their bounds
    ("d1_dfto", 1, 900, None, [1e-3, 1e-2, 0.05, 0.3, 2.0], 16, "dfto"),
    ("d2_dfto", 2, 1500, None, [1e-3, 1e-2, 0.03, 0.1, 0.3, 1.0], 32, "dfto"),
    ("d3_dfto", 3, 1500, None, [1e-3, 1e-2, 0.05, 0.2, 1.0], 32, "dfto"),
    ("d4_dfto_256_terms", 4, 1000, None, [0.05, 0.2, 1.0], 32, "dfto"),
    ("d5_dfto_bi_243_terms", 5, 1000, 400, [0.05, 0.3, 2.0], 32, "dfto"),
    ("d2_dfto_h2l_only", 2, 1500, None, [0.03, 0.1, 0.3, 1.0], 32, "dfto", 0, 4),
    ("d3_dfto_h2l_only", 3, 1500, None, [0.1, 0.3, 1.0, 3.0], 32, "dfto", 0, 4),
    ("d3_dfto_dl_only", 3, 1500, None, [0.1, 0.3, 1.0, 3.0], 32, "dfto", 0, 2),
    ("d3_dfto_dh_only", 3, 1500, None, [0.1, 0.3, 1.0, 3.0], 32, "dfto", 0, 1),
    ("d6_dfto_bi", 6, 900, 300, [0.1, 0.5, 3.0], 32, "dfto"),
    # an order limit without compiled tensor kernels: the generic kernels
    ("d3_dfto_plimit4_generic", 3, 1500, None, [1e-2, 0.05, 0.2, 1.0], 32, "dfto", 4),
    # the leaf sizes the autotuner picks at the benchmark's sizes, on inputs large
    # enough for several query batches per work unit (leaf 256: four batches of 64)
    # and runs cut into several slices whose partial sums are added afterwards
    ("d3_leaf256_mid", 3, 20000, None, list(np.logspace(-3, 0, 10)), 256, "dito"),
    ("d3_leaf128_mid", 3, 12000, None, list(np.logspace(-3, 0, 10)), 128, "dito"),
    ("d5_leaf128_mid", 5, 8000, None, list(np.logspace(-3, 0, 8)), 128, "dito"),
    ("d8_leaf256_mid_bi", 8, 9000, 3000, list(np.logspace(-2, 0.3, 6)), 256, "dito"),
]


def _inputs(D, N, M, seed):
    r, w, q = mixture((seed, D), N, D, 4, (0.02, 0.1), weights=(0.5, 1.5), m_queries=M)
    return r, w, (r if M is None else q)


def _check_stats(st, ref, method, pair_evals):
    """The call's statistics against the oracle's run: the histogram of the
    chosen orders (Figure 6) bit-exact from the oracle's trace, and the token
    deposits and withdrawals (section 5) from its ledger of resolved pairs,
    within the rounding of a sum taken in another order."""
    from oracle.bounds import need
    hist = np.zeros((3, 16), dtype=np.int64)
    for hk, lvl, Q, R, code, p in ref.trace:
        if code in (DT.DH, DT.DL, DT.H2L):
            hist[code - DT.DH, p] += 1
    got = np.array([[st.p_hist[x][p] for p in range(16)] for x in range(3)])
    assert np.array_equal(got, hist), (got, hist)
    dep = wd = 0.0
    if method != "dfd":
        W = float(ref.rtree.W[0])
        for hk, Q, R, code, E, L, WR, t in ref.ledger:
            v = -WR if code == DT.BASE else need(E, WR, L, W, ref.eps_alg)
            dep += max(-v, 0.0)
            wd += max(v, 0.0)
    assert abs(st.tokens_deposited - dep) <= 1e-10 * max(dep, 1e-300), (st.tokens_deposited, dep)
    assert abs(st.tokens_withdrawn - wd) <= 1e-10 * max(wd, 1e-300), (st.tokens_withdrawn, wd)
    assert st.pair_evals_per_s == pytest.approx(pair_evals / (st.t_total_ms * 1e-3), rel=1e-12)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_dualtree_parity(case):
    name, D, N, M, hs, leaf, method = case[:7]
    plimit = case[7] if len(case) > 7 else 0
    mask = case[8] if len(case) > 8 else 7
    banner("dualtree", name)
    r, w, q = _inputs(D, N, M, 70 + D)
    hs = np.array(hs)
    c = ctx()
    G = c.gauss_sum(q, r, w, hs, 0.01, method=method, leaf_size=leaf, keep_trace=1, plimit=plimit,
                    fmm_mask=mask)
    ref = DT.dualtree(q, r, w, hs, 0.01, leaf_size=leaf, method=method, trace=True,
                      plimit=plimit or None, fmm_mask=mask, ledger=True)
    _check_stats(c.stats(), ref, method, q.shape[0] * r.shape[0] * len(hs))
    if mask != 7:
        # the restricted method carries the series prunes of the run
        code = {1: 1, 2: 2, 4: 3}[mask]
        assert ref.counts[:, code].sum() > 20, ref.counts.sum(axis=0)

    # tree, bit-exact
    for which, t in ((0, ref.rtree), (1, ref.qtree)):
        gt = c.get_tree(which, D)
        assert np.array_equal(gt["perm"], t.perm)
        assert np.array_equal(gt["begin"], t.begin) and np.array_equal(gt["count"], t.count)
        assert np.array_equal(gt["left"], t.left)
        for k in ("lo", "hi", "ctr", "rinf"):
            assert np.array_equal(gt[k], getattr(t, k)), k
        if which == 0:
            assert np.array_equal(gt["W"], t.W) and np.array_equal(gt["wmin"], t.wmin)

    # decisions, bit-exact
    got = c.get_trace()
    want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert got.shape == want.shape, (got.shape, want.shape)
    g_s, w_s = key(got.astype(np.int64)), key(want)
    if not np.array_equal(g_s, w_s):
        bad = np.nonzero(np.any(g_s != w_s, axis=1))[0][:5]
        raise AssertionError("trace mismatch at %s: gpu %s oracle %s" % (bad, g_s[bad], w_s[bad]))
    assert np.array_equal(c.pair_counts(len(hs)), ref.counts)

    # values
    exact = gauss_sum_exhaustive(q, r, w, hs)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01


SPHERE_CASES = [
    # (name, D, N, M, hs, leaf)
    ("d2", 2, 1500, None, [0.01, 0.05, 0.2, 1.0], 32),
    ("d3", 3, 1500, None, [0.01, 0.05, 0.2, 1.0], 32),
    ("d8_bi", 8, 900, 400, [0.05, 0.3, 2.0], 32),
]


@pytest.mark.parametrize("case", SPHERE_CASES, ids=[c[0] for c in SPHERE_CASES])
def test_dualtree_sphere_rect_parity(case):
    """Sphere-rectangle node bounds: node radii and the decision trace
    bit-exact with the oracle's, values within rounding of it, Theorem 2."""
    name, D, N, M, hs, leaf = case
    banner("dualtree sphere_rect", name)
    r, w, q = _inputs(D, N, M, 90 + D)
    hs = np.array(hs)
    c = ctx()
    G = c.gauss_sum(q, r, w, hs, 0.01, leaf_size=leaf, keep_trace=1, node_bounds="sphere_rect")
    ref = DT.dualtree(q, r, w, hs, 0.01, leaf_size=leaf, trace=True, node_bounds="sphere_rect")
    for which, t in ((0, ref.rtree), (1, ref.qtree)):
        gt = c.get_tree(which, D)
        assert np.array_equal(gt["rad"], t.rad)
    got = c.get_trace().astype(np.int64)
    want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert np.array_equal(key(got), key(want))
    exact = gauss_sum_exhaustive(q, r, w, hs)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01


FAR_FIRST_CASES = [
    # (name, D, N, M, hs, leaf, method, node_bounds)
    ("d2", 2, 1500, None, [1e-3, 0.01, 0.05, 0.2, 1.0], 32, "dito", "box"),
    ("d3", 3, 1500, None, [1e-3, 0.01, 0.05, 0.2, 1.0], 32, "dito", "box"),
    ("d3_bi_leaf64", 3, 1300, 600, [0.02, 0.1, 0.5], 64, "dito", "box"),
    ("d5", 5, 1000, None, [0.01, 0.1, 0.5, 3.0], 32, "dito", "box"),
    ("d3_dfto", 3, 1500, None, [1e-3, 1e-2, 0.05, 0.2, 1.0], 32, "dfto", "box"),
    ("d3_dfdo", 3, 1200, None, [1e-2, 0.1, 1.0], 32, "dfdo", "box"),
    ("d2_sphere_rect", 2, 1500, None, [0.01, 0.05, 0.2, 1.0], 32, "dito", "sphere_rect"),
]


@pytest.mark.parametrize("case", FAR_FIRST_CASES, ids=[c[0] for c in FAR_FIRST_CASES])
def test_dualtree_far_first_parity(case):
    """The best-first walk (pair_order="far_first": every query node's list in
    decreasing dmin^2, ties by reference node, at every level): the decision
    trace bit-exact with the oracle's run in the same order, values within
    rounding of it, Theorem 2; and the order does change decisions."""
    name, D, N, M, hs, leaf, method, nb = case
    banner("dualtree far_first", name)
    r, w, q = _inputs(D, N, M, 110 + D)
    hs = np.array(hs)
    c = ctx()
    G = c.gauss_sum(q, r, w, hs, 0.01, leaf_size=leaf, keep_trace=1, method=method, node_bounds=nb,
                    pair_order="far_first")
    ref = DT.dualtree(q, r, w, hs, 0.01, leaf_size=leaf, trace=True, method=method, node_bounds=nb,
                      pair_order="far_first")
    got = c.get_trace().astype(np.int64)
    want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.array_equal(key(got), key(want))
    assert np.array_equal(c.pair_counts(len(hs)), ref.counts)
    exact = gauss_sum_exhaustive(q, r, w, hs)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01
    tree = DT.dualtree(q, r, w, hs, 0.01, leaf_size=leaf, method=method, node_bounds=nb)
    if method != "dfd":
        assert not np.array_equal(tree.counts, ref.counts)


def test_dualtree_torch_device_and_repeat():
    import torch
    banner("dualtree torch repeat")
    r, w, _ = mixture((81, 3), 4000, 3, 8, (0.01, 0.1))
    hs = np.logspace(-3, 0, 10)
    rt = torch.from_numpy(r).cuda()
    wt = torch.from_numpy(w).cuda()
    ht = torch.from_numpy(hs).cuda()
    G1 = ctx().gauss_sum(rt, rt, wt, ht, 0.01).cpu().numpy()
    G2 = ctx().gauss_sum(rt, rt, wt, ht, 0.01).cpu().numpy()
    assert np.array_equal(G1, G2)   # deterministic: no float atomics
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G1 - exact) / exact).max() <= 0.01


def _sorted_trace(c):
    t = c.get_trace().astype(np.int64)
    return t[np.lexsort(t.T[::-1])]


def test_dualtree_bandwidth_chunks():
    """Bandwidths never interact in the traversal: any split of the sweep
    (h_chunk) makes the same decisions; values differ only by the summation
    order of the base tiles.  20 bandwidths span two base-tile blocks of 16,
    and chunks of 3 and 7 split both blocks across chunks."""
    banner("dualtree chunks")
    r, w, _ = mixture((91, 3), 3000, 3, 8, (0.01, 0.1))
    hs = np.logspace(-3, 0, 20)
    c = ctx()
    G0 = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32, keep_trace=1)
    tr0 = _sorted_trace(c)
    pc0 = c.pair_counts(len(hs))
    st0 = c.stats()
    assert st0.h_chunks == 1
    assert 0 < st0.base_dist_evals <= st0.base_pair_evals
    for chunk in (1, 3, 7):
        G = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32, keep_trace=1, h_chunk=chunk)
        st = c.stats()
        assert st.h_chunks == -(-len(hs) // chunk)
        assert st.base_pair_evals == st0.base_pair_evals
        assert np.array_equal(_sorted_trace(c), tr0)
        assert np.array_equal(c.pair_counts(len(hs)), pc0)
        assert (np.abs(G - G0) / G0).max() <= 1e-12, chunk
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G0 - exact) / exact).max() <= 0.01


def test_dualtree_frontier_cap_retry():
    """A frontier cap below the full sweep's frontier makes the library halve
    the bandwidth chunk and redo it; the decisions and values are those of the
    uncapped call.  A cap no single bandwidth fits in is an overflow error."""
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    banner("dualtree frontier cap")
    r, w, _ = mixture((92, 2), 2000, 2, 6, (0.01, 0.1))
    hs = np.logspace(-2.5, 0, 6)
    c = ctx()
    G0 = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=16, keep_trace=1)
    tr0 = _sorted_trace(c)
    peak = c.stats().frontier_peak
    # the largest frontier of one bandwidth: from single-bandwidth runs
    one = 0
    for k in range(len(hs)):
        c.gauss_sum(r, r, w, hs[k:k + 1], 0.01, leaf_size=16)
        one = max(one, c.stats().frontier_peak)
    assert one < peak
    G = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=16, keep_trace=1, max_frontier=one)
    st = c.stats()
    assert st.h_chunks > 1 and st.frontier_peak <= one
    assert np.array_equal(_sorted_trace(c), tr0)
    assert (np.abs(G - G0) / G0).max() <= 1e-12
    with pytest.raises(g.GaussSumError) as ei:
        c.gauss_sum(r, r, w, hs, 0.01, leaf_size=16, max_frontier=one - 1)
    assert ei.value.status == _lib.GS_EOVERFLOW


def test_autotune_picks_and_caches_a_configuration():
    """autotune=1 times the leaf sizes and the exhaustive path once per
    workload signature, then reuses the choice; every candidate is a correct
    method, so the result meets Theorem 2 whichever is chosen."""
    import paper_1206_6857_amd as g
    banner("autotune")
    c = g.Context(0)
    r, w, _ = mixture((93, 3), 6000, 3, 6, (0.01, 0.1))
    hs = np.logspace(-3, 0, 6)
    G1 = c.gauss_sum(r, r, w, hs, 0.01, autotune=1)
    st1 = c.stats()
    assert st1.autotune_trials >= 5
    assert st1.tuned_method in (g.GS_DUALTREE, g.GS_EXHAUSTIVE)
    assert st1.tuned_leaf_size in (32, 64, 128, 256) or st1.tuned_method == g.GS_EXHAUSTIVE
    G2 = c.gauss_sum(r, r, w, hs, 0.01, autotune=1)
    st2 = c.stats()
    assert st2.autotune_trials == 0
    assert (st2.tuned_method, st2.tuned_leaf_size) == (st1.tuned_method, st1.tuned_leaf_size)
    assert np.array_equal(G1, G2)
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G2 - exact) / exact).max() <= 0.01
    # another signature (bandwidth range) is tuned on its own
    c.gauss_sum(r, r, w, hs * 10, 0.01, autotune=1)
    assert c.stats().autotune_trials > 0
    c.close()


def test_dfto_rejects_unsupported_options():
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    r, w, _ = _inputs(2, 300, None, 5)
    c = ctx()
    for kw in (dict(node_bounds="sphere_rect"), dict(log_pairs=1)):
        with pytest.raises(g.GaussSumError) as e:
            c.gauss_sum(r, r, w, [0.1], 0.01, method="dfto", **kw)
        assert e.value.status == _lib.GS_EINVAL
    r3, w3, _ = _inputs(3, 300, None, 5)
    with pytest.raises(g.GaussSumError) as e:
        c.gauss_sum(r3, r3, w3, [0.1], 0.01, method="dfto", plimit=7)  # 7^3 terms > 286
    assert e.value.status == _lib.GS_EINVAL


def test_repeated_calls_alternating_inputs():
    """Calls alternate between two inputs of the same size, so every call
    reuses the previous call's buffers: every tree is bit-exact with the
    oracle's tree of its own input and every result equals the first result
    for the same input."""
    from oracle.kdtree import build_kdtree
    D, N, M, leaf = 3, 2500, 900, 32
    data = [_inputs(D, N, M, 300 + k) for k in range(2)]
    hs = np.array([0.02, 0.1, 0.5])
    c = ctx()
    first = {}
    for call, k in enumerate([0, 1, 0, 1, 0, 1]):
        banner("alternating inputs", call, k)
        r, w, q = data[k]
        G = c.gauss_sum(q, r, w, hs, 0.01, leaf_size=leaf, keep_trace=1)
        for which, x, wt in ((0, r, w), (1, q, None)):
            want = build_kdtree(x, wt, leaf)
            gt = c.get_tree(which, D)
            assert np.array_equal(gt["perm"], want.perm), (call, which)
            assert np.array_equal(gt["begin"], want.begin) and np.array_equal(gt["left"], want.left)
            for f in ("lo", "hi", "ctr", "rinf"):
                assert np.array_equal(gt[f], getattr(want, f)), (call, which, f)
            if which == 0:
                assert np.array_equal(gt["W"], want.W) and np.array_equal(gt["wmin"], want.wmin)
        if k in first:
            assert np.array_equal(G, first[k]), call
        else:
            first[k] = G


def test_kernel_timing_modes():
    """kernel_timing=1 times every kernel class, 2 only the base-case tiles
    (the exhaustive tiles on that path), 0 none; other values are rejected."""
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    r, w, _ = _inputs(3, 4000, None, 9)
    c = ctx()
    hs = [0.01, 0.1, 1.0]
    c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32, kernel_timing=1)
    st = c.stats()
    assert st.k_ms[_lib.K_BASE] > 0 and st.k_ms[_lib.K_DECIDE] > 0 and st.k_ms[_lib.K_TREE] > 0
    c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32, kernel_timing=2)
    st = c.stats()
    assert st.k_ms[_lib.K_BASE] > 0 and st.k_launches[_lib.K_BASE] == 1
    assert st.k_ms[_lib.K_DECIDE] == 0 and st.k_ms[_lib.K_TREE] == 0 and st.k_ms[_lib.K_SERIES] == 0
    c.gauss_sum(r, r, w, hs, 0.01, leaf_size=32)
    assert c.stats().k_ms[_lib.K_BASE] == 0
    with pytest.raises(g.GaussSumError) as e:
        c.gauss_sum(r, r, w, hs, 0.01, kernel_timing=3)
    assert e.value.status == _lib.GS_EINVAL


FULL_BLOCK_CASES = [
    # (D, N, log10 h range, seed): 20 bandwidths, leaf 128; the leaf pairs' base
    # cases span 1..16 bandwidths of the first 16-bandwidth block (hundreds of
    # entries with all 16), and 1..4 of the second
    (3, 6000, (-2.0, -0.5), 94),
    (5, 5000, (-1.6, -0.2), 95),
    (8, 4000, (-1.2, 0.0), 96),
]


@pytest.mark.parametrize("case", FULL_BLOCK_CASES, ids=["d%d" % c[0] for c in FULL_BLOCK_CASES])
def test_base_tiles_full_bandwidth_blocks(case):
    """Base entries whose masks fill whole 16-bandwidth blocks (every mask size
    1..16 occurs, on the MFMA and the difference-form paths): decisions
    bit-exact with the oracle, values within the rounding tolerance of its G~,
    Theorem 2 against the exhaustive sum, and a chunked sweep (chunks of 7
    split the first block) gives the same values."""
    D, N, (lo, hi), seed = case
    banner("base tiles full blocks", D)
    r, w, _ = mixture((seed, D), N, D, 6, (0.01, 0.1), weights=(0.5, 1.5))
    hs = np.logspace(lo, hi, 20)
    c = ctx()
    G = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=128, keep_trace=1)
    st = c.stats()
    got = _sorted_trace(c)
    ref = DT.dualtree(r, r, w, hs, 0.01, leaf_size=128, trace=True)
    want = np.array(ref.trace, dtype=np.int64).reshape(-1, 6)
    assert np.array_equal(got, want[np.lexsort(want.T[::-1])])
    assert np.array_equal(c.pair_counts(len(hs)), ref.counts)
    # the base cases of one (Q, R) fill a whole block somewhere
    base = want[want[:, 4] == 4]
    per_block = {}
    for h, _, q, rr, _, _ in base:
        per_block[(q, rr, h // 16)] = per_block.get((q, rr, h // 16), 0) + 1
    assert max(per_block.values()) == 16
    assert 0 < st.base_mfma_pair_evals < st.base_pair_evals, (st.base_mfma_pair_evals, st.base_pair_evals)
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01
    G7 = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=128, h_chunk=7)
    assert (np.abs(G7 - G) / exact).max() <= 1e-12


def test_base_tiles_mfma_and_difference_paths():
    """The base tiles take a bandwidth's squared distances from the MFMA norm
    expansion only where its rounding bound admits it, else from the
    difference form; on a set whose bandwidths run from far below to far above
    the leaf extents both paths carry work, and the values stay within the
    rounding tolerance of the oracle's run with the same decisions.  Each
    bandwidth's path and value do not depend on the other bandwidths of the
    call (a chunked sweep gives the same values)."""
    banner("base tiles mfma paths")
    r, w, _ = mixture((93, 5), 6000, 5, 6, (0.01, 0.1), weights=(0.5, 1.5))
    hs = np.logspace(-3, 0.3, 12)
    c = ctx()
    G = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=128, keep_trace=1)
    st = c.stats()
    assert 0 < st.base_mfma_pair_evals < st.base_pair_evals, (st.base_mfma_pair_evals, st.base_pair_evals)
    ref = DT.dualtree(r, r, w, hs, 0.01, leaf_size=128, trace=True)
    assert np.array_equal(c.pair_counts(len(hs)), ref.counts)
    exact = gauss_sum_exhaustive(r, r, w, hs)
    assert (np.abs(G - ref.G) / exact).max() <= TOL_ROUND
    assert (np.abs(G - exact) / exact).max() <= 0.01
    G1 = c.gauss_sum(r, r, w, hs, 0.01, leaf_size=128, h_chunk=1)
    assert (np.abs(G1 - G) / exact).max() <= 1e-12
