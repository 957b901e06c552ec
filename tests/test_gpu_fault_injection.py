"""Error paths of the C ABI under injected allocation failures.

gs_options.debug_fail_alloc = k makes the k-th device workspace request of a
call fail as an out-of-memory would.  For every k up to the number of requests
a clean call makes (gs_stats.workspace_requests), the call either returns
GS_ENOMEM with a message, or absorbs the failure by traversing fewer
bandwidths at a time (then it makes the same decisions and its values agree to
rounding); and the next clean call on the same context returns exactly the
clean result.  The failure is forced from the host: no kernel sees anything
unusual.
"""
import numpy as np
import pytest

from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner, ctx

pytestmark = pytest.mark.gpu

HS = np.array([0.01, 0.05, 0.3])
EPS = 0.01


def _inputs(device):
    r, w, q = mixture((77, 2), 1500, 2, 4, (0.02, 0.1), weights=(0.5, 1.5), m_queries=600)
    if device:
        import torch
        dev = torch.device("cuda:0")
        return (torch.from_numpy(r).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(q).to(dev),
                torch.from_numpy(HS).to(dev))
    return r, w, q, HS


def _as_np(G):
    return G.cpu().numpy() if hasattr(G, "cpu") else np.asarray(G)


@pytest.mark.parametrize("method,device", [("dito", False), ("dito", True), ("dfto", False),
                                           ("exhaustive", False)])
def test_every_injected_failure_leaves_the_context_usable(method, device):
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    banner("fault injection", method, "device" if device else "host")
    r, w, q, hs = _inputs(device)
    c = ctx()
    opts = dict(method=method, leaf_size=32)
    G0 = _as_np(c.gauss_sum(q, r, w, hs, EPS, **opts))
    n = c.stats().workspace_requests
    assert n >= 5
    failed = absorbed = 0
    for k in range(1, n + 1):
        try:
            G = _as_np(c.gauss_sum(q, r, w, hs, EPS, debug_fail_alloc=k, **opts))
        except g.GaussSumError as e:
            assert e.status == _lib.GS_ENOMEM, (k, str(e))
            assert "allocation failed" in str(e), (k, str(e))
            failed += 1
        else:
            # a failed allocation inside the traversal is retried with fewer
            # bandwidths per chunk: same decisions, rounding-level differences
            assert c.stats().h_chunks > 1, k
            assert (np.abs(G - G0) / G0).max() <= 1e-12, k
            absorbed += 1
        G1 = _as_np(c.gauss_sum(q, r, w, hs, EPS, **opts))
        assert np.array_equal(G1, G0), k
        assert c.stats().workspace_requests == n, k
    assert failed + absorbed == n and failed >= 1
    # beyond the last request nothing fails
    G = _as_np(c.gauss_sum(q, r, w, hs, EPS, debug_fail_alloc=n + 1, **opts))
    assert np.array_equal(G, G0)


def test_injected_failures_with_the_learned_policy():
    """The learned policy's inference buffers are workspace requests too.  A
    context of its own holds a seeded network (any parameters: the policy only
    chooses among actions the bound admits)."""
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    banner("fault injection", "learned policy")
    rng = np.random.default_rng(31)
    params = np.concatenate([rng.normal(0, 0.35, _lib.POLICY_PARAMS), rng.normal(0, 1, 16),
                             rng.uniform(0.5, 2.0, 16), [3.0, 2.5]]).astype(np.float32)
    r, w, q, hs = _inputs(False)
    c = g.Context(0)
    try:
        c.policy_set_params(params)
        opts = dict(policy="learned", leaf_size=32)
        G0 = c.gauss_sum(q, r, w, hs, EPS, **opts)
        assert c.stats().policy_calls > 0
        n = c.stats().workspace_requests
        failed = 0
        for k in range(1, n + 1):
            try:
                G = c.gauss_sum(q, r, w, hs, EPS, debug_fail_alloc=k, **opts)
            except g.GaussSumError as e:
                assert e.status == _lib.GS_ENOMEM, (k, str(e))
                failed += 1
            else:
                assert c.stats().h_chunks > 1, k
                assert (np.abs(G - G0) / G0).max() <= 1e-12, k
            assert np.array_equal(c.gauss_sum(q, r, w, hs, EPS, **opts), G0), k
        assert failed >= 1
    finally:
        c.close()


def test_injected_failures_in_lscv():
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    banner("fault injection", "lscv")
    x, _, _ = mixture((78, 2), 1200, 2, 4, (0.02, 0.1))
    hs = np.array([0.01, 0.03, 0.1])
    c = ctx()
    s0, b0 = c.lscv(x, hs, 0.01)
    n = c.stats().workspace_requests
    assert n >= 5
    for k in sorted({1, 2, n // 3, n // 2, n - 1, n}):
        try:
            c.lscv(x, hs, 0.01, debug_fail_alloc=k)
        except g.GaussSumError as e:
            assert e.status == _lib.GS_ENOMEM, (k, str(e))
        s1, b1 = c.lscv(x, hs, 0.01)
        assert np.array_equal(s1, s0) and np.array_equal(b1, b0), k


def test_negative_debug_fail_alloc_is_rejected():
    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    banner("fault injection", "rejects")
    r, w, q, hs = _inputs(False)
    c = ctx()
    with pytest.raises(g.GaussSumError) as ei:
        c.gauss_sum(q, r, w, hs, EPS, debug_fail_alloc=-1)
    assert ei.value.status == _lib.GS_EINVAL
