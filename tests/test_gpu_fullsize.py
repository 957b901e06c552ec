"""Theorem 2 at the full sizes of the benchmark workloads, in the launch
configurations the benchmark uses (autotuned leaf size and method), on
sampled queries that the FP64 exhaustive oracle evaluates one by one.

Samples: random queries plus the extreme points of every coordinate (cluster
edges and isolated points) and the first and last query."""
import numpy as np
import pytest

from oracle.exhaustive import gauss_sum_exhaustive
from paper_1206_6857_amd.datagen import workload
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _sample(q, n, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(q.shape[0], n, replace=False).tolist())
    for d in range(q.shape[1]):
        idx.add(int(np.argmin(q[:, d])))
        idx.add(int(np.argmax(q[:, d])))
    idx.update((0, q.shape[0] - 1))
    return np.array(sorted(idx))


def _check(cfg, D=None, n_sample=200, **opts):
    import torch
    import paper_1206_6857_amd as g
    wl = workload(cfg, D=D)
    banner("fullsize", wl.name, opts)
    dev = torch.device("cuda:0")
    rd = torch.from_numpy(wl.refs).to(dev)
    qd = rd if wl.monochromatic else torch.from_numpy(wl.queries).to(dev)
    wd = torch.from_numpy(wl.weights).to(dev)
    hd = torch.from_numpy(wl.bandwidths).to(dev)
    c = g.Context(0)
    G = c.gauss_sum(qd, rd, wd, hd, wl.eps, **opts).cpu().numpy()
    st = c.stats()
    idx = _sample(wl.queries, n_sample, cfg)
    exact = gauss_sum_exhaustive(wl.queries[idx], wl.refs, wl.weights, wl.bandwidths)
    ok = exact > 1e-290
    rel = np.abs(G[:, idx][ok] - exact[ok]) / exact[ok]
    c.close()
    assert rel.max() <= wl.eps, (wl.name, opts, rel.max(), st.tuned_leaf_size, st.tuned_method)
    return st


def test_fullsize_d2_all_queries():
    import paper_1206_6857_amd as g
    wl = workload(0)
    banner("fullsize", wl.name)
    c = g.Context(0)
    for opts in (dict(autotune=1), dict(leaf_size=64), dict(leaf_size=128)):
        G = c.gauss_sum(wl.refs, wl.refs, wl.weights, wl.bandwidths, wl.eps, **opts)
        exact = gauss_sum_exhaustive(wl.refs, wl.refs, wl.weights, wl.bandwidths)
        assert (np.abs(G - exact) / exact).max() <= wl.eps, opts
    c.close()


@pytest.mark.parametrize("opts", [dict(autotune=1), dict(leaf_size=64), dict(leaf_size=128),
                                  dict(leaf_size=256), dict(autotune=1, method="dualtree", h_chunk=3),
                                  dict(leaf_size=256, method="dfto"), dict(leaf_size=256, method="dfdo")],
                         ids=["autotune", "leaf64", "leaf128", "leaf256", "chunked", "dfto", "dfdo"])
def test_fullsize_d3_bench_workload(opts):
    _check(1, n_sample=300, **opts)


def test_fullsize_d5_32h():
    _check(2, n_sample=60, autotune=1)


@pytest.mark.parametrize("opts", [dict(autotune=1), dict(leaf_size=64)], ids=["autotune", "leaf64"])
def test_fullsize_d16_bichromatic(opts):
    _check(3, n_sample=150, **opts)


@pytest.mark.parametrize("D", [2, 3])
def test_fullsize_million_points_64h(D):
    _check(4, D=D, n_sample=24, leaf_size=128)
