"""gs_exhaustive_noalloc, the exhaustive sum whose intermediates live in a
fixed device array of the library, against gauss_sum's exhaustive path (the
allocating entry point running the same kernels): bit-identical outputs on two
calls in a row, the second on a smaller input, so that nothing the first call
left in the array leaks into the second.  Also its error paths."""
import os
import re

import numpy as np
import pytest

from paper_1206_6857_amd import _lib
from paper_1206_6857_amd.datagen import mixture
from tests.gpu_util import banner

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_noalloc_source_allocates_nothing():
    """The entry point's file calls no allocator and no workspace request."""
    src = open(os.path.join(ROOT, "paper_1206_6857_amd", "csrc", "noalloc.hip")).read()
    code = re.sub(r"//.*", "", src)
    for name in ("hipMalloc", "hipFree", "hipHostMalloc", "hipMallocAsync", "hipExtMalloc",
                 "ws.get", "WS(", "hipMemset"):
        assert name not in code, name


def _inputs(seed, D, N, M, mono):
    r, w, _ = mixture((seed, D), N, D, 4, 0.05)
    q = r if mono else mixture((seed + 1, D), M, D, 4, 0.05)[0]
    return q, r, w


@pytest.mark.gpu
def test_noalloc_matches_allocating_entry_point_twice():
    import torch
    import paper_1206_6857_amd as g
    dev = torch.device("cuda:0")
    c = g.Context(0)
    # (D, N, M, bandwidths, monochromatic): the second call is smaller in every size
    cases = [(3, 6000, 4100, np.logspace(-3, 0, 9), False),
             (2, 900, 900, np.array([0.002, 0.05, 0.7]), True)]
    for D, N, M, hs, mono in cases:
        banner("noalloc", D, N, M, len(hs), "mono" if mono else "bichro")
        q, r, w = _inputs(7 + D, D, N, M, mono)
        rd = torch.from_numpy(r).to(dev)
        qd = rd if mono else torch.from_numpy(q).to(dev)
        wd = torch.from_numpy(w).to(dev)
        out = torch.full((len(hs), qd.shape[0]), float("nan"), dtype=torch.float64, device=dev)
        c.exhaustive_noalloc(qd, rd, wd, hs, out)
        want = c.gauss_sum(qd, rd, wd, torch.from_numpy(hs).to(dev), 0.01, method="exhaustive")
        torch.cuda.synchronize()
        assert torch.equal(out, want), (D, N, M)
    c.close()


@pytest.mark.gpu
def test_noalloc_error_paths():
    import torch
    import paper_1206_6857_amd as g
    dev = torch.device("cuda:0")
    banner("noalloc errors")
    c = g.Context(0)
    q, r, w = _inputs(3, 2, 500, 300, False)
    qd, rd, wd = (torch.from_numpy(a).to(dev) for a in (q, r, w))
    hs = np.array([0.1])
    out = torch.empty((1, 300), dtype=torch.float64, device=dev)
    # a host array where device memory is required
    with pytest.raises(g.GaussSumError) as e:
        c.exhaustive_noalloc(q, rd, wd, hs, out)
    assert e.value.status == _lib.GS_EINVAL
    # invalid values, found on the device
    bad = qd.clone()
    bad[17, 1] = float("nan")
    with pytest.raises(g.GaussSumError) as e:
        c.exhaustive_noalloc(bad, rd, wd, hs, out)
    assert e.value.status == _lib.GS_EINVAL
    wneg = wd.clone()
    wneg[5] = -1.0
    with pytest.raises(g.GaussSumError) as e:
        c.exhaustive_noalloc(qd, rd, wneg, hs, out)
    assert e.value.status == _lib.GS_EINVAL
    with pytest.raises(g.GaussSumError) as e:
        c.exhaustive_noalloc(qd, rd, wd, np.array([0.1, 0.0]), torch.empty((2, 300), dtype=torch.float64, device=dev))
    assert e.value.status == _lib.GS_EINVAL
    # more scratch than the fixed array holds: 10^6 references, 10^5 queries, 64 bandwidths
    big_r = torch.rand((1000000, 3), dtype=torch.float64, device=dev)
    big_w = torch.ones(1000000, dtype=torch.float64, device=dev)
    big_q = torch.rand((100000, 3), dtype=torch.float64, device=dev)
    big_out = torch.empty((64, 100000), dtype=torch.float64, device=dev)
    with pytest.raises(g.GaussSumError) as e:
        c.exhaustive_noalloc(big_q, big_r, big_w, np.logspace(-3, 0, 64), big_out)
    assert e.value.status == _lib.GS_EOVERFLOW
    assert "scratch" in str(e.value)
    del big_r, big_w, big_q, big_out
    # the context and the array still serve a valid call
    c.exhaustive_noalloc(qd, rd, wd, hs, out)
    want = c.gauss_sum(qd, rd, wd, torch.from_numpy(hs).to(dev), 0.01, method="exhaustive")
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    c.close()
