"""Helpers for GPU tests: a shared context, and a flushed banner naming each case."""
import sys

import pytest

_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        import torch
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        import paper_1206_6857_amd as g
        _ctx = g.Context(0)
    return _ctx


def banner(*parts):
    print("[case]", *parts, file=sys.stderr, flush=True)
