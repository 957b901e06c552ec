"""The C ABI library loads and exports every function include/gausssum.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1206_6857_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gausssum.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"^#.*$", "", src, flags=re.M)  # preprocessor lines
    return sorted(set(re.findall(r"\b(\w+)\s*\([^;{]*\)\s*;", src)) - {"if", "sizeof"})


def test_header_declarations_match_binding_list():
    assert _declared() == sorted(_lib.EXPORTED)


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_default_options():
    import paper_1206_6857_amd as g
    o = g.gs_default_options()
    assert o.struct_size == ctypes.sizeof(_lib.GsOptions)
    assert (o.leaf_size, o.plimit, o.method, o.policy, o.monochromatic, o.blocking) == (64, 0, 0, 0, -1, 1)
    assert abs(o.eps_round_share - 0.1) < 1e-15
