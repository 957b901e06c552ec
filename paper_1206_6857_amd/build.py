"""Compile the HIP library libgausssum.so for gfx950, in-tree.

Every translation unit is compiled with hipcc for gfx950 only.  Packed FP32
instructions are disabled for all device code.  Units whose double-precision
arithmetic decides pruning (the traversal, the tree builder and the host
orchestration) are compiled without floating-point contraction, so that every
addition and multiplication is a separately rounded IEEE operation.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgausssum.so")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-Wno-unused-command-line-argument"]
NO_CONTRACT = ["-ffp-contract=off"]

# (source, extra flags)
SOURCES = [
    ("k_stage.hip", []),
    ("k_exhaustive.hip", []),
    ("k_tree.hip", NO_CONTRACT),
    ("k_decide.hip", NO_CONTRACT),
    ("k_series.hip", []),
    ("k_series_fast.hip", []),
    ("k_base.hip", []),
    ("k_policy.hip", []),
    ("k_lscv.hip", []),
    ("policy.cpp", []),
    ("noalloc.hip", []),
    ("dualtree.hip", NO_CONTRACT),
    ("capi.cpp", NO_CONTRACT),
]


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = jobs or min(8, os.cpu_count() or 4)

    def compile_one(item):
        src, extra = item
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compilation of %s failed:\n%s%s" % (src, r.stdout, r.stderr))
        return obj

    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
