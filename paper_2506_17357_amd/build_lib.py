"""Build libtga.so (the C-ABI device library) with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "api.hip")
DEPS = [os.path.join(HERE, "csrc", f) for f in ("api.hip", "kernels.hip", "tga_internal.h")]
LIB = os.path.join(HERE, "libtga.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # keep the device code free of packed fp32 instructions (the device pass
    # honours the feature; only hipcc's host pass warns that it does not know it)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def ensure_built(verbose: bool = False) -> str:
    """Build when the library is missing or older than any of its sources."""
    if is_stale():
        build(verbose=verbose)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS + [os.path.join(ROOT, "include", "tga.h")])


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
