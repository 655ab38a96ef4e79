"""Build the HIP libraries (gfx950) in-tree with hipcc: libck.so (the tables)
and libck_ceilings.so (the random-access ceilings the benchmark measures)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libck.so")
CEIL_LIB = os.path.join(HERE, "libck_ceilings.so")
SOURCES = ["ck_kernels.hip", "ck_api.hip"]
CEIL_SOURCES = ["ceilings.hip"]
HEADERS = ["ck_internal.h", os.path.join("..", "..", "include", "ck.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CK_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off for all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def _link(sources, lib, verbose):
    objs = []
    for src in sources:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


def build(verbose: bool = False) -> str:
    _link(CEIL_SOURCES, CEIL_LIB, verbose)
    return _link(SOURCES, LIB, verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
