"""Build libpa.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1809_07592_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpa.so")

SOURCES = ["pa_kernels.hip", "pa_plan.cpp", "pa_api.cpp", "pa_serve.cpp", "pa_tune.cpp", "pa_graph.cpp", "pa_fft.hip", "pa_fft_host.cpp", "pa_probe.hip", "pa_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Always recompiles libpa.so (atomically replaces the old file): every
    source to an object in parallel, then one link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    tmp = LIB + ".tmp%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="pa_build_") as objdir:
        def compile_one(src):
            obj = os.path.join(objdir, src + ".o")
            cmd = [hipcc()] + compile_flags + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj
        workers = max(1, min(len(SOURCES), os.cpu_count() or 4, 16))
        with ThreadPoolExecutor(workers) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
