"""Compile libnqs.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Each source is compiled to an object of its own, in parallel, then the
objects are linked; no device code crosses translation units.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnqs.so")

SOURCES = ["nqs_api.hip", "nqs_kernels.hip", "nqs_join.hip", "nqs_server.hip", "nqs_table.cpp",
           "nqs_host.cpp"]
# the host-only part, buildable without the device code (sanitizer test)
HOST_SOURCES = ["nqs_table.cpp", "nqs_host.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="nqs_build_") as work:
        def compile_one(src):
            obj = os.path.join(work, src + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj

        jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
               "-lpthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
