"""Builds libbc.so (HIP kernels + host library) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbc.so")
SOURCES = ["bc_kernels.hip", "bc_host.cpp", "bc_server.cpp", "bc_server_hip.cpp"]
# the roofline denominators' microbenchmarks, a library of their own
PEAKS_LIB = os.path.join(HERE, "libbc_peaks.so")
PEAKS_SOURCES = ["bc_peaks.hip"]

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    _build_lib(SOURCES, LIB, verbose)
    _build_lib(PEAKS_SOURCES, PEAKS_LIB, verbose)
    return LIB


def _build_lib(sources, lib, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src in sources:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
               "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
