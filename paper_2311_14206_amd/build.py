"""Build libsdr.so (HIP for gfx950) in place.

    python -m paper_2311_14206_amd.build

Compiles the HIP kernels and the C++ host driver with hipcc, and the
host-only small-dense code with g++, into ``paper_2311_14206_amd/libsdr.so``.  Packed FP32 instructions are disabled
(``-packed-fp32-ops``); every source is rebuilt on each call.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdr.so")

SOURCES = ["sdr_kernels.hip", "sdr_solver.cpp", "dense.cpp", "sdr_noalloc.hip"]
HOST_ONLY = {"dense.cpp"}

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src in SOURCES:  # the sources compile in parallel
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        if src in HOST_ONLY:
            # host-only small-dense code: g++ (it vectorises this code's loops
            # markedly better than the HIP toolchain's host compiler), AVX2/FMA,
            # inline complex products
            cmd = [os.environ.get("CXX", "g++"), "-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3",
                   "-fcx-limited-range", "-fopenmp-simd", "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
