"""Build libmdlts.so for gfx950 in-tree (paper_2310_07607_amd/lib/).

Host C++ (forest, tables, planner) is compiled with g++ and no FP
contraction, the HIP sources with hipcc for gfx950, and both are linked into
one shared library with a plain C ABI (include/mdlts.h).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libmdlts.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
             # packed FP32 instructions are kept out of all device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(LIBDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host_o = os.path.join(LIBDIR, "host.o")
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall", *inc, "-c",
          os.path.join(CSRC, "host.cpp"), "-o", host_o])
    dev_o = os.path.join(LIBDIR, "mdlts.o")
    _run([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, "mdlts.hip"), "-o", dev_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", dev_o, host_o, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
