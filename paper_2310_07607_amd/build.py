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
             # the first 16 dwords of kernel arguments arrive in scalar
             # registers at wave start (no dependent load before the first
             # memory access; 1-3 % per substep launch)
             "-mllvm", "-amdgpu-kernarg-preload-count=16",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _run_all(cmds):
    """Run the compile commands concurrently; raise if any fails."""
    procs = []
    for cmd in cmds:
        print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])


def build(verbose=True):
    os.makedirs(LIBDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host_o = os.path.join(LIBDIR, "host.o")
    dev_o = os.path.join(LIBDIR, "mdlts.o")
    # the substep kernels, one translation unit per polynomial degree
    var_o = [os.path.join(LIBDIR, f"variants_p{p}.o") for p in (1, 2, 3)]
    cmds = [["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall", *inc, "-c",
             os.path.join(CSRC, "host.cpp"), "-o", host_o],
            [HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, "mdlts.hip"), "-o", dev_o]]
    for p, o in zip((1, 2, 3), var_o):
        cmds.append([HIPCC, *HIP_FLAGS, *inc, f"-DMDLTS_DEGREE={p}", "-c", os.path.join(CSRC, "variants.hip"),
                     "-o", o])
    _run_all(cmds)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", dev_o, *var_o, host_o, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
