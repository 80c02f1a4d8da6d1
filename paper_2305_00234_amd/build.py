"""Build the gfx950 HIP library (libccprfdtd.so) in-tree with hipcc.

Usage: python -m paper_2305_00234_amd.build  (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libccprfdtd.so")
ARCH = os.environ.get("CCPR_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ccpr_kernels.hip", "ccpr_solver.cpp", "ccpr_engine.cpp", "ccpr_filter.hip"]

# -packed-fp32-ops: no v_pk_*_f32 from the compiler (they are avoided on this
# hardware); -ffp-contract=fast lets hipcc fuse a*b+c into FMA.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", "-c", "-x", "hip", path, "-o", obj] + HIPFLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
