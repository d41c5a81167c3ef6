"""Compile the gfx950 HIP library ``libcrk.so`` in-tree.

hipcc builds the kernels and the C ABI (``csrc/crk.hip``, ``csrc/crk_backward.hip``,
``csrc/gravity.hip``, ``csrc/extras.hip``, ``csrc/step.hip``, ``csrc/devtree.hip``);
g++ builds the
host tree (``csrc/tree.cpp``, OpenMP).  Packed FP32 instructions are switched
off for all device code.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcrk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused within a source expression only: device code shared
    # by several kernels (and by both sides of a pair) rounds the same way in
    # every one of them
    "-ffp-contract=on",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False):
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for name in ("crk", "crk_backward", "gravity", "extras", "step", "devtree"):
        obj = os.path.join(bdir, name + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, name + ".hip"), "-o", obj], verbose)
        objs.append(obj)
    obj_tree = os.path.join(bdir, "tree.o")
    _run(["g++", "-std=c++17", "-O3", "-fopenmp", "-fPIC", "-I", CSRC, "-c",
          os.path.join(CSRC, "tree.cpp"), "-o", obj_tree], verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, obj_tree,
          "-lgomp"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
