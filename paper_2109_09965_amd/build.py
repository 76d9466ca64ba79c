"""Build libcgks.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcgks.so")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             # no packed FP32 instructions in generated code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    obj_prep = os.path.join(CSRC, "mesh_prep.o")
    obj_api = os.path.join(CSRC, "cgks_api.o")
    cmds = [
        ["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-I", os.path.join(ROOT, "include"), "-c",
         os.path.join(CSRC, "mesh_prep.cpp"), "-o", obj_prep],
        ["hipcc"] + HIP_FLAGS + ["-c", os.path.join(CSRC, "cgks_api.hip"), "-o", obj_api],
        ["hipcc", "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", obj_api, obj_prep, "-o", LIB + ".tmp"],
    ]
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.check_call(c)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
