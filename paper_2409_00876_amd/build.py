"""Builds libpgsgd.so, the HIP library for gfx950, in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB_PATH = os.path.join(HERE, "libpgsgd.so")
SOURCES = ["capi.hip", "layout_kernels.hip", "batch_kernels.hip", "local_kernels.hip", "stress_kernels.hip", "gfa.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # packed FP32 instructions stay off: plain scalar FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-o", LIB_PATH + ".tmp",
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
