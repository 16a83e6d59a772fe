"""Build the HIP library paper_1711_10984_amd/liblbm.so for gfx950 (MI355X).

FMA contraction is off so that the FP64 path evaluates every expression in the order written;
packed FP32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", "lbm_kernels.hip"), os.path.join(HERE, "csrc", "lbm_api.hip")]
LIB = os.path.join(HERE, "liblbm.so")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(os.path.dirname(HERE), "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + hipcc_flags() + ["-shared", "-o", tmp] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
