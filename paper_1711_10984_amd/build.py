"""Build the HIP library paper_1711_10984_amd/liblbm.so for gfx950 (MI355X).

FP64 kernels and the host side are compiled without floating-point contraction, so that the FP64 path
evaluates every expression in the order written.  The FP32 and FP16-storage kernels contract a * b + c into a
fused multiply-add within a source expression only (-ffp-contract=on), so every instantiation of a kernel (the
stepping and the stage-exporting one) rounds alike.  Packed FP32 instructions are disabled everywhere.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
# (source, floating-point contraction)
SRC = [("lbm_kernels_f64.hip", "off"), ("lbm_kernels_f32.hip", "on"), ("lbm_kernels_f16.hip", "on"),
       ("lbm_adjoint_f64.hip", "off"), ("lbm_adjoint_f32.hip", "on"),
       ("lbm_api.hip", "off")]
LIB = os.path.join(HERE, "liblbm.so")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(os.path.dirname(HERE), "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src, contract in SRC:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc] + hipcc_flags() + ["-ffp-contract=" + contract, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L" + rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
