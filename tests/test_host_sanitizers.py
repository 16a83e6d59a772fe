"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, no GPU calls): lbm_api.hip
is compiled with the sanitizers on its host side only, linked with the kernel objects of the normal build, and
the plain C caller tests/c_abi_check.c (built with the same sanitizers) runs the host-only entry points against
it: workspace layout of one lattice and of an uneven batch, a rejected configuration, the tuning tables and the
kernel names.  The HIP runtime's own allocations at exit are outside this check (leak detection off)."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_host_entry_points_clean_under_sanitizers(tmp_path):
    from paper_1711_10984_amd import build as B
    hipcc, clang = os.path.join(ROCM, "bin", "hipcc"), os.path.join(ROCM, "lib", "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    objs = sorted(glob.glob(os.path.join(B.HERE, "_build", "lbm_*.o")))
    kernels = [o for o in objs if not o.endswith("lbm_api.o")]
    if len(kernels) < 5:
        B.build()
        kernels = [o for o in sorted(glob.glob(os.path.join(B.HERE, "_build", "lbm_*.o"))) if not o.endswith("lbm_api.o")]
    api = tmp_path / "api.o"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-sanitize-recover=undefined", "-g", "-O1"]
    r = subprocess.run([hipcc] + B.hipcc_flags() + ["-ffp-contract=off"] + san +
                       ["-c", os.path.join(B.CSRC, "lbm_api.hip"), "-o", str(api)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lib = tmp_path / "liblbm_san.so"
    r = subprocess.run([clang + "++", "-shared", "-fsanitize=address,undefined", "-o", str(lib)] + kernels +
                       [str(api), "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx",
                        "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = tmp_path / "c_abi_check_san"
    r = subprocess.run([clang, "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", str(exe),
                        str(lib), "-Wl,-rpath," + str(tmp_path)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    got = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    assert got["single_rc"] == "0" and got["batch_rc"] == "0" and got["bad_rc"] == "-1"
    assert got["wave_kernel"] == "k_wave"
