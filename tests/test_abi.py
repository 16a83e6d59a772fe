"""The C ABI without a GPU: the library loads, exports every function include/lbm.h declares, the binding's
constants match the header, and configuration checks (host-only) reject bad input with a message."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _lbm():
    from paper_1711_10984_amd import lbm
    return lbm


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(lbm_[a-z_]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lbm = _lbm()
    lib = lbm.load_library()
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(lbm.EXPORTED) == names


def test_header_constants_match_binding():
    lbm = _lbm()
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(LBM_[A-Z0-9_]+)\s+(-?\d+)", text))
    for k, v in defs.items():
        assert getattr(lbm, k) == int(v), k


def test_struct_layouts():
    lbm = _lbm()
    assert C.sizeof(lbm.lbm_config) == 6 * 4 + 12 * 8
    assert C.sizeof(lbm.lbm_droplet) == 6 * 8 + 8
    assert C.sizeof(lbm.lbm_obs) == 8 + 5 * 8 + 8


def _cfg(**kw):
    lbm = _lbm()
    p = dict(nx=64, ny=48)
    p.update(kw)
    return lbm.make_config(p, kw.pop("precision", 0) if "precision" in kw else 0)


def test_workspace_bytes_scales_with_lattice():
    lbm = _lbm()
    b1 = lbm.lbm_workspace_bytes([_cfg(nx=256, ny=256)], [1])
    b2 = lbm.lbm_workspace_bytes([_cfg(nx=512, ny=512)], [1])
    # 25 planes of 8 bytes per node dominate
    assert 25 * 8 * 256 * 256 <= b1 < 2 * 25 * 8 * 256 * 256
    assert 3.5 < b2 / b1 < 4.5
    # FP32 halves the field pool (the fixed-size stage-export scratch aside)
    b64 = lbm.lbm_workspace_bytes([lbm.make_config(dict(nx=2048, ny=2048), lbm.LBM_FP64)], [64])
    b32 = lbm.lbm_workspace_bytes([lbm.make_config(dict(nx=2048, ny=2048), lbm.LBM_FP32)], [64])
    assert 0.5 < b32 / b64 < 0.6
    # FP16 population storage: 9 x 2 B + 7 x 4 B per node in the pool instead of 25 x 4 B
    b16 = lbm.lbm_workspace_bytes([lbm.make_config(dict(nx=2048, ny=2048), lbm.LBM_FP16)], [64])
    assert 0.6 < b16 / b32 < 0.75
    # a batch needs the sum
    bb = lbm.lbm_workspace_bytes([_cfg(nx=256, ny=256), _cfg(nx=100, ny=37)], [2, 0])
    assert bb > b1


@pytest.mark.parametrize("bad,msg", [
    (dict(nx=2), "nx and ny"),
    (dict(tau=0.5), "tau"),
    (dict(b=0.0), "b must be positive"),
    (dict(advection=7), "advection"),
    (dict(D=float("nan")), "finite"),
])
def test_invalid_configs_rejected(bad, msg):
    lbm = _lbm()
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_workspace_bytes([_cfg(**bad)], [0])
    assert ei.value.code == lbm.LBM_E_INVAL
    assert msg in str(ei.value)


def test_mixed_precision_and_droplet_limits_rejected():
    lbm = _lbm()
    a = lbm.make_config(dict(nx=16, ny=16), lbm.LBM_FP64)
    b = lbm.make_config(dict(nx=16, ny=16), lbm.LBM_FP32)
    with pytest.raises(lbm.LBMError, match="same precision"):
        lbm.lbm_workspace_bytes([a, b], [0, 0])
    with pytest.raises(lbm.LBMError, match="droplet count"):
        lbm.lbm_workspace_bytes([a], [lbm.LBM_MAXDROP + 1])


def test_init_rejects_bad_workspace_before_any_device_call():
    lbm = _lbm()
    cfg = _cfg(nx=16, ny=16)
    import numpy as np
    z = np.zeros(256)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_init_batch([cfg], 0, 1 << 20, 0, z, z, None, [0], [])
    assert ei.value.code == lbm.LBM_E_INVAL
    with pytest.raises(lbm.LBMError, match="256-byte aligned"):
        lbm.lbm_init_batch([cfg], 0x1008, 1 << 20, 0, z, z, None, [0], [])
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_init_batch([cfg], 0x100000, 16, 0, z, z, None, [0], [])
    assert ei.value.code == lbm.LBM_E_NOMEM


def test_kernel_names():
    lbm = _lbm()
    assert [lbm.lbm_kernel_name(lbm.LBM_PATH_SPLIT, i) for i in range(3)] == ["k_lb", "k_fd", "k_reduce"]
    assert [lbm.lbm_kernel_name(lbm.LBM_PATH_FUSED, i) for i in range(3)] == ["k_step", "k_reduce", ""]


def test_unknown_precision_rejected():
    lbm = _lbm()
    with pytest.raises(lbm.LBMError, match="precision must be"):
        lbm.lbm_workspace_bytes([lbm.make_config(dict(nx=16, ny=16), 3)], [0])


def test_header_compiles_as_c99_and_a_c_caller_agrees_with_the_binding(tmp_path):
    """include/lbm.h is a C header: a C99 program (pedantic, warnings as errors) builds against it, links the
    library and gets the same answers from the host-only entry points as the Python binding."""
    import shutil
    import subprocess
    lbm = _lbm()
    lib = lbm.load_library()
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "c_abi_check"
    libdir = os.path.dirname(lbm.LIB_PATH)
    cmd = [gcc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", str(exe), lbm.LIB_PATH,
           "-Wl,-rpath," + libdir]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.split(" ", 1) for line in out.strip().splitlines())
    cfgs = [lbm.make_config(dict(nx=256, ny=256, tau=1.0, a=-0.001, b=0.001, B0=0.006, B1=-0.05, D=0.1,
                                 Gamma=1.0, t_star=2.0e6), lbm.LBM_FP64),
            lbm.make_config(dict(nx=100, ny=37, tau=1.0, a=-0.001, b=0.001, B0=0.006, B1=-0.05, D=0.1,
                                 Gamma=1.0, t_star=2.0e6), lbm.LBM_FP64)]
    assert int(got["single_rc"]) == 0 and int(got["batch_rc"]) == 0
    assert int(got["single_bytes"]) == lbm.lbm_workspace_bytes(cfgs[:1], [1])
    assert int(got["batch_bytes"]) == lbm.lbm_workspace_bytes(cfgs, [1, 0])
    assert int(got["bad_rc"]) == lbm.LBM_E_INVAL and got["bad_has_message"] == "1"
    assert int(got["sizeof_config"]) == C.sizeof(lbm.lbm_config)
    assert int(got["sizeof_droplet"]) == C.sizeof(lbm.lbm_droplet)
    assert int(got["sizeof_obs"]) == C.sizeof(lbm.lbm_obs)
    assert int(got["first_tune_row"]) == lbm.lbm_tune_rows()[0]
    assert got["wave_kernel"] == lbm.lbm_kernel_name(lbm.LBM_PATH_WAVE, 0)
    del lib
