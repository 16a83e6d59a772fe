"""Thin Python binding of the C ABI in include/lbm.h (liblbm.so, HIP for gfx950).

Only argument marshalling lives here: every step of the timestep runs in the library's kernels.
PyTorch provides the device workspace and the HIP stream.  Functions keep the C names
(``lbm_init_batch``, ``lbm_step``, ``lbm_fields``, ...); :class:`Sim` bundles them for one batch.
There is no fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY selects another build of the same sources (e.g. a tuning variant); default: the in-tree build.
LIB_PATH = os.environ.get("LBM_LIBRARY", os.path.join(_HERE, "liblbm.so"))

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_UNSTABLE, LBM_E_STATE = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32, LBM_FP16 = 0, 1, 2
LBM_WALLS_NONE, LBM_WALLS_Y = 0, 1
LBM_ADV_PAPER, LBM_ADV_FLUX = 0, 1
LBM_PATH_FUSED, LBM_PATH_SPLIT, LBM_PATH_WAVE = 0, 1, 2
LBM_MAXDROP = 256
LBM_NSTAGE = 22
STAGES = ["mu", "X", "Fx", "Fy", "n", "ux", "uy", "phi_h", "c_h", "M", "X_h", "phi_new", "c_new"] + [
    f"fstar{i}" for i in range(9)
]
EXPORTED = ["lbm_workspace_bytes", "lbm_init_batch", "lbm_init", "lbm_step", "lbm_set_graph", "lbm_sync",
            "lbm_get_step", "lbm_fields", "lbm_observables", "lbm_droplets", "lbm_debug_stage",
            "lbm_time_kernels", "lbm_time_launches", "lbm_kernel_name", "lbm_set_path", "lbm_get_path", "lbm_set_seg_rows",
            "lbm_get_seg_rows", "lbm_set_strip_width", "lbm_get_strip_width", "lbm_tune_rows", "lbm_tune_widths",
            "lbm_autotune", "lbm_step_noalloc", "lbm_adjoint_bytes", "lbm_adjoint_forward",
            "lbm_adjoint_backward", "lbm_destroy", "lbm_last_error"]
LBM_SEG_ROWS_MIN, LBM_SEG_ROWS_MAX, LBM_TUNE_NROWS = 16, 4096, 16
LBM_STRIP_W_MIN, LBM_STRIP_W_MAX, LBM_TUNE_NWIDTHS = 32, 54, 1
LBM_NOALLOC_SCRATCH_BYTES = 16 << 20
PATH_NAMES = {LBM_PATH_FUSED: "fused", LBM_PATH_SPLIT: "split", LBM_PATH_WAVE: "wave"}


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32), ("advection", C.c_int32),
                ("walls", C.c_int32), ("reserved", C.c_int32), ("tau", C.c_double), ("n0", C.c_double),
                ("a", C.c_double), ("b", C.c_double),
                ("B0", C.c_double), ("B1", C.c_double), ("D", C.c_double), ("Gamma", C.c_double),
                ("gamma", C.c_double), ("A0", C.c_double), ("t_star", C.c_double), ("c0", C.c_double)]


class lbm_droplet(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("R", C.c_double), ("Rs", C.c_double),
                ("ex", C.c_double), ("ey", C.c_double), ("active", C.c_int32), ("reserved", C.c_int32)]


class lbm_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("sum_phi", C.c_double), ("sum_c", C.c_double),
                ("min_B", C.c_double), ("max_u", C.c_double), ("nonfinite", C.c_int32), ("ndrop", C.c_int32)]


_lib = None


def load_library(path: Optional[str] = None):
    """Load liblbm.so (built by paper_1711_10984_amd/build.py).  Raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    try:
        # torch first: its HIP runtime (same soname) is then the one the library binds to.  Loaded the other way
        # round, the process would hold two HIP runtimes and torch's device memory would be foreign to ours.
        import torch  # noqa: F401
    except ImportError:
        pass
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    lib = C.CDLL(p)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    lib.lbm_workspace_bytes.argtypes = [C.c_int32, C.POINTER(lbm_config), C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
    lib.lbm_init_batch.argtypes = [C.c_int32, C.POINTER(lbm_config), vp, C.c_size_t, vp, dp, dp, dp,
                                   C.POINTER(C.c_int32), C.POINTER(lbm_droplet), C.c_int64, C.POINTER(vp)]
    lib.lbm_init.argtypes = [C.POINTER(lbm_config), vp, C.c_size_t, vp, dp, dp, dp, C.c_int32,
                             C.POINTER(lbm_droplet), C.c_int64, C.POINTER(vp)]
    lib.lbm_step.argtypes = [vp, C.c_int64]
    lib.lbm_set_graph.argtypes = [vp, C.c_int32]
    lib.lbm_sync.argtypes = [vp]
    lib.lbm_get_step.argtypes = [vp]
    lib.lbm_get_step.restype = C.c_int64
    lib.lbm_fields.argtypes = [vp, C.c_int32, dp, dp, dp, dp, dp, dp]
    lib.lbm_observables.argtypes = [vp, C.c_int32, C.POINTER(lbm_obs), dp]
    lib.lbm_droplets.argtypes = [vp, C.c_int32, C.POINTER(lbm_droplet)]
    lib.lbm_debug_stage.argtypes = [vp, C.c_int32, dp]
    lib.lbm_time_kernels.argtypes = [vp, C.c_int64, dp]
    lib.lbm_time_launches.argtypes = [vp, C.c_int32, dp]
    lib.lbm_kernel_name.argtypes = [C.c_int32, C.c_int32]
    lib.lbm_kernel_name.restype = C.c_char_p
    lib.lbm_set_path.argtypes = [vp, C.c_int32]
    lib.lbm_get_path.argtypes = [vp]
    lib.lbm_get_path.restype = C.c_int32
    lib.lbm_set_seg_rows.argtypes = [vp, C.c_int32]
    lib.lbm_get_seg_rows.argtypes = [vp]
    lib.lbm_get_seg_rows.restype = C.c_int32
    lib.lbm_set_strip_width.argtypes = [vp, C.c_int32]
    lib.lbm_get_strip_width.argtypes = [vp]
    lib.lbm_get_strip_width.restype = C.c_int32
    lib.lbm_tune_rows.argtypes = []
    lib.lbm_tune_rows.restype = C.POINTER(C.c_int32)
    lib.lbm_tune_widths.argtypes = []
    lib.lbm_tune_widths.restype = C.POINTER(C.c_int32)
    lib.lbm_autotune.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
    lib.lbm_step_noalloc.argtypes = [C.POINTER(lbm_config), vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.c_int32,
                                     vp, C.c_int64, C.c_int64]
    lib.lbm_adjoint_bytes.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    lib.lbm_adjoint_forward.argtypes = [vp, vp, C.c_size_t, C.c_int32, C.c_int64, C.c_int32, dp]
    lib.lbm_adjoint_backward.argtypes = [vp, vp, C.c_size_t, dp, dp]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.restype = C.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(rc: int, allow=()) -> int:
    if rc != LBM_OK and rc not in allow:
        raise LBMError(rc, lbm_last_error())
    return rc


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(p: dict, precision: int = LBM_FP64) -> lbm_config:
    """lbm_config from a parameter dict (keys as in include/lbm.h; nx, ny required)."""
    return lbm_config(nx=int(p["nx"]), ny=int(p["ny"]), precision=int(precision),
                      advection=int(p.get("advection", 0)), walls=int(p.get("walls", 0)), reserved=0,
                      tau=p.get("tau", 1.0), n0=p.get("n0", 1.0),
                      a=p.get("a", -0.001), b=p.get("b", 0.001), B0=p.get("B0", 0.006), B1=p.get("B1", -0.05),
                      D=p.get("D", 0.1), Gamma=p.get("Gamma", 1.0), gamma=p.get("gamma", 0.0),
                      A0=p.get("A0", 0.0), t_star=p.get("t_star", 2.0e6), c0=p.get("c0", 0.0))


def make_droplet(d: dict) -> lbm_droplet:
    return lbm_droplet(x=d["x"], y=d["y"], R=d["R"], Rs=d.get("Rs", 0.0), ex=d.get("ex", 1.0), ey=d.get("ey", 0.0),
                       active=int(d.get("active", 0)), reserved=0)


# ---- functions with the C names (argument marshalling only) ----------------------------------------
def lbm_last_error() -> str:
    return load_library().lbm_last_error().decode()


def lbm_workspace_bytes(cfgs: Sequence[lbm_config], ndrop: Sequence[int]) -> int:
    arr = (lbm_config * len(cfgs))(*cfgs)
    nd = (C.c_int32 * len(ndrop))(*ndrop)
    out = C.c_size_t(0)
    _check(load_library().lbm_workspace_bytes(len(cfgs), arr, nd, C.byref(out)))
    return int(out.value)


def lbm_init_batch(cfgs: Sequence[lbm_config], workspace_ptr: int, workspace_bytes: int, stream_ptr: int,
                   phi0: np.ndarray, c0: np.ndarray, f_pre: Optional[np.ndarray], ndrop: Sequence[int],
                   drops: Sequence[lbm_droplet], step: int = 0) -> int:
    arr = (lbm_config * len(cfgs))(*cfgs)
    nd = (C.c_int32 * len(ndrop))(*ndrop)
    dr = (lbm_droplet * max(1, len(drops)))(*drops)
    h = C.c_void_p(0)
    _check(load_library().lbm_init_batch(len(cfgs), arr, C.c_void_p(workspace_ptr), workspace_bytes,
                                         C.c_void_p(stream_ptr), _dptr(phi0), _dptr(c0), _dptr(f_pre), nd, dr,
                                         int(step), C.byref(h)))
    return int(h.value)


def lbm_step(ctx: int, n: int) -> None:
    _check(load_library().lbm_step(C.c_void_p(ctx), int(n)))


def lbm_set_graph(ctx: int, steps_per_graph: int) -> None:
    _check(load_library().lbm_set_graph(C.c_void_p(ctx), int(steps_per_graph)))


def lbm_sync(ctx: int) -> None:
    _check(load_library().lbm_sync(C.c_void_p(ctx)))


def lbm_get_step(ctx: int) -> int:
    return int(load_library().lbm_get_step(C.c_void_p(ctx)))


def lbm_fields(ctx: int, inst: int, f_pre=None, phi=None, c=None, n=None, ux=None, uy=None) -> int:
    """Returns LBM_OK, or LBM_E_UNSTABLE when a returned value is non-finite (the arrays are filled)."""
    return _check(load_library().lbm_fields(C.c_void_p(ctx), inst, _dptr(f_pre), _dptr(phi), _dptr(c), _dptr(n),
                                            _dptr(ux), _dptr(uy)), allow=(LBM_E_UNSTABLE,))


def lbm_observables(ctx: int, inst: int, drop_out: Optional[np.ndarray]):
    o = lbm_obs()
    rc = _check(load_library().lbm_observables(C.c_void_p(ctx), inst, C.byref(o), _dptr(drop_out)),
                allow=(LBM_E_UNSTABLE,))
    return o, rc


def lbm_droplets(ctx: int, inst: int, ndrop: int) -> List[lbm_droplet]:
    arr = (lbm_droplet * max(1, ndrop))()
    _check(load_library().lbm_droplets(C.c_void_p(ctx), inst, arr))
    return list(arr[:ndrop])


def lbm_debug_stage(ctx: int, inst: int, out: np.ndarray) -> None:
    _check(load_library().lbm_debug_stage(C.c_void_p(ctx), inst, _dptr(out)))


def lbm_time_kernels(ctx: int, n: int) -> np.ndarray:
    out = np.zeros(3)
    _check(load_library().lbm_time_kernels(C.c_void_p(ctx), int(n), _dptr(out)))
    return out


def lbm_time_launches(ctx: int, launches: int) -> np.ndarray:
    out = np.zeros(3)
    _check(load_library().lbm_time_launches(C.c_void_p(ctx), int(launches), _dptr(out)))
    return out


def lbm_adjoint_bytes(ctx: int, nsteps: int, every: int) -> int:
    n = C.c_size_t(0)
    _check(load_library().lbm_adjoint_bytes(C.c_void_p(ctx), int(nsteps), int(every), C.byref(n)))
    return int(n.value)


def lbm_adjoint_forward(ctx: int, ws: int, nbytes: int, drop: int, nsteps: int, every: int) -> float:
    J = np.zeros(1)
    _check(load_library().lbm_adjoint_forward(C.c_void_p(ctx), C.c_void_p(ws), nbytes, int(drop), int(nsteps),
                                              int(every), _dptr(J)))
    return float(J[0])


def lbm_adjoint_backward(ctx: int, ws: int, nbytes: int, shape):
    dA0 = np.zeros(1)
    dc0 = np.zeros(shape)
    _check(load_library().lbm_adjoint_backward(C.c_void_p(ctx), C.c_void_p(ws), nbytes, _dptr(dA0), _dptr(dc0)))
    return float(dA0[0]), dc0


def lbm_kernel_name(path: int, which: int) -> str:
    return load_library().lbm_kernel_name(path, which).decode()


def lbm_set_path(ctx: int, path: int) -> None:
    _check(load_library().lbm_set_path(C.c_void_p(ctx), int(path)))


def lbm_get_path(ctx: int) -> int:
    return int(load_library().lbm_get_path(C.c_void_p(ctx)))


def lbm_set_seg_rows(ctx: int, rows: int) -> None:
    _check(load_library().lbm_set_seg_rows(C.c_void_p(ctx), int(rows)))


def lbm_get_seg_rows(ctx: int) -> int:
    return int(load_library().lbm_get_seg_rows(C.c_void_p(ctx)))


def lbm_set_strip_width(ctx: int, width: int) -> None:
    _check(load_library().lbm_set_strip_width(C.c_void_p(ctx), int(width)))


def lbm_get_strip_width(ctx: int) -> int:
    return int(load_library().lbm_get_strip_width(C.c_void_p(ctx)))


def lbm_tune_rows():
    p = load_library().lbm_tune_rows()
    return [int(p[i]) for i in range(LBM_TUNE_NROWS)]


def lbm_tune_widths():
    p = load_library().lbm_tune_widths()
    return [int(p[i]) for i in range(LBM_TUNE_NWIDTHS)]


def lbm_autotune(ctx: int, launches: int, both_paths: bool = True):
    """Returns (rows, path, {"fused:rows" / "wave:rows": ms per launch}) for the candidates tried."""
    rows, path = C.c_int32(0), C.c_int32(0)
    nw, nr = LBM_TUNE_NWIDTHS, LBM_TUNE_NROWS
    ms = np.zeros(2 * nw * nr + 1)
    _check(load_library().lbm_autotune(C.c_void_p(ctx), int(launches), int(bool(both_paths)), C.byref(rows),
                                       C.byref(path), _dptr(ms)))
    heights, widths = lbm_tune_rows(), lbm_tune_widths()
    times = {}
    for pi, name in enumerate(("fused", "wave")):
        for wi, w in enumerate(widths):
            for k, r in enumerate(heights):
                v = ms[(pi * nw + wi) * nr + k]
                if v >= 0:
                    times[f"{name}:{w}x{r}"] = float(v)
    if ms[2 * nw * nr] >= 0:
        times["split"] = float(ms[2 * nw * nr])
    return int(rows.value), int(path.value), times


def lbm_step_noalloc(cfg: lbm_config, stream_ptr: int, f_ptrs, phi_ptrs, c_ptrs, ndrop: int, drops_ptr: int,
                     step: int, nsteps: int) -> int:
    """The allocation-free step (device pointers in, nothing allocated); returns the error code (no raise), so
    that callers and tests see LBM_E_INVAL / LBM_E_NOMEM directly."""
    pair = lambda p: (C.c_void_p * 2)(C.c_void_p(p[0]), C.c_void_p(p[1]))
    return int(load_library().lbm_step_noalloc(C.byref(cfg), C.c_void_p(stream_ptr), pair(f_ptrs), pair(phi_ptrs),
                                               pair(c_ptrs), int(ndrop), C.c_void_p(drops_ptr), int(step),
                                               int(nsteps)))


def lbm_destroy(ctx: int) -> None:
    load_library().lbm_destroy(C.c_void_p(ctx))


# ---- convenience object -----------------------------------------------------------------------------
class Sim:
    """A batch of periodic lattices advanced on one GPU (a single lattice is a batch of one).

    params: list of parameter dicts (nx, ny and the lbm_config fields), phi0 / c0: lists of (ny, nx)
    arrays, drops: list of lists of droplet dicts.  torch owns the workspace and the stream.
    """

    def __init__(self, params: List[dict], phi0: List[np.ndarray], c0: List[np.ndarray],
                 drops: Optional[List[List[dict]]] = None, precision: int = LBM_FP64,
                 f_pre: Optional[List[np.ndarray]] = None, step: int = 0, device: str = "cuda:0",
                 graph_steps: Optional[int] = None, path: int = LBM_PATH_FUSED):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU (torch.cuda.is_available() is False)")
        load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.params = [dict(p) for p in params]
        self.n = len(params)
        drops = drops if drops is not None else [[] for _ in range(self.n)]
        self.ndrop = [len(d) for d in drops]
        self.cfgs = [make_config(p, precision) for p in params]
        self.precision = precision
        nbytes = lbm_workspace_bytes(self.cfgs, self.ndrop)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in params]
        cat = lambda arrs: np.ascontiguousarray(np.concatenate([np.asarray(a, np.float64).ravel() for a in arrs]))
        fp = cat(f_pre) if f_pre is not None else None
        dl = [make_droplet(d) for ds in drops for d in ds]
        torch.cuda.synchronize(self.device)
        self.ctx = lbm_init_batch(self.cfgs, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream, cat(phi0),
                                  cat(c0), fp, self.ndrop, dl, step)
        lbm_set_path(self.ctx, path)
        # the library's default: 20-step graphs on the (non-default) stream
        self.graph_steps = 20
        if graph_steps is not None:
            self.set_graph(graph_steps)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_sync(self.ctx)
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step_count(self) -> int:
        return lbm_get_step(self.ctx)

    def step(self, n: int) -> None:
        lbm_step(self.ctx, n)

    def sync(self) -> None:
        lbm_sync(self.ctx)

    def set_graph(self, steps_per_graph: int) -> None:
        """Steps per hipGraph replay (0: eager launches); the graphs are captured by this call."""
        lbm_set_graph(self.ctx, steps_per_graph)
        self.graph_steps = steps_per_graph

    def fields(self, inst: int = 0) -> Dict[str, np.ndarray]:
        ny, nx = self.shapes[inst]
        out = {"f": np.empty((9, ny, nx)), "phi": np.empty((ny, nx)), "c": np.empty((ny, nx)),
               "n": np.empty((ny, nx)), "ux": np.empty((ny, nx)), "uy": np.empty((ny, nx))}
        lbm_fields(self.ctx, inst, out["f"], out["phi"], out["c"], out["n"], out["ux"], out["uy"])
        return out

    def observables(self, inst: int = 0) -> dict:
        nd = self.ndrop[inst]
        d = np.zeros((max(1, nd), 5))
        o, rc = lbm_observables(self.ctx, inst, d)
        return {"step": o.step, "mass": o.mass, "sum_phi": o.sum_phi, "sum_c": o.sum_c, "min_B": o.min_B,
                "max_u": o.max_u, "nonfinite": bool(o.nonfinite), "unstable": rc == LBM_E_UNSTABLE,
                "com": d[:nd, 0:2].copy(), "vel": d[:nd, 2:4].copy(), "drop_mass": d[:nd, 4].copy()}

    def droplets(self, inst: int = 0) -> List[dict]:
        return [dict(x=d.x, y=d.y, R=d.R, Rs=d.Rs, ex=d.ex, ey=d.ey, active=d.active)
                for d in lbm_droplets(self.ctx, inst, self.ndrop[inst])]

    def stages(self, inst: int = 0) -> Dict[str, np.ndarray]:
        ny, nx = self.shapes[inst]
        buf = np.empty((LBM_NSTAGE, ny, nx))
        lbm_debug_stage(self.ctx, inst, buf)
        return {name: buf[i] for i, name in enumerate(STAGES)}

    def set_path(self, path: int) -> None:
        lbm_set_path(self.ctx, path)

    def tune_rows(self):
        return lbm_tune_rows()

    @property
    def path(self) -> int:
        return lbm_get_path(self.ctx)

    @property
    def seg_rows(self) -> int:
        return lbm_get_seg_rows(self.ctx)

    def set_seg_rows(self, rows: int) -> None:
        lbm_set_seg_rows(self.ctx, rows)

    @property
    def strip_width(self) -> int:
        return lbm_get_strip_width(self.ctx)

    def set_strip_width(self, width: int) -> None:
        lbm_set_strip_width(self.ctx, width)

    def autotune(self, launches: int = 5, both_paths: bool = True):
        """Pick the kernel path (fused or wave sweep with its strip width and segment height, or the split pair)
        by timing each candidate (the state is unchanged).  Returns (rows, path, times); the chosen width is
        `strip_width`.  Keys of times: "fused:WxH", "wave:WxH", "split"."""
        return lbm_autotune(self.ctx, launches, both_paths)

    def time_kernels(self, n: int) -> Dict[str, float]:
        """Average ms per launch of each kernel of the current path (hipEvents on the library's stream)."""
        ms = lbm_time_kernels(self.ctx, n)
        path = lbm_get_path(self.ctx)
        return {lbm_kernel_name(path, i): float(ms[i]) for i in range(3) if lbm_kernel_name(path, i)}

    def time_launches(self, launches: int) -> Dict[str, float]:
        """Device ms per launch of the current path's main kernels from back-to-back launches (state unchanged)."""
        ms = lbm_time_launches(self.ctx, launches)
        path = lbm_get_path(self.ctx)
        names = [lbm_kernel_name(path, i) for i in range(3) if lbm_kernel_name(path, i)]
        return {k: float(ms[i]) for i, k in enumerate(names)}

    def adjoint_forward(self, drop: int, nsteps: int, every: int = 100) -> float:
        """Advance nsteps steps keeping checkpoints every `every` steps (the adjoint workspace is a torch
        uint8 tensor held by this object) and return J = x_CM(end) - x_CM(start) of droplet `drop`."""
        nbytes = lbm_adjoint_bytes(self.ctx, nsteps, every)
        with self.torch.cuda.device(self.device):
            self.adj_ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        return lbm_adjoint_forward(self.ctx, self.adj_ws.data_ptr(), nbytes, drop, nsteps, every)

    def adjoint_backward(self):
        """(dJ/dA0, dJ/dc at the start) of the last adjoint_forward (the library's adjoint kernels)."""
        return lbm_adjoint_backward(self.ctx, self.adj_ws.data_ptr(), self.adj_ws.numel(), self.shapes[0])


def com_displacement(A0, psi0, params: dict, phi0: np.ndarray, drops: List[dict], nsteps: int, every: int = 100,
                     drop: int = 0, precision: int = LBM_FP64, path: int = -1):
    """J = x-displacement of droplet `drop`'s centre of mass over nsteps steps as a differentiable function of the
    production rate A0 (0-d tensor) and the initial surfactant field psi0 ([ny][nx] tensor); the gradient comes
    from the library's adjoint (lbm_adjoint_backward).  path -1 picks the kernel path with the autotuner."""
    return _ComDisplacement.apply(A0, psi0, params, phi0, drops, nsteps, every, drop, precision, path)


def _make_com_displacement():
    import torch

    class ComDisplacement(torch.autograd.Function):
        @staticmethod
        def forward(ctx, A0, psi0, params, phi0, drops, nsteps, every, drop, precision, path):
            p = dict(params, A0=float(A0.detach().cpu()))
            c0 = np.ascontiguousarray(psi0.detach().cpu().numpy(), dtype=np.float64)
            sim = Sim([p], [phi0], [c0], [drops], precision=precision, graph_steps=20,
                      path=LBM_PATH_FUSED if path < 0 else path)
            if path < 0:
                sim.autotune(10, both_paths=True)
            J = sim.adjoint_forward(drop, nsteps, every)
            ctx.sim = sim
            ctx.psi_device, ctx.psi_dtype = psi0.device, psi0.dtype
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            # the context stays alive with ctx (a second backward, e.g. with retain_graph, repeats the first);
            # it is released when autograd frees ctx
            dA0, dc0 = ctx.sim.adjoint_backward()
            g = gJ.detach().cpu().double()
            gA0 = (g * dA0).to(torch.float64)
            gpsi = (g * torch.from_numpy(dc0)).to(device=ctx.psi_device, dtype=ctx.psi_dtype)
            return gA0, gpsi, None, None, None, None, None, None, None, None

    return ComDisplacement


class _LazyFunction:
    def __init__(self):
        self.fn = None

    def apply(self, *args):
        if self.fn is None:
            self.fn = _make_com_displacement()
        return self.fn.apply(*args)


_ComDisplacement = _LazyFunction()
