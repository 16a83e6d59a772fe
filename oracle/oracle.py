"""ctypes wrapper of the FP64 CPU oracle (oracle/lbm_oracle.c).

TEST INFRASTRUCTURE: a plain reference of the hybrid lattice-Boltzmann /
finite-difference scheme of Fadda et al. (arXiv:1711.10984, Sec. 2).  It is
independent of the HIP library (no shared source, no shared helpers); only the
public data formats agree: fields are row-major [ny][nx] with x fastest and
populations are [9][ny][nx] in the D2Q9 order rest, E, N, W, S, NE, NW, SW, SE.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_ORACLE_LIB points the wrapper at another build of the same source (the mutation test uses it
# to check that the pins fail when a mistake is planted in the oracle).
_LIB_PATH = os.environ.get("LBM_ORACLE_LIB", os.path.join(_HERE, "liblbm_oracle.so"))
_lib = None

STAGES = ["mu", "X", "Fx", "Fy", "n", "ux", "uy", "phi_h", "c_h", "M", "X_h", "phi_new", "c_new"] + [
    f"fstar{i}" for i in range(9)
]


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("advection", C.c_int32), ("walls", C.c_int32),
                ("tau", C.c_double), ("n0", C.c_double),
                ("a", C.c_double), ("b", C.c_double), ("B0", C.c_double), ("B1", C.c_double),
                ("D", C.c_double), ("Gamma", C.c_double),
                ("gamma", C.c_double), ("A0", C.c_double), ("t_star", C.c_double), ("c0", C.c_double)]


class _Drop(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("R", C.c_double), ("Rs", C.c_double),
                ("ex", C.c_double), ("ey", C.c_double), ("active", C.c_int32), ("reserved", C.c_int32)]


class _ObsHead(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("sum_phi", C.c_double), ("sum_c", C.c_double),
                ("min_B", C.c_double), ("max_u", C.c_double), ("nonfinite", C.c_int32), ("ndrop", C.c_int32)]


@dataclass
class Params:
    """Model parameters in lattice units (Sec. 2 of the paper)."""
    nx: int
    ny: int
    tau: float = 1.0
    n0: float = 1.0
    a: float = -0.001
    b: float = 0.001
    B0: float = 0.006
    B1: float = -0.05
    D: float = 0.1
    Gamma: float = 1.0
    gamma: float = 0.0
    A0: float = 0.0
    t_star: float = 2.0e6
    c0: float = 0.0
    advection: int = 0  # 0: Eqs. (16)-(17) as printed, 1: conservative flux form
    walls: int = 0  # 0: periodic in y, 1: plates at y = -1/2 and y = ny - 1/2


@dataclass
class Drop:
    x: float
    y: float
    R: float
    Rs: float = 0.0
    ex: float = 1.0
    ey: float = 0.0
    active: int = 0


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        lib.orc_new.restype = C.c_void_p
        lib.orc_new.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_int64, C.c_int, C.POINTER(_Drop)]
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_run.argtypes = [C.c_void_p, C.c_int64]
        lib.orc_stage_count.restype = C.c_int
        lib.orc_num_threads.restype = C.c_int
        lib.orc_threads_for.restype = C.c_int
        lib.orc_threads_for.argtypes = [C.c_int, C.c_int]
        lib.orc_stages.argtypes = [C.c_void_p, dp]
        lib.orc_get_step.restype = C.c_int64
        lib.orc_get_step.argtypes = [C.c_void_p]
        lib.orc_get_drops.argtypes = [C.c_void_p, C.POINTER(_Drop)]
        lib.orc_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
        lib.orc_observables.argtypes = [C.c_void_p, C.POINTER(_ObsHead), dp]
        lib.orc_grad9.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        lib.orc_lap9.argtypes = [C.c_int, C.c_int, dp, dp]
        lib.orc_div9.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c_params(p: Params) -> _Params:
    d = asdict(p)
    return _Params(nx=d["nx"], ny=d["ny"], advection=d["advection"], walls=d["walls"], tau=d["tau"], n0=d["n0"],
                   a=d["a"], b=d["b"], B0=d["B0"], B1=d["B1"], D=d["D"], Gamma=d["Gamma"], gamma=d["gamma"],
                   A0=d["A0"], t_star=d["t_star"], c0=d["c0"])


class OracleSim:
    """One lattice (periodic, or bounded by plates in y) advanced by the oracle."""

    def __init__(self, p: Params, phi0: np.ndarray, c0: np.ndarray, drops: Sequence[Drop] = (),
                 f_pre: Optional[np.ndarray] = None, step: int = 0):
        lib = load()
        self.p = p
        shape = (p.ny, p.nx)
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(shape)
        c0 = np.ascontiguousarray(c0, dtype=np.float64).reshape(shape)
        fp = None
        if f_pre is not None:
            fp = np.ascontiguousarray(f_pre, dtype=np.float64).reshape((9,) + shape)
        self.ndrop = len(drops)
        arr = (_Drop * max(1, self.ndrop))()
        for k, d in enumerate(drops):
            arr[k] = _Drop(d.x, d.y, d.R, d.Rs, d.ex, d.ey, int(d.active), 0)
        self._cp = _c_params(p)
        h = lib.orc_new(C.byref(self._cp), _ptr(fp), _ptr(phi0), _ptr(c0), int(step), self.ndrop, arr)
        if not h:
            raise ValueError("oracle rejected the configuration")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    @property
    def step_count(self) -> int:
        return int(load().orc_get_step(self._h))

    def run(self, nsteps: int) -> None:
        load().orc_run(self._h, int(nsteps))

    def fields(self) -> dict:
        p = self.p
        N = (p.ny, p.nx)
        out = {"f": np.empty((9,) + N), "phi": np.empty(N), "c": np.empty(N), "n": np.empty(N),
               "ux": np.empty(N), "uy": np.empty(N)}
        load().orc_fields(self._h, *[_ptr(out[k]) for k in ("f", "phi", "c", "n", "ux", "uy")])
        return out

    def stages(self) -> dict:
        """Intermediate planes of the next step (the state is not advanced)."""
        p = self.p
        ns = load().orc_stage_count()
        buf = np.empty((ns, p.ny, p.nx))
        load().orc_stages(self._h, _ptr(buf))
        return {name: buf[i] for i, name in enumerate(STAGES)}

    def drops(self) -> List[Drop]:
        arr = (_Drop * max(1, self.ndrop))()
        load().orc_get_drops(self._h, arr)
        return [Drop(a.x, a.y, a.R, a.Rs, a.ex, a.ey, a.active) for a in arr[: self.ndrop]]

    def observables(self) -> dict:
        head = _ObsHead()
        d = np.zeros((max(1, self.ndrop), 5))
        load().orc_observables(self._h, C.byref(head), _ptr(d))
        return {"step": head.step, "mass": head.mass, "sum_phi": head.sum_phi, "sum_c": head.sum_c,
                "min_B": head.min_B, "max_u": head.max_u, "nonfinite": bool(head.nonfinite),
                "com": d[: self.ndrop, 0:2].copy(), "vel": d[: self.ndrop, 2:4].copy(),
                "drop_mass": d[: self.ndrop, 4].copy()}


def grad9(g: np.ndarray):
    g = np.ascontiguousarray(g, dtype=np.float64)
    ny, nx = g.shape
    gx, gy = np.empty_like(g), np.empty_like(g)
    load().orc_grad9(nx, ny, _ptr(g), _ptr(gx), _ptr(gy))
    return gx, gy


def lap9(g: np.ndarray):
    g = np.ascontiguousarray(g, dtype=np.float64)
    ny, nx = g.shape
    out = np.empty_like(g)
    load().orc_lap9(nx, ny, _ptr(g), _ptr(out))
    return out


def div9(k: np.ndarray, X: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    ny, nx = k.shape
    out = np.empty_like(k)
    load().orc_div9(nx, ny, _ptr(k), _ptr(X), _ptr(out))
    return out


def num_threads(nx: int = 0, ny: int = 0) -> int:
    """Threads the oracle's OpenMP loops use in this process (for an nx x ny lattice if given: small lattices
    run on one thread)."""
    if nx and ny:
        return int(load().orc_threads_for(int(nx), int(ny)))
    return int(load().orc_num_threads())
