"""Seeded synthetic inputs (initial fields, droplet tables, parameter sets).

This module holds no arithmetic of the timestep: it only builds the initial
conditions that both the HIP library and the CPU oracle start from, so that
the two sides can be compared on identical inputs.  Shapes and parameter
values follow the paper's runs (Fadda et al., arXiv:1711.10984): R = 12..32
droplets in a phi = -1 matrix, surfactant 0.05..0.15 inside, a = -b = -0.001,
D = 0.1, tau = 0.6 for active runs (Sec. 4), gamma = 1.5e-3 and
A0 = gamma / 1e7 (Sec. 4).

Fields are float64 numpy arrays of shape (ny, nx), x fastest.  Noise is
U(-0.005, 0.005) from numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

# Parameter sets (lattice units).
PAPER_EQUILIBRIUM = dict(tau=1.0, n0=1.0, a=-0.001, b=0.001, B0=0.006, B1=-0.05, D=0.1, Gamma=1.0,
                         gamma=0.0, A0=0.0, t_star=2.0e6, c0=0.0, advection=0)
# Active-droplet set: tau = 0.6, gamma = 1.5e-3, A0 = gamma / 1e7 (Sec. 4); B0 = 0.01 (a Table 1 pair)
# keeps B(c) = B0 + B1 c > 0 for c up to 0.2.
ACTIVE = dict(PAPER_EQUILIBRIUM, tau=0.6, B0=0.01, gamma=1.5e-3, A0=1.5e-10)
# Sharp-interface stress set (a = -0.0625, b = 0.0625, kappa = 0.04, no surfactant coupling).
KAPPA_SET = dict(PAPER_EQUILIBRIUM, a=-0.0625, b=0.0625, B0=0.04, B1=0.0)


@dataclass
class DropSpec:
    x: float
    y: float
    R: float
    Rs: float
    ex: float = 1.0
    ey: float = 0.0
    active: int = 1
    psi_front: float = 0.15  # surfactant on the half facing e_hat
    psi_back: float = 0.05


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    params: dict
    phi0: np.ndarray
    c0: np.ndarray
    drops: List[DropSpec]
    steps: int = 0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def param_dict(self) -> dict:
        return dict(self.params, nx=self.nx, ny=self.ny)

    def drop_dicts(self) -> List[dict]:
        return [dict(x=d.x, y=d.y, R=d.R, Rs=d.Rs, ex=d.ex, ey=d.ey, active=d.active) for d in self.drops]


def _minimg(d: np.ndarray, L: int) -> np.ndarray:
    return (d + 0.5 * L) % L - 0.5 * L


def droplet_fields(nx: int, ny: int, drops: List[DropSpec], psi_out: float = 0.0, xi: float = 2.0,
                   phi_eq: float = 1.0, noise: float = 0.005, seed: int = 0):
    """phi0 = phi_eq * tanh(2 (R - d) / xi) about the nearest droplet (Eq. 20 profile),
    psi0 = psi_in (1 + phi0/phi_eq)/2 + psi_out (1 - phi0/phi_eq)/2 + U(-noise, noise),
    psi_in = psi_front on the half facing e_hat, psi_back on the other half."""
    phi = np.full((ny, nx), -1.0)
    psi_in = np.zeros((ny, nx))
    best = np.full((ny, nx), np.inf)
    # Each droplet updates only a periodic window of half-width h around its centre.  Beyond distance
    # R_max + 10 xi from every centre the profile rounds to -1.0 exactly (tanh saturates in double precision
    # past 19) and psi_in is multiplied by 0.0, and every node a window covers is covered by its nearest
    # droplet's window too, so the result is the same, bit for bit, as evaluating every droplet everywhere.
    h = int(math.ceil(max(d.R for d in drops) + 10.0 * xi + 1.0)) if drops else 0
    windowed = 2 * h + 2 <= min(nx, ny)
    for d in drops:
        if windowed:
            cx, cy = int(math.floor(d.x)), int(math.floor(d.y))
            xs = np.arange(cx - h, cx + h + 2) % nx
            ys = np.arange(cy - h, cy + h + 2) % ny
            sub = np.ix_(ys, xs)
            x = xs.astype(np.float64)[None, :]
            y = ys.astype(np.float64)[:, None]
        else:
            sub = (slice(None), slice(None))
            y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
        dx = _minimg(x - d.x, nx)
        dy = _minimg(y - d.y, ny)
        r = np.hypot(dx, dy)
        prof = np.tanh(2.0 * (d.R - r) / xi)
        closer = r < best[sub]
        best[sub] = np.where(closer, r, best[sub])
        phi[sub] = np.where(closer, prof, phi[sub])
        front = dx * d.ex + dy * d.ey >= 0.0
        psi_in[sub] = np.where(closer, np.where(front, d.psi_front, d.psi_back), psi_in[sub])
    frac_in = 0.5 * (1.0 + phi)
    psi = psi_in * frac_in + psi_out * (1.0 - frac_in)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        psi = psi + rng.uniform(-noise, noise, size=(ny, nx))
    return np.ascontiguousarray(phi_eq * phi), np.ascontiguousarray(psi)


def c1_equilibrium(seed: int = 1001, params: dict | None = None) -> Workload:
    """64x64 periodic, one R = 12 droplet, psi = 0.1 inside / 0 outside + noise, tau = 1, Gamma = 0.1,
    paper's equilibrium free-energy set, no source (Sec. 3 parameters)."""
    nx = ny = 64
    p = dict(PAPER_EQUILIBRIUM, Gamma=0.1) if params is None else dict(params)
    d = DropSpec(x=32.0, y=32.0, R=12.0, Rs=3.0, active=0, psi_front=0.1, psi_back=0.1)
    phi, psi = droplet_fields(nx, ny, [d], seed=seed)
    return Workload("c1_64x64_equilibrium_droplet", nx, ny, p, phi, psi, [d], steps=2000)


def c2_single_active(seed: int = 1002, n: int = 256) -> Workload:
    """n x n periodic, one self-propelled droplet R = 30 (R scaled with n/256), surfactant halves
    0.15 (front, +x) / 0.05, source radius R/4, active parameter set."""
    R = 30.0 * n / 256.0
    d = DropSpec(x=n / 2.0, y=n / 2.0, R=R, Rs=R / 4.0, ex=1.0, ey=0.0, active=1)
    phi, psi = droplet_fields(n, n, [d], seed=seed)
    return Workload(f"c2_{n}x{n}_single_active_droplet", n, n, dict(ACTIVE), phi, psi, [d], steps=50000)


def plates_single_active(seed: int = 1006, nx: int = 512, ny: int = 256, R: float = 32.0) -> Workload:
    """The plate geometry of Sec. 4: a droplet of radius R at the centre of an nx x ny box between two plates
    (walls at y = -1/2 and y = ny - 1/2, x periodic), surfactant initially 0.1 everywhere, B0 = 0.006,
    B1 = -0.05, tau = 0.6, consumption 1.5e-3 and production A0 = 1.5e-10 in a disk of radius R/4 touching
    the interface from inside on the +x side."""
    d = DropSpec(x=nx / 2.0, y=ny / 2.0, R=R, Rs=R / 4.0, ex=1.0, ey=0.0, active=1, psi_front=0.1, psi_back=0.1)
    phi, psi = droplet_fields(nx, ny, [d], psi_out=0.1, seed=seed)
    params = dict(PAPER_EQUILIBRIUM, tau=0.6, gamma=1.5e-3, A0=1.5e-10, walls=1)
    return Workload(f"plates_{nx}x{ny}_single_active_droplet", nx, ny, params, phi, psi, [d], steps=100000)


def c3_batch(seed: int = 1003) -> List[Workload]:
    """32 two-droplet instances (R = 24, Ly = 256) of uneven widths: head-on separations
    d in {2.5, 3, 4, 6} R (Lx = 256, 256, 384, 512), vertical offsets {0, R/2, R}, active-active and
    active-passive (the passive droplet has no surfactant and no source), plus 8 seed replicas at
    512 x 256 (d in {2.5, 3, 4, 6} R, offsets {0, R})."""
    R = 24.0
    Ly = 256
    out: List[Workload] = []
    lx_of = {2.5: 256, 3.0: 256, 4.0: 384, 6.0: 512}
    k = 0

    def make(dmult, off, passive, lx, s):
        cx, cy = lx / 2.0, Ly / 2.0
        sep = dmult * R
        left = DropSpec(cx - sep / 2.0, cy - off / 2.0, R, R / 4.0, ex=1.0, ey=0.0, active=1)
        if passive:
            right = DropSpec(cx + sep / 2.0, cy + off / 2.0, R, R / 4.0, ex=-1.0, ey=0.0, active=0,
                             psi_front=0.0, psi_back=0.0)
        else:
            right = DropSpec(cx + sep / 2.0, cy + off / 2.0, R, R / 4.0, ex=-1.0, ey=0.0, active=1)
        phi, psi = droplet_fields(lx, Ly, [left, right], seed=s)
        tag = "ap" if passive else "aa"
        return Workload(f"c3_{lx}x{Ly}_d{dmult}R_off{off / R:g}R_{tag}", lx, Ly, dict(ACTIVE), phi, psi,
                        [left, right], steps=20000)

    for dmult in (2.5, 3.0, 4.0, 6.0):
        for off in (0.0, R / 2.0, R):
            for passive in (False, True):
                out.append(make(dmult, off, passive, lx_of[dmult], seed + k))
                k += 1
    for dmult in (2.5, 3.0, 4.0, 6.0):
        for off in (0.0, R):
            out.append(make(dmult, off, False, 512, seed + 100 + k))
            k += 1
    return out


def c5_emulsion(seed: int = 1005, n: int = 2048, ndrop: int = 64, R: float = 20.0) -> Workload:
    """n x n periodic dilute emulsion: ndrop active droplets of radius R at seeded random positions with
    minimum-image centre distance >= 5R (gap >= 3R), seeded random orientation, asymmetric surfactant
    halves 0.15 / 0.05, source radius R/4, active parameter set."""
    rng = np.random.default_rng(seed)
    centres: List[tuple] = []
    tries = 0
    while len(centres) < ndrop:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place droplets")
        cx, cy = rng.uniform(0, n), rng.uniform(0, n)
        ok = True
        for (px, py) in centres:
            dx = (cx - px + 0.5 * n) % n - 0.5 * n
            dy = (cy - py + 0.5 * n) % n - 0.5 * n
            if dx * dx + dy * dy < (5.0 * R) ** 2:
                ok = False
                break
        if ok:
            centres.append((cx, cy))
    drops = []
    for (cx, cy) in centres:
        th = rng.uniform(0.0, 2.0 * math.pi)
        drops.append(DropSpec(cx, cy, R, R / 4.0, ex=math.cos(th), ey=math.sin(th), active=1))
    phi, psi = droplet_fields(n, n, drops, seed=seed + 1)
    return Workload(f"c5_{n}x{n}_emulsion_{ndrop}drops", n, n, dict(ACTIVE), phi, psi, drops, steps=100000)


def crop_workload(w: Workload, x0: int, y0: int, size: int, seed: int = 1105) -> Workload:
    """A separate size x size periodic run seeded with the droplets of ``w`` whose centres fall in
    [x0, x0+size) x [y0, y0+size), positions shifted to the crop."""
    drops = []
    for d in w.drops:
        if x0 <= d.x < x0 + size and y0 <= d.y < y0 + size:
            drops.append(replace(d, x=d.x - x0, y=d.y - y0))
    phi, psi = droplet_fields(size, size, drops, seed=seed)
    return Workload(f"{w.name}_crop{size}", size, size, dict(w.params), phi, psi, drops, steps=w.steps)


def random_state(nx: int, ny: int, seed: int, f_amp: float = 0.02, phi_amp: float = 0.9, c_mean: float = 0.1,
                 c_amp: float = 0.04):
    """Random smooth-ish fields and populations for stage-level comparisons on tiny grids."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = w[:, None, None] * (1.0 + rng.uniform(-f_amp, f_amp, size=(9, ny, nx)))
    phi = rng.uniform(-phi_amp, phi_amp, size=(ny, nx))
    c = c_mean + rng.uniform(-c_amp, c_amp, size=(ny, nx))
    return np.ascontiguousarray(f), np.ascontiguousarray(phi), np.ascontiguousarray(c)
