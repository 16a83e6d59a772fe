"""Pins of the oracle's lattice-Boltzmann half (Sec. 2.2, Eqs. 10-15).

* Moments of the collision (Eqs. 11-13): for any tau, sum f* = n, sum f* e = n u + F/2 and
  sum f* ee = (1-w) sum f ee + w (n cs^2 I + n u u) + (1 - w/2)(u F + F u), w = 1/tau.  These hold only
  with the 1/2 in the second-order equilibrium term and with the Guo forcing of Eq. (13).
* Streaming (Eq. 10): a population at r moves to r + e_i in one step.
* Mass conservation.
* Shear-wave decay at nu = (tau - 1/2)/3 (Eq. 15) and sound speed cs = 1/sqrt(3) (textbook LB).
"""
import numpy as np
import pytest

from oracle import OracleSim, Params
from paper_1711_10984_amd.workloads import random_state
from tests.lbhelpers import EX, EY, WT, feq, moments


def _quiet_params(nx, ny, **kw):
    """a = b = B0 = B1 = 0 and uniform c: the thermodynamic force vanishes identically."""
    d = dict(nx=nx, ny=ny, tau=1.0, a=0.0, b=0.0, B0=0.0, B1=0.0, D=0.0, Gamma=1.0, gamma=0.0, A0=0.0)
    d.update(kw)
    return Params(**d)


@pytest.mark.parametrize("tau", [1.0, 0.6, 1.7])
def test_collision_moments(tau):
    nx, ny = 8, 7
    f, phi, c = random_state(nx, ny, seed=11, f_amp=0.3)
    p = Params(nx=nx, ny=ny, tau=tau, a=-0.02, b=0.03, B0=0.05, B1=-0.2, D=0.1, Gamma=1.0)
    s = OracleSim(p, phi, c, f_pre=f)
    st = s.stages()
    n0, mx0, my0, pxx0, pxy0, pyy0 = moments(f)
    Fx, Fy, n, ux, uy = st["Fx"], st["Fy"], st["n"], st["ux"], st["uy"]
    assert np.max(np.abs(Fx)) > 1e-3 and np.max(np.abs(Fy)) > 1e-3  # the force is really on
    # Eq. (11): n = sum f, n u = sum f e + F/2
    assert np.allclose(n, n0, rtol=0, atol=1e-15)
    assert np.allclose(n * ux, mx0 + 0.5 * Fx, rtol=0, atol=1e-15)
    assert np.allclose(n * uy, my0 + 0.5 * Fy, rtol=0, atol=1e-15)
    fs = np.stack([st[f"fstar{i}"] for i in range(9)])
    n1, mx1, my1, pxx1, pxy1, pyy1 = moments(fs)
    w = 1.0 / tau
    assert np.allclose(n1, n, rtol=0, atol=1e-14)
    assert np.allclose(mx1, n * ux + 0.5 * Fx, rtol=0, atol=1e-14)
    assert np.allclose(my1, n * uy + 0.5 * Fy, rtol=0, atol=1e-14)
    g = 1.0 - 0.5 * w
    assert np.allclose(pxx1, (1 - w) * pxx0 + w * (n / 3 + n * ux * ux) + g * 2 * ux * Fx, rtol=0, atol=1e-14)
    assert np.allclose(pyy1, (1 - w) * pyy0 + w * (n / 3 + n * uy * uy) + g * 2 * uy * Fy, rtol=0, atol=1e-14)
    assert np.allclose(pxy1, (1 - w) * pxy0 + w * (n * ux * uy) + g * (ux * Fy + uy * Fx), rtol=0, atol=1e-14)


def test_equilibrium_is_fixed_point_at_tau_one():
    """With F = 0 and tau = 1 the post-collision state is f^eq(n, u) itself."""
    nx, ny = 6, 5
    rng = np.random.default_rng(5)
    n = 1 + 0.1 * rng.random((ny, nx))
    ux = 0.05 * rng.standard_normal((ny, nx))
    uy = 0.05 * rng.standard_normal((ny, nx))
    f = feq(n, 0 * n, 0 * n) + 0.01 * rng.standard_normal((9, ny, nx)) * WT[:, None, None]
    n0, mx, my, *_ = moments(f)
    s = OracleSim(_quiet_params(nx, ny), np.zeros((ny, nx)), np.full((ny, nx), 0.1), f_pre=f)
    st = s.stages()
    fs = np.stack([st[f"fstar{i}"] for i in range(9)])
    assert np.allclose(fs, feq(n0, mx / n0, my / n0), rtol=0, atol=1e-15)


def test_streaming_direction():
    """A mass bump at r0 (F = 0, u = 0) is carried by each population to r0 + e_i (Eq. 10)."""
    nx, ny = 7, 6
    f = np.broadcast_to(WT[:, None, None], (9, ny, nx)).copy()
    x0, y0 = 3, 2
    f[:, y0, x0] *= 1.1
    s = OracleSim(_quiet_params(nx, ny, tau=0.8), np.zeros((ny, nx)), np.full((ny, nx), 0.1), f_pre=f)
    s.run(1)
    f1 = s.fields()["f"]
    for i in range(9):
        exp = np.full((ny, nx), WT[i])
        exp[(y0 + EY[i]) % ny, (x0 + EX[i]) % nx] = 1.1 * WT[i]
        assert np.allclose(f1[i], exp, rtol=0, atol=1e-15), i


def test_mass_conservation_droplet():
    from paper_1711_10984_amd.workloads import c1_equilibrium
    w = c1_equilibrium()
    s = OracleSim(Params(nx=w.nx, ny=w.ny, **w.params), w.phi0, w.c0)
    m0 = s.observables()["mass"]
    s.run(300)
    m1 = s.observables()["mass"]
    assert abs(m1 - m0) / m0 < 1e-13


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_shear_wave_decay(tau):
    """u_x = U sin(2 pi y / L) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3 (Eq. 15)."""
    L = 64
    nx, ny = 4, L
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    U = 1e-4
    k = 2 * np.pi / L
    f = feq(np.ones((ny, nx)), U * np.sin(k * y), np.zeros((ny, nx)))
    s = OracleSim(_quiet_params(nx, ny, tau=tau), np.zeros((ny, nx)), np.full((ny, nx), 0.1), f_pre=f)

    def amp():
        ux = s.fields()["ux"][:, 0]
        return 2.0 / L * np.sum(ux * np.sin(k * np.arange(L)))

    s.run(100)
    a1 = amp()
    s.run(1000)
    a2 = amp()
    nu = -np.log(a2 / a1) / (k * k * 1000)
    assert abs(nu / ((tau - 0.5) / 3) - 1) < 0.01


def test_sound_speed():
    """A standing density wave oscillates at omega = cs k, cs^2 = 1/3 (Eq. 12)."""
    L = 64
    nx, ny = L, 3
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    k = 2 * np.pi / L
    eps = 1e-5
    f = feq(1 + eps * np.cos(k * x), np.zeros((ny, nx)), np.zeros((ny, nx)))
    # c = 0: an advected surfactant would add its own osmotic pressure (-grad c in Eq. 14)
    s = OracleSim(_quiet_params(nx, ny, tau=0.6), np.zeros((ny, nx)), np.zeros((ny, nx)), f_pre=f)
    amps = []
    for t in range(400):
        n = s.fields()["n"][0]
        amps.append(np.sum((n - 1) * np.cos(k * np.arange(nx))) * 2 / nx)
        s.run(1)
    a = np.array(amps)
    # zero crossings, linearly interpolated
    zs = [t + a[t] / (a[t] - a[t + 1]) for t in range(len(a) - 1) if a[t] * a[t + 1] < 0]
    half_periods = np.diff(zs)
    omega = np.pi / np.mean(half_periods)
    assert abs(omega / (k / np.sqrt(3)) - 1) < 0.005
