"""Pins of the oracle's finite-difference half (Sec. 2.3, Eqs. 16-19) and the activity terms.

* Upwind advection by a uniform velocity: amplification 1 - u (1 - e^{-ik}) per axis (u > 0),
  1 - u (e^{ik} - 1) (u < 0): the textbook first-order upwind scheme.  The conservative flux form has the
  same symbol (face velocity = u, face value taken from the upwind node), which fixes its upwind side.
* Centred velocity divergence: phi0 (1 - U sin k cos kx) for u_x = U sin kx, in both forms (in the flux
  form the face velocity is the mean of the two nodes, whose difference is the centred one).
* Time level of c in B(c) and in grad c of Eq. (18): a state whose force vanishes identically while
  lap phi does not (phi a period-4 staircase along x, so |grad phi| is uniform, a = b = 0, B(c) = 0 at the
  uniform c), moved by a small positive velocity.  Then B(c^{n+1/2}) = -B1 c div u is first order in u,
  and the first-order response of phi^{n+1} follows by hand; with B(c^n) = 0 that term would vanish.
* Linear response of one Fourier mode, derived by hand from Eqs. (3), (11), (14), (16)-(19)
  with the 9-point symbols: pins a, b (at time level n), B(c) = B0 + B1 c, Gamma, D, gamma, the
  half-force velocity and the centred divergence in the advection.
* Exact budget identities: the printed advection changes sum(phi) by exactly
  1/2 sum_r phi sum_a Delta_a^2 |u_a|; the flux form conserves it; diffusion conserves it; the
  surfactant budget is sum c^{n+1} = sum c^{1/2} - gamma (sum c^{1/2} - N c0) + A(n) N_Theta.
* Source disk and ramp A(n) = A0 min(n, t*) in closed form (Sec. 2.1, Sec. 4).
"""
import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from paper_1711_10984_amd.workloads import c1_equilibrium, c2_single_active
from tests.lbhelpers import feq, sym_lap, WT


def _flow_only(nx, ny, **kw):
    d = dict(nx=nx, ny=ny, tau=0.8, a=0.0, b=0.0, B0=0.0, B1=0.0, D=0.0, Gamma=1.0, gamma=0.0, A0=0.0)
    d.update(kw)
    return Params(**d)


@pytest.mark.parametrize("advection", [0, 1])
@pytest.mark.parametrize("u0", [(0.03, 0.02), (-0.03, 0.02), (0.03, -0.04), (-0.02, -0.01)])
def test_upwind_uniform_velocity(u0, advection):
    nx, ny = 16, 12
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    phi = np.cos(kx * x + ky * y)
    f = feq(np.ones((ny, nx)), np.full((ny, nx), u0[0]), np.full((ny, nx), u0[1]))
    s = OracleSim(_flow_only(nx, ny, advection=advection), phi, np.full((ny, nx), 0.1), f_pre=f)
    st = s.stages()
    ux, uy = st["ux"][0, 0], st["uy"][0, 0]
    assert abs(ux - u0[0]) < 1e-15 and abs(uy - u0[1]) < 1e-15
    gx = 1 - ux * (1 - np.exp(-1j * kx)) if ux > 0 else 1 - ux * (np.exp(1j * kx) - 1)
    gy = 1 - uy * (1 - np.exp(-1j * ky)) if uy > 0 else 1 - uy * (np.exp(1j * ky) - 1)
    G = gx + gy - 1  # one Euler step: the two axis increments add
    expect = np.real(G * np.exp(1j * (kx * x + ky * y)))
    assert np.max(np.abs(st["phi_new"] - expect)) < 1e-14


@pytest.mark.parametrize("advection", [0, 1])
def test_centred_velocity_divergence(advection):
    nx, ny = 16, 10
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi / nx, 2 * np.pi * 2 / ny
    U, V = 0.02, 0.015
    f = feq(np.ones((ny, nx)), U * np.sin(kx * x), V * np.sin(ky * y))
    phi0, cbar = 0.7, 0.1
    s = OracleSim(_flow_only(nx, ny, advection=advection), np.full((ny, nx), phi0), np.full((ny, nx), cbar),
                  f_pre=f)
    st = s.stages()
    div = U * np.sin(kx) * np.cos(kx * x) + V * np.sin(ky) * np.cos(ky * y)
    assert np.max(np.abs(st["phi_new"] - phi0 * (1 - div))) < 1e-15
    assert np.max(np.abs(st["c_new"] - cbar * (1 - div))) < 1e-15


def _fourier(g, symbol):
    return np.real(np.fft.ifft2(np.fft.fft2(g) * symbol))


def test_time_level_of_c_in_the_phi_update():
    """Eq. (18) takes B(c) and grad c at n + 1/2.  Base state: phi a staircase (p0, p0, p1, p1) repeating along
    x, uniform c = cbar, a = b = 0 and B0 = -B1 cbar (exact in binary), fluid at rest.  Then mu = 0, the 9-point
    grad phi is +-(p1 - p0)/2 everywhere so X is uniform, and the force vanishes identically, while lap phi = +-
    (p1 - p0) does not.  Populations at equilibrium with a velocity eps u1, u1 > 0 everywhere (so the upwind side
    is the backward difference on both axes): c^{1/2} = cbar (1 - D0.u), B(c^{1/2}) = -B1 cbar eps D0.u1, and to
    first order in eps
        phi^{n+1} - phi = eps [ -(phi D0.u1 + u1 . Dminus phi)
                                + Gamma B1 cbar lap9( (D0.u1) lap9 phi + grad9(D0.u1) . grad9 phi ) ],
    with D0 the 3-point centred divergence, Dminus the backward difference, and the 9-point operators applied
    here through their Fourier symbols.  Reading B(c^n) instead drops the (D0.u1) lap9 phi term; reading grad c^n
    drops the other."""
    from tests.lbhelpers import sym_grad, sym_lap, wavenumbers
    nx, ny = 16, 12
    p0, p1 = -0.3, 0.5
    phi = np.tile(np.array([p0, p0, p1, p1]), (ny, nx // 4))
    cbar, B1, Gamma = 0.25, -0.5, 0.7
    p = Params(nx=nx, ny=ny, tau=0.8, a=0.0, b=0.0, B0=-B1 * cbar, B1=B1, D=0.1, Gamma=Gamma, gamma=0.0)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    u1x = 1.0 + 0.5 * np.sin(2 * np.pi * x / nx + 0.3) + 0.2 * np.cos(2 * np.pi * y / ny)
    u1y = 1.0 + 0.4 * np.cos(2 * np.pi * (x / nx + 2 * y / ny))
    eps = 1e-7
    s = OracleSim(p, phi, np.full((ny, nx), cbar), f_pre=feq(np.ones((ny, nx)), eps * u1x, eps * u1y))
    st = s.stages()
    assert np.all(st["mu"] == 0.0) and np.all(st["Fx"] == 0.0) and np.all(st["Fy"] == 0.0)
    kx, ky = wavenumbers(ny, nx)
    div = _fourier(u1x, 1j * np.sin(kx)) + _fourier(u1y, 1j * np.sin(ky))
    dmx, dmy = _fourier(phi, 1 - np.exp(-1j * kx)), _fourier(phi, 1 - np.exp(-1j * ky))
    gsx, gsy = sym_grad(ny, nx)
    lap = sym_lap(ny, nx)
    lap_phi = _fourier(phi, lap)
    grad_term = _fourier(div, gsx) * _fourier(phi, gsx) + _fourier(div, gsy) * _fourier(phi, gsy)
    advect = -(phi * div + u1x * dmx + u1y * dmy)
    want = advect + Gamma * B1 * cbar * _fourier(div * lap_phi + grad_term, lap)
    got = (st["phi_new"] - phi) / eps
    assert np.max(np.abs(got - want)) < 1e-6
    # the alternative readings differ from this by far more than the tolerance
    b_at_n = advect + Gamma * B1 * cbar * _fourier(grad_term, lap)
    gradc_at_n = advect + Gamma * B1 * cbar * _fourier(div * lap_phi, lap)
    assert np.max(np.abs(b_at_n - want)) > 1e-2 and np.max(np.abs(gradc_at_n - want)) > 1e-2


def _odd_response(p, base_phi, base_c, dphi, dc, eps):
    """Odd part in eps of one step's (phi, c) response, divided by eps."""
    out = []
    for sgn in (+1, -1):
        s = OracleSim(p, base_phi + sgn * eps * dphi, base_c + sgn * eps * dc)
        st = s.stages()
        out.append((st["phi_new"], st["c_new"]))
    return (out[0][0] - out[1][0]) / (2 * eps), (out[0][1] - out[1][1]) / (2 * eps)


def _upwind_remainder(u1x, u1y, mode_field, kx, ky, eps):
    """The upwind difference chosen by the sign of u = eps u1 equals the centred one minus
    |u| Delta^2 / 2, whose part odd in eps is eps * (|u1x| Delta_x^2 + |u1y| Delta_y^2) mode / 2
    (relative to the mode): second order in size, but it survives the odd extraction."""
    return 0.5 * eps * (np.abs(u1x) * 2 * (np.cos(kx) - 1) + np.abs(u1y) * 2 * (np.cos(ky) - 1)) * mode_field


@pytest.mark.parametrize("mode", [(1, 0), (2, 3), (5, 1), (4, 4)])
def test_linear_response_phi_mode(mode):
    nx, ny = 16, 12
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * mode[0] / nx, 2 * np.pi * mode[1] / ny
    cosm = np.cos(kx * x + ky * y)
    a, b, B0, B1, Gamma, D, gam, c0 = -0.02, 0.05, 0.03, -0.1, 0.8, 0.3, 0.01, 0.02
    phi0, cbar = 0.6, 0.12
    p = Params(nx=nx, ny=ny, tau=0.7, a=a, b=b, B0=B0, B1=B1, D=D, Gamma=Gamma, gamma=gam, c0=c0)
    eps = 1e-5
    Rp, Rc = _odd_response(p, np.full((ny, nx), phi0), np.full((ny, nx), cbar), cosm, 0 * cosm, eps)
    lam = (8 * np.cos(kx) + 8 * np.cos(ky) + 4 * np.cos(kx) * np.cos(ky) - 20) / 6
    sx = np.sin(kx) * (2 + np.cos(ky)) / 3
    sy = np.sin(ky) * (2 + np.cos(kx)) / 3
    sigma = sx * np.sin(kx) + sy * np.sin(ky)
    Beff = B0 + B1 * cbar
    g = a + 3 * b * phi0 ** 2 - Beff * lam          # mu_phi linearised (Eq. 3)
    h = 1 - phi0 ** 2 * g * sigma / 2               # advection by u = F/2 (Eqs. 11, 14, 16)
    G = h + Gamma * lam * (a * h + 3 * b * phi0 ** 2 - Beff * lam * h)   # Eq. (18), b (phi^n)^3
    Gc = -cbar * (phi0 * g * sigma / 2) * (1 + D * lam - gam)            # Eqs. (17), (19)
    sinm = np.sin(kx * x + ky * y)
    w = _upwind_remainder(0.5 * phi0 * g * sx * sinm, 0.5 * phi0 * g * sy * sinm, cosm, kx, ky, eps)
    Lphi = 1 + Gamma * sym_lap(ny, nx) * (a - Beff * sym_lap(ny, nx))  # Eq. (18) acting on phi^{1/2}
    corr = np.real(np.fft.ifft2(np.fft.fft2(w) * Lphi))
    assert np.max(np.abs(Rp - G * cosm - corr)) < 1e-9
    assert np.max(np.abs(Rc - Gc * cosm)) < 1e-9
    # the time level of the cubic term is visible at this tolerance:
    G_half = h + Gamma * lam * (a * h + 3 * b * phi0 ** 2 * h - Beff * lam * h)
    assert abs(G - G_half) > 1e-6


@pytest.mark.parametrize("mode", [(1, 0), (3, 2), (6, 5)])
def test_linear_response_c_mode(mode):
    nx, ny = 16, 12
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * mode[0] / nx, 2 * np.pi * mode[1] / ny
    cosm = np.cos(kx * x + ky * y + 0.4)
    a, b, B0, B1, Gamma, D, gam = -0.02, 0.05, 0.03, -0.1, 0.8, 0.3, 0.01
    phi0, cbar = -0.5, 0.12
    p = Params(nx=nx, ny=ny, tau=0.9, a=a, b=b, B0=B0, B1=B1, D=D, Gamma=Gamma, gamma=gam)
    eps = 1e-5
    Rp, Rc = _odd_response(p, np.full((ny, nx), phi0), np.full((ny, nx), cbar), 0 * cosm, cosm, eps)
    lam = (8 * np.cos(kx) + 8 * np.cos(ky) + 4 * np.cos(kx) * np.cos(ky) - 20) / 6
    sx = np.sin(kx) * (2 + np.cos(ky)) / 3
    sy = np.sin(ky) * (2 + np.cos(kx)) / 3
    sigma = sx * np.sin(kx) + sy * np.sin(ky)
    Beff = B0 + B1 * cbar
    hc = 1 - cbar * sigma / 2                      # F = -grad c, u = F/2
    Gp = -(phi0 * sigma / 2) * (1 + Gamma * lam * (a - Beff * lam))
    Gc = hc * (1 + D * lam - gam)
    sinm = np.sin(kx * x + ky * y + 0.4)
    w = _upwind_remainder(0.5 * sx * sinm, 0.5 * sy * sinm, cosm, kx, ky, eps)
    Lc = 1 + D * sym_lap(ny, nx) - gam             # Eq. (19) acting on c^{1/2}
    corr = np.real(np.fft.ifft2(np.fft.fft2(w) * Lc))
    assert np.max(np.abs(Rp - Gp * cosm)) < 1e-9
    assert np.max(np.abs(Rc - Gc * cosm - corr)) < 1e-9


def _d2abs(u, axis):
    a = np.abs(u)
    return np.roll(a, -1, axis) - 2 * a + np.roll(a, 1, axis)


@pytest.mark.parametrize("advection", [0, 1])
def test_phi_and_c_budget_identities(advection):
    w = c1_equilibrium()
    prm = dict(w.params, advection=advection)
    s = OracleSim(Params(nx=w.nx, ny=w.ny, **prm), w.phi0, w.c0)
    s.run(20)
    fl = s.fields()
    st = s.stages()
    ux, uy = st["ux"], st["uy"]
    drift_phi = 0.5 * np.sum(fl["phi"] * (_d2abs(ux, 1) + _d2abs(uy, 0)))
    drift_c = 0.5 * np.sum(fl["c"] * (_d2abs(ux, 1) + _d2abs(uy, 0)))
    dphi = st["phi_new"].sum() - fl["phi"].sum()
    dc = st["c_new"].sum() - fl["c"].sum()
    if advection == 0:
        assert abs(drift_phi) > 1e-4  # the printed scheme really is non-conservative here
        assert abs(dphi - drift_phi) < 1e-11
        assert abs(dc - drift_c) < 1e-11
    else:
        assert abs(dphi) < 1e-11
        assert abs(dc) < 1e-11
    # the half step alone
    if advection == 0:
        assert abs(st["phi_h"].sum() - fl["phi"].sum() - drift_phi) < 1e-11


def test_surfactant_budget_with_source():
    w = c2_single_active(n=96)
    prm = dict(w.params, A0=2e-5, gamma=3e-3, c0=0.01)
    s = OracleSim(Params(nx=w.nx, ny=w.ny, **prm), w.phi0, w.c0, [Drop(**d) for d in w.drop_dicts()])
    s.run(7)
    st = s.stages()
    d = s.drops()[0]
    px, py = d.x + (d.R - d.Rs) * d.ex, d.y + (d.R - d.Rs) * d.ey
    y, x = np.mgrid[0:w.ny, 0:w.nx].astype(float)
    dx = (x - px + w.nx / 2) % w.nx - w.nx / 2
    dy = (y - py + w.ny / 2) % w.ny - w.ny / 2
    ntheta = int(np.sum(dx * dx + dy * dy <= d.Rs ** 2))
    assert ntheta > 15  # Rs = 2.8 at this size
    A = prm["A0"] * min(7, prm["t_star"])
    sch = st["c_h"].sum()
    N = w.nx * w.ny
    expect = sch - prm["gamma"] * (sch - N * prm["c0"]) + A * ntheta
    assert abs(st["c_new"].sum() - expect) < 1e-11


@pytest.mark.parametrize("centre,t_star", [((10.3, 7.6), 1e6), ((0.4, 13.2), 0.5), ((20.9, 0.2), 1e6)])
def test_source_disk_closed_form(centre, t_star):
    """phi = -1 and uniform c: no force, no flow, no phi >= 0 nodes (the centre stays put), so two
    steps are c1 = c - gamma (c - c0) and c2 = c1 - gamma (c1 - c0) + A0 min(1, t*) [|r - r_P| <= Rs]."""
    nx, ny = 23, 17
    gam, c0, A0, cbar = 0.05, 0.02, 0.01, 0.1
    p = Params(nx=nx, ny=ny, tau=1.0, a=-0.001, b=0.001, B0=0.006, B1=-0.05, D=0.1, Gamma=1.0,
               gamma=gam, A0=A0, c0=c0, t_star=t_star)
    th = 0.7
    drop = Drop(x=centre[0], y=centre[1], R=8.0, Rs=3.0, ex=np.cos(th), ey=np.sin(th), active=1)
    s = OracleSim(p, np.full((ny, nx), -1.0), np.full((ny, nx), cbar), [drop])
    s.run(1)
    c1 = cbar - gam * (cbar - c0)
    assert np.max(np.abs(s.fields()["c"] - c1)) < 1e-16
    s.run(1)
    px, py = centre[0] + 5.0 * np.cos(th), centre[1] + 5.0 * np.sin(th)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx = (x - px + nx / 2) % nx - nx / 2
    dy = (y - py + ny / 2) % ny - ny / 2
    inside = (dx * dx + dy * dy <= 9.0)
    c2 = c1 - gam * (c1 - c0) + A0 * min(1.0, t_star) * inside
    assert inside.sum() >= 25
    assert np.max(np.abs(s.fields()["c"] - c2)) < 1e-16
    # passive droplets carry no source
    drop.active = 0
    s = OracleSim(p, np.full((ny, nx), -1.0), np.full((ny, nx), cbar), [drop])
    s.run(2)
    assert np.max(np.abs(s.fields()["c"] - (c1 - gam * (c1 - c0)))) < 1e-16
