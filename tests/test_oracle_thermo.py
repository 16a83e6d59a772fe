"""Pins of the chemical potential and the thermodynamic force against the paper's other formulas.

* mu_phi (Eq. 3) is the variational derivative of the free energy (Eq. 1):
  mu = a phi + b phi^3 - div(B(c) grad phi), with B(c) = B0 + B1 c.
* The force density of Eq. (14), F = -phi grad mu_phi - c grad mu_c, equals -div P of the non-ideal
  pressure tensor P_ab = p0' delta_ab + B(c) d_a phi d_b phi with p0' given by Eq. (9)
  (without the ideal-gas part p^i).
Both sides are compared on smooth, long-wavelength fields, where the 9-point stencils agree with the
continuum derivatives (evaluated spectrally) up to their O(k^2) truncation; every term is made
comparable in size so that a wrong sign or a missing term fails.
"""
import numpy as np

from oracle import OracleSim, Params


def _spectral(ny, nx):
    ky = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    kx = 2 * np.pi * np.fft.fftfreq(nx)[None, :]

    def dx(g):
        return np.real(np.fft.ifft2(np.fft.fft2(g) * 1j * kx))

    def dy(g):
        return np.real(np.fft.ifft2(np.fft.fft2(g) * 1j * ky))

    return dx, dy


def _smooth_state(L=128):
    y, x = np.mgrid[0:L, 0:L].astype(float)
    k = 2 * np.pi / L
    phi = 0.8 * np.sin(k * x + 0.3) * np.cos(k * y) + 0.3 * np.cos(2 * k * y + 0.7)
    c = 0.2 + 0.1 * np.cos(k * x - 0.4) * np.sin(k * y + 0.2) + 0.05 * np.sin(2 * k * x)
    return phi, c


PRM = dict(tau=1.0, a=-0.01, b=0.02, B0=6.0, B1=-15.0, D=0.1, Gamma=1.0)


def test_mu_is_variational_derivative():
    L = 128
    phi, c = _smooth_state(L)
    st = OracleSim(Params(nx=L, ny=L, **PRM), phi, c).stages()
    dx, dy = _spectral(L, L)
    B = PRM["B0"] + PRM["B1"] * c
    mu_ref = PRM["a"] * phi + PRM["b"] * phi ** 3 - (dx(B * dx(phi)) + dy(B * dy(phi)))
    scale = np.max(np.abs(mu_ref))
    term = np.max(np.abs(PRM["B1"] * (dx(c) * dx(phi) + dy(c) * dy(phi))))
    assert term > 0.1 * scale  # a sign error in this term would exceed the tolerance 60-fold
    assert np.max(np.abs(st["mu"] - mu_ref)) < 3e-3 * scale
    X_ref = 0.5 * PRM["B1"] * (dx(phi) ** 2 + dy(phi) ** 2)
    assert np.max(np.abs(st["X"] - X_ref)) < 3e-3 * np.max(np.abs(X_ref))


def test_force_is_minus_divergence_of_pressure_tensor():
    L = 128
    phi, c = _smooth_state(L)
    st = OracleSim(Params(nx=L, ny=L, **PRM), phi, c).stages()
    dx, dy = _spectral(L, L)
    a, b, B0, B1 = PRM["a"], PRM["b"], PRM["B0"], PRM["B1"]
    B = B0 + B1 * c
    px, py = dx(phi), dy(phi)
    lap = dx(px) + dy(py)
    # Eq. (9) without the ideal-gas term
    p0 = (a / 2 * phi ** 2 + 3 * b / 4 * phi ** 4 - B * phi * lap - B1 * phi * (dx(c) * px + dy(c) * py)
          + c - B0 / 2 * (px * px + py * py))
    # Eq. (8): P_ab = p0 delta_ab + B d_a phi d_b phi ; F_a = -d_b P_ab (Eq. 14)
    Fx_ref = -(dx(p0) + dx(B * px * px) + dy(B * px * py))
    Fy_ref = -(dy(p0) + dx(B * py * px) + dy(B * py * py))
    scale = max(np.max(np.abs(Fx_ref)), np.max(np.abs(Fy_ref)))
    assert np.max(np.abs(st["Fx"] - Fx_ref)) < 5e-3 * scale
    assert np.max(np.abs(st["Fy"] - Fy_ref)) < 5e-3 * scale
    # the surfactant's own pressure and the B1 terms matter at this tolerance
    assert np.max(np.abs(dx(c))) > 0.05 * scale


def test_bracket_M_equals_mu_at_rest():
    """With populations whose momentum cancels half the force, u = 0, the half step leaves phi and c
    unchanged and the bracket M of Eq. (18) is mu_phi of Eq. (3) (b phi^3 is taken at time n anyway)."""
    from tests.lbhelpers import EX, EY, WT

    L = 128
    phi, c = _smooth_state(L)
    p = Params(nx=L, ny=L, **PRM)
    st0 = OracleSim(p, phi, c).stages()
    mx, my = -0.5 * st0["Fx"], -0.5 * st0["Fy"]
    f = np.stack([WT[i] * (1 + 3 * (EX[i] * mx + EY[i] * my)) for i in range(9)])
    st = OracleSim(p, phi, c, f_pre=f).stages()
    assert np.max(np.abs(st["ux"])) < 1e-15 and np.max(np.abs(st["uy"])) < 1e-15
    scale = np.max(np.abs(st["mu"]))
    assert np.max(np.abs(st["M"] - st["mu"])) < 1e-12 * scale
    assert np.max(np.abs(st["X_h"] - st["X"])) < 1e-12 * np.max(np.abs(st["X"]))
