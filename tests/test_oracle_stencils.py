"""Pins of the oracle's discrete operators against their Fourier symbols (closed forms).

The isotropic 9-point gradient sum_i (w_i/cs^2) e_i g(r+e_i) has symbol
i sin(kx)(2+cos ky)/3 along x; the 9-point Laplacian has symbol
(8 cos kx + 8 cos ky + 4 cos kx cos ky - 20)/6 (D2Q9 weights, Sec. 2.2).  A swapped
axis, a wrong sign or a wrong neighbour index changes the symbol and fails here.
"""
import numpy as np
import pytest

from oracle import grad9, lap9, div9
from tests.lbhelpers import spec_grad, spec_lap, sym_grad, sym_lap, wavenumbers

SHAPES = [(8, 8), (6, 10), (9, 7), (3, 5), (16, 12)]


@pytest.mark.parametrize("shape", SHAPES)
def test_grad9_symbol(shape):
    rng = np.random.default_rng(1)
    g = rng.standard_normal(shape)
    gx, gy = grad9(g)
    ex, ey = spec_grad(g)
    assert np.max(np.abs(gx - ex)) < 1e-13
    assert np.max(np.abs(gy - ey)) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
def test_lap9_symbol(shape):
    rng = np.random.default_rng(2)
    g = rng.standard_normal(shape)
    assert np.max(np.abs(lap9(g) - spec_lap(g))) < 1e-13


def test_plane_wave_eigenfunction():
    """A single plane wave cos(k.r) is an eigenfunction of the Laplacian with eigenvalue
    lambda(k), and its gradient is -s(k) sin(k.r)."""
    ny, nx = 12, 8
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for mx_, my_ in [(1, 0), (0, 1), (1, 2), (3, 5), (4, 6)]:
        kx, ky = 2 * np.pi * mx_ / nx, 2 * np.pi * my_ / ny
        g = np.cos(kx * x + ky * y + 0.3)
        lam = (8 * np.cos(kx) + 8 * np.cos(ky) + 4 * np.cos(kx) * np.cos(ky) - 20) / 6
        assert np.allclose(lap9(g), lam * g, atol=1e-13)
        gx, gy = grad9(g)
        sx = np.sin(kx) * (2 + np.cos(ky)) / 3
        sy = np.sin(ky) * (2 + np.cos(kx)) / 3
        assert np.allclose(gx, -sx * np.sin(kx * x + ky * y + 0.3), atol=1e-13)
        assert np.allclose(gy, -sy * np.sin(kx * x + ky * y + 0.3), atol=1e-13)


def test_small_k_limits():
    """Second-order consistency: s(k) = k + O(k^3), lambda(k) = -|k|^2 + O(k^4)."""
    for k in [1e-2, 2e-2]:
        sx = np.sin(k) * 3 / 3
        lam = (8 * np.cos(k) + 8 + 4 * np.cos(k) - 20) / 6
        assert abs(sx - k) < k ** 3
        assert abs(lam + k * k) < k ** 4


@pytest.mark.parametrize("shape", [(8, 8), (7, 9)])
def test_div9_product_rule(shape):
    """Div(k, X) = 1/2 [lap(kX) - X lap(k) + k lap(X)] holds exactly for the link form
    sum_i (2w_i/cs^2)(k+k_i)/2 (X_i - X); with the Laplacian pinned above this pins Div."""
    rng = np.random.default_rng(3)
    k = 1 + 0.3 * rng.standard_normal(shape)
    X = rng.standard_normal(shape)
    lhs = div9(k, X)
    rhs = 0.5 * (spec_lap(k * X) - X * spec_lap(k) + k * spec_lap(X))
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_div9_constant_coefficient_and_conservation():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((10, 6))
    k = np.full_like(X, 0.37)
    assert np.max(np.abs(div9(k, X) - 0.37 * spec_lap(X))) < 1e-13
    kv = 1 + rng.random(X.shape)
    # telescoping link fluxes: the total is zero
    assert abs(div9(kv, X).sum()) < 1e-12
    # no flux for uniform X
    assert np.max(np.abs(div9(kv, np.full_like(X, 2.5)))) == 0.0
