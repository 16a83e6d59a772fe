"""Test-side helpers: textbook D2Q9 constants and Fourier symbols of the discrete operators.

Used to build inputs and closed-form expectations; independent of both the oracle and
the HIP library.
"""
import numpy as np

# D2Q9 links in the public order rest, E, N, W, S, NE, NW, SW, SE.
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


def feq(n, ux, uy):
    """Textbook second-order D2Q9 equilibrium, cs^2 = 1/3, shape (9, ...)."""
    n, ux, uy = np.broadcast_arrays(np.asarray(n, float), np.asarray(ux, float), np.asarray(uy, float))
    out = np.empty((9,) + n.shape)
    usq = ux * ux + uy * uy
    for i in range(9):
        eu = EX[i] * ux + EY[i] * uy
        out[i] = WT[i] * n * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * usq)
    return out


def wavenumbers(ny, nx):
    ky = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    kx = 2 * np.pi * np.fft.fftfreq(nx)[None, :]
    return np.broadcast_arrays(kx, ky)


def sym_grad(ny, nx):
    """Fourier symbols (i*sx, i*sy) of the isotropic 9-point gradient."""
    kx, ky = wavenumbers(ny, nx)
    return 1j * np.sin(kx) * (2 + np.cos(ky)) / 3, 1j * np.sin(ky) * (2 + np.cos(kx)) / 3


def sym_lap(ny, nx):
    kx, ky = wavenumbers(ny, nx)
    return (8 * np.cos(kx) + 8 * np.cos(ky) + 4 * np.cos(kx) * np.cos(ky) - 20) / 6


def apply_symbol(g, s):
    return np.real(np.fft.ifft2(np.fft.fft2(g) * s))


def spec_grad(g):
    sx, sy = sym_grad(*g.shape)
    return apply_symbol(g, sx), apply_symbol(g, sy)


def spec_lap(g):
    return apply_symbol(g, sym_lap(*g.shape))


def moments(f):
    n = f.sum(0)
    mx = np.tensordot(EX, f, 1)
    my = np.tensordot(EY, f, 1)
    pxx = np.tensordot(EX * EX, f, 1)
    pxy = np.tensordot(EX * EY, f, 1)
    pyy = np.tensordot(EY * EY, f, 1)
    return n, mx, my, pxx, pxy, pyy


def mode_amplitude(field, kx_index, ky_index):
    """Complex amplitude of exp(i(kx x + ky y)) in a real field (ny, nx), normalised so that
    A cos(k.r + th) has amplitude A e^{i th}."""
    F = np.fft.fft2(field)
    ny, nx = field.shape
    return 2.0 * F[ky_index % ny, kx_index % nx] / (nx * ny)
