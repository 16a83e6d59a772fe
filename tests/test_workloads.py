"""The seeded input generators: the windowed droplet-field construction equals the direct definition (every
droplet's Eq. 20 profile evaluated at every node, nearest droplet wins, first one on ties) bit for bit."""
import numpy as np

from paper_1711_10984_amd import workloads as W


def _direct(nx, ny, drops, psi_out, xi, noise, seed):
    phi = np.full((ny, nx), -1.0)
    psi_in = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            best, k_best = np.inf, -1
            for k, d in enumerate(drops):
                dx = (i - d.x + 0.5 * nx) % nx - 0.5 * nx
                dy = (j - d.y + 0.5 * ny) % ny - 0.5 * ny
                r = np.hypot(dx, dy)
                if r < best:
                    best, k_best, bdx, bdy = r, k, dx, dy
            if k_best >= 0:
                d = drops[k_best]
                phi[j, i] = np.tanh(2.0 * (d.R - best) / xi)
                psi_in[j, i] = d.psi_front if bdx * d.ex + bdy * d.ey >= 0.0 else d.psi_back
    frac = 0.5 * (1.0 + phi)
    psi = psi_in * frac + psi_out * (1.0 - frac)
    psi = psi + np.random.default_rng(seed).uniform(-noise, noise, size=(ny, nx))
    return phi, psi


def test_windowed_droplet_fields_equal_direct_definition():
    rng = np.random.default_rng(11)
    nx, ny = 150, 110
    drops = [W.DropSpec(x=rng.uniform(0, nx), y=rng.uniform(0, ny), R=rng.uniform(2.0, 14.0), Rs=1.0,
                        ex=float(np.cos(k)), ey=float(np.sin(k)), active=1, psi_front=0.15, psi_back=0.05)
             for k in range(6)]
    drops.append(W.DropSpec(x=0.2, y=ny - 0.3, R=9.0, Rs=2.0, ex=0.0, ey=1.0))  # across both seams
    for xi in (2.0, 1.5):
        phi, psi = W.droplet_fields(nx, ny, drops, psi_out=0.02, xi=xi, seed=7)
        rphi, rpsi = _direct(nx, ny, drops, 0.02, xi, 0.005, 7)
        assert np.array_equal(phi, rphi) and np.array_equal(psi, rpsi)
