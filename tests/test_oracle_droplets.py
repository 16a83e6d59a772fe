"""Pins of the oracle's droplet bookkeeping and observables against closed forms (Sec. 4).

* Centre of mass of several droplets: r_CM = sum phi r / sum phi over phi >= 0, each node assigned to the
  nearest previous centre (minimum image, ties to the lowest droplet index), offsets unwrapped about that
  centre, the new centre wrapped back into the lattice.  Disks whose node sets are point-symmetric about a
  node have their centre there whatever the weights; one disk straddles both periodic edges of a
  non-square lattice, and one node lies exactly halfway between two previous centres.
* Observables at time n: with a = b = B0 = B1 = 0 and uniform c the thermodynamic force vanishes
  identically, so populations at equilibrium f^eq(n0, u) carry exactly the velocity u.  A uniform u gives
  v_CM = u for every droplet and max|u| = |u|; a velocity odd about a droplet's symmetry axis gives zero
  there.  sum n = N n0, sum phi and sum c follow from the node counts and the Fourier sums of the fields;
  min B(c) = B0 + B1 max c for B1 < 0 and B0 + B1 min c for B1 > 0.
"""
import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from tests.lbhelpers import feq


def _disk_nodes(nx, ny, cx, cy, r2):
    """Nodes (x, y) within squared distance r2 (minimum image) of the node (cx, cy); integer arithmetic."""
    out = []
    for y in range(ny):
        for x in range(nx):
            dx = (x - cx + nx // 2) % nx - nx // 2
            dy = (y - cy + ny // 2) % ny - ny // 2
            if dx * dx + dy * dy <= r2:
                out.append((x, y))
    return out


def _minimg(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def test_several_droplets_nearest_previous_centre_ties_and_edges():
    nx, ny = 40, 30
    phi = np.full((ny, nx), -1.0)
    corner = _disk_nodes(nx, ny, 0, 0, 12)          # straddles x = 0 and y = 0
    left = _disk_nodes(nx, ny, 12, 15, 9)
    right = _disk_nodes(nx, ny, 22, 15, 9)
    for x, y in corner + left + right:
        phi[y, x] = 0.8
    phi[15, 17] = 0.5   # halfway between the previous centres (12, 15) and (22, 15): a tie
    phi[4, 30] = 0.0    # phi = 0 belongs to a droplet but weighs nothing
    phi[5, 30] = -1e-9  # phi < 0 is outside every droplet
    assert len(left) == len(right) == 29 and len(corner) == 37
    drops = [Drop(x=39.0, y=29.5, R=4.0), Drop(x=12.0, y=15.0, R=3.0), Drop(x=22.0, y=15.0, R=3.0)]
    s = OracleSim(Params(nx=nx, ny=ny), phi, np.zeros((ny, nx)), drops)
    got = s.drops()
    # the corner disk is symmetric about the node (0, 0): its centre is there, wrapped into [0, L)
    assert 0.0 <= got[0].x < nx and 0.0 <= got[0].y < ny
    assert abs(_minimg(got[0].x, nx)) < 1e-12 and abs(_minimg(got[0].y, ny)) < 1e-12
    # the tie goes to the lower index: droplet 1 takes the bridge node, droplet 2 keeps its symmetric disk
    m = 0.8 * len(left)
    assert abs(got[1].x - (12.0 + 0.5 * 5.0 / (m + 0.5))) < 1e-13
    assert abs(got[1].y - 15.0) < 1e-13
    assert abs(got[2].x - 22.0) < 1e-13 and abs(got[2].y - 15.0) < 1e-13
    # listed in the other order, the other droplet (again the lower index) takes the bridge node
    s = OracleSim(Params(nx=nx, ny=ny), phi, np.zeros((ny, nx)), [drops[0], drops[2], drops[1]])
    got = s.drops()
    assert abs(got[1].x - (22.0 - 0.5 * 5.0 / (m + 0.5))) < 1e-13
    assert abs(got[2].x - 12.0) < 1e-13


def test_assignment_uses_the_previous_centres():
    """A node nearer to droplet 0's previous centre than to droplet 1's belongs to droplet 0, although it is
    nearer to droplet 1's disk: the new centres follow from the assignment, not the other way round."""
    nx, ny = 36, 20
    phi = np.full((ny, nx), -1.0)
    a = _disk_nodes(nx, ny, 8, 10, 4)
    b = _disk_nodes(nx, ny, 24, 10, 4)
    for x, y in a + b:
        phi[y, x] = 1.0
    phi[10, 18] = 1.0   # distance 4 to the previous centre (14, 10) of droplet 0, 6 to (24, 10)
    s = OracleSim(Params(nx=nx, ny=ny), phi, np.zeros((ny, nx)),
                  [Drop(x=14.0, y=10.0, R=2.0), Drop(x=24.0, y=10.0, R=2.0)])
    got = s.drops()
    na = len(a)
    assert abs(got[0].x - (na * 8.0 + 18.0) / (na + 1)) < 1e-13
    assert abs(got[1].x - 24.0) < 1e-13


def _still_params(nx, ny, **kw):
    """a = b = B0 = B1 = 0: mu = 0 and X = 0, so the force is -grad c, zero for uniform c."""
    d = dict(nx=nx, ny=ny, tau=0.8, a=0.0, b=0.0, B0=0.0, B1=0.0, D=0.1, Gamma=1.0)
    d.update(kw)
    return Params(**d)


def _two_disks(nx, ny):
    phi = np.full((ny, nx), -1.0)
    d0 = _disk_nodes(nx, ny, 9, 8, 10)
    d1 = _disk_nodes(nx, ny, 25, 16, 16)
    for x, y in d0:
        phi[y, x] = 0.8
    for x, y in d1:
        phi[y, x] = 0.6
    return phi, d0, d1


def test_observables_uniform_velocity():
    nx, ny = 36, 24
    U, V, n0, cbar = 0.031, -0.017, 1.3, 0.07
    phi, d0, d1 = _two_disks(nx, ny)
    f = feq(np.full((ny, nx), n0), np.full((ny, nx), U), np.full((ny, nx), V))
    s = OracleSim(_still_params(nx, ny), phi, np.full((ny, nx), cbar),
                  [Drop(x=9.0, y=8.0, R=3.0), Drop(x=25.0, y=16.0, R=4.0)], f_pre=f)
    ob = s.observables()
    N = nx * ny
    assert abs(ob["mass"] - N * n0) < 1e-12 * N
    n_in0, n_in1 = len(d0), len(d1)
    assert abs(ob["sum_phi"] - (0.8 * n_in0 + 0.6 * n_in1 - (N - n_in0 - n_in1))) < 1e-12 * N
    assert abs(ob["sum_c"] - N * cbar) < 1e-14 * N
    assert abs(ob["max_u"] - np.hypot(U, V)) < 1e-15
    assert np.max(np.abs(ob["vel"] - np.array([[U, V], [U, V]]))) < 1e-15
    assert abs(ob["drop_mass"][0] - 0.8 * n_in0) < 1e-12 and abs(ob["drop_mass"][1] - 0.6 * n_in1) < 1e-12
    assert not ob["nonfinite"]
    assert ob["min_B"] == 0.0


def test_observables_odd_velocity_and_extremes():
    """u_x = U sin(2 pi (y - 8) / ny): odd about droplet 0's row, so its v_x vanishes; max|u| = U at the rows
    a quarter period away (ny divisible by 4).  c = cbar + eps cos(2 pi x / nx): sum c = N cbar, and min B
    is reached at the largest c (B1 < 0) or the smallest (B1 > 0)."""
    nx, ny = 36, 24
    U = 0.02
    phi, d0, d1 = _two_disks(nx, ny)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    ux = U * np.sin(2 * np.pi * (y - 8) / ny)
    f = feq(np.ones((ny, nx)), ux, np.zeros((ny, nx)))
    s = OracleSim(_still_params(nx, ny), phi, np.full((ny, nx), 0.05),
                  [Drop(x=9.0, y=8.0, R=3.0), Drop(x=25.0, y=16.0, R=4.0)], f_pre=f)
    ob = s.observables()
    assert abs(ob["vel"][0, 0]) < 1e-16 and ob["vel"][0, 1] == 0.0
    assert ob["vel"][1, 0] > 1e-3  # droplet 1 sits where u_x > 0
    assert abs(ob["max_u"] - U) < 1e-16
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    cbar, eps = 0.1, 0.03
    c = cbar + eps * np.cos(2 * np.pi * x / nx)
    for B0, B1, cext in ((0.01, -0.05, cbar + eps), (0.01, 0.05, cbar - eps)):
        s = OracleSim(Params(nx=nx, ny=ny, B0=B0, B1=B1), phi, c, [Drop(x=9.0, y=8.0, R=3.0)])
        ob = s.observables()
        assert abs(ob["min_B"] - (B0 + B1 * cext)) < 1e-17
        assert abs(ob["sum_c"] - nx * ny * cbar) < 1e-12


def test_observables_flag_nonfinite_values():
    nx, ny = 12, 10
    phi, c = np.full((ny, nx), -1.0), np.full((ny, nx), 0.1)
    f = feq(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    assert not OracleSim(Params(nx=nx, ny=ny), phi, c, f_pre=f).observables()["nonfinite"]
    f[5, 3, 4] = np.inf
    assert OracleSim(Params(nx=nx, ny=ny), phi, c, f_pre=f).observables()["nonfinite"]
    c[2, 2] = np.nan
    assert OracleSim(Params(nx=nx, ny=ny), phi, c).observables()["nonfinite"]
