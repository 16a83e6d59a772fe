"""Pins of the oracle's bounding walls: plates halfway between node rows at y = -1/2 and y = ny - 1/2
(Sec. 2.2 names the walls, Sec. 2.3 fixes neutral wetting, n.grad mu_phi = n.grad mu_c = 0; the reading,
halfway bounce-back plus mirror ghosts, is stated in the oracle's header).

* Mirror equivalence: a state that is invariant and symmetric in x evolves between the plates exactly as
  rows 0..L-1 of the 2L-periodic lattice whose initial data are mirrored about y = -1/2.  For such states
  halfway bounce-back coincides with periodic streaming across the mirror plane, and every mirror ghost
  with the real neighbour; equality is bitwise because the arithmetic is exactly y-reflection symmetric.
* No slip: the slowest shear mode between the plates, u_x = U sin(pi (y + 1/2) / L), decays at
  nu (pi / L)^2 with nu = (tau - 1/2)/3 (Eq. 15; Stokes flow between plates).
* Conservation with x- and y-varying states: bounce-back keeps sum f; the mirror ghosts give no
  diffusive flux through the plates and the reversed ghost velocity no advective flux in the flux form,
  so sum phi and sum c are kept without source and consumption.
* The two plates are treated alike: a state symmetric about the mid-plane stays symmetric, bitwise.
"""
import numpy as np
import pytest

from oracle import OracleSim, Params
from lbhelpers import feq
from paper_1711_10984_amd import workloads as W

REFL_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]  # direction i -> its mirror image under y -> -y
FIELDS = ("f", "phi", "c", "n", "ux", "uy")


def _params(nx, ny, walls, advection=0, **kw):
    d = dict(W.ACTIVE, nx=nx, ny=ny, walls=walls, advection=advection, tau=0.8, Gamma=0.7, A0=0.0, gamma=0.0)
    d.update(kw)
    return Params(**{k: v for k, v in d.items() if k in Params.__dataclass_fields__})


def _mirror_rows(a, f_like=False):
    """Rows 0..L-1 followed by their mirror image about y = L - 1/2 (directions reflected for f)."""
    if f_like:
        return np.concatenate([a, a[REFL_Y][:, ::-1, :]], axis=1)
    return np.concatenate([a, a[::-1, :]], axis=0)


def _x_invariant_state(nx, L, seed):
    rng = np.random.default_rng(seed)
    phi = np.repeat(rng.uniform(-0.9, 0.9, size=(L, 1)), nx, axis=1)
    c = np.repeat(0.1 + rng.uniform(-0.04, 0.04, size=(L, 1)), nx, axis=1)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    prof = w[:, None] * (1.0 + rng.uniform(-0.02, 0.02, size=(9, L)))
    prof[3], prof[6], prof[7] = prof[1], prof[5], prof[8]  # symmetric in x: W = E, NW = NE, SW = SE
    f = np.repeat(prof[:, :, None], nx, axis=2)
    return np.ascontiguousarray(f), np.ascontiguousarray(phi), np.ascontiguousarray(c)


@pytest.mark.parametrize("advection", [0, 1])
def test_mirror_equivalence_with_doubled_periodic_lattice(advection):
    nx, L = 6, 13
    f, phi, c = _x_invariant_state(nx, L, seed=5)
    walled = OracleSim(_params(nx, L, 1, advection), phi, c, [], f_pre=f)
    doubled = OracleSim(_params(nx, 2 * L, 0, advection), np.ascontiguousarray(_mirror_rows(phi)),
                        np.ascontiguousarray(_mirror_rows(c)), [], f_pre=np.ascontiguousarray(_mirror_rows(f, True)))
    for _ in range(3):
        walled.run(15)
        doubled.run(15)
        a, b = walled.fields(), doubled.fields()
        for k in FIELDS:
            bk = b[k][:, :L, :] if k == "f" else b[k][:L, :]
            assert np.array_equal(a[k], bk), (k, float(np.max(np.abs(a[k] - bk))))


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_channel_shear_mode_decays_at_nu_k2(tau):
    nx, L = 4, 32
    k = np.pi / L
    y = np.arange(L)[:, None] * np.ones((1, nx))
    U = 1e-4
    f = feq(np.ones((L, nx)), U * np.sin(k * (y + 0.5)), np.zeros((L, nx)))
    p = Params(nx=nx, ny=L, tau=tau, a=0.0, b=0.0, B0=0.0, B1=0.0, D=0.0, Gamma=1.0, walls=1)
    s = OracleSim(p, np.zeros((L, nx)), np.full((L, nx), 0.1), [], f_pre=np.ascontiguousarray(f))
    mode = np.sin(k * (np.arange(L) + 0.5))

    def amp():
        return 2.0 / L * np.sum(s.fields()["ux"][:, 0] * mode)

    s.run(200)
    a1 = amp()
    s.run(2000)
    a2 = amp()
    nu = -np.log(a2 / a1) / (k * k * 2000)
    print(f"tau {tau}: measured nu / (tau - 1/2)/3 = {nu / ((tau - 0.5) / 3):.5f}")
    assert abs(nu / ((tau - 0.5) / 3) - 1) < 0.02
    # the flow never crosses the plates: no y-velocity develops
    assert np.max(np.abs(s.fields()["uy"])) < 1e-12


@pytest.mark.parametrize("advection", [1])
def test_sums_conserved_between_plates(advection):
    nx, ny = 23, 17
    f, phi, c = W.random_state(nx, ny, seed=8, phi_amp=0.5)
    s = OracleSim(_params(nx, ny, 1, advection), phi, c, [], f_pre=f)
    o0 = s.observables()
    s.run(30)
    o1 = s.observables()
    N = nx * ny
    assert abs(o1["mass"] - o0["mass"]) < 1e-13 * N
    assert abs(o1["sum_phi"] - o0["sum_phi"]) < 1e-12 * N
    assert abs(o1["sum_c"] - o0["sum_c"]) < 1e-12 * N


def test_plates_are_treated_alike():
    nx, ny = 11, 14
    f, phi, c = W.random_state(nx, ny, seed=9, phi_amp=0.5)
    half = ny // 2
    phi = np.ascontiguousarray(_mirror_rows(phi[:half]))
    c = np.ascontiguousarray(_mirror_rows(c[:half]))
    f = np.ascontiguousarray(_mirror_rows(f[:, :half], True))
    s = OracleSim(_params(nx, ny, 1, 0), phi, c, [], f_pre=f)
    s.run(25)
    F = s.fields()
    for k in ("phi", "c", "n", "ux"):
        assert np.array_equal(F[k], F[k][::-1]), k
    assert np.array_equal(F["uy"], -F["uy"][::-1])
    assert np.array_equal(F["f"], F["f"][REFL_Y][:, ::-1])
