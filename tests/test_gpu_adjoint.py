"""Reverse mode (lbm_adjoint_forward / lbm_adjoint_backward): derivative of a droplet's centre-of-mass
x-displacement with respect to the production rate A0 and the initial surfactant field.

Checks, all against central finite differences of the forward map (the adjoint holds the production-disk
membership, the upwind sides and the droplet masks fixed; a perturbation of 1e-6 moves none of them here):
* C4 workload (256^2 active droplet, 2000 steps, checkpoints every 100): 16 seeded nodes of dJ/dpsi and
  dJ/dA0 against FP64 differences of the GPU forward path, step 1e-6 (relative 1e-3 x A0 for A0);
* the oracle's own differences on a smaller active droplet: dJ/dA0 and two random directional derivatives of
  dJ/dpsi (independent of the GPU's forward arithmetic).  The directions are supported near the droplet: a
  perturbation of the whole field also moves u where it is close to zero far from the droplet, flips upwind
  sides there, and the differences then see the kinks of the piecewise-smooth map (they converge to the
  adjoint only erratically, 1e-4 .. 1e-2 at h = 1e-4 .. 1e-7 for such directions, against 2e-6 at h = 1e-6
  for directions near the droplet);
* between plates: J, dJ/dA0 and dJ/dpsi at nodes on and next to both plates against the oracle's
  differences, on all three paths;
* the same on a 70 x 37 lattice, periodic and between plates, whose sides are not multiples of the adjoint
  kernels' tiles;
* FP32 adjoint against the FP64 one, periodic and between plates; the torch.autograd wrapper; the state is restored and a second
  backward pass repeats the first bit for bit; the checkpoint interval and the kernel path leave the gradients
  unchanged bit for bit.
"""
import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from paper_1711_10984_amd import workloads as W

pytestmark = pytest.mark.gpu


def _minimg(d, L):
    return (d + 0.5 * L) % L - 0.5 * L


def gpu_J(w, c0, A0=None, nsteps=2000, precision=0):
    from paper_1711_10984_amd import lbm
    p = w.param_dict() if A0 is None else dict(w.param_dict(), A0=A0)
    s = lbm.Sim([p], [w.phi0], [c0], [w.drop_dicts()], precision=precision, graph_steps=20)
    x0 = s.droplets()[0]["x"]
    s.step(nsteps)
    J = _minimg(s.droplets()[0]["x"] - x0, w.nx)
    s.close()
    return J


def adjoint(w, nsteps, every, precision=0, path=0):
    from paper_1711_10984_amd import lbm
    s = lbm.Sim([w.param_dict()], [w.phi0], [w.c0], [w.drop_dicts()], precision=precision, graph_steps=20,
                path=path)
    J = s.adjoint_forward(0, nsteps, every)
    dA0, dc0 = s.adjoint_backward()
    return s, J, dA0, dc0


def seeded_nodes(w, n=16, seed=44):
    rng = np.random.default_rng(seed)
    d = w.drops[0]
    out = []
    while len(out) < n // 2:  # half of them in and around the droplet
        x, y = rng.integers(0, w.nx), rng.integers(0, w.ny)
        if np.hypot(_minimg(x - d.x, w.nx), _minimg(y - d.y, w.ny)) < 1.5 * d.R:
            out.append((int(y), int(x)))
    while len(out) < n:
        out.append((int(rng.integers(0, w.ny)), int(rng.integers(0, w.nx))))
    return out


def test_c4_gradients_against_fp64_differences():
    w = W.c2_single_active()
    N, h = 2000, 1e-6
    s, J, dA0, dc0 = adjoint(w, N, 100)
    assert abs(J - gpu_J(w, w.c0, nsteps=N)) == 0.0  # the recorded forward pass is the ordinary run
    s.close()
    fd = []
    for (y, x) in seeded_nodes(w):
        cp, cm = w.c0.copy(), w.c0.copy()
        cp[y, x] += h
        cm[y, x] -= h
        fd.append((gpu_J(w, cp, nsteps=N) - gpu_J(w, cm, nsteps=N)) / (2 * h))
    ad = np.array([dc0[y, x] for (y, x) in seeded_nodes(w)])
    fd = np.array(fd)
    print("dJ/dpsi adjoint", ad, "\ndJ/dpsi differences", fd)
    scale = np.max(np.abs(fd))
    assert scale > 0
    assert np.max(np.abs(ad - fd)) <= 1e-4 * scale + 1e-7
    A0 = w.params["A0"]
    hA = 1e-3 * A0
    fdA = (gpu_J(w, w.c0, A0 + hA, N) - gpu_J(w, w.c0, A0 - hA, N)) / (2 * hA)
    print("dJ/dA0 adjoint", dA0, "differences", fdA)
    assert abs(dA0 - fdA) <= 1e-4 * abs(fdA)


def _oracle_J(w, c0, A0, nsteps):
    p = dict(w.params, A0=A0)
    o = OracleSim(Params(nx=w.nx, ny=w.ny, **p), w.phi0, c0, [Drop(**d) for d in w.drop_dicts()])
    x0 = o.drops()[0].x
    o.run(nsteps)
    return _minimg(o.drops()[0].x - x0, w.nx)


@pytest.mark.parametrize("path", [0, 2])
def test_gradients_against_oracle_differences(path):
    w = W.c2_single_active(n=64, seed=45)
    w.params["A0"] = 2e-6  # a production rate that moves the droplet within the short run
    N = 200
    s, J, dA0, dc0 = adjoint(w, N, 50, path=path)
    s.close()
    A0 = w.params["A0"]
    assert abs(J - _oracle_J(w, w.c0, A0, N)) < 1e-12
    hA = 1e-3 * A0
    fdA = (_oracle_J(w, w.c0, A0 + hA, N) - _oracle_J(w, w.c0, A0 - hA, N)) / (2 * hA)
    print("dJ/dA0 adjoint", dA0, "oracle differences", fdA)
    assert abs(dA0 - fdA) <= 1e-5 * abs(fdA)
    rng = np.random.default_rng(46)
    h = 1e-6
    d = w.drops[0]
    yy, xx = np.mgrid[0:w.ny, 0:w.nx]
    near = np.hypot(_minimg(xx - d.x, w.nx), _minimg(yy - d.y, w.ny)) < 12
    for _ in range(2):
        v = np.where(near, rng.uniform(-1.0, 1.0, size=w.c0.shape), 0.0)
        fd = (_oracle_J(w, w.c0 + h * v, A0, N) - _oracle_J(w, w.c0 - h * v, A0, N)) / (2 * h)
        ad = float(np.sum(dc0 * v))
        print("directional derivative adjoint", ad, "oracle differences", fd)
        assert abs(ad - fd) <= 2e-5 * abs(fd) + 1e-9


def _near_wall_workload():
    """A droplet of radius 10 three nodes from the lower plate (64 x 40, plates at y = -1/2 and 39.5), production
    on the +x side, surfactant 0.1 everywhere."""
    d = W.DropSpec(x=32.0, y=13.0, R=10.0, Rs=2.5, ex=1.0, ey=0.0, active=1, psi_front=0.1, psi_back=0.1)
    phi, psi = W.droplet_fields(64, 40, [d], psi_out=0.1, seed=51)
    params = dict(W.PAPER_EQUILIBRIUM, tau=0.6, gamma=1.5e-3, A0=2e-6, walls=1)
    return W.Workload("plates_64x40_near_wall", 64, 40, params, phi, psi, [d])


@pytest.mark.parametrize("path", [0, 1, 2])
def test_walls_gradients_against_oracle_differences(path):
    """Reverse mode between plates: J agrees with the oracle's forward run; dJ/dA0 and dJ/dc(n0) at single
    nodes agree with the oracle's central differences.  The nodes include both plate rows and the rows next to
    them, below the droplet and far from it, so the mirror and bounce-back transposes are exercised.  Single
    nodes, not random directions: the fluid is nearly at rest along the plates, and a direction spread over
    many nodes there flips upwind sides within h = 1e-5 (single-node differences agree to 1e-5 between
    h = 1e-6 and 1e-7)."""
    w = _near_wall_workload()
    N = 200
    s, J, dA0, dc0 = adjoint(w, N, 50, path=path)
    s.close()
    A0 = w.params["A0"]
    assert abs(J - _oracle_J(w, w.c0, A0, N)) < 1e-12
    # steps of 1e-3 A0 and more flip upwind sides along the plates (the differences move by 1 % between
    # steps of 1e-3 and 3e-3 A0); at 1e-4 and 1e-5 A0 they agree with each other to 1e-15
    hA = 1e-4 * A0
    fdA = (_oracle_J(w, w.c0, A0 + hA, N) - _oracle_J(w, w.c0, A0 - hA, N)) / (2 * hA)
    print("walls: dJ/dA0 adjoint", dA0, "oracle differences", fdA)
    assert abs(dA0 - fdA) <= 1e-5 * abs(fdA)
    h = 1e-6
    for y, x in ((0, 32), (1, 32), (2, 30), (0, 5), (39, 32), (38, 20), (13, 42), (13, 22)):
        v = np.zeros_like(w.c0)
        v[y, x] = 1.0
        fd = (_oracle_J(w, w.c0 + h * v, A0, N) - _oracle_J(w, w.c0 - h * v, A0, N)) / (2 * h)
        print("walls: dJ/dc", (y, x), "adjoint", dc0[y, x], "oracle differences", fd)
        assert abs(dc0[y, x] - fd) <= 2e-5 * abs(fd) + 1e-9


def _ragged_workload(walls):
    """A 70 x 37 lattice, so that the adjoint kernels' 64 x 4 tiles are ragged in both directions (a second tile
    column of 6 nodes, a last tile row of 1), with a radius-8 droplet across the tile boundary at x = 63 | 64 and,
    without walls, across the periodic edge in y (with plates it sits two nodes above the lower one)."""
    y = 33.0 if walls == 0 else 10.0
    d = W.DropSpec(x=62.0, y=y, R=8.0, Rs=2.0, ex=1.0, ey=0.0, active=1, psi_front=0.1, psi_back=0.1)
    phi, psi = W.droplet_fields(70, 37, [d], psi_out=0.1, seed=52 + walls)
    params = dict(W.PAPER_EQUILIBRIUM, tau=0.6, gamma=1.5e-3, A0=2e-6, walls=walls)
    return W.Workload(f"ragged_70x37_walls{walls}", 70, 37, params, phi, psi, [d])


# Single nodes on the ragged tile edges (x = 64 .. 69, the last row), on both sides of the tile boundary
# x = 63 | 64, near the droplet and far from it.  Only nodes where the oracle's own differences at h = 1e-6 and
# 1e-7 agree to 5e-6: the map is piecewise smooth (upwind sides flip where u is near 0, as inside a droplet
# between plates), and there the differences do not converge to the derivative.
RAGGED_NODES = {0: ((36, 64), (36, 69), (0, 69), (0, 64), (36, 63), (33, 68), (28, 64), (1, 64), (20, 10)),
                1: ((36, 69), (0, 69), (0, 64), (5, 64), (3, 66), (13, 69), (10, 69))}


@pytest.mark.parametrize("walls,path", [(0, 2), (1, 0)])
def test_ragged_tiles_against_oracle_differences(walls, path):
    """Reverse mode on a lattice whose sides are not multiples of the adjoint kernels' tile (64 x 4): J agrees
    with the oracle's forward run; dJ/dA0 and dJ/dc(n0) at the nodes of RAGGED_NODES agree with the oracle's
    central differences (the bounds of the test between plates)."""
    w = _ragged_workload(walls)
    N = 200
    s, J, dA0, dc0 = adjoint(w, N, 50, path=path)
    s.close()
    A0 = w.params["A0"]
    assert abs(J - _oracle_J(w, w.c0, A0, N)) < 1e-12
    hA = 1e-4 * A0
    fdA = (_oracle_J(w, w.c0, A0 + hA, N) - _oracle_J(w, w.c0, A0 - hA, N)) / (2 * hA)
    print("ragged: dJ/dA0 adjoint", dA0, "oracle differences", fdA)
    assert abs(dA0 - fdA) <= 1e-5 * abs(fdA)
    h = 1e-6
    for y, x in RAGGED_NODES[walls]:
        v = np.zeros_like(w.c0)
        v[y, x] = 1.0
        fd = (_oracle_J(w, w.c0 + h * v, A0, N) - _oracle_J(w, w.c0 - h * v, A0, N)) / (2 * h)
        print("ragged: dJ/dc", (y, x), "adjoint", dc0[y, x], "oracle differences", fd)
        assert abs(dc0[y, x] - fd) <= 2e-5 * abs(fd) + 1e-9


def test_fp32_adjoint_tracks_fp64():
    w = W.c2_single_active()
    s64, J64, dA64, dc64 = adjoint(w, 2000, 100, precision=0)
    s64.close()
    s32, J32, dA32, dc32 = adjoint(w, 2000, 100, precision=1)
    s32.close()
    rel = float(np.linalg.norm(dc32 - dc64) / np.linalg.norm(dc64))
    print("fp32 vs fp64: J", J32, J64, "dA0", dA32, dA64, "dJ/dpsi relative L2", rel)
    assert abs(J32 - J64) < 1e-3
    assert abs(dA32 - dA64) <= 1e-2 * abs(dA64)
    assert rel < 1e-2


def test_fp32_adjoint_tracks_fp64_between_plates():
    """The FP32 adjoint between plates (the mirror signs and the ring rows beyond a plate in FP32) against the FP64
    one on the near-wall workload, with the bounds of the periodic FP32 check."""
    w = _near_wall_workload()
    s64, J64, dA64, dc64 = adjoint(w, 200, 50, precision=0)
    s64.close()
    s32, J32, dA32, dc32 = adjoint(w, 200, 50, precision=1)
    s32.close()
    rel = float(np.linalg.norm(dc32 - dc64) / np.linalg.norm(dc64))
    print("walls, fp32 vs fp64: J", J32, J64, "dA0", dA32, dA64, "dJ/dpsi relative L2", rel)
    assert abs(J32 - J64) < 1e-3
    assert abs(dA32 - dA64) <= 1e-2 * abs(dA64)
    assert rel < 1e-2


def test_state_restored_and_backward_repeatable():
    w = W.c2_single_active(n=96, seed=47)
    w.params["A0"] = 1e-6
    s, J, dA0, dc0 = adjoint(w, 120, 40)
    f1 = s.fields()
    dA0b, dc0b = s.adjoint_backward()
    assert dA0b == dA0 and np.array_equal(dc0b, dc0)
    f2 = s.fields()
    for k in ("f", "phi", "c"):
        assert np.array_equal(f1[k], f2[k])
    ref = gpu_J(w, w.c0, nsteps=120)
    assert J == ref
    s.close()


@pytest.mark.parametrize("every,path", [(1, 1), (7, 2), (100, 0)])
def test_interval_and_path_leave_gradients_unchanged(every, path):
    """The checkpoint interval (dividing the run or not, longer than it) and the kernel path only change the
    schedule of the recompute: the gradients are bit for bit those of a run with interval 20 on the fused path."""
    w = W.c2_single_active(n=64, seed=49)
    w.params["A0"] = 2e-6
    s0, J0, dA0_0, dc0_0 = adjoint(w, 60, 20, path=0)
    s0.close()
    s, J, dA0, dc0 = adjoint(w, 60, every, path=path)
    s.close()
    assert J == J0 and dA0 == dA0_0 and np.array_equal(dc0, dc0_0)


def test_torch_autograd_wrapper():
    import torch
    from paper_1711_10984_amd import lbm
    w = W.c2_single_active(n=64, seed=48)
    A0 = torch.tensor(2e-6, dtype=torch.float64, requires_grad=True)
    psi = torch.tensor(w.c0, dtype=torch.float64, requires_grad=True)
    J = lbm.com_displacement(A0, psi, w.param_dict(), w.phi0, w.drop_dicts(), nsteps=100, every=25)
    (3.0 * J).backward()
    w.params["A0"] = 2e-6
    s, Jr, dA0, dc0 = adjoint(w, 100, 25)
    s.close()
    assert float(J.detach()) == Jr
    assert float(A0.grad) == 3.0 * dA0
    assert np.array_equal(psi.grad.numpy(), 3.0 * dc0)


def test_torch_autograd_wrapper_second_backward():
    """With retain_graph the wrapper's backward can run twice (the library context lives as long as autograd
    keeps the node): the second pass accumulates exactly the same gradients again."""
    import torch
    from paper_1711_10984_amd import lbm
    w = W.c2_single_active(n=64, seed=49)
    A0 = torch.tensor(2e-6, dtype=torch.float64, requires_grad=True)
    psi = torch.tensor(w.c0, dtype=torch.float64, requires_grad=True)
    J = lbm.com_displacement(A0, psi, w.param_dict(), w.phi0, w.drop_dicts(), nsteps=60, every=20)
    J.backward(retain_graph=True)
    g1, p1 = float(A0.grad), psi.grad.clone()
    J.backward()
    assert float(A0.grad) == 2.0 * g1
    assert torch.equal(psi.grad, 2.0 * p1)
