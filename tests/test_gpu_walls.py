"""Bounding walls on the GPU (LBM_WALLS_Y: plates at y = -1/2 and y = ny - 1/2, halfway bounce-back,
mirror ghosts; the same reading as the oracle's) against the FP64 oracle.

FP64 is bitwise equal to the oracle stage by stage and over many steps, on every kernel path, including
lattices only 3 or 4 rows high (where both plates fall inside one strip or tile) and the plate geometry of
Sec. 4 (512 x 256, R = 32).
"""
import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from paper_1711_10984_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("f", "phi", "c", "n", "ux", "uy")
PATHS = [0, 1, 2]
REFL_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]


def gpu_sim(w, precision=0, graph_steps=None, step=0, f_pre=None, path=0):
    from paper_1711_10984_amd import lbm
    return lbm.Sim([w.param_dict()], [w.phi0], [w.c0], [w.drop_dicts()], precision=precision,
                   graph_steps=graph_steps, step=step, f_pre=None if f_pre is None else [f_pre], path=path)


def oracle_sim(w, step=0, f_pre=None):
    return OracleSim(Params(nx=w.nx, ny=w.ny, **w.params), w.phi0, w.c0, [Drop(**d) for d in w.drop_dicts()],
                     f_pre=f_pre, step=step)


def rel_inf(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def walled_random(nx, ny, seed, ndrop=2, advection=0):
    f, phi, c = W.random_state(nx, ny, seed)
    rng = np.random.default_rng(seed + 7)
    drops = [W.DropSpec(x=rng.uniform(0, nx), y=rng.uniform(0, ny), R=min(nx, ny) / 3, Rs=min(nx, ny) / 6,
                        ex=np.cos(k), ey=np.sin(k), active=int(k % 2 == 0)) for k in range(ndrop)]
    p = dict(W.ACTIVE, A0=1e-3, gamma=0.01, c0=0.02, Gamma=0.7, tau=0.8, walls=1, advection=advection)
    return W.Workload(f"walled_{nx}x{ny}", nx, ny, p, phi, c, drops), f


@pytest.mark.parametrize("path,rows", [(0, None), (1, None), (2, None), (2, 16)])
@pytest.mark.parametrize("shape", [(5, 3), (7, 4), (70, 37), (130, 19), (55, 129), (64, 16)])
def test_stages_with_walls_match_oracle_bitwise(shape, path, rows):
    """Every stage plane bitwise; with 16-row strips the upper plate lies in a short last segment of the wave
    kernel on the 19- and 37-row lattices."""
    nx, ny = shape
    w, f = walled_random(nx, ny, seed=nx * 100 + ny + 5)
    sim = gpu_sim(w, f_pre=f, step=3, path=path)
    if rows is not None:
        sim.set_seg_rows(rows)
    got = sim.stages()
    ref = oracle_sim(w, step=3, f_pre=f).stages()
    for k in ref:
        assert np.array_equal(got[k], ref[k]), (k, float(np.max(np.abs(got[k] - ref[k]))))
    sim.close()


@pytest.mark.parametrize("path", PATHS)
def test_populations_round_trip_through_the_device_layout(path):
    """lbm_fields returns the pre-collision populations it was given, also next to the plates where the
    stored layout holds them bounced back."""
    w, f = walled_random(37, 11, seed=3)
    sim = gpu_sim(w, f_pre=f, path=path)
    assert np.array_equal(sim.fields()["f"], f)
    sim.close()


@pytest.mark.parametrize("advection,path,rows", [(0, 0, None), (1, 0, None), (0, 1, None), (0, 2, None),
                                                (1, 2, None), (0, 2, 16), (1, 2, 16)])
def test_walled_random_state_300_steps(advection, path, rows):
    w, f = walled_random(61, 29, seed=17, advection=advection)
    w.params["A0"] = 1e-5
    sim = gpu_sim(w, f_pre=f, path=path, graph_steps=10)
    if rows is not None:
        sim.set_seg_rows(rows)  # the upper plate in the second, 13-row segment
    ref = oracle_sim(w, f_pre=f)
    sim.step(300)
    ref.run(300)
    g, r = sim.fields(), ref.fields()
    for k in FIELDS:
        assert np.array_equal(g[k], r[k]), (k, rel_inf(g[k], r[k]))
    for a, b in zip(sim.droplets(), ref.drops()):
        assert abs(a["x"] - b.x) < 1e-12 * w.nx and abs(a["y"] - b.y) < 1e-12 * w.ny
    sim.close()


@pytest.mark.parametrize("path", [0, 2])
def test_plate_geometry_512x256_matches_oracle(path):
    """Sec. 4 geometry: a droplet of radius 32 in a 512 x 256 box between plates, 200 steps."""
    w = W.plates_single_active()
    sim = gpu_sim(w, graph_steps=20, path=path)
    ref = oracle_sim(w)
    sim.step(200)
    ref.run(200)
    g, r = sim.fields(), ref.fields()
    errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
    assert all(v <= 1e-12 for v in errs.values()), errs
    dg, dr = sim.droplets()[0], ref.drops()[0]
    assert abs(dg["x"] - dr.x) < 1e-10 and abs(dg["y"] - dr.y) < 1e-10
    og, orr = sim.observables(), ref.observables()
    assert abs(og["mass"] - orr["mass"]) < 1e-12 * orr["mass"]
    sim.close()


def test_walls_fp32_against_fp64_oracle():
    w, f = walled_random(48, 40, seed=23)
    w.params["A0"] = 1e-5
    sim = gpu_sim(w, precision=1, f_pre=f)
    ref = oracle_sim(w, f_pre=f)
    sim.step(200)
    ref.run(200)
    g, r = sim.fields(), ref.fields()
    errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
    print("walls fp32 relative errors", errs)
    assert errs["f"] < 1e-5 and errs["phi"] < 1e-5 and errs["n"] < 1e-5 and errs["c"] < 1e-4
    sim.close()


def test_mirror_equivalence_on_the_gpu():
    """An x-invariant, x-symmetric state between plates equals the mirror-doubled periodic lattice, bitwise
    (the oracle-side pin of the same property, run through the kernels)."""
    from paper_1711_10984_amd import lbm
    nx, L = 70, 24
    rng = np.random.default_rng(4)
    phi = np.repeat(rng.uniform(-0.9, 0.9, size=(L, 1)), nx, axis=1)
    c = np.repeat(0.1 + rng.uniform(-0.04, 0.04, size=(L, 1)), nx, axis=1)
    wts = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    prof = wts[:, None] * (1.0 + rng.uniform(-0.02, 0.02, size=(9, L)))
    prof[3], prof[6], prof[7] = prof[1], prof[5], prof[8]
    f = np.repeat(prof[:, :, None], nx, axis=2)
    p = dict(W.ACTIVE, tau=0.8, Gamma=0.7, A0=0.0, gamma=0.0)
    a = lbm.Sim([dict(p, nx=nx, ny=L, walls=1)], [phi], [c], [[]], f_pre=[np.ascontiguousarray(f)], path=2)
    b = lbm.Sim([dict(p, nx=nx, ny=2 * L, walls=0)], [np.concatenate([phi, phi[::-1]])],
                [np.concatenate([c, c[::-1]])], [[]],
                f_pre=[np.ascontiguousarray(np.concatenate([f, f[REFL_Y][:, ::-1]], axis=1))], path=2)
    a.step(50)
    b.step(50)
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        assert np.array_equal(fa[k], fb[k][:, :L] if k == "f" else fb[k][:L]), k
    a.close()
    b.close()
