"""FP16 population storage (LBM_FP16): populations kept as the FP16-rounded deviation f_i - w_i n0 from
the rest state, fields and arithmetic in FP32.

* Storage semantics, exactly: from the rest state f_i = fp32(w_i n0) (deviation 0 in both) the FP32 and
  the FP16 runs compute the same post-collision deviations d*_i in FP32, so one step later phi and c agree
  bit for bit, and every population of the FP16 run is fp16(d*_i), widened back as fp32(fp16(d*_i)) +
  fp32(w_i n0) and pulled along e_i.  d*_i comes from the FP32 run's stage export (d*_i + w_i n0 in double);
  the storage is emulated with numpy's IEEE float16/float32 arithmetic.  The export comes from a separate
  instantiation of the kernel; FP32 contracts multiply-adds only within a source expression, so it rounds as
  the stepping kernel does.
* Accuracy against the FP64 oracle: storing a population rounds it by at most 2^-11 |d_i| (d_i the
  deviation).  The equilibrium-droplet workload starts far from equilibrium: in the oracle run |u| reaches
  0.08 and |d_i| 0.11 (45 % of w_i n0) within the first 200 steps, so the storage error is up to
  2^-11 x 0.11 = 5.4e-5 absolute, about 1e-4 of the largest population, per population and step.  With
  tau = 1 the collision replaces each population by its equilibrium every step, so these errors do not
  pile up in f; they reach n and u, and through the advection phi and c.  The bounds allow 3 x 1e-4 for
  f, n and c, 1e-3 for phi (an O(1) field advected by u) and 5e-3 for u (relative to max |u|).
"""
import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from paper_1711_10984_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("f", "phi", "c", "n", "ux", "uy")
WGT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]  # D2Q9 directions (x, y)


def sim_of(w, precision, path, graph_steps=None, f_pre=None):
    from paper_1711_10984_amd import lbm
    return lbm.Sim([w.param_dict()], [w.phi0], [w.c0], [w.drop_dicts()], precision=precision,
                   graph_steps=graph_steps, path=path, f_pre=None if f_pre is None else [f_pre])


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("path", [0, 1, 2])
def test_storage_rounding_after_one_step_is_exact(path):
    from paper_1711_10984_amd import lbm
    w = W.c2_single_active(n=96, seed=41)
    # the rest populations rounded to FP32: both storages then hold a deviation of exactly 0
    rest = np.broadcast_to(np.float32(WGT * float(w.params.get("n0", 1.0))).astype(np.float64)[:, None, None],
                           (9, w.ny, w.nx)).copy()
    s32, s16 = sim_of(w, lbm.LBM_FP32, path, f_pre=rest), sim_of(w, lbm.LBM_FP16, path, f_pre=rest)
    st = s32.stages()
    s32.step(1)
    s16.step(1)
    a, b = s32.fields(), s16.fields()
    assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["c"], b["c"])
    wn = np.float32(WGT * float(w.params.get("n0", 1.0)))
    emulated = np.empty_like(b["f"])
    for i, (ex, ey) in enumerate(E):
        dev = np.float32(st[f"fstar{i}"] - np.float64(wn[i]))  # exact: the export is fp32 d* + fp32 w n0
        assert np.array_equal(dev.astype(np.float64) + np.float64(wn[i]), st[f"fstar{i}"])
        stored = (np.float32(np.float16(dev)) + wn[i]).astype(np.float64)
        emulated[i] = np.roll(stored, (ey, ex), axis=(0, 1))  # pulled: f_i(r) = f*_i(r - e_i)
    assert np.array_equal(b["f"], emulated), int(np.count_nonzero(b["f"] != emulated))
    # the rounding is really there: FP16 differs from FP32 somewhere
    assert not np.array_equal(b["f"], a["f"])
    s32.close()
    s16.close()


@pytest.mark.parametrize("path", [0, 2])
def test_fp16_against_fp64_oracle(path):
    from paper_1711_10984_amd import lbm
    w = W.c1_equilibrium()
    sim = sim_of(w, lbm.LBM_FP16, path)
    ref = OracleSim(Params(nx=w.nx, ny=w.ny, **w.params), w.phi0, w.c0, [Drop(**d) for d in w.drop_dicts()])
    sim.step(200)
    ref.run(200)
    g, r = sim.fields(), ref.fields()
    errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
    print("fp16 storage: relative errors after 200 steps", errs)
    assert errs["f"] < 3e-4 and errs["n"] < 3e-4 and errs["c"] < 3e-4
    assert errs["phi"] < 1e-3 and errs["ux"] < 5e-3 and errs["uy"] < 5e-3
    dg, dr = sim.droplets()[0], ref.drops()[0]
    assert abs(dg["x"] - dr.x) < 1e-2 and abs(dg["y"] - dr.y) < 1e-2
    sim.close()


def test_fp16_active_droplet_tracks_fp64():
    """C2 single active droplet, 2000 steps: the FP16-storage centre of mass stays within 0.01 lattice
    units of the FP64 run (same GPU kernels), and the lattice mass within 1e-5 relative."""
    from paper_1711_10984_amd import lbm
    w = W.c2_single_active()
    s64, s16 = sim_of(w, lbm.LBM_FP64, 0, 20), sim_of(w, lbm.LBM_FP16, 0, 20)
    m0 = s64.observables()["mass"]
    s64.step(2000)
    s16.step(2000)
    d64, d16 = s64.droplets()[0], s16.droplets()[0]
    print("fp16 vs fp64 centre of mass after 2000 steps:", d16["x"] - d64["x"], d16["y"] - d64["y"])
    assert abs(d16["x"] - d64["x"]) < 1e-2 and abs(d16["y"] - d64["y"]) < 1e-2
    assert abs(s16.observables()["mass"] - m0) < 1e-5 * m0
    s64.close()
    s16.close()
