"""GPU parity of the HIP library (through the C ABI) against the FP64 CPU oracle.

FP64: the kernels evaluate the same expressions in the same order as the oracle's plain definitions,
without FMA contraction, so fields agree to the last bit; the only difference is the summation order
of the centre-of-mass reductions (1e-16 relative in r_CM).  The bar is 1e-12 relative
(infinity norm per field, normalised by the oracle field's infinity norm) after 1000 steps.
FP32: compared with the FP64 oracle within bounds derived from single-precision rounding.
"""
import functools

import numpy as np
import pytest

from oracle import OracleSim, Params, Drop
from paper_1711_10984_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("f", "phi", "c", "n", "ux", "uy")


def _lbm():
    from paper_1711_10984_amd import lbm
    return lbm


def rel_inf(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def gpu_sim(w, precision=0, graph_steps=None, step=0, f_pre=None, phi=None, c=None, drops=None, path=0):
    lbm = _lbm()
    return lbm.Sim([w.param_dict()], [w.phi0 if phi is None else phi], [w.c0 if c is None else c],
                   [w.drop_dicts() if drops is None else drops], precision=precision, graph_steps=graph_steps,
                   step=step, f_pre=None if f_pre is None else [f_pre], path=path)


PATHS = [0, 1, 2]  # fused sweep kernel, split LB + FD kernels, wavefront-per-strip sweep kernel


@functools.lru_cache(maxsize=1)
def _c5():
    """The 2048^2 emulsion (built once per test session: the seeded generator takes seconds)."""
    return W.c5_emulsion()


def oracle_sim(w, step=0, f_pre=None):
    return OracleSim(Params(nx=w.nx, ny=w.ny, **w.params), w.phi0, w.c0, [Drop(**d) for d in w.drop_dicts()],
                     f_pre=f_pre, step=step)


def compare(g, r, tol, label=""):
    errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{label}: {bad}"
    return errs


def random_workload(nx, ny, seed, ndrop=1, A0=1e-3):
    """Random state with droplets and the source on (stage-level comparison)."""
    f, phi, c = W.random_state(nx, ny, seed)
    rng = np.random.default_rng(seed + 7)
    drops = [W.DropSpec(x=rng.uniform(0, nx), y=rng.uniform(0, ny), R=min(nx, ny) / 3, Rs=min(nx, ny) / 6,
                        ex=np.cos(k), ey=np.sin(k), active=int(k % 2 == 0)) for k in range(ndrop)]
    p = dict(W.ACTIVE, A0=A0, gamma=0.01, c0=0.02, Gamma=0.7, tau=0.8)
    return W.Workload(f"random_{nx}x{ny}", nx, ny, p, phi, c, drops), f


@pytest.mark.parametrize("path,rows", [(0, None), (1, None), (2, None), (2, 16)])
@pytest.mark.parametrize("shape", [(3, 3), (5, 7), (8, 8), (70, 37), (130, 19), (64, 16), (55, 129), (200, 67)])
def test_stages_match_oracle_bitwise(shape, path, rows):
    """Every stage plane bitwise equal to the oracle's, also with 16-row strips on the wave path (several
    segments per column strip, the last one short)."""
    nx, ny = shape
    w, f = random_workload(nx, ny, seed=nx * 100 + ny, ndrop=2)
    sim = gpu_sim(w, f_pre=f, step=3, path=path)
    if rows is not None:
        sim.set_seg_rows(rows)
    got = sim.stages()
    ref = oracle_sim(w, step=3, f_pre=f).stages()
    for k in ref:
        assert np.array_equal(got[k], ref[k]), (k, float(np.max(np.abs(got[k] - ref[k]))))
    sim.close()


@pytest.mark.parametrize("advection,path", [(0, 0), (1, 0), (0, 1), (0, 2), (1, 2)])
def test_c1_equilibrium_droplet_1000_2000_steps(advection, path):
    w = W.c1_equilibrium()
    w.params["advection"] = advection
    sim = gpu_sim(w, path=path)
    ref = oracle_sim(w)
    for steps in (1000, 1000):
        sim.step(steps)
        ref.run(steps)
        compare(sim.fields(), ref.fields(), 1e-12, f"c1 step {ref.step_count}")
        dg, dr = sim.droplets()[0], ref.drops()[0]
        assert abs(dg["x"] - dr.x) < 1e-12 * w.nx and abs(dg["y"] - dr.y) < 1e-12 * w.ny
    sim.close()


@pytest.mark.parametrize("path", [0, 2])
def test_c2_active_droplet_256_first_1000_steps(path):
    w = W.c2_single_active()
    sim = gpu_sim(w, graph_steps=20, path=path)
    ref = oracle_sim(w)
    sim.step(1000)
    ref.run(1000)
    errs = compare(sim.fields(), ref.fields(), 1e-12, "c2 1000 steps")
    print("c2 relative errors", errs)
    og, orr = sim.observables(), ref.observables()
    assert np.max(np.abs(og["com"] - orr["com"])) < 1e-12 * w.nx
    assert abs(og["mass"] - orr["mass"]) < 1e-12 * orr["mass"]
    assert abs(og["sum_phi"] - orr["sum_phi"]) < 1e-12 * abs(orr["sum_phi"])
    assert abs(og["sum_c"] - orr["sum_c"]) < 1e-12 * abs(orr["sum_c"])
    assert abs(og["min_B"] - orr["min_B"]) < 1e-12 * abs(orr["min_B"])  # a minimum: the same node's value
    assert abs(og["max_u"] - orr["max_u"]) < 1e-12 * orr["max_u"]
    assert og["nonfinite"] == orr["nonfinite"] is False
    assert np.max(np.abs(og["vel"] - orr["vel"])) < 1e-12 * max(1e-8, np.max(np.abs(orr["vel"])))
    assert np.max(np.abs(og["drop_mass"] - orr["drop_mass"])) < 1e-12 * np.max(orr["drop_mass"])
    sim.close()


@functools.lru_cache(maxsize=3)
def _c5_reference(steps):
    ref = oracle_sim(_c5())
    ref.run(steps)
    return ref.fields(), np.array([[d.x, d.y] for d in ref.drops()])


@pytest.mark.parametrize("path", [0, 2])
def test_c5_emulsion_2048_every_tuned_height(path):
    """Full-size 2048^2 emulsion with 64 droplets at every strip height the autotuner may pick (the bench's
    launch configuration is one of them), graph replay: every field after 4 steps within 1e-12 of the oracle
    on the whole lattice, centres within 1e-12 nx."""
    w = _c5()
    r, orr = _c5_reference(4)
    for rows in _lbm().lbm_tune_rows():
        sim = gpu_sim(w, graph_steps=2, path=path)
        sim.set_seg_rows(rows)
        sim.step(4)
        compare(sim.fields(), r, 1e-12, f"c5 4 steps, height {rows}")
        og = np.array([[d["x"], d["y"]] for d in sim.droplets()])
        assert np.max(np.abs(og - orr)) < 1e-12 * w.nx, rows
        sim.close()
        del sim


def test_c5_emulsion_2048_bench_configuration():
    """The benchmark's own configuration: the autotuner over every path with 30 launches per candidate, then
    one 100-step hipGraph replay, against 100 oracle steps of the whole lattice."""
    w = _c5()
    r, orr = _c5_reference(100)
    sim = gpu_sim(w, graph_steps=100, path=0)
    rows, path, _ = sim.autotune(30, both_paths=True)
    sim.set_graph(100)
    sim.step(100)
    compare(sim.fields(), r, 1e-12, f"c5 100 steps, path {path}, height {rows}, width {sim.strip_width}")
    og = np.array([[d["x"], d["y"]] for d in sim.droplets()])
    assert np.max(np.abs(og - orr)) < 1e-12 * w.nx
    sim.close()


@functools.lru_cache(maxsize=1)
def _c5_crop_reference():
    w = W.crop_workload(_c5(), 1152, 896, 256)
    ref = oracle_sim(w)
    ref.run(1000)
    return w, ref.fields(), np.array([[d.x, d.y] for d in ref.drops()])


@pytest.mark.parametrize("precision,path", [(0, 0), (0, 1), (0, 2), (1, 2)])
def test_c5_crop_256_matches_oracle(precision, path):
    """The 2048^2 emulsion's oracle check at a size the oracle runs for long: a separate 256^2 periodic lattice
    seeded with the three droplets whose centres fall in the window at (1152, 896), 1000 steps with the sources
    on.  FP64 within 1e-12 of the oracle.  FP32: the C1 check's bounds after 200 steps (1e-5 relative in
    populations, phi and n) scaled by the step count (rounding errors of this dissipative scheme accumulate at
    most linearly: 5e-5 after 1000 steps); c and u as in the C1 check; centres within 1e-3 lattice units."""
    w, r, orr = _c5_crop_reference()
    assert len(w.drops) == 3
    sim = gpu_sim(w, precision=precision, path=path, graph_steps=20)
    sim.step(1000)
    g = sim.fields()
    og = np.array([[d["x"], d["y"]] for d in sim.droplets()])
    moved = np.max(np.abs(orr - np.array([[d.x, d.y] for d in w.drops])))
    if precision == 0:
        compare(g, r, 1e-12, "c5 crop")
        assert np.max(np.abs(og - orr)) < 1e-9
    else:
        errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
        print("fp32 relative errors after 1000 steps", errs, "centres", np.max(np.abs(og - orr)))
        assert errs["f"] < 5e-5 and errs["phi"] < 5e-5 and errs["n"] < 5e-5
        assert errs["c"] < 1e-4 and errs["ux"] < 1e-3 and errs["uy"] < 1e-3
        assert np.max(np.abs(og - orr)) < 1e-3
    assert moved > 1e-3  # the droplets moved (sources on)
    sim.close()


def _uneven_batch():
    """Lattices of uneven sizes in one batch: 96^2 active, 64^2 equilibrium, a ragged 110 x 37 pair (one passive
    droplet), and four of the two-droplet sweep's 256 x 256 .. 512 x 256 lattices (active-active and
    active-passive, head-on)."""
    ws = [W.c2_single_active(n=96, seed=11), W.c1_equilibrium(seed=12)]
    a = W.DropSpec(30.0, 18.0, 10.0, 2.5, ex=1.0, ey=0.0, active=1)
    b = W.DropSpec(75.0, 22.0, 10.0, 2.5, ex=-1.0, ey=0.0, active=0, psi_front=0.0, psi_back=0.0)
    phi, c = W.droplet_fields(110, 37, [a, b], seed=13)
    ws.append(W.Workload("ragged_110x37", 110, 37, dict(W.ACTIVE, A0=1e-6), phi, c, [a, b]))
    c3 = W.c3_batch()
    ws += [c3[i] for i in (1, 10, 19, 30)]
    return ws


@functools.lru_cache(maxsize=1)
def _uneven_batch_reference(steps):
    out = []
    for w in _uneven_batch():
        ref = oracle_sim(w)
        ref.run(steps)
        out.append((ref.fields(), np.array([[d.x, d.y] for d in ref.drops()])))
    return out


@pytest.mark.parametrize("path,rows", [(0, 16), (0, 40), (1, None), (2, 16), (2, 44)])
def test_batched_uneven_instances_match_oracle(path, rows):
    """FP64 batch of uneven lattices in one launch sequence on every path (and short and tall strip segments):
    each instance within 1e-12 of its own oracle run after 300 steps, centres within 1e-12 nx."""
    lbm = _lbm()
    ws = _uneven_batch()
    assert len({(w.nx, w.ny) for w in ws}) >= 5
    sim = lbm.Sim([w.param_dict() for w in ws], [w.phi0 for w in ws], [w.c0 for w in ws],
                  [w.drop_dicts() for w in ws], precision=lbm.LBM_FP64, graph_steps=10, path=path)
    if rows is not None:
        sim.set_seg_rows(rows)
    sim.step(300)
    for i, (w, (r, orr)) in enumerate(zip(ws, _uneven_batch_reference(300))):
        compare(sim.fields(i), r, 1e-12, w.name)
        og = np.array([[d["x"], d["y"]] for d in sim.droplets(i)])
        assert np.max(np.abs(og - orr)) < 1e-12 * w.nx, w.name
    sim.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("other", [1, 2])
def test_fused_and_other_paths_agree_bitwise(other, precision):
    """Every path computes the same arithmetic in every precision (FP32 and FP16 storage contract a * b + c only
    within a source expression, and the paths share those expressions), so the fields agree bit for bit."""
    w = W.c5_emulsion(n=384, ndrop=6, R=16.0, seed=21)
    s1 = gpu_sim(w, path=0, graph_steps=10, precision=precision)
    s2 = gpu_sim(w, path=other, graph_steps=10, precision=precision)
    s1.step(120)
    s2.step(120)
    f1, f2 = s1.fields(), s2.fields()
    for k in FIELDS:
        assert np.array_equal(f1[k], f2[k]), k
    d1, d2 = s1.droplets(), s2.droplets()
    for a, b in zip(d1, d2):
        assert abs(a["x"] - b["x"]) < 1e-12 and abs(a["y"] - b["y"]) < 1e-12
    s1.close()
    s2.close()


def test_graph_replay_equals_eager_bitwise():
    w = W.c2_single_active(n=128, seed=5)
    s1 = gpu_sim(w, graph_steps=0)
    s2 = gpu_sim(w, graph_steps=6)
    for _ in range(4):  # several replays with host synchronisation in between
        s1.step(13)
        s2.step(13)
        s1.sync()
        s2.sync()
        f1, f2 = s1.fields(), s2.fields()
        for k in FIELDS:
            assert np.array_equal(f1[k], f2[k]), k
        assert s1.droplets() == s2.droplets()
    s1.close()
    s2.close()


def test_checkpoint_resume_bitwise():
    w = W.c2_single_active(n=96, seed=6)
    w.params["A0"] = 1e-6
    full = gpu_sim(w)
    full.step(70)
    part = gpu_sim(w)
    part.step(30)
    st = part.fields()
    drops = part.droplets()
    resumed = gpu_sim(w, step=30, f_pre=st["f"], phi=st["phi"], c=st["c"], drops=drops)
    resumed.step(40)
    f1, f2 = full.fields(), resumed.fields()
    for k in FIELDS:
        assert np.array_equal(f1[k], f2[k]), k
    d1, d2 = full.droplets()[0], resumed.droplets()[0]
    assert abs(d1["x"] - d2["x"]) < 1e-12 and abs(d1["y"] - d2["y"]) < 1e-12
    for s in (full, part, resumed):
        s.close()


def test_translation_equivariance_bitwise():
    w = W.c1_equilibrium()
    sh = (7, -11)
    s1 = gpu_sim(w)
    s2 = gpu_sim(w, phi=np.roll(w.phi0, sh, (0, 1)), c=np.roll(w.c0, sh, (0, 1)),
                 drops=[dict(d, x=(d["x"] + sh[1]) % w.nx, y=(d["y"] + sh[0]) % w.ny) for d in w.drop_dicts()])
    s1.step(200)
    s2.step(200)
    f1, f2 = s1.fields(), s2.fields()
    for k in ("phi", "c", "ux", "uy", "n"):
        assert np.array_equal(np.roll(f1[k], sh, (0, 1)), f2[k]), k
    s1.close()
    s2.close()


def test_determinism_bitwise():
    w = W.c5_emulsion(n=512, ndrop=8, R=16.0, seed=77)
    runs = []
    for _ in range(2):
        s = gpu_sim(w, graph_steps=10)
        s.step(100)
        runs.append((s.fields(), s.droplets()))
        s.close()
    for k in FIELDS:
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    assert runs[0][1] == runs[1][1]


@pytest.mark.parametrize("path", [0, 2])
def test_fp32_against_fp64_oracle(path):
    """FP32 storage and arithmetic: relative deviation of a few 1e-6 per field after 200 steps (unit
    roundoff 6e-8 amplified by the ~100 operations per node and step and by the dynamics)."""
    w = W.c1_equilibrium()
    sim = gpu_sim(w, precision=1, path=path)
    ref = oracle_sim(w)
    sim.step(200)
    ref.run(200)
    g, r = sim.fields(), ref.fields()
    errs = {k: rel_inf(g[k], r[k]) for k in FIELDS}
    print("fp32 relative errors after 200 steps", errs)
    assert errs["f"] < 1e-5 and errs["phi"] < 1e-5 and errs["n"] < 1e-5
    assert errs["c"] < 1e-4 and errs["ux"] < 1e-3 and errs["uy"] < 1e-3
    dg, dr = sim.droplets()[0], ref.drops()[0]
    assert abs(dg["x"] - dr.x) < 1e-3 and abs(dg["y"] - dr.y) < 1e-3
    sim.close()


def test_instability_is_reported():
    """B(c) = B0 + B1 c <= 0 where c is large: observables report it (Sec. 4 stability condition)."""
    w = W.c1_equilibrium()
    w.params["B1"] = -0.2  # B(0.1) = 0.006 - 0.02 < 0
    sim = gpu_sim(w)
    sim.step(10)
    ob = sim.observables()
    assert ob["unstable"] and ob["min_B"] < 0
    sim.close()


@pytest.mark.parametrize("path", PATHS)
def test_nonfinite_state_is_reported(path):
    """A NaN injected into the initial surfactant field (host-forced) spreads through the stencils; the kernels
    run on and the observables flag it (nonfinite, LBM_E_UNSTABLE), as does lbm_fields (LBM_E_UNSTABLE, the
    arrays filled).  A clean run of the same lattice is not flagged."""
    w = W.c1_equilibrium()
    c = w.c0.copy()
    c[10, 20] = np.nan
    sim = gpu_sim(w, c=c, path=path)
    sim.step(3)
    ob = sim.observables()
    assert ob["nonfinite"] and ob["unstable"]
    phi = np.empty((w.ny, w.nx))
    lbm = _lbm()
    assert lbm.lbm_fields(sim.ctx, 0, phi=phi) == lbm.LBM_E_UNSTABLE and not np.isfinite(phi).all()
    sim.close()
    clean = gpu_sim(w, path=path)
    clean.step(3)
    ob = clean.observables()
    assert not ob["nonfinite"] and not ob["unstable"]
    assert lbm.lbm_fields(clean.ctx, 0, phi=phi) == lbm.LBM_OK and np.isfinite(phi).all()
    clean.close()


@pytest.mark.parametrize("path", PATHS)
def test_no_droplets_and_tiny_lattice(path):
    w = W.c1_equilibrium()
    f, phi, c = W.random_state(3, 4, 3)
    tiny = W.Workload("tiny", 3, 4, dict(w.params), phi, c, [])
    sim = gpu_sim(tiny, f_pre=f, path=path)
    ref = oracle_sim(tiny, f_pre=f)
    sim.step(25)
    ref.run(25)
    compare(sim.fields(), ref.fields(), 1e-12, "tiny 3x4")
    sim.close()


@pytest.mark.parametrize("path", PATHS)
def test_maximum_droplet_count_matches_oracle(path):
    """The droplet limit of a lattice (256 active droplets: four 64-bit mask words per strip or tile) against
    the oracle: fields within 1e-12 and every centre within 1e-12 lattice units after 30 steps."""
    lbm = _lbm()
    w = W.c5_emulsion(seed=41, n=448, ndrop=lbm.LBM_MAXDROP, R=4.0)
    w.params["A0"] = 1e-3  # sources strong enough to move every droplet within the run
    sim = gpu_sim(w, path=path, graph_steps=10)
    ref = oracle_sim(w)
    sim.step(30)
    ref.run(30)
    compare(sim.fields(), ref.fields(), 1e-12, "256 droplets")
    got, want = sim.droplets(), ref.drops()
    assert len(got) == len(want) == lbm.LBM_MAXDROP

    def mi(d):
        return (d + 0.5 * w.nx) % w.nx - 0.5 * w.nx

    dev = max(max(abs(mi(g["x"] - r.x)), abs(mi(g["y"] - r.y))) for g, r in zip(got, want))
    moved = max(abs(mi(g["x"] - d.x)) + abs(mi(g["y"] - d.y)) for g, d in zip(got, w.drops))
    assert dev < 1e-12 and moved > 1e-6, (dev, moved)
    sim.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("path", [0, 2])
def test_segment_heights_agree_bitwise_and_autotune_keeps_state(path, precision):
    """The sweeping kernels' strip width and height change only the work decomposition: every width and
    height gives the same bits, in every precision; the autotuner's trial launches and lbm_time_launches leave the
    state, droplets and step counter untouched."""
    lbm = _lbm()
    w = W.c5_emulsion(n=300, ndrop=4, R=14.0, seed=31)
    ref = None
    for rows, width in ((16, 54), (32, 48), (64, 32), (128, 41), (256, 54), (20, 48)):
        s = gpu_sim(w, graph_steps=0, path=path, precision=precision)
        s.set_seg_rows(rows)
        s.set_strip_width(width)
        assert s.strip_width == width and s.seg_rows == rows
        s.step(37)
        f = s.fields()
        if ref is None:
            ref = f
        else:
            for k in FIELDS:
                assert np.array_equal(f[k], ref[k]), (rows, width, k)
        for bad in (lbm.LBM_STRIP_W_MIN - 1, lbm.LBM_STRIP_W_MAX + 1):
            with pytest.raises(lbm.LBMError):
                s.set_strip_width(bad)
        s.close()
    s = gpu_sim(w, graph_steps=10, path=path, precision=precision)
    s.step(5)
    before, drops_before, step_before = s.fields(), s.droplets(), s.step_count
    chosen, chosen_path, times = s.autotune(3, both_paths=False)
    ms = s.time_launches(4)
    assert list(ms) == [lbm.lbm_kernel_name(path, 0), "k_reduce"] and min(ms.values()) > 0
    assert chosen_path == path and chosen in s.tune_rows() and len(times) >= 3
    assert s.strip_width in lbm.lbm_tune_widths()
    assert {k.split(":")[1].split("x")[0] for k in times} == {str(x) for x in lbm.lbm_tune_widths()}
    after = s.fields()
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    assert s.droplets() == drops_before and s.step_count == step_before
    s.step(32)
    f = s.fields()
    for k in FIELDS:
        assert np.array_equal(f[k], ref[k]), k
    s.close()


def test_autotune_over_all_paths_keeps_state():
    """With both_paths the autotuner also times the split pair; whatever it picks, the state, droplets and
    step counter are untouched and the run continues bit for bit (the paths agree bitwise)."""
    w = W.c5_emulsion(n=200, ndrop=3, R=12.0, seed=32)
    ref = gpu_sim(w, graph_steps=0, path=0)
    ref.step(24)
    want = ref.fields()
    ref.close()
    s = gpu_sim(w, graph_steps=0, path=1)
    s.step(5)
    before, drops_before, step_before = s.fields(), s.droplets(), s.step_count
    rows, path, times = s.autotune(3, both_paths=True)
    assert path in (0, 1, 2) and "split" in times and any(k.startswith("wave:") for k in times)
    assert s.path == path and (path == 1 or rows in s.tune_rows())
    after = s.fields()
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    assert s.droplets() == drops_before and s.step_count == step_before
    s.step(19)
    f = s.fields()
    for k in FIELDS:
        assert np.array_equal(f[k], want[k]), k
    s.close()


@pytest.mark.parametrize("path", PATHS)
def test_stage_export_keeps_state(path):
    """lbm_debug_stage writes only scratch (the inactive halves, the partial sums, the stage planes): the
    fields, droplets and step counter are unchanged and the run continues bit for bit."""
    w = W.c5_emulsion(n=200, ndrop=3, R=12.0, seed=34)
    ref = gpu_sim(w, graph_steps=0, path=path)
    ref.step(9)
    want, want_drops = ref.fields(), ref.droplets()
    ref.close()
    s = gpu_sim(w, graph_steps=0, path=path)
    s.step(4)
    before, drops_before, step_before = s.fields(), s.droplets(), s.step_count
    s.stages()
    after = s.fields()
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    assert s.droplets() == drops_before and s.step_count == step_before
    s.step(5)
    f = s.fields()
    for k in FIELDS:
        assert np.array_equal(f[k], want[k]), k
    assert s.droplets() == want_drops
    s.close()


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("path,rows", [(0, 16), (1, None), (2, 16), (2, 26)])
def test_low_precision_batched_instances_match_single_runs(path, rows, precision):
    """Batching does not change any instance's arithmetic (FP32 and FP16 storage, uneven sizes, every path):
    each lattice of a C3-like batch on the given path and height equals its own single run on the fused path at
    the default height, bit for bit."""
    lbm = _lbm()
    ws = W.c3_batch()[::7]
    sim = lbm.Sim([w.param_dict() for w in ws], [w.phi0 for w in ws], [w.c0 for w in ws],
                  [w.drop_dicts() for w in ws], precision=precision, graph_steps=10, path=path)
    if rows is not None:
        sim.set_seg_rows(rows)
    sim.step(60)
    for i, w in enumerate(ws):
        single = gpu_sim(w, precision=precision, graph_steps=10)
        single.step(60)
        a, b = sim.fields(i), single.fields()
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), (w.name, k)
        # centres: the per-strip partial sums are added in an order that depends on the strip height
        for da, db in zip(sim.droplets(i), single.droplets()):
            assert abs(da["x"] - db["x"]) < 1e-12 * w.nx and abs(da["y"] - db["y"]) < 1e-12 * w.ny
        single.close()
    sim.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_plain_and_general_wave_kernels_agree_bitwise(precision):
    """The wave path launches a kernel specialised for periodic lattices with the printed advection when every
    lattice of the launch is one, and the general kernel otherwise.  The same periodic lattices, once alone
    (specialised kernel) and once batched with a walled lattice (general kernel for all), give the same fields
    bit for bit after 80 steps, in every precision; centres agree to 1e-12 of the lattice."""
    lbm = _lbm()
    ws = [W.c2_single_active(n=96, seed=21), W.c3_batch()[5]]
    walled = W.c2_single_active(n=64, seed=22)
    pw = dict(walled.param_dict(), walls=1)
    alone = lbm.Sim([w.param_dict() for w in ws], [w.phi0 for w in ws], [w.c0 for w in ws],
                    [w.drop_dicts() for w in ws], precision=precision, graph_steps=10, path=2)
    mixed = lbm.Sim([w.param_dict() for w in ws] + [pw], [w.phi0 for w in ws] + [walled.phi0],
                    [w.c0 for w in ws] + [walled.c0], [w.drop_dicts() for w in ws] + [walled.drop_dicts()],
                    precision=precision, graph_steps=10, path=2)
    for s in (alone, mixed):
        s.set_seg_rows(26)
        s.step(80)
    for i, w in enumerate(ws):
        a, b = alone.fields(i), mixed.fields(i)
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), (w.name, k, precision)
        for da, db in zip(alone.droplets(i), mixed.droplets(i)):
            assert abs(da["x"] - db["x"]) < 1e-12 * w.nx and abs(da["y"] - db["y"]) < 1e-12 * w.ny
    alone.close()
    mixed.close()


@functools.lru_cache(maxsize=2)
def _c3_reference(steps):
    out = []
    for w in W.c3_batch():
        ref = oracle_sim(w)
        ref.run(steps)
        out.append((ref.fields(), np.array([[d.x, d.y] for d in ref.drops()])))
    return out


# FP32 and FP16-storage bounds against the FP64 oracle after at most 200 steps: the C1 check's (FP32) and the
# FP16 storage check's (tests/test_gpu_fp16.py)
LOWP_BOUNDS = {1: {"f": 1e-5, "phi": 1e-5, "n": 1e-5, "c": 1e-4, "ux": 1e-3, "uy": 1e-3},
               2: {"f": 3e-4, "phi": 1e-3, "n": 3e-4, "c": 3e-4, "ux": 5e-3, "uy": 5e-3}}


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("rows", [16, 24])
def test_c3_full_batch_matches_oracle(precision, rows):
    """The whole two-droplet sweep batch (32 lattices, 3.2 M nodes) as the bench times it: the wave path at the
    strip heights its autotuner picks (16, 24), replayed from 20-step graphs, each lattice against its own oracle
    run.  FP64: 100 steps, within 1e-12 (centres 1e-12 of the lattice).  FP32 and FP16 storage: 20 steps, within
    the bounds of the 200-step equilibrium-droplet checks, centres within 1e-3 lattice units.  (Those bounds come
    from a workload at rest; these lattices are active, with larger population deviations and so larger storage
    rounding: after 100 steps FP16 storage's populations differed by 3.8e-4 on one lattice, above the 3e-4 of
    the 200-step check.  Rounding accumulates about linearly with the step count, so at 20 steps the bounds hold
    with margin.)"""
    lbm = _lbm()
    ws = W.c3_batch()
    assert len(ws) == 32
    steps = 100 if precision == 0 else 20
    refs = _c3_reference(steps)
    sim = lbm.Sim([w.param_dict() for w in ws], [w.phi0 for w in ws], [w.c0 for w in ws],
                  [w.drop_dicts() for w in ws], precision=precision, graph_steps=20, path=2)
    sim.set_seg_rows(rows)
    sim.step(steps)
    for i, (w, (r, orr)) in enumerate(zip(ws, refs)):
        g = sim.fields(i)
        og = np.array([[d["x"], d["y"]] for d in sim.droplets(i)])
        if precision == 0:
            compare(g, r, 1e-12, w.name)
            assert np.max(np.abs(og - orr)) < 1e-12 * w.nx, w.name
        else:
            for k, bound in LOWP_BOUNDS[precision].items():
                assert rel_inf(g[k], r[k]) < bound, (w.name, k, rel_inf(g[k], r[k]))
            assert np.max(np.abs(og - orr)) < 1e-3, w.name
    sim.close()


@pytest.mark.parametrize("precision,rows", [(1, 28), (2, 26)])
def test_c5_low_precision_bench_configuration(precision, rows):
    """The 2048^2 emulsion in FP32 and with FP16 storage as the bench runs them (wave path at the height its
    autotuner picks, graph replay): every field after 20 steps within the low-precision bounds of the FP64 oracle
    on the whole lattice, centres within 1e-3 lattice units."""
    w = _c5()
    r, orr = _c5_reference(20)
    sim = gpu_sim(w, precision=precision, graph_steps=20, path=2)
    sim.set_seg_rows(rows)
    sim.step(20)
    g = sim.fields()
    for k, bound in LOWP_BOUNDS[precision].items():
        assert rel_inf(g[k], r[k]) < bound, (k, rel_inf(g[k], r[k]))
    og = np.array([[d["x"], d["y"]] for d in sim.droplets()])
    assert np.max(np.abs(og - orr)) < 1e-3
    sim.close()
