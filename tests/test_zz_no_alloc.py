"""lbm_step_noalloc, the entry point for callers that cannot allocate: its scratch is a static device array, the
caller passes only the state.  On the GPU it must give the same bits as lbm_step on the same state, over two
calls in a row (the second on a smaller lattice, so that the shared scratch holds the first call's leftovers).
The host-side rejections need no GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_1711_10984_amd import workloads as W

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


def _lbm():
    from paper_1711_10984_amd import lbm
    return lbm


def _stored_pops(f_pre, precision, n0=1.0):
    """The documented device layout of the populations: f*_i(r) = f_i(r + e_i) (periodic), FP64 as is, FP32 the
    deviation f* - (float)(w_i n0) rounded to float, FP16 the half of (float)f* - (float)(w_i n0)."""
    fs = np.stack([np.roll(f_pre[i], (-EY[i], -EX[i]), axis=(0, 1)) for i in range(9)])
    if precision == 0:
        return np.ascontiguousarray(fs)
    if precision == 2:
        wn32 = np.float32(WT * n0)[:, None, None]
        return np.ascontiguousarray((fs.astype(np.float32) - wn32).astype(np.float16))
    wn = np.float32(WT * n0).astype(np.float64)[:, None, None]
    return np.ascontiguousarray((fs - wn).astype(np.float32))


def _pre_collision(stored, precision, n0=1.0):
    if precision == 2:  # widened in float, as the library reads FP16 storage back
        fs = (stored.astype(np.float32) + np.float32(WT * n0)[:, None, None]).astype(np.float64)
    else:
        fs = stored.astype(np.float64)
        if precision != 0:
            fs = fs + np.float32(WT * n0).astype(np.float64)[:, None, None]
    return np.stack([np.roll(fs[i], (EY[i], EX[i]), axis=(0, 1)) for i in range(9)])


def _noalloc_run(torch, lbm, w, f_pre, drops, precision, nsteps):
    dt = torch.float64 if precision == 0 else torch.float32
    ft = torch.float16 if precision == 2 else dt
    npdt = np.float64 if precision == 0 else np.float32
    dev = torch.device("cuda:0")
    f = [torch.from_numpy(_stored_pops(f_pre, precision)).to(dev), torch.zeros((9, w.ny, w.nx), dtype=ft, device=dev)]
    phi = [torch.from_numpy(w.phi0.astype(npdt)).to(dev), torch.zeros((w.ny, w.nx), dtype=dt, device=dev)]
    c = [torch.from_numpy(w.c0.astype(npdt)).to(dev), torch.zeros((w.ny, w.nx), dtype=dt, device=dev)]
    table = (lbm.lbm_droplet * len(drops))(*[lbm.make_droplet(d) for d in drops])
    raw = np.frombuffer(bytes(table), dtype=np.uint8).copy()
    dd = torch.from_numpy(raw).to(dev)
    cfg = lbm.make_config(w.param_dict(), precision)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    rc = lbm.lbm_step_noalloc(cfg, stream.cuda_stream, [t.data_ptr() for t in f], [t.data_ptr() for t in phi],
                              [t.data_ptr() for t in c], len(drops), dd.data_ptr(), 0, nsteps)
    assert rc == lbm.LBM_OK, lbm.lbm_last_error()
    stream.synchronize()
    k = nsteps % 2
    out = (lbm.lbm_droplet * len(drops)).from_buffer_copy(dd.cpu().numpy().tobytes())
    return {"f": _pre_collision(f[k].cpu().numpy(), precision), "phi": phi[k].cpu().numpy().astype(np.float64),
            "c": c[k].cpu().numpy().astype(np.float64)}, [(d.x, d.y) for d in out]


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_noalloc_equals_lbm_step_on_two_calls_in_a_row(precision):
    import torch
    lbm = _lbm()
    rng = np.random.default_rng(70 + precision)
    cases = [(W.c2_single_active(n=96, seed=71), 37), (W.c1_equilibrium(seed=72), 24)]
    assert cases[1][0].nodes < cases[0][0].nodes
    for w, nsteps in cases:
        f_pre = WT[:, None, None] * (1.0 + rng.uniform(-0.01, 0.01, size=(9, w.ny, w.nx)))
        sim = lbm.Sim([w.param_dict()], [w.phi0], [w.c0], [w.drop_dicts()], precision=precision, f_pre=[f_pre],
                      graph_steps=0, path=lbm.LBM_PATH_WAVE)
        sim.set_seg_rows(40)
        start = sim.droplets()   # the centres after lbm_init's first pass: the state's r_CM at step 0
        got, centres = _noalloc_run(torch, lbm, w, f_pre, start, precision, nsteps)
        sim.step(nsteps)
        want = sim.fields()
        for k in ("f", "phi", "c"):
            assert np.array_equal(got[k], want[k]), (w.name, k, float(np.max(np.abs(got[k] - want[k]))))
        assert centres == [(d["x"], d["y"]) for d in sim.droplets()], w.name
        sim.close()


def test_noalloc_rejects_bad_arguments_before_any_device_call():
    lbm = _lbm()
    w = W.c1_equilibrium()
    cfg = lbm.make_config(w.param_dict(), 0)
    ok = [256, 512]
    assert lbm.lbm_step_noalloc(cfg, 0, [0, 512], ok, ok, 0, 0, 0, 1) == lbm.LBM_E_INVAL
    assert lbm.lbm_step_noalloc(cfg, 0, [256 + 8, 512], ok, ok, 0, 0, 0, 1) == lbm.LBM_E_INVAL
    assert lbm.lbm_step_noalloc(cfg, 0, ok, ok, ok, 1, 0, 0, 1) == lbm.LBM_E_INVAL
    assert lbm.lbm_step_noalloc(cfg, 0, ok, ok, ok, 0, 0, -1, 1) == lbm.LBM_E_INVAL
    bad = lbm.make_config(dict(w.param_dict(), tau=0.4), 0)
    assert lbm.lbm_step_noalloc(bad, 0, ok, ok, ok, 0, 0, 0, 1) == lbm.LBM_E_INVAL
    big = lbm.make_config(dict(w.param_dict(), nx=8192, ny=8192), 0)
    assert lbm.lbm_step_noalloc(big, 0, ok, ok, ok, 256, 256, 0, 1) == lbm.LBM_E_NOMEM
    assert "LBM_NOALLOC_SCRATCH_BYTES" in lbm.lbm_last_error()
