"""Self-propulsion in the plate geometry of Sec. 4, on the GPU path (FP64).

A droplet of radius 32 in the middle of a 512 x 256 box between two plates, surfactant 0.1 everywhere, B0 = 0.006,
tau = 0.6.  The two signs of B1 (-0.05 and +0.05) run as one batch.  The fluid first relaxes for 2e5 steps without
production or consumption.  Then consumption (gamma = 1.5e-3) and production A(t) = A0 t (A0 = gamma / 1e7) in a
disk of radius R/4 touching the interface from inside on the +x side are switched on, with the ramp counted from
the switch (Sec. 4).  Checked over the next 4e5 steps:
* B1 < 0: the droplet moves along +x, towards the production side; its velocity grows while the production rate
  ramps up (each 1e5-step displacement exceeds the previous one); it stays on the mid-plane;
* the B1 < 0 droplet is faster than the B1 > 0 one;
* the bulk surfactant relaxes to c0 under consumption; B(c) > 0 everywhere (the stability condition of Sec. 4).
The paper also reports +x motion for B1 > 0.  With these parameters the B1 > 0 droplet drifts slowly towards -x
instead.  This is not asserted: the paper leaves the source-disk size, c0 and the source position open.
"""
import numpy as np
import pytest

from paper_1711_10984_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_active_droplet_between_plates():
    from paper_1711_10984_amd import lbm
    w = W.plates_single_active()
    B1s = (-0.05, 0.05)
    relax = [dict(w.param_dict(), B1=b, A0=0.0, gamma=0.0) for b in B1s]
    s = lbm.Sim(relax, [w.phi0] * 2, [w.c0] * 2, [w.drop_dicts()] * 2, graph_steps=100)
    s.autotune(10, both_paths=True)
    s.step(200000)
    F = [s.fields(i) for i in range(2)]
    D = [s.droplets(i)[0] for i in range(2)]
    s.close()
    active = [dict(w.param_dict(), B1=b) for b in B1s]
    drops = [[dict(D[i], ex=1.0, ey=0.0, active=1)] for i in range(2)]
    s = lbm.Sim(active, [F[i]["phi"] for i in range(2)], [F[i]["c"] for i in range(2)], drops,
                f_pre=[F[i]["f"] for i in range(2)], graph_steps=100)
    s.autotune(10, both_paths=True)
    x0 = [D[i]["x"] for i in range(2)]
    traj = [[], []]
    for _ in range(4):
        s.step(100000)
        for i in range(2):
            d = s.droplets(i)[0]
            o = s.observables(i)
            assert not o["unstable"] and o["min_B"] > 0.0
            traj[i].append((d["x"] - x0[i], d["y"]))
    bulk = []
    for i in range(2):
        Fi = s.fields(i)
        bulk.append(float(np.mean(Fi["c"][Fi["phi"] < -0.9])))
    s.close()
    print("B1 = -0.05:", traj[0])
    print("B1 = +0.05:", traj[1])
    print("bulk c:", bulk)
    dx_neg = [t[0] for t in traj[0]]
    steps = np.diff([0.0] + dx_neg)
    assert dx_neg[-1] > 2.0
    assert np.all(steps > 0) and np.all(np.diff(steps) > 0)
    assert max(abs(t[1] - w.ny / 2) for t in traj[0]) < 0.1
    assert abs(traj[1][-1][0]) < 0.5 * dx_neg[-1]
    assert max(bulk) < 1e-3  # c0 = 0
