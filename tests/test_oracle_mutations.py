"""Sensitivity of the oracle's pins: plant a plausible mistake in a copy of the oracle (on the CPU), build
it, and check that the fast pin suite fails.  Eight of them always run (about 30 s); all of them (about two
minutes) with LBM_MUTATION_CHECK=1.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
PINS = ["tests/test_oracle_thermo.py", "tests/test_oracle_stencils.py", "tests/test_oracle_lb.py",
        "tests/test_oracle_fd.py", "tests/test_oracle_equilibrium.py", "tests/test_oracle_walls.py",
        "tests/test_oracle_droplets.py"]

MUTATIONS = [
    ("equilibrium without the 1/2", "4.5 * eu * eu", "9.0 * eu * eu"),
    ("forcing sign", "(exd - ux[k])", "(exd + ux[k])"),
    ("velocity without half force", "(mx + 0.5 * Fx[k])", "(mx + Fx[k])"),
    ("force: sign of grad c", "-(phi[k] * gmx[k]) - gcx[k]", "-(phi[k] * gmx[k]) + gcx[k]"),
    ("force: sign of c grad X", "- c[k] * gXx[k]", "+ c[k] * gXx[k]"),
    ("force: sign of phi grad mu", "(-(phi[k] * gmy[k])", "((phi[k] * gmy[k])"),
    ("upwind side reversed", "ux[k] > 0.0 ? gc - g[kW] : g[kE] - gc", "ux[k] > 0.0 ? g[kE] - gc : gc - g[kW]"),
    ("centred divergence sign", "0.5 * (ux[kE] - ux[kW])", "0.5 * (ux[kW] - ux[kE])"),
    ("cubic term at the half step", "p->b * (pn * pn * pn)", "p->b * (ph[k] * ph[k] * ph[k])"),
    ("gradient axes mixed", "gy[k] = (4.0 * (N - S)", "gy[k] = (4.0 * (E - Wv)"),
    ("Laplacian centre weight", "- 20.0 * g[k]", "- 16.0 * g[k]"),
    ("streaming reversed", "idx(p, x + EX[i], yy)] = fstar", "idx(p, x - EX[i], y - EY[i])] = fstar"),
    ("source disk radius", "<= d->Rs * d->Rs", "< d->Rs * d->Rs * 0.5"),
    ("consumption sign", "- p->gamma * (ch[k] - p->c0)", "+ p->gamma * (ch[k] - p->c0)"),
    ("link mobility from one end", "(kc + kf[ki])", "(2.0 * kc)"),
    ("sign of X in mu_c", "    X[k] = halfB1 *", "    X[k] = -halfB1 *"),
    ("B1 dropped from B(c) in mu", "double B = p->B0 + p->B1 * c[k];", "double B = p->B0;"),
    ("B1 dropped from B(c) in M", "double Bh = p->B0 + p->B1 * ch[k];", "double Bh = p->B0;"),
    ("mu: sign of grad phi . grad c", "- p->B1 * (gpx[k] * gcx[k] + gpy[k] * gcy[k])",
     "+ p->B1 * (gpx[k] * gcx[k] + gpy[k] * gcy[k])"),
    ("M: sign of grad c . grad phi", "- p->B1 * (gchx[k] * gphx[k] + gchy[k] * gphy[k])",
     "+ p->B1 * (gchx[k] * gphx[k] + gchy[k] * gphy[k])"),
    ("mobility Gamma ignored", "ph[k] + p->Gamma * lM[k]", "ph[k] + lM[k]"),
    ("surfactant diffusion dropped", "(ch[k] + p->D * lch[k])", "(ch[k])"),
    ("ramp not clipped at t*", "(tn < p->t_star ? tn : p->t_star)", "(tn)"),
    ("momentum from the wrong diagonals", "double my = (fi[2] + (fi[5] + fi[6])) - (fi[4] + (fi[7] + fi[8]));",
     "double my = (fi[2] + (fi[5] + fi[8])) - (fi[4] + (fi[7] + fi[6]));"),
    ("centre of mass unweighted", "sx[k] += v * dx;", "sx[k] += dx;"),
    ("relaxation rate", "double omega = 1.0 / p->tau;", "double omega = 1.0 / (p->tau + 0.1);"),
    ("walls: bounce-back to the mirror diagonal", "OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6}",
     "OPP[9] = {0, 3, 4, 1, 2, 8, 7, 6, 5}"),
    ("walls: mirror ghost one row off", "if (y < 0) y = -1 - y;", "if (y < 0) y = -y;"),
    ("walls: top plate mirrored off by one", "if (y >= p->ny) y = 2 * p->ny - 1 - y;",
     "if (y >= p->ny) y = 2 * p->ny - 2 - y;"),
    ("walls: ghost velocity not reversed", "(p->walls && y == 0) ? -uy[kS] : uy[kS]",
     "(p->walls && y == 0) ? uy[kS] : uy[kS]"),
    ("B(c) of Eq. (18) at time n", "double Bh = p->B0 + p->B1 * ch[k];", "double Bh = p->B0 + p->B1 * s->c[k];"),
    ("flux form: face value from the downwind node (x)",
     "double Fr = uxr * (uxr >= 0.0 ? gc : g[kE]);\n        double Fl = uxl * (uxl >= 0.0 ? g[kW] : gc);",
     "double Fr = uxr * (uxr >= 0.0 ? g[kE] : gc);\n        double Fl = uxl * (uxl >= 0.0 ? gc : g[kW]);"),
    ("flux form: face value from the downwind node (y)",
     "double Ft = uyt * (uyt >= 0.0 ? gc : g[kN]);\n        double Fb = uyb * (uyb >= 0.0 ? g[kS] : gc);",
     "double Ft = uyt * (uyt >= 0.0 ? g[kN] : gc);\n        double Fb = uyb * (uyb >= 0.0 ? gc : g[kS]);"),
    ("flux form: face velocity from one node", "double uxr = 0.5 * (ux[k] + ux[kE]), uxl = 0.5 * (ux[kW] + ux[k]);",
     "double uxr = ux[k], uxl = ux[kW];"),
    ("centre of mass: ties to the highest index", "if (best < 0 || d2 < bd) {", "if (best < 0 || d2 <= bd) {"),
    ("centre of mass: x offset not unwrapped", "double dx = minimg((double)x - s->drop[k].x, (double)p->nx);",
     "double dx = (double)x - s->drop[k].x;"),
    ("centre of mass: y offset wrapped with the x period",
     "double dy = minimg((double)y - s->drop[k].y, yperiod(p));",
     "double dy = minimg((double)y - s->drop[k].y, (double)p->nx);"),
    ("centre of mass: new centre not wrapped", "s->drop[k].x = wrapd(s->drop[k].x + sx[k] / sw[k], (double)p->nx);",
     "s->drop[k].x = s->drop[k].x + sx[k] / sw[k];"),
    ("centre of mass: nodes assigned to the nearest production disk",
     "double dx = minimg(x - s->drop[k].x, (double)s->p.nx);\n    double dy = minimg(y - s->drop[k].y, yperiod(&s->p));",
     "double dx = minimg(x - s->drop[k].x - (s->drop[k].R - s->drop[k].Rs) * s->drop[k].ex, (double)s->p.nx);\n"
     "    double dy = minimg(y - s->drop[k].y - (s->drop[k].R - s->drop[k].Rs) * s->drop[k].ey, yperiod(&s->p));"),
    ("observables: min B with the sign of B1 reversed", "p->B0 + p->B1 * s->c[k]", "p->B0 - p->B1 * s->c[k]"),
    ("observables: max|u| from u_x only", "double um = sqrt(vx[k] * vx[k] + vy[k] * vy[k]);",
     "double um = fabs(vx[k]);"),
    ("observables: droplet velocity unweighted", "su[d] += v * vx[k];", "su[d] += vx[k];"),
    ("observables: droplet velocity components swapped", "su[d] += v * vx[k];\n          sv[d] += v * vy[k];",
     "su[d] += v * vy[k];\n          sv[d] += v * vx[k];"),
    ("observables: sum c over phi", "sc += s->c[k];", "sc += s->phi[k];"),
]


# always run: one planted mistake from each part of the step (about 20 s); LBM_MUTATION_CHECK=1 runs them all
DEFAULT = {"equilibrium without the 1/2", "force: sign of grad c", "upwind side reversed", "Laplacian centre weight",
           "consumption sign", "walls: mirror ghost one row off", "B(c) of Eq. (18) at time n",
           "centre of mass: ties to the highest index"}


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new):
    if name not in DEFAULT and os.environ.get("LBM_MUTATION_CHECK") != "1":
        pytest.skip("set LBM_MUTATION_CHECK=1 (all mutations, about two minutes)")
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    with tempfile.TemporaryDirectory() as d:
        c_file = os.path.join(d, "mutant.c")
        lib = os.path.join(d, "libmutant.so")
        with open(c_file, "w") as fh:
            fh.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", lib,
                        c_file, "-lm"], check=True)
        env = dict(os.environ, LBM_ORACLE_LIB=lib, LBM_MUTATION_CHECK="0")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow", "-p", "no:cacheprovider"]
                           + PINS, cwd=ROOT, env=env, capture_output=True, text=True)
        assert r.returncode != 0, f"the pins did not notice: {name}"
