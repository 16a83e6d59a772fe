/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE, not the product.
 *
 * A plain, slow, FP64 CPU reference of one timestep of the hybrid
 * lattice-Boltzmann / finite-difference scheme for a ternary mixture with a
 * surfactant source, after Fadda, Gonnella, Lamura, Tiribocchi, "Lattice
 * Boltzmann study of chemically-driven self-propelled droplets" (EPJ E 2017,
 * arXiv:1711.10984), Sec. 2.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no source with the
 * HIP library; the two agree only on the public data formats (D2Q9 direction
 * order, row-major [ny][nx] fields with x fastest).
 *
 * Every step is written out in full-size arrays, in the order the paper states
 * the scheme, with periodic wrap by explicit index arithmetic.  No blocking, no
 * fusion.  Rows may be spread over OpenMP threads (each node is independent);
 * every reduction is serial in row-major order.
 *
 * Readings of the paper where it is silent or garbled (each one is listed in
 * the design notes):
 *  - Eq. (12): the second-order term of the equilibrium carries the usual 1/2,
 *    i.e. 4.5 (e.u)^2 - 1.5 u^2; without it the equilibrium has the wrong
 *    second moment (Sec. 2.2 states it is the 2nd-order Maxwell-Boltzmann
 *    expansion).
 *  - "centred scheme" for gradients of phi, c, mu and X: the isotropic D2Q9
 *    9-point gradient and Laplacian; the velocity divergence in the advection
 *    step (Eqs. 16-17) uses the 3-point centred difference; the concentration
 *    derivatives there are first-order upwind per axis by the sign of u_alpha.
 *  - Eq. (5)/(19): c grad(ln c) = grad c, so the surfactant flux
 *    D c grad(mu_c) is evaluated log-free as D lap(c) + div(D c grad X) with
 *    X = (B1/2)|grad phi|^2 (conservative link form); the force Eq. (14) uses
 *    the same identity, -c grad mu_c = -grad c - c grad X.
 *  - Time levels follow Eqs. (16)-(19) literally: b (phi^n)^3, B(c^{n+1/2}),
 *    u^n in the advection.  Both halves of a step read the state at time n.
 *  - Mobility Gamma multiplies the Laplacian of the bracket in Eq. (18) (the
 *    paper uses 1).
 *  - Source: A(n) = A0 min(n, t*) at the update n -> n+1 (Sec. 4), a closed
 *    disk of radius Rs around r_P = r_CM + (R - Rs) e_hat, minimum-image
 *    distance; consumption -gamma (c^{n+1/2} - c0) with constant c0.
 *  - Centre of mass (Sec. 4): over nodes with phi >= 0, each node assigned to
 *    the nearest previous centre (minimum image), offsets unwrapped about it.
 *  - Bounding walls (optional, walls = 1; Sec. 2.2 defers their implementation
 *    to a reference not reproduced, Sec. 2.3 fixes neutral wetting): solid
 *    plates halfway between node rows, at y = -1/2 and y = ny - 1/2; x stays
 *    periodic.  Populations: halfway bounce-back, a population streamed into a
 *    plate returns to its node in the opposite direction.  Every scalar field
 *    that enters a stencil (phi, c, mu, X and their half-step counterparts, M)
 *    is continued across a plate by its mirror image, g(x, -1) = g(x, 0) and
 *    g(x, ny) = g(x, ny - 1): this is n.grad(phi) = 0 (neutral wetting) and,
 *    link by link, zero diffusive flux through the plate (n.grad mu_phi =
 *    n.grad mu_c = 0).  In the advection stencil the ghost velocity is the
 *    mirror image with u_y reversed (no flow through the plate).  Droplet
 *    distances and centres are not periodic in y.
 *
 * Every function here is pinned by the CPU tests against closed forms,
 * textbook cases, exact identities or the paper's printed values.  Two
 * readings follow the paper's words but have no printed value to compare
 * with: the source geometry (Rs, r_P) and the droplet velocity as the
 * phi-weighted mean of u; the tests pin that the oracle computes them as
 * stated here, not that the paper computed them so.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXDROP 256

typedef struct {
  int32_t nx, ny;
  int32_t advection; /* 0: Eqs. (16)-(17) as printed; 1: conservative face-upwind flux form */
  int32_t walls;     /* 0: periodic in y; 1: plates at y = -1/2 and y = ny - 1/2 */
  double tau, n0;
  double a, b, B0, B1, D, Gamma;
  double gamma, A0, t_star, c0;
} orc_params;

typedef struct {
  double x, y;   /* current centre of mass r_CM */
  double R, Rs;  /* droplet radius, source radius */
  double ex, ey; /* unit vector from centre towards the source */
  int32_t active;
  int32_t reserved;
} orc_drop;

typedef struct {
  int64_t step;
  double mass, sum_phi, sum_c, min_B, max_u;
  int32_t nonfinite, ndrop;
} orc_obs_head;

/* D2Q9 links: rest, E, N, W, S, NE, NW, SW, SE (Sec. 2.2). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6}; /* e_OPP[i] = -e_i */
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Stage planes exported by orc_stages, in this order. */
enum {
  ST_MU, ST_X, ST_FX, ST_FY, ST_N, ST_UX, ST_UY, ST_PHIH, ST_CH, ST_M, ST_XH,
  ST_PHINEW, ST_CNEW, ST_FSTAR0, ST_COUNT = ST_FSTAR0 + 9
};

typedef struct {
  orc_params p;
  int64_t step;
  int ndrop;
  orc_drop drop[ORC_MAXDROP];
  double *f;      /* [9][N] pre-collision populations at time n */
  double *phi, *c; /* [N] */
} orc_sim;

/* Threads only pay off on large lattices; results do not depend on the thread count. */
#define PAR(p) ((long)(p)->nx * (long)(p)->ny >= 16384L)

/* Periodic wrap of an index at most one lattice length out of range. */
static inline int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
static inline size_t idx(const orc_params* p, int x, int y) {
  return (size_t)wrapi(y, p->ny) * (size_t)p->nx + (size_t)wrapi(x, p->nx);
}
/* Neighbour of a scalar field in a stencil: periodic in x; in y periodic, or with walls the mirror
   image across the plate (row -1 reads row 0, row ny reads row ny - 1). */
static inline size_t idxs(const orc_params* p, int x, int y) {
  if (p->walls) {
    if (y < 0) y = -1 - y;
    if (y >= p->ny) y = 2 * p->ny - 1 - y;
  }
  return idx(p, x, y);
}
/* Period of the y coordinate for droplet distances and centres (none with walls). */
static inline double yperiod(const orc_params* p) { return p->walls ? INFINITY : (double)p->ny; }

/* Minimum-image offset for a coordinate difference on a ring of length L. */
static double minimg(double d, double L) {
  if (d >= 0.5 * L) return d - L;
  if (d < -0.5 * L) return d + L;
  return d;
}
static double wrapd(double v, double L) {
  if (isinf(L)) return v;
  double r = fmod(v, L);
  if (r < 0.0) r += L;
  if (r >= L) r -= L;
  return r;
}

/* ---------------- stencils (Sec. 2.3, "centred scheme") ---------------- */
/* Isotropic gradient  sum_i (w_i / cs^2) e_i g(r + e_i). */
static void grad9(const orc_params* p, const double* g, double* gx, double* gy) {
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double E = g[idxs(p, x + 1, y)], Wv = g[idxs(p, x - 1, y)];
      double N = g[idxs(p, x, y + 1)], S = g[idxs(p, x, y - 1)];
      double NE = g[idxs(p, x + 1, y + 1)], NW = g[idxs(p, x - 1, y + 1)];
      double SW = g[idxs(p, x - 1, y - 1)], SE = g[idxs(p, x + 1, y - 1)];
      size_t k = idxs(p, x, y);
      gx[k] = (4.0 * (E - Wv) + ((NE - NW) + (SE - SW))) * (1.0 / 12.0);
      gy[k] = (4.0 * (N - S) + ((NE - SE) + (NW - SW))) * (1.0 / 12.0);
    }
}

/* Isotropic Laplacian  sum_{i>0} (2 w_i / cs^2) (g(r + e_i) - g(r)). */
static void lap9(const orc_params* p, const double* g, double* out) {
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double E = g[idxs(p, x + 1, y)], Wv = g[idxs(p, x - 1, y)];
      double N = g[idxs(p, x, y + 1)], S = g[idxs(p, x, y - 1)];
      double NE = g[idxs(p, x + 1, y + 1)], NW = g[idxs(p, x - 1, y + 1)];
      double SW = g[idxs(p, x - 1, y - 1)], SE = g[idxs(p, x + 1, y - 1)];
      size_t k = idxs(p, x, y);
      out[k] = (4.0 * ((E + Wv) + (N + S)) + ((NE + NW) + (SE + SW)) - 20.0 * g[k]) * (1.0 / 6.0);
    }
}

/* Conservative divergence of k grad X on the D2Q9 links:
 * sum_{i>0} (2 w_i / cs^2) * (k(r) + k(r+e_i))/2 * (X(r+e_i) - X(r)). */
static void div9(const orc_params* p, const double* kf, const double* X, double* out) {
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k0 = idxs(p, x, y);
      double kc = kf[k0], Xc = X[k0];
      double t[9];
      for (int i = 1; i < 9; ++i) {
        size_t ki = idxs(p, x + EX[i], y + EY[i]);
        t[i] = (kc + kf[ki]) * (X[ki] - Xc);
      }
      /* axis links weigh 4/12, diagonal links 1/12 */
      out[k0] = (4.0 * ((t[1] + t[3]) + (t[2] + t[4])) + ((t[5] + t[6]) + (t[7] + t[8]))) * (1.0 / 12.0);
    }
}

/* ---------------- droplet bookkeeping (Sec. 4, r_CM) ---------------- */
static int nearest_drop(const orc_sim* s, double x, double y) {
  int best = -1;
  double bd = 0.0;
  for (int k = 0; k < s->ndrop; ++k) {
    double dx = minimg(x - s->drop[k].x, (double)s->p.nx);
    double dy = minimg(y - s->drop[k].y, yperiod(&s->p));
    double d2 = dx * dx + dy * dy;
    if (best < 0 || d2 < bd) {
      best = k;
      bd = d2;
    }
  }
  return best;
}

/* S10: new centres from phi over phi >= 0, assigned to the nearest previous centre. */
static void update_centres(orc_sim* s, const double* phi) {
  const orc_params* p = &s->p;
  double sw[ORC_MAXDROP], sx[ORC_MAXDROP], sy[ORC_MAXDROP];
  for (int k = 0; k < s->ndrop; ++k) sw[k] = sx[k] = sy[k] = 0.0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double v = phi[(size_t)y * p->nx + x];
      if (!(v >= 0.0)) continue;
      int k = nearest_drop(s, (double)x, (double)y);
      if (k < 0) continue;
      double dx = minimg((double)x - s->drop[k].x, (double)p->nx);
      double dy = minimg((double)y - s->drop[k].y, yperiod(p));
      sw[k] += v;
      sx[k] += v * dx;
      sy[k] += v * dy;
    }
  for (int k = 0; k < s->ndrop; ++k) {
    if (sw[k] > 0.0) {
      s->drop[k].x = wrapd(s->drop[k].x + sx[k] / sw[k], (double)p->nx);
      s->drop[k].y = wrapd(s->drop[k].y + sy[k] / sw[k], yperiod(p));
    }
  }
}

/* Number of active source disks that contain node (x, y), Sec. 2.1 / Sec. 4. */
static int source_count(const orc_sim* s, int x, int y) {
  int cnt = 0;
  for (int k = 0; k < s->ndrop; ++k) {
    const orc_drop* d = &s->drop[k];
    if (!d->active) continue;
    double px = d->x + (d->R - d->Rs) * d->ex;
    double py = d->y + (d->R - d->Rs) * d->ey;
    double dx = minimg((double)x - px, (double)s->p.nx);
    double dy = minimg((double)y - py, yperiod(&s->p));
    if (dx * dx + dy * dy <= d->Rs * d->Rs) ++cnt;
  }
  return cnt;
}

/* ---------------- one timestep ---------------- */
/* S1-S4: force and velocity at time n from (f, phi, c).  Outputs full arrays. */
static void force_and_velocity(const orc_sim* s, double* mu, double* X, double* Fx, double* Fy,
                               double* n, double* ux, double* uy) {
  const orc_params* p = &s->p;
  size_t N = (size_t)p->nx * p->ny;
  double* gpx = malloc(N * sizeof(double));
  double* gpy = malloc(N * sizeof(double));
  double* gcx = malloc(N * sizeof(double));
  double* gcy = malloc(N * sizeof(double));
  double* lp = malloc(N * sizeof(double));
  double* gmx = malloc(N * sizeof(double));
  double* gmy = malloc(N * sizeof(double));
  double* gXx = malloc(N * sizeof(double));
  double* gXy = malloc(N * sizeof(double));
  const double* phi = s->phi;
  const double* c = s->c;

  /* S1: gradients and Laplacian at time n (Eq. 3) */
  grad9(p, phi, gpx, gpy);
  grad9(p, c, gcx, gcy);
  lap9(p, phi, lp);
  /* S2: mu_phi (Eq. 3) and X = (B1/2)|grad phi|^2, the gradient part of mu_c (Eq. 5) */
  double halfB1 = 0.5 * p->B1;
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    double ph = phi[k];
    double B = p->B0 + p->B1 * c[k];
    mu[k] = ((p->a * ph + p->b * (ph * ph * ph)) - B * lp[k]) - p->B1 * (gpx[k] * gcx[k] + gpy[k] * gcy[k]);
    X[k] = halfB1 * (gpx[k] * gpx[k] + gpy[k] * gpy[k]);
  }
  /* S3: F = -phi grad mu_phi - c grad mu_c = -phi grad mu - grad c - c grad X (Eq. 14) */
  grad9(p, mu, gmx, gmy);
  grad9(p, X, gXx, gXy);
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    Fx[k] = (-(phi[k] * gmx[k]) - gcx[k]) - c[k] * gXx[k];
    Fy[k] = (-(phi[k] * gmy[k]) - gcy[k]) - c[k] * gXy[k];
  }
  /* S4: moments with half the force (Eq. 11) */
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    double fi[9];
    for (int i = 0; i < 9; ++i) fi[i] = s->f[(size_t)i * N + k];
    /* sums grouped by mirror pairs, so that x- and y-reflections of the lattice are exact
       symmetries of the rounded arithmetic (axis links 1/3 and 2/4, diagonals 5/6, 7/8) */
    double nn = ((fi[0] + (fi[2] + fi[4])) + (fi[1] + fi[3])) + ((fi[5] + fi[6]) + (fi[7] + fi[8]));
    double mx = (fi[1] + (fi[5] + fi[8])) - (fi[3] + (fi[6] + fi[7])); /* links with e_x = +1 minus e_x = -1 */
    double my = (fi[2] + (fi[5] + fi[6])) - (fi[4] + (fi[7] + fi[8])); /* links with e_y = +1 minus e_y = -1 */
    n[k] = nn;
    ux[k] = (mx + 0.5 * Fx[k]) / nn;
    uy[k] = (my + 0.5 * Fy[k]) / nn;
  }
  free(gpx); free(gpy); free(gcx); free(gcy); free(lp);
  free(gmx); free(gmy); free(gXx); free(gXy);
}

/* Advection half-step, Eqs. (16)-(17), for one scalar g with velocity u^n. */
static void advect(const orc_params* p, const double* g, const double* ux, const double* uy, double* out) {
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = idx(p, x, y);
      size_t kE = idxs(p, x + 1, y), kW = idxs(p, x - 1, y);
      size_t kN = idxs(p, x, y + 1), kS = idxs(p, x, y - 1);
      double gc = g[k];
      /* y-velocity of the neighbours; across a plate the mirror image with the sign reversed */
      double uyN = (p->walls && y == p->ny - 1) ? -uy[kN] : uy[kN];
      double uyS = (p->walls && y == 0) ? -uy[kS] : uy[kS];
      if (p->advection == 0) {
        /* centred velocity divergence, upwind concentration gradient */
        double divu = 0.5 * (ux[kE] - ux[kW]) + 0.5 * (uyN - uyS);
        double dgx = ux[k] > 0.0 ? gc - g[kW] : g[kE] - gc;
        double dgy = uy[k] > 0.0 ? gc - g[kS] : g[kN] - gc;
        out[k] = gc - ((gc * divu + ux[k] * dgx) + uy[k] * dgy);
      } else {
        /* conservative form: face velocity = mean of the two nodes, upwind face value */
        double uxr = 0.5 * (ux[k] + ux[kE]), uxl = 0.5 * (ux[kW] + ux[k]);
        double uyt = 0.5 * (uy[k] + uyN), uyb = 0.5 * (uyS + uy[k]);
        double Fr = uxr * (uxr >= 0.0 ? gc : g[kE]);
        double Fl = uxl * (uxl >= 0.0 ? g[kW] : gc);
        double Ft = uyt * (uyt >= 0.0 ? gc : g[kN]);
        double Fb = uyb * (uyb >= 0.0 ? g[kS] : gc);
        out[k] = gc - ((Fr - Fl) + (Ft - Fb));
      }
    }
}

/* One full step n -> n+1.  If st != NULL the intermediate planes are exported
 * (and the state is left unchanged). */
static void do_step(orc_sim* s, double* st) {
  const orc_params* p = &s->p;
  size_t N = (size_t)p->nx * p->ny;
  double* mu = malloc(N * sizeof(double));
  double* X = malloc(N * sizeof(double));
  double* Fx = malloc(N * sizeof(double));
  double* Fy = malloc(N * sizeof(double));
  double* n = malloc(N * sizeof(double));
  double* ux = malloc(N * sizeof(double));
  double* uy = malloc(N * sizeof(double));
  double* fstar = malloc(9 * N * sizeof(double));
  double* fnew = malloc(9 * N * sizeof(double));
  double* ph = malloc(N * sizeof(double));
  double* ch = malloc(N * sizeof(double));
  double* gphx = malloc(N * sizeof(double));
  double* gphy = malloc(N * sizeof(double));
  double* gchx = malloc(N * sizeof(double));
  double* gchy = malloc(N * sizeof(double));
  double* lph = malloc(N * sizeof(double));
  double* lch = malloc(N * sizeof(double));
  double* M = malloc(N * sizeof(double));
  double* lM = malloc(N * sizeof(double));
  double* Xh = malloc(N * sizeof(double));
  double* kD = malloc(N * sizeof(double));
  double* dv = malloc(N * sizeof(double));
  double* phinew = malloc(N * sizeof(double));
  double* cnew = malloc(N * sizeof(double));

  /* S1-S4 */
  force_and_velocity(s, mu, X, Fx, Fy, n, ux, uy);

  /* S5: BGK collision with the equilibrium of Eq. (12) and the forcing of Eq. (13) */
  double omega = 1.0 / p->tau;
  double coef = 1.0 - 1.0 / (2.0 * p->tau);
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    double usq = ux[k] * ux[k] + uy[k] * uy[k];
    for (int i = 0; i < 9; ++i) {
      double exd = (double)EX[i], eyd = (double)EY[i];
      double eu = exd * ux[k] + eyd * uy[k];
      double eF = exd * Fx[k] + eyd * Fy[k];
      double feq = W[i] * n[k] * (((1.0 + 3.0 * eu) + 4.5 * eu * eu) - 1.5 * usq);
      double Fi = coef * W[i] * (3.0 * ((exd - ux[k]) * Fx[k] + (eyd - uy[k]) * Fy[k]) + 9.0 * eu * eF);
      double fi = s->f[(size_t)i * N + k];
      fstar[(size_t)i * N + k] = (fi - omega * (fi - feq)) + Fi;
    }
  }
  /* S6: streaming f_i(r + e_i, n + 1) = f*_i(r) (Eq. 10); with walls, a population that would enter a
     plate is bounced back: f_OPP[i](r, n + 1) = f*_i(r) */
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x)
      for (int i = 0; i < 9; ++i) {
        int yy = y + EY[i];
        if (p->walls && (yy < 0 || yy >= p->ny))
          fnew[(size_t)OPP[i] * N + idx(p, x, y)] = fstar[(size_t)i * N + idx(p, x, y)];
        else
          fnew[(size_t)i * N + idx(p, x + EX[i], yy)] = fstar[(size_t)i * N + idx(p, x, y)];
      }

  /* S7: Euler advection half-step with u^n (Eqs. 16-17) */
  advect(p, s->phi, ux, uy, ph);
  advect(p, s->c, ux, uy, ch);

  /* S8: phi diffusion step (Eq. 18) */
  grad9(p, ph, gphx, gphy);
  grad9(p, ch, gchx, gchy);
  lap9(p, ph, lph);
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    double pn = s->phi[k];
    double Bh = p->B0 + p->B1 * ch[k];
    M[k] = ((p->a * ph[k] + p->b * (pn * pn * pn)) - Bh * lph[k]) - p->B1 * (gchx[k] * gphx[k] + gchy[k] * gphy[k]);
  }
  lap9(p, M, lM);
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) phinew[k] = ph[k] + p->Gamma * lM[k];

  /* S9: surfactant diffusion, consumption and production (Eq. 19) */
  double halfB1 = 0.5 * p->B1;
#pragma omp parallel for schedule(static) if (PAR(p))
  for (long k = 0; k < (long)N; ++k) {
    Xh[k] = halfB1 * (gphx[k] * gphx[k] + gphy[k] * gphy[k]);
    kD[k] = p->D * ch[k];
  }
  lap9(p, ch, lch);
  div9(p, kD, Xh, dv);
  double tn = (double)s->step;
  double A = p->A0 * (tn < p->t_star ? tn : p->t_star);
#pragma omp parallel for schedule(static) if (PAR(p))
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      double src = A * (double)source_count(s, x, y);
      cnew[k] = (((ch[k] + p->D * lch[k]) + dv[k]) - p->gamma * (ch[k] - p->c0)) + src;
    }

  if (st) {
    memcpy(st + (size_t)ST_MU * N, mu, N * sizeof(double));
    memcpy(st + (size_t)ST_X * N, X, N * sizeof(double));
    memcpy(st + (size_t)ST_FX * N, Fx, N * sizeof(double));
    memcpy(st + (size_t)ST_FY * N, Fy, N * sizeof(double));
    memcpy(st + (size_t)ST_N * N, n, N * sizeof(double));
    memcpy(st + (size_t)ST_UX * N, ux, N * sizeof(double));
    memcpy(st + (size_t)ST_UY * N, uy, N * sizeof(double));
    memcpy(st + (size_t)ST_PHIH * N, ph, N * sizeof(double));
    memcpy(st + (size_t)ST_CH * N, ch, N * sizeof(double));
    memcpy(st + (size_t)ST_M * N, M, N * sizeof(double));
    memcpy(st + (size_t)ST_XH * N, Xh, N * sizeof(double));
    memcpy(st + (size_t)ST_PHINEW * N, phinew, N * sizeof(double));
    memcpy(st + (size_t)ST_CNEW * N, cnew, N * sizeof(double));
    memcpy(st + (size_t)ST_FSTAR0 * N, fstar, 9 * N * sizeof(double));
  } else {
    memcpy(s->f, fnew, 9 * N * sizeof(double));
    memcpy(s->phi, phinew, N * sizeof(double));
    memcpy(s->c, cnew, N * sizeof(double));
    s->step += 1;
    /* S10: centres of mass from phi^{n+1} */
    update_centres(s, s->phi);
  }

  free(mu); free(X); free(Fx); free(Fy); free(n); free(ux); free(uy);
  free(fstar); free(fnew); free(ph); free(ch); free(gphx); free(gphy); free(gchx); free(gchy);
  free(lph); free(lch); free(M); free(lM); free(Xh); free(kD); free(dv); free(phinew); free(cnew);
}

/* ---------------- public entry points (ctypes) ---------------- */
orc_sim* orc_new(const orc_params* p, const double* f_pre, const double* phi, const double* c,
                 int64_t step, int ndrop, const orc_drop* drops) {
  if (p->nx < 3 || p->ny < 3 || ndrop < 0 || ndrop > ORC_MAXDROP) return NULL;
  orc_sim* s = calloc(1, sizeof(orc_sim));
  s->p = *p;
  s->step = step;
  s->ndrop = ndrop;
  size_t N = (size_t)p->nx * p->ny;
  s->f = malloc(9 * N * sizeof(double));
  s->phi = malloc(N * sizeof(double));
  s->c = malloc(N * sizeof(double));
  if (f_pre) {
    memcpy(s->f, f_pre, 9 * N * sizeof(double));
  } else {
    /* initial populations at rest with density n0 */
    for (int i = 0; i < 9; ++i)
      for (size_t k = 0; k < N; ++k) s->f[(size_t)i * N + k] = W[i] * p->n0;
  }
  memcpy(s->phi, phi, N * sizeof(double));
  memcpy(s->c, c, N * sizeof(double));
  for (int k = 0; k < ndrop; ++k) s->drop[k] = drops[k];
  /* initial centres: one S10 pass on phi^0 about the given centres */
  update_centres(s, s->phi);
  return s;
}

void orc_free(orc_sim* s) {
  if (!s) return;
  free(s->f); free(s->phi); free(s->c);
  free(s);
}

void orc_run(orc_sim* s, int64_t nsteps) {
  for (int64_t t = 0; t < nsteps; ++t) do_step(s, NULL);
}

int orc_stage_count(void) { return ST_COUNT; }

/* Threads the OpenMP loops run on (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads the loops of an nx x ny lattice run on (small lattices run on one). */
int orc_threads_for(int nx, int ny) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  return PAR(&p) ? orc_num_threads() : 1;
}

void orc_stages(orc_sim* s, double* out) { do_step(s, out); }

int64_t orc_get_step(const orc_sim* s) { return s->step; }

void orc_get_drops(const orc_sim* s, orc_drop* out) {
  for (int k = 0; k < s->ndrop; ++k) out[k] = s->drop[k];
}

/* Fields at time n; n and u from S1-S4 applied to the current state. */
void orc_fields(const orc_sim* s, double* f, double* phi, double* c, double* n, double* ux, double* uy) {
  const orc_params* p = &s->p;
  size_t N = (size_t)p->nx * p->ny;
  if (f) memcpy(f, s->f, 9 * N * sizeof(double));
  if (phi) memcpy(phi, s->phi, N * sizeof(double));
  if (c) memcpy(c, s->c, N * sizeof(double));
  if (n || ux || uy) {
    double* mu = malloc(N * sizeof(double));
    double* X = malloc(N * sizeof(double));
    double* Fx = malloc(N * sizeof(double));
    double* Fy = malloc(N * sizeof(double));
    double* nn = malloc(N * sizeof(double));
    double* vx = malloc(N * sizeof(double));
    double* vy = malloc(N * sizeof(double));
    force_and_velocity(s, mu, X, Fx, Fy, nn, vx, vy);
    if (n) memcpy(n, nn, N * sizeof(double));
    if (ux) memcpy(ux, vx, N * sizeof(double));
    if (uy) memcpy(uy, vy, N * sizeof(double));
    free(mu); free(X); free(Fx); free(Fy); free(nn); free(vx); free(vy);
  }
}

/* Conserved sums and droplet observables at time n.
 * drop_out: per droplet {x_cm, y_cm, vx, vy, sum_phi}. */
void orc_observables(const orc_sim* s, orc_obs_head* head, double* drop_out) {
  const orc_params* p = &s->p;
  size_t N = (size_t)p->nx * p->ny;
  double* nn = malloc(N * sizeof(double));
  double* vx = malloc(N * sizeof(double));
  double* vy = malloc(N * sizeof(double));
  orc_fields(s, NULL, NULL, NULL, nn, vx, vy);
  double mass = 0.0, sp = 0.0, sc = 0.0, minB = INFINITY, maxu = 0.0;
  int nonfinite = 0;
  double sw[ORC_MAXDROP], su[ORC_MAXDROP], sv[ORC_MAXDROP];
  for (int k = 0; k < s->ndrop; ++k) sw[k] = su[k] = sv[k] = 0.0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      double fi[9];
      for (int i = 0; i < 9; ++i) {
        fi[i] = s->f[(size_t)i * N + k];
        if (!isfinite(fi[i])) nonfinite = 1;
      }
      mass += nn[k];
      sp += s->phi[k];
      sc += s->c[k];
      if (!isfinite(s->phi[k]) || !isfinite(s->c[k])) nonfinite = 1;
      double B = p->B0 + p->B1 * s->c[k];
      if (B < minB) minB = B;
      double um = sqrt(vx[k] * vx[k] + vy[k] * vy[k]);
      if (um > maxu) maxu = um;
      double v = s->phi[k];
      if (v >= 0.0) {
        int d = nearest_drop(s, (double)x, (double)y);
        if (d >= 0) {
          sw[d] += v;
          su[d] += v * vx[k];
          sv[d] += v * vy[k];
        }
      }
    }
  head->step = s->step;
  head->mass = mass;
  head->sum_phi = sp;
  head->sum_c = sc;
  head->min_B = minB;
  head->max_u = maxu;
  head->nonfinite = nonfinite;
  head->ndrop = s->ndrop;
  for (int k = 0; k < s->ndrop; ++k) {
    drop_out[5 * k + 0] = s->drop[k].x;
    drop_out[5 * k + 1] = s->drop[k].y;
    drop_out[5 * k + 2] = sw[k] > 0.0 ? su[k] / sw[k] : 0.0;
    drop_out[5 * k + 3] = sw[k] > 0.0 ? sv[k] / sw[k] : 0.0;
    drop_out[5 * k + 4] = sw[k];
  }
  free(nn); free(vx); free(vy);
}

/* Stencil primitives, exported for the Fourier-symbol pins. */
void orc_grad9(int nx, int ny, const double* g, double* gx, double* gy) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  grad9(&p, g, gx, gy);
}
void orc_lap9(int nx, int ny, const double* g, double* out) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  lap9(&p, g, out);
}
void orc_div9(int nx, int ny, const double* k, const double* X, double* out) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  div9(&p, k, X, out);
}
