/* Drives the oracle through its C interface on edge-case lattices, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (the oracle source is compiled into this program).  Exit status 0 and no sanitizer
 * report mean: no out-of-bounds access, use after free, leak or undefined behaviour on these cases. */
#include "lbm_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double urand(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int nx, int ny, int walls, int advection, int ndrop, int steps) {
  const size_t n = (size_t)nx * ny;
  double* phi = malloc(n * sizeof(double));
  double* c = malloc(n * sizeof(double));
  double* f = malloc(9 * n * sizeof(double));
  double* out = malloc((size_t)ST_COUNT * n * sizeof(double));
  double* fo = malloc(9 * n * sizeof(double));
  double* fields[6];
  for (int k = 0; k < 6; ++k) fields[k] = malloc(n * sizeof(double));
  double* dout = malloc((size_t)(ndrop > 0 ? ndrop : 1) * 5 * sizeof(double));
  orc_drop drops[8];
  static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (size_t i = 0; i < n; ++i) {
    phi[i] = 1.8 * urand() - 0.9;
    c[i] = 0.05 + 0.1 * urand();
    for (int k = 0; k < 9; ++k) f[k * n + i] = w[k] * (1.0 + 0.04 * (urand() - 0.5));
  }
  for (int k = 0; k < ndrop; ++k) {
    drops[k].x = k == 0 ? 0.2 : urand() * nx;  /* the first one on the periodic edge */
    drops[k].y = k == 0 ? ny - 0.3 : urand() * ny;
    drops[k].R = 1.0 + 0.3 * (nx < ny ? nx : ny) * urand();
    drops[k].Rs = 0.25 * drops[k].R;
    drops[k].ex = 1.0;
    drops[k].ey = 0.0;
    drops[k].active = k % 2 == 0;
    drops[k].reserved = 0;
  }
  orc_params p = {nx, ny, advection, walls, 0.8, 1.0, -0.001, 0.001, 0.006, -0.05, 0.1, 0.7,
                  0.01, 1e-3, 50.0, 0.02};
  orc_sim* s = orc_new(&p, f, phi, c, 3, ndrop, drops);
  if (!s) return 1;
  orc_stages(s, out);
  orc_run(s, steps);
  orc_fields(s, fo, fields[0], fields[1], fields[2], fields[3], fields[4]);
  orc_obs_head head;
  orc_observables(s, &head, dout);
  orc_drop got[8];
  if (ndrop > 0) orc_get_drops(s, got);
  printf("%dx%d walls=%d adv=%d drops=%d: mass %.12f nonfinite %d\n", nx, ny, walls, advection, ndrop, head.mass,
         head.nonfinite);
  orc_free(s);
  free(phi);
  free(c);
  free(f);
  free(out);
  free(fo);
  for (int k = 0; k < 6; ++k) free(fields[k]);
  free(dout);
  return head.nonfinite != 0;
}

int main(void) {
  int bad = 0;
  bad |= run_case(3, 3, 0, 0, 2, 10);
  bad |= run_case(3, 4, 1, 1, 1, 10);
  bad |= run_case(5, 7, 1, 0, 3, 12);
  bad |= run_case(37, 4, 1, 1, 2, 15);
  bad |= run_case(64, 48, 0, 0, 5, 20);
  bad |= run_case(64, 48, 1, 1, 5, 20);
  bad |= run_case(17, 3, 0, 1, 0, 8);
  return bad;
}
