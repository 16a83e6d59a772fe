/* Plain C99 caller of the library (no GPU calls): include/lbm.h must compile as C and the host-only entry
 * points must answer as the Python binding does.  Prints one "key value" pair per line. */
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static lbm_config config(int32_t nx, int32_t ny, int32_t precision) {
  lbm_config c;
  memset(&c, 0, sizeof c);
  c.nx = nx;
  c.ny = ny;
  c.precision = precision;
  c.advection = LBM_ADV_PAPER;
  c.walls = LBM_WALLS_NONE;
  c.tau = 1.0;
  c.n0 = 1.0;
  c.a = -0.001;
  c.b = 0.001;
  c.B0 = 0.006;
  c.B1 = -0.05;
  c.D = 0.1;
  c.Gamma = 1.0;
  c.t_star = 2.0e6;
  return c;
}

int main(void) {
  lbm_config cfg[2];
  int32_t ndrop[2] = {1, 0};
  size_t bytes = 0;
  int rc;
  cfg[0] = config(256, 256, LBM_FP64);
  cfg[1] = config(100, 37, LBM_FP64);
  rc = lbm_workspace_bytes(1, cfg, ndrop, &bytes);
  printf("single_rc %d\nsingle_bytes %zu\n", rc, bytes);
  rc = lbm_workspace_bytes(2, cfg, ndrop, &bytes);
  printf("batch_rc %d\nbatch_bytes %zu\n", rc, bytes);
  cfg[0].nx = 2;
  rc = lbm_workspace_bytes(1, cfg, ndrop, &bytes);
  printf("bad_rc %d\nbad_has_message %d\n", rc, (int)(strlen(lbm_last_error()) > 0));
  printf("sizeof_config %zu\nsizeof_droplet %zu\nsizeof_obs %zu\n", sizeof(lbm_config), sizeof(lbm_droplet),
         sizeof(lbm_obs));
  printf("first_tune_row %d\nwave_kernel %s\n", (int)lbm_tune_rows()[0], lbm_kernel_name(LBM_PATH_WAVE, 0));
  return 0;
}
