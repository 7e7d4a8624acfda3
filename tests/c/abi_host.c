/* Plain C99 use of the libpd ABI without a device: version, grid creation,
   field validation (every field kind, fourth-order table length, y component),
   valley selection, error statuses and messages.  Prints one line per check;
   the exit status is the number of failed checks. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "pd.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  printf("%s %s\n", cond ? "ok  " : "FAIL", what);
  if (!cond) ++failures;
}

int main(void) {
  pd_grid g = NULL;
  pd_info info;
  pd_field f;
  double A[50];
  int i;

  expect(strstr(pd_version(), "gfx950") != NULL, "version names the target");
  expect(pd_create_grid(0, 8, -1.0, 1.0, -1.0, 1.0, PD_FP64, PD_SCHEME_STRANG, &g) == PD_ERR_INVALID && g == NULL,
         "nx = 0 rejected");
  expect(strlen(pd_last_error()) > 0, "error message set");
  expect(pd_create_grid(64, 64, -2.0, 2.0, -2.0, 2.0, PD_FP32, PD_SCHEME_STRANG4, &g) == PD_OK && g != NULL,
         "fourth-order grid created");

  memset(&f, 0, sizeof f);
  f.kind = PD_FIELD_SIN2;
  f.E0 = 0.1;
  f.omega = 0.5;
  f.cycles = 8;
  expect(pd_check_field(g, &f, 1000, &info) == PD_OK, "sin2 field accepted");
  expect(info.stages == 5 && info.elliptic == 0 && info.n_masked == 1 && info.valley == PD_VALLEYS_BOTH,
         "info: stages, polarisation, masked point, valley");
  expect(fabs(info.dt - 8 * 2 * M_PI / 0.5 / 1000) < 1e-15, "info: dt");
  expect(pd_check_field(g, &f, 20, &info) == PD_ERR_INVALID, "step condition dt E_max <= pi enforced");

  f.ellipticity = 0.5;
  expect(pd_check_field(g, &f, 1000, &info) == PD_OK && info.elliptic == 1, "y component reported");

  memset(&f, 0, sizeof f);
  f.kind = PD_FIELD_TABLE;
  for (i = 0; i < 50; ++i) A[i] = 0.01 * i;
  f.A_mid = A;
  f.n_table = 10;
  f.t_i = 0.0;
  f.t_f = 1.0;
  expect(pd_check_field(g, &f, 10, &info) == PD_ERR_INVALID, "fourth-order table needs 5 samples per step");
  f.n_table = 50;
  expect(pd_check_field(g, &f, 10, &info) == PD_OK, "fourth-order table with 5 N samples accepted");

  expect(pd_set_valley(g, PD_VALLEY_KMINUS) == PD_OK, "valley K- selected before a field");
  expect(pd_get_info(g, &info) == PD_OK && info.valley == PD_VALLEY_KMINUS, "info: valley");
  expect(pd_set_valley(g, 9) == PD_ERR_INVALID, "unknown valley rejected");
  expect(pd_propagate(g, -1, NULL) == PD_ERR_STATE, "propagate before a field: state error");
  expect(pd_snapshot(g, NULL, 0, NULL, NULL) == PD_ERR_STATE, "snapshot before a field: state error");
  expect(pd_solve_bytes(g, 1000) > 0, "closed-form footprint");
  pd_destroy_grid(g);
  pd_destroy_grid(NULL);
  return failures;
}
