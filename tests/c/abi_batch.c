/* Plain C99 batch on the device through the libpd ABI, with no other runtime in the
   process.  Four members: three second-order Strang solves of fields along x (two FP32,
   one FP64; they share the persistent kernel) and one midpoint solve (its own launch
   beside it), on ragged grids under sin^2 pulses.  Each member is first solved alone
   (pd_propagate, pd_density); then the batch runs every whole solve twice
   (pd_batch_run: capture, then a replay of the graph), then again in epochs of uneven
   per-member limits (pd_batch_step_each) after pd_rewind.  Every rho and every n(p) of
   the batch must equal the member's solve alone bit for bit.  Prints one line per
   failed check and "batch ok"; the exit status is the number of failures. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pd.h"

#define M 4

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAIL %s: %s\n", what, pd_last_error());
    ++failures;
  }
}

int main(void) {
  const int nx[M] = {37, 64, 45, 29}, ny[M] = {29, 50, 45, 33};
  const int prec[M] = {PD_FP32, PD_FP64, PD_FP32_FAST, PD_FP64};
  const int scheme[M] = {PD_SCHEME_STRANG, PD_SCHEME_STRANG, PD_SCHEME_STRANG, PD_SCHEME_MIDPOINT};
  const long long steps[M] = {1500, 2200, 900, 1300};
  const double e0[M] = {0.1, 0.2, 0.15, 0.12};
  pd_grid g[M];
  pd_field f[M];
  double rho_alone[M], rho[M], *n_alone[M], *n = NULL;
  pd_batch b = NULL;
  pd_batch_info info;
  int i, round, finished[M];
  long long limits[M];

  for (i = 0; i < M; ++i) {
    memset(&f[i], 0, sizeof f[i]);
    f[i].kind = PD_FIELD_SIN2;
    f[i].E0 = e0[i];
    f[i].omega = 0.5;
    f[i].cycles = 3 + i;
    g[i] = NULL;
    expect(pd_create_grid(nx[i], ny[i], -2.0, 2.0, -1.5, 1.5, prec[i], scheme[i], &g[i]) == PD_OK, "pd_create_grid");
    if (!g[i]) return 1;
    n_alone[i] = malloc(sizeof(double) * nx[i] * ny[i]);
    expect(pd_set_field(g[i], &f[i], steps[i]) == PD_OK, "pd_set_field");
    expect(pd_propagate(g[i], -1, NULL) == PD_OK, "pd_propagate");
    expect(pd_density(g[i], n_alone[i], 0, &rho_alone[i], NULL) == PD_OK, "pd_density");
    expect(pd_rewind(g[i]) == PD_OK, "pd_rewind");
  }
  n = malloc(sizeof(double) * 64 * 50);

  expect(pd_batch_create(&b) == PD_OK && b, "pd_batch_create");
  for (i = 0; i < M; ++i) expect(pd_batch_add(b, g[i]) == PD_OK, "pd_batch_add");
  for (round = 0; round < 2; ++round) {
    expect(pd_batch_run(b, rho, NULL) == PD_OK, "pd_batch_run");
    expect(pd_batch_get_info(b, &info) == PD_OK && info.graph_captured == 1 && info.n_grids == M,
           "graph captured");
    expect(info.separate_launches == 1, "the midpoint member runs its own launch");
    for (i = 0; i < M; ++i) {
      expect(rho[i] == rho_alone[i], "pd_batch_run rho equals the solve alone");
      expect(pd_density(g[i], n, 0, NULL, NULL) == PD_OK, "pd_density after the batch");
      expect(memcmp(n, n_alone[i], sizeof(double) * nx[i] * ny[i]) == 0, "pd_batch_run n(p) equals the solve alone");
    }
  }

  /* epochs: uneven limits, a member held back in the first epoch */
  for (i = 0; i < M; ++i) {
    expect(pd_rewind(g[i]) == PD_OK, "pd_rewind before the epochs");
    rho[i] = -1.0;
  }
  for (round = 0; round < 20; ++round) {
    int all = 1;
    for (i = 0; i < M; ++i) limits[i] = round == 0 && i == 1 ? 0 : 137 + 211 * i;
    expect(pd_batch_step_each(b, limits, rho, finished, NULL) == PD_OK, "pd_batch_step_each");
    for (i = 0; i < M; ++i) all = all && finished[i];
    if (all) break;
  }
  for (i = 0; i < M; ++i) {
    expect(finished[i] == 1, "every member finished");
    expect(rho[i] == rho_alone[i], "epoch rho equals the solve alone");
    expect(pd_density(g[i], n, 0, NULL, NULL) == PD_OK, "pd_density after the epochs");
    expect(memcmp(n, n_alone[i], sizeof(double) * nx[i] * ny[i]) == 0, "epoch n(p) equals the solve alone");
  }
  {
    long long bad[M] = {10, -1, 10, 10};
    expect(pd_batch_step_each(b, bad, NULL, NULL, NULL) == PD_ERR_INVALID, "a negative limit is rejected");
  }

  pd_batch_destroy(b);
  for (i = 0; i < M; ++i) {
    pd_destroy_grid(g[i]);
    free(n_alone[i]);
  }
  free(n);
  if (!failures) printf("batch ok\n");
  return failures;
}
