/* Plain C99 solve on the device through the libpd ABI, with no other runtime in the
   process: a ragged 37 x 29 grid on [-2,2] x [-1.5,1.5] under the sin^2 pulse
   E0 = 0.1, omega = 0.5, 4 cycles, N = 1500 steps, in two pd_propagate calls (a
   third of the steps, then the rest; state kept in device memory between them) on
   the default stream, then pd_density and pd_density_static into host memory.  After
   the first call the state is also saved to host memory (pd_save_state) and a second
   handle loads it (pd_load_state) and finishes the solve; its n(p) and rho must equal
   the first handle's bit for bit.
   Usage: abi_device <precision> <scheme> (pd_precision and pd_scheme values).
   Prints "rho <value>", "rho_static <value>" and "n <index> <value>" for every point
   (%.17g); the exit status is nonzero if a call fails or the two densities differ. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pd.h"

#define NX 37
#define NY 29

static int check(pd_status s, const char* what) {
  if (s != PD_OK) {
    printf("FAIL %s: status %d: %s\n", what, (int)s, pd_last_error());
    return 1;
  }
  return 0;
}

int main(int argc, char** argv) {
  pd_grid g = NULL, g2 = NULL;
  pd_field f;
  pd_info info;
  static double n[NX * NY], n_static[NX * NY], n2[NX * NY];
  double rho = 0.0, rho_static = 0.0, rho2 = 0.0;
  void* saved = NULL;
  size_t state_bytes = 0;
  long long saved_at = 0;
  const long long N = 1500;
  int k;
  if (argc != 3) {
    printf("FAIL usage: abi_device <precision> <scheme>\n");
    return 2;
  }
  if (check(pd_create_grid(NX, NY, -2.0, 2.0, -1.5, 1.5, atoi(argv[1]), atoi(argv[2]), &g), "pd_create_grid"))
    return 1;
  memset(&f, 0, sizeof f);
  f.kind = PD_FIELD_SIN2;
  f.E0 = 0.1;
  f.omega = 0.5;
  f.cycles = 4;
  if (check(pd_set_field(g, &f, N), "pd_set_field")) return 1;
  if (check(pd_propagate(g, N / 3, NULL), "pd_propagate (first third)")) return 1;
  if (check(pd_get_info(g, &info), "pd_get_info")) return 1;
  if (info.steps_done != N / 3) {
    printf("FAIL steps_done %lld after the first call\n", info.steps_done);
    return 1;
  }
  state_bytes = pd_state_bytes(g);
  saved = malloc(state_bytes);
  if (!saved || check(pd_save_state(g, saved, state_bytes, &saved_at, NULL), "pd_save_state")) return 1;
  if (saved_at != N / 3) {
    printf("FAIL pd_save_state reports step %lld\n", saved_at);
    return 1;
  }
  if (check(pd_propagate(g, -1, NULL), "pd_propagate (rest)")) return 1;
  if (check(pd_density(g, n, 0, &rho, NULL), "pd_density")) return 1;
  if (check(pd_density_static(g, n_static, 0, &rho_static, NULL), "pd_density_static")) return 1;
  if (check(pd_create_grid(NX, NY, -2.0, 2.0, -1.5, 1.5, atoi(argv[1]), atoi(argv[2]), &g2), "pd_create_grid (2)") ||
      check(pd_set_field(g2, &f, N), "pd_set_field (2)") ||
      check(pd_load_state(g2, saved, state_bytes, saved_at, NULL), "pd_load_state") ||
      check(pd_propagate(g2, -1, NULL), "pd_propagate (restarted)") ||
      check(pd_density(g2, n2, 0, &rho2, NULL), "pd_density (restarted)"))
    return 1;
  pd_destroy_grid(g2);
  free(saved);
  if (rho2 != rho || memcmp(n, n2, sizeof n) != 0) {
    printf("FAIL the restarted solve differs\n");
    return 1;
  }
  printf("rho %.17g\nrho_static %.17g\n", rho, rho_static);
  for (k = 0; k < NX * NY; ++k) printf("n %d %.17g\n", k, n[k]);
  pd_destroy_grid(g);
  if (rho != rho_static || memcmp(n, n_static, sizeof n) != 0) {
    printf("FAIL pd_density_static differs from pd_density\n");
    return 1;
  }
  return 0;
}
