/* Drives the oracle's entry points over every field kind, both schemes, second and
   fourth order, both valleys and a y component, on small grids, so that a build with
   AddressSanitizer and UndefinedBehaviorSanitizer sees every path (test_sanitizers.py).
   Exits 0 if every result is finite and every occupation lies in [0, 1]. */
#include <stdio.h>

#include "../../oracle/oracle.c"

static int check_grid(const oracle_problem* f, int nx, int ny) {
  double n[64], dev[64];
  long long idx[3] = {0, 5, (long long)nx * ny - 1};
  if (oracle_solve_grid(f, nx, ny, -2.0, 2.0, -1.5, 1.5, NULL, 0, n, dev, 1) < 0) return 1;
  for (int k = 0; k < nx * ny; ++k)
    if (!(n[k] >= 0.0 && n[k] <= 1.0) || !(dev[k] == dev[k])) return 2;
  double rho = oracle_density(nx, ny, -2.0, 2.0, -1.5, 1.5, n, 0);
  double rho_c = oracle_density(nx, ny, -2.0, 2.0, -1.5, 1.5, n, 1);
  if (!(rho >= 0.0) || !(rho_c >= 0.0)) return 3;
  if (oracle_solve_grid(f, nx, ny, -2.0, 2.0, -1.5, 1.5, idx, 3, n, dev, 1) < 0) return 4;
  double px[2] = {0.3, -0.7}, py[2] = {0.1, 0.0};
  if (oracle_snapshot_points(f, f->n_steps / 2, 2, px, py, n, 1) < 0) return 5;
  double psi[4];
  if (oracle_state_at(f, f->n_steps / 3, 0.2, 0.4, psi) < 0) return 6;
  if (oracle_final_state(f, 0.2, 0.4, psi) < 0) return 7;
  return 0;
}

int main(void) {
  enum { N = 120 };
  static double A_mid[5 * N], Ay_mid[5 * N];  /* stages x steps values at fourth order */
  int rc;
  for (int scheme = 0; scheme <= 1; ++scheme)
    for (int order = 2; order <= 4; order += 2)
      for (int valley = -1; valley <= 1; valley += 2)
        for (int kind = 0; kind <= 3; ++kind) {
          oracle_problem f;
          memset(&f, 0, sizeof f);
          f.field_kind = kind;
          f.E0 = 0.3;
          f.omega = 0.7;
          f.cycles = 2;
          f.t_end = 9.0;
          f.phi = 0.4;
          f.omega_rise = 0.2;
          f.omega_fall = 0.3;
          f.duration = 12.0;
          f.n_steps = N;
          f.scheme = scheme;
          f.valley = valley;
          f.order = order;
          f.ellipticity = kind == 2 ? 0.0 : 0.5;
          if (kind == 2) {  /* a caller table, with a y component */
            const int stages = order == 4 ? 5 : 1;
            for (int k = 0; k < stages * N; ++k) A_mid[k] = 0.2 * sin(0.05 * k);
            for (int k = 0; k < stages * N; ++k) Ay_mid[k] = 0.1 * cos(0.03 * k);
            f.A_mid = A_mid;
            f.Ay_mid = Ay_mid;
            f.t_i = 0.0;
            f.t_f = 10.0;
            f.A_in = 0.0;
            f.A_out = 0.05;
            f.Ay_in = 0.1;
            f.Ay_out = 0.02;
          }
          static double tab[5 * N];
          double a_in, a_out, dt;
          if (kind != 2 && oracle_field_table(&f, tab, &a_in, &a_out, &dt) != 0) return 10;
          if ((rc = check_grid(&f, 8, 7)) != 0) {
            fprintf(stderr, "scheme %d order %d valley %d field %d: check %d\n", scheme, order, valley, kind, rc);
            return rc;
          }
        }
  double c[5], sigma[5];
  if (oracle_composition(4, c, sigma) != 5 || oracle_composition(2, c, sigma) != 1) return 11;
  puts("oracle paths ok");
  return 0;
}
