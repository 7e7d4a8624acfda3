/* Drives the host-side logic of libpd (argument checks, the field sampling of every
   field kind for every scheme, with and without a y component, pd_check_field's
   bounds, batch membership, launch validation, fault specifications, per-thread
   error messages) without a device, so that a build of the library's host code with
   AddressSanitizer and UndefinedBehaviorSanitizer sees those paths
   (test_sanitizers.py).  Prints one line per failed check; exits with the number of
   failures, 0 on success. */
#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pd.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAIL %s\n", what);
    ++failures;
  }
}

static int all_finite(const double* v, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* One field of each kind, with or without a y component; table arrays sized for
   five stages. */
static void make_field(pd_field* f, int kind, int elliptic, long long n_steps, double* ax, double* ay) {
  memset(f, 0, sizeof *f);
  f->kind = kind;
  f->E0 = 0.2;
  f->omega = 0.6;
  f->cycles = 3;
  f->t_end = 7.0;
  f->phi = 0.3;
  f->omega_rise = 0.2;
  f->omega_fall = 0.25;
  f->duration = 40.0;
  f->ellipticity = elliptic ? 0.6 : 0.0;
  if (kind == PD_FIELD_TABLE) {
    for (long long k = 0; k < 5 * n_steps; ++k) {
      ax[k] = 0.1 * sin(0.01 * (double)k);
      ay[k] = 0.05 * cos(0.02 * (double)k);
    }
    f->A_mid = ax;
    f->Ay_mid = elliptic ? ay : NULL;
    f->t_i = -1.0;
    f->t_f = 9.0;
    f->A_in = 0.01;
    f->A_out = -0.02;
    f->Ay_in = 0.05;
    f->Ay_out = 0.04;
  }
}

static void check_sampling(void) {
  enum { N = 300 };
  static double ax[5 * N], ay[5 * N], sx[5 * N + 1], sy[5 * N + 1];
  for (int scheme = 0; scheme <= 3; ++scheme) {
    int stages = scheme >= PD_SCHEME_STRANG4 ? 5 : 1;
    for (int kind = 0; kind <= 3; ++kind)
      for (int elliptic = 0; elliptic <= 1; ++elliptic) {
        pd_field f;
        double ends[6], t_i, t_f, a_in, a_out;
        make_field(&f, kind, elliptic, N, ax, ay);
        f.n_table = (long long)stages * N;
        sx[stages * N] = 12345.0; /* sentinel: nothing is written past stages * N */
        expect(pd_sample_field_xy(&f, N, scheme, sx, sy, ends) == PD_OK, "pd_sample_field_xy accepts the field");
        expect(all_finite(sx, stages * N) && all_finite(sy, stages * N) && all_finite(ends, 6),
               "samples are finite");
        expect(sx[stages * N] == 12345.0, "no write past stages * N samples");
        if (kind == PD_FIELD_TABLE) expect(sx[7] == ax[7], "table samples returned unchanged");
        if (stages == 1) {
          f.n_table = N;
          expect(pd_sample_field(&f, N, sx, &t_i, &t_f, &a_in, &a_out) == PD_OK, "pd_sample_field");
          expect(pd_sample_field(&f, N, NULL, NULL, NULL, NULL, NULL) == PD_OK, "pd_sample_field, NULL outputs");
        }
        expect(pd_sample_field_xy(&f, N, scheme, NULL, NULL, NULL) == PD_OK, "pd_sample_field_xy, NULL outputs");
        if (kind == PD_FIELD_TABLE)
          expect(pd_sample_field_xy(&f, N + 1, scheme, sx, sy, ends) == PD_ERR_INVALID, "short table rejected");
      }
  }
  pd_field bad;
  make_field(&bad, PD_FIELD_SIN2, 0, N, ax, ay);
  bad.cycles = 1;
  expect(pd_sample_field(&bad, N, sx, NULL, NULL, NULL, NULL) == PD_ERR_INVALID, "sin2 with one cycle rejected");
  make_field(&bad, PD_FIELD_PULSE, 0, N, ax, ay);
  bad.duration = 1.0;
  expect(pd_sample_field(&bad, N, sx, NULL, NULL, NULL, NULL) == PD_ERR_INVALID, "pulse shorter than its edges");
  make_field(&bad, 9, 0, N, ax, ay);
  expect(pd_sample_field(&bad, N, sx, NULL, NULL, NULL, NULL) == PD_ERR_INVALID, "unknown field kind");
  expect(pd_sample_field(NULL, N, sx, NULL, NULL, NULL, NULL) == PD_ERR_INVALID, "NULL field");
  make_field(&bad, PD_FIELD_SIN2, 0, N, ax, ay);
  expect(pd_sample_field(&bad, 0, sx, NULL, NULL, NULL, NULL) == PD_ERR_INVALID, "zero steps");
  expect(pd_sample_field_xy(&bad, N, 7, sx, sy, NULL) == PD_ERR_INVALID, "unknown scheme");
}

static void check_grids(void) {
  enum { N = 2000 };
  static double ax[5 * N], ay[5 * N];
  for (int precision = 0; precision <= 2; ++precision)
    for (int scheme = 0; scheme <= 3; ++scheme) {
      pd_grid g = NULL;
      pd_info info;
      int stages = scheme >= PD_SCHEME_STRANG4 ? 5 : 1;
      expect(pd_create_grid(33, 17, -2.0, 2.0, -1.0, 1.5, precision, scheme, &g) == PD_OK && g, "grid created");
      if (!g) continue;
      for (int kind = 0; kind <= 3; ++kind)
        for (int elliptic = 0; elliptic <= 1; ++elliptic) {
          pd_field f;
          make_field(&f, kind, elliptic, N, ax, ay);
          f.n_table = (long long)stages * N;
          expect(pd_check_field(g, &f, N, &info) == PD_OK, "field accepted");
          expect(info.stages == stages && info.elliptic == elliptic && info.n_points == 33 * 17,
                 "info: stages, y component, points");
          expect(isfinite(info.dt) && info.dt > 0 && isfinite(info.E_max) && info.A_min <= info.A_max,
                 "info: dt, E_max, A range");
          expect(pd_check_field(g, &f, N, NULL) == PD_OK, "NULL info");
          expect(pd_solve_bytes(g, N) > 0, "footprint");
        }
      expect(pd_set_launch(g, 3, 256, 0, 0) == PD_ERR_INVALID, "three points per lane rejected");
      expect(pd_set_launch(g, 1, 100, 0, 0) == PD_ERR_INVALID, "block of 100 threads rejected");
      expect(pd_set_launch(g, 0, 0, 9, 0) == PD_ERR_INVALID, "unknown table stage rejected");
      expect(pd_set_launch(g, 0, 0, 0, -5) == PD_ERR_INVALID, "negative chunk rejected");
      expect(pd_bind_state(g, (void*)(size_t)4096, 16) == PD_ERR_INVALID, "state buffer too small rejected");
      expect(pd_bind_state(g, NULL, 0) == PD_OK, "binding NULL unbinds");
      expect(pd_resume(g, 5) == PD_ERR_STATE, "resume before a field");
      {
        static unsigned char host[33 * 17 * 4 * 8];
        long long done = -1;
        expect(pd_save_state(g, host, sizeof host, &done, NULL) == PD_ERR_STATE && done == -1,
               "save before a field");
        expect(pd_save_state(g, NULL, sizeof host, &done, NULL) == PD_ERR_INVALID, "save to NULL");
        expect(pd_load_state(g, host, pd_state_bytes(g), 5, NULL) == PD_ERR_STATE, "load before a field");
        expect(pd_load_state(g, NULL, pd_state_bytes(g), 5, NULL) == PD_ERR_INVALID, "load from NULL");
      }
      expect(pd_rewind(g) == PD_ERR_STATE, "rewind before a field");
      expect(pd_density(g, NULL, 0, NULL, NULL) != PD_OK, "density before a field");
      expect(pd_get_info(g, NULL) == PD_ERR_INVALID, "NULL info to pd_get_info");
      pd_destroy_grid(g);
    }
  pd_grid g = NULL;
  expect(pd_create_grid(65537, 4, -1, 1, -1, 1, PD_FP32, 0, &g) == PD_ERR_INVALID && !g, "nx above 65536");
  expect(pd_create_grid(4, 4, 1, -1, -1, 1, PD_FP32, 0, &g) == PD_ERR_INVALID && !g, "empty range");
  expect(pd_create_grid(4, 4, -1, 1, -1, NAN, PD_FP32, 0, &g) == PD_ERR_INVALID && !g, "NaN range");
  expect(pd_create_grid(4, 4, -1, 1, -1, 1, 5, 0, &g) == PD_ERR_INVALID && !g, "unknown precision");
  expect(pd_create_grid(4, 4, -1, 1, -1, 1, PD_FP32, 0, NULL) == PD_ERR_INVALID, "NULL out");
}

static void check_batches(void) {
  pd_batch b = NULL;
  pd_grid g[3] = {NULL, NULL, NULL}, out[4];
  pd_batch_info bi;
  expect(pd_batch_create(&b) == PD_OK && b, "batch created");
  if (!b) return;
  for (int i = 0; i < 3; ++i) expect(pd_create_grid(16 + i, 9, -1, 1, -1, 1, PD_FP32, 0, &g[i]) == PD_OK, "member grid");
  expect(pd_batch_add(b, g[0]) == PD_OK && pd_batch_add(b, g[1]) == PD_OK, "members added");
  expect(pd_batch_add(b, g[0]) != PD_OK, "a member twice rejected");
  expect(pd_batch_size(b) == 2, "size 2");
  expect(pd_batch_members(b, out, 4) == PD_OK && out[0] == g[0] && out[1] == g[1], "members in order");
  expect(pd_batch_remove(b, g[0]) == PD_OK && pd_batch_size(b) == 1, "member removed");
  expect(pd_batch_remove(b, g[2]) != PD_OK, "removing a stranger rejected");
  expect(pd_batch_add(b, g[2]) == PD_OK && pd_batch_size(b) == 2, "member added after a removal");
  expect(pd_batch_set_launch(b, 3, 256) == PD_ERR_INVALID, "batch: three points per lane rejected");
  expect(pd_batch_get_info(b, &bi) == PD_OK, "batch info");
  expect(pd_batch_run(b, NULL, NULL) != PD_OK, "run with members that have no field");
  expect(pd_batch_clear(b) == PD_OK && pd_batch_size(b) == 0, "batch cleared");
  expect(pd_batch_add(NULL, g[0]) == PD_ERR_INVALID && pd_batch_size(NULL) == 0, "NULL batch");
  pd_batch_destroy(b);
  pd_batch_destroy(NULL);
  for (int i = 0; i < 3; ++i) pd_destroy_grid(g[i]);
}

static void check_faults(void) {
  const char* good[] = {"", "alloc@3", "launch@1", "launch@1000000"};
  const char* bad[] = {"alloc", "none", "alloc@0", "launch@", "fire@2", "alloc@x", "launch@-2", "alloc@3x"};
  for (size_t i = 0; i < sizeof good / sizeof *good; ++i) expect(pd_set_fault(good[i]) == PD_OK, good[i]);
  for (size_t i = 0; i < sizeof bad / sizeof *bad; ++i) expect(pd_set_fault(bad[i]) == PD_ERR_INVALID, bad[i]);
  expect(pd_set_fault(NULL) == PD_OK, "NULL clears the fault");
}

/* Error messages are per thread: each thread's failing call leaves its own text. */
static void* thread_body(void* arg) {
  long id = (long)arg;
  char want[64];
  for (int rep = 0; rep < 200; ++rep) {
    pd_grid g = NULL;
    int code = (int)(1000 + 1000 * id + rep); /* never a valid precision or scheme */
    if (id % 2) {
      pd_create_grid(4, 4, -1, 1, -1, 1, code, 0, &g);
      snprintf(want, sizeof want, "unknown precision %d", code);
    } else {
      pd_create_grid(4, 4, -1, 1, -1, 1, PD_FP32, code, &g);
      snprintf(want, sizeof want, "unknown scheme %d", code);
    }
    if (g || strcmp(pd_last_error(), want) != 0) return (void*)1;
    if (pd_create_grid(8, 8, -1, 1, -1, 1, PD_FP64, (int)(id % 4), &g) != PD_OK || !g) return (void*)2;
    pd_destroy_grid(g);
  }
  return NULL;
}

static void check_threads(void) {
  pthread_t t[8];
  for (long i = 0; i < 8; ++i) pthread_create(&t[i], NULL, thread_body, (void*)i);
  for (int i = 0; i < 8; ++i) {
    void* r = NULL;
    pthread_join(t[i], &r);
    expect(r == NULL, "per-thread error messages");
  }
}

int main(void) {
  check_sampling();
  check_grids();
  check_batches();
  check_faults();
  check_threads();
  if (!failures) printf("host paths ok\n");
  return failures;
}
