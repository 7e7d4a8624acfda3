/*
 * Plain FP64 CPU oracle for electron-hole pair production in graphene
 * (Fillion-Gourdeau et al., arXiv:1607.03062).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, imports or calls it, and it shares no code,
 * header or table with the product library.
 *
 * What it computes, per momentum point p (Sec. II, Eq. (1)):
 *
 *     n(p) = | u_out^dagger(p)  U_p(t_f, t_i)  v_in(p) |^2
 *
 * with unit-normalised adiabatic spinors (Sec. II, Eqs. (3)-(4), divided by
 * sqrt(2E) so that n lies in [0,1]), U_p the evolution operator of the
 * massless momentum-space Dirac equation (Sec. II, Eq. (2)), replaced by the
 * product of N short-time operators (Sec. III, Eq. (9)).  Two short-time
 * operators are provided:
 *
 *   scheme 1, MIDPOINT: the paper's own step, the exact exponential of the
 *     Hamiltonian frozen at the midpoint of the step (Sec. III, Eqs. (11)-(12)),
 *     written as the explicit 2x2 matrix of Eq. (13):
 *         U = cos(dt E) I - i (sigma.P / E) sin(dt E),  P = p + A(t_{k+1/2}).
 *   scheme 0, STRANG: the same midpoint Hamiltonian sigma_x P_x + sigma_y p_y
 *     split symmetrically into its sigma_y and sigma_x parts:
 *         U = exp(-i dt p_y sigma_y / 2) exp(-i dt P_x sigma_x) exp(-i dt p_y sigma_y / 2).
 *     Both are second order in dt (Sec. III: local error O(dt^3)).
 *   order 4: either step composed by Suzuki's fractal decomposition, which
 *     the paper names as the way to higher order (Sec. III, after Eq. (12)):
 *         S4(dt) = S(c1 dt) S(c2 dt) S(c3 dt) S(c4 dt) S(c5 dt),
 *         c = (p, p, 1 - 4p, p, p),  p = 1 / (4 - 4^(1/3)),
 *     each stage S(c dt) a second-order step over its own sub-interval with
 *     A taken at that sub-interval's midpoint (the coefficients satisfy
 *     sum c = 1 and sum c^3 = 0, which cancels the dt^3 error of the
 *     symmetric second-order step).
 *
 * Fields: linear along x (Sec. II), or elliptic with a y component
 * (Sec. V mentions circular polarisation as an extension); then
 * P = (p_x + A_x, p_y + A_y) everywhere, including the spinors.
 *
 * Snapshots: the state after k of the N steps projected on the positive-energy
 * eigenvector of sigma.P(t_k), P(t_k) = p + A(t_i + k dt) (the instantaneous
 * adiabatic occupation, which at k = N is n(p)).
 *
 * Conventions where the paper is silent (units hbar = v_F = e = 1; node grid
 * p_j = p_min + j (p_max - p_min)/n, j < n, point index k = j*nx + i; step
 * midpoints t_i + (k + 1/2) dt; n := 0 at a point where E_in or E_out
 * vanishes, such points are counted as masked; density
 * rho = 4 dx dy / (2 pi)^2 * sum n, the factor 4 for spin x valley).
 *
 * Arithmetic: FP64 only, real components (a1, b1, a2, b2) of the spinor
 * psi = (a1 + i b1, a2 + i b2), no complex type, libm sin/cos/sqrt, every
 * step evaluated directly (no angle addition, no merging of the half steps
 * of neighbouring Strang steps).  Build with -ffp-contract=off so that the
 * compiler does not fuse multiplies and adds.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_FIELD_SIN2 0     /* E(t) = E0 sin^2(pi t / T) sin(w t), T = cycles 2 pi / w, t in [0, T] */
#define OR_FIELD_CONSTANT 1 /* E(t) = E0 on [0, t_end] */
#define OR_FIELD_TABLE 2    /* caller's A at the step midpoints, plus t_i, t_f, A_in, A_out */
#define OR_FIELD_PULSE 3    /* the paper's rise / flat / fall laser pulse, Sec. IV, Eq. (14) */

#define OR_SCHEME_STRANG 0
#define OR_SCHEME_MIDPOINT 1

typedef struct {
  int field_kind;
  double E0, omega;
  int cycles;
  double t_end;
  const double* A_mid; /* TABLE: n_steps values A(t_i + (k + 1/2) dt) */
  double t_i, t_f, A_in, A_out; /* TABLE */
  double phi, omega_rise, omega_fall, duration; /* PULSE */
  long long n_steps;
  int scheme;
  int valley; /* +1 for K+, -1 for K- */
  int order;  /* 2 (or 0) or 4 */
  double ellipticity; /* SIN2, PULSE, CONSTANT: amplitude of E_y relative to E0 */
  const double* Ay_mid; /* TABLE: NULL (A_y = 0) or stages * n_steps values of A_y */
  double Ay_in, Ay_out; /* TABLE */
} oracle_problem;

/* ------------------------------------------------------------------------ */
/* Composition: stage coefficients c[j] and stage midpoints sigma[j] (in units of
   dt from the start of the step); returns the number of stages. */
int oracle_composition(int order, double c[5], double sigma[5]) {
  int S;
  if (order == 4) {
    double p = 1.0 / (4.0 - cbrt(4.0));
    c[0] = p;
    c[1] = p;
    c[2] = 1.0 - 4.0 * p;
    c[3] = p;
    c[4] = p;
    S = 5;
  } else {
    c[0] = 1.0;
    S = 1;
  }
  double start = 0.0;
  for (int j = 0; j < S; ++j) {
    sigma[j] = start + 0.5 * c[j];
    start += c[j];
  }
  return S;
}

static int stages_of(const oracle_problem* f) {
  double c[5], sg[5];
  return oracle_composition(f->order, c, sg);
}

/* ------------------------------------------------------------------------ */
/* Field: gauge A_0 = 0, E = -dA/dt, A = -int_{t_i}^t E (Sec. II, after Eq. (2)) */

static double one_minus_cos(double x) {
  /* 1 - cos x written as 2 sin^2(x/2): no cancellation near x = 0 */
  double s = sin(0.5 * x);
  return 2.0 * s * s;
}

/* sin^2 pulse: E = E0 sin^2(pi t/T) sin(w t) = (E0/2) sin(w t) - (E0/4)[sin((w+W)t) + sin((w-W)t)],
   W = 2 pi / T, so int_0^t E = E0 [ (1-cos w t)/(2w) - (1-cos(w+W)t)/(4(w+W)) - (1-cos(w-W)t)/(4(w-W)) ]. */
static double sin2_A(double E0, double w, int cycles, double t) {
  double T = cycles * 2.0 * M_PI / w;
  double W = 2.0 * M_PI / T;
  double I = one_minus_cos(w * t) / (2.0 * w) - one_minus_cos((w + W) * t) / (4.0 * (w + W)) -
             one_minus_cos((w - W) * t) / (4.0 * (w - W));
  return -E0 * I;
}

static double sin2_E(double E0, double w, int cycles, double t) {
  double T = cycles * 2.0 * M_PI / w;
  double s = sin(M_PI * t / T);
  return E0 * s * s * sin(w * t);
}

/* y component of the elliptic sin^2 pulse: E_y = e E0 sin^2(pi t/T) cos(w t)
   = (e E0/2) cos(w t) - (e E0/4)[cos((w+W)t) + cos((w-W)t)], so
   int_0^t E_y = e E0 [ sin(w t)/(2w) - sin((w+W)t)/(4(w+W)) - sin((w-W)t)/(4(w-W)) ]. */
static double sin2_Ay(double E0y, double w, int cycles, double t) {
  double T = cycles * 2.0 * M_PI / w;
  double W = 2.0 * M_PI / T;
  double I = sin(w * t) / (2.0 * w) - sin((w + W) * t) / (4.0 * (w + W)) - sin((w - W) * t) / (4.0 * (w - W));
  return -E0y * I;
}

static double sin2_Ey(double E0y, double w, int cycles, double t) {
  double T = cycles * 2.0 * M_PI / w;
  double s = sin(M_PI * t / T);
  return E0y * s * s * cos(w * t);
}

/* The paper's pulse, Sec. IV, Eq. (14), with t_i = 0, t_f = duration:
     rise  t in [0, tr]:        E0 sin^2(Wr t) cos(w t + phi),   tr = pi / (2 Wr)
     flat  t in [tr, t_f - tf]: E0 cos(w t + phi)
     fall  t in [t_f - tf, t_f]: E0 cos^2(Wf (t - t_f + tf)) cos(w t + phi),  tf = pi / (2 Wf)
   (the fall factor is taken so that the envelope goes from 1 to 0 across the
   fall window; the equation as printed does not vanish at t_f).  A is the
   closed-form antiderivative, piece by piece, continuous at the joins. */
static double pulse_env_int(double w, double phi, double W, double shift, int fall, double a, double b) {
  /* int_a^b env(t) cos(w t + phi) dt with env = sin^2(W (t - shift)) (rise) or cos^2(W (t - shift)) (fall).
     sin^2 u = (1 - cos 2u)/2, cos^2 u = (1 + cos 2u)/2;
     cos(2W(t-s)) cos(w t + phi) = [cos((w+2W)t + phi - 2Ws) + cos((w-2W)t + phi + 2Ws)]/2. */
  double sgn = fall ? 1.0 : -1.0;
  double base = (sin(w * b + phi) - sin(w * a + phi)) / w;
  double w1 = w + 2.0 * W, p1 = phi - 2.0 * W * shift;
  double w2 = w - 2.0 * W, p2 = phi + 2.0 * W * shift;
  double t1 = (sin(w1 * b + p1) - sin(w1 * a + p1)) / w1;
  double t2 = (fabs(w2) > 0.0) ? (sin(w2 * b + p2) - sin(w2 * a + p2)) / w2 : (b - a) * cos(p2);
  return 0.5 * base + sgn * 0.25 * (t1 + t2);
}

static double pulse_A_phase(const oracle_problem* f, double phi, double t) {
  double w = f->omega, tf_ = f->duration;
  double tr = M_PI / (2.0 * f->omega_rise), tfall = M_PI / (2.0 * f->omega_fall);
  double t_fall0 = tf_ - tfall;
  double I = 0.0;
  if (t <= 0.0) return 0.0;
  if (t > tf_) t = tf_;
  /* rise */
  double b = t < tr ? t : tr;
  I += pulse_env_int(w, phi, f->omega_rise, 0.0, 0, 0.0, b);
  if (t > tr) {
    double b2 = t < t_fall0 ? t : t_fall0;
    if (b2 > tr) I += (sin(w * b2 + phi) - sin(w * tr + phi)) / w;
    if (t > t_fall0) I += pulse_env_int(w, phi, f->omega_fall, t_fall0, 1, t_fall0, t);
  }
  return -f->E0 * I;
}

static double pulse_A(const oracle_problem* f, double t) { return pulse_A_phase(f, f->phi, t); }

/* Elliptic pulse: E_y = e E0 env(t) sin(w t + phi) = e E0 env(t) cos(w t + phi - pi/2). */
static double pulse_Ay(const oracle_problem* f, double t) {
  return f->ellipticity * pulse_A_phase(f, f->phi - 0.5 * M_PI, t);
}

static double pulse_E_phase(const oracle_problem* f, double phi, double t) {
  double w = f->omega, tf_ = f->duration;
  double tr = M_PI / (2.0 * f->omega_rise), tfall = M_PI / (2.0 * f->omega_fall);
  if (t < 0.0 || t > tf_) return 0.0;
  double env;
  if (t < tr) {
    double s = sin(f->omega_rise * t);
    env = s * s;
  } else if (t > tf_ - tfall) {
    double c = cos(f->omega_fall * (t - tf_ + tfall));
    env = c * c;
  } else {
    env = 1.0;
  }
  return f->E0 * env * cos(w * t + phi);
}

static double pulse_E(const oracle_problem* f, double t) { return pulse_E_phase(f, f->phi, t); }

void oracle_times(const oracle_problem* f, double* t_i, double* t_f) {
  switch (f->field_kind) {
    case OR_FIELD_SIN2: *t_i = 0.0; *t_f = f->cycles * 2.0 * M_PI / f->omega; break;
    case OR_FIELD_CONSTANT: *t_i = 0.0; *t_f = f->t_end; break;
    case OR_FIELD_PULSE: *t_i = 0.0; *t_f = f->duration; break;
    default: *t_i = f->t_i; *t_f = f->t_f; break;
  }
}

/* Vector potential A_x(t).  For TABLE only the endpoints are defined (A_in, A_out). */
double oracle_A(const oracle_problem* f, double t) {
  switch (f->field_kind) {
    case OR_FIELD_SIN2: {
      double T = f->cycles * 2.0 * M_PI / f->omega;
      if (t <= 0.0) return 0.0;
      if (t >= T) t = T;
      return sin2_A(f->E0, f->omega, f->cycles, t);
    }
    case OR_FIELD_CONSTANT:
      if (t <= 0.0) return 0.0;
      if (t >= f->t_end) t = f->t_end;
      return -f->E0 * t;
    case OR_FIELD_PULSE: return pulse_A(f, t);
    default: return t <= f->t_i ? f->A_in : f->A_out;
  }
}

/* Vector potential A_y(t) (zero for linear polarisation). */
double oracle_Ay(const oracle_problem* f, double t) {
  switch (f->field_kind) {
    case OR_FIELD_SIN2: {
      double T = f->cycles * 2.0 * M_PI / f->omega;
      if (t <= 0.0) return 0.0;
      if (t >= T) t = T;
      return sin2_Ay(f->ellipticity * f->E0, f->omega, f->cycles, t);
    }
    case OR_FIELD_CONSTANT:
      if (t <= 0.0) return 0.0;
      if (t >= f->t_end) t = f->t_end;
      return -f->ellipticity * f->E0 * t;
    case OR_FIELD_PULSE: return pulse_Ay(f, t);
    default: return t <= f->t_i ? f->Ay_in : f->Ay_out;
  }
}

/* Electric field E_y(t) (used only by the pins). */
double oracle_Ey(const oracle_problem* f, double t) {
  switch (f->field_kind) {
    case OR_FIELD_SIN2: {
      double T = f->cycles * 2.0 * M_PI / f->omega;
      if (t < 0.0 || t > T) return 0.0;
      return sin2_Ey(f->ellipticity * f->E0, f->omega, f->cycles, t);
    }
    case OR_FIELD_CONSTANT: return (t < 0.0 || t > f->t_end) ? 0.0 : f->ellipticity * f->E0;
    case OR_FIELD_PULSE: return f->ellipticity * pulse_E_phase(f, f->phi - 0.5 * M_PI, t);
    default: return 0.0;
  }
}

/* Electric field E_x(t) (used only by the quadrature pin of A). */
double oracle_E(const oracle_problem* f, double t) {
  switch (f->field_kind) {
    case OR_FIELD_SIN2: {
      double T = f->cycles * 2.0 * M_PI / f->omega;
      if (t < 0.0 || t > T) return 0.0;
      return sin2_E(f->E0, f->omega, f->cycles, t);
    }
    case OR_FIELD_CONSTANT: return (t < 0.0 || t > f->t_end) ? 0.0 : f->E0;
    case OR_FIELD_PULSE: return pulse_E(f, t);
    default: return 0.0;
  }
}

/* A at the sample times of every stage of every step, t_i + (k + sigma_j) dt
   (k < N, j < stages; for second order the step midpoints), index k * stages + j,
   plus the end values A(t_i), A(t_f).  Ay may be NULL. */
typedef struct {
  double Ax_in, Ax_out, Ay_in, Ay_out, dt;
} field_ends;

static void field_table(const oracle_problem* f, double* Ax, double* Ay, field_ends* e) {
  double t_i, t_f, c[5], sg[5];
  oracle_times(f, &t_i, &t_f);
  int S = oracle_composition(f->order, c, sg);
  long long N = f->n_steps;
  double dt = (t_f - t_i) / (double)N;
  e->dt = dt;
  if (f->field_kind == OR_FIELD_TABLE) {
    memcpy(Ax, f->A_mid, (size_t)(N * S) * sizeof(double));
    if (Ay) {
      if (f->Ay_mid)
        memcpy(Ay, f->Ay_mid, (size_t)(N * S) * sizeof(double));
      else
        memset(Ay, 0, (size_t)(N * S) * sizeof(double));
    }
    e->Ax_in = f->A_in;
    e->Ax_out = f->A_out;
    e->Ay_in = f->Ay_mid ? f->Ay_in : 0.0;
    e->Ay_out = f->Ay_mid ? f->Ay_out : 0.0;
    return;
  }
  for (long long k = 0; k < N; ++k)
    for (int j = 0; j < S; ++j) {
      double t = t_i + ((double)k + sg[j]) * dt;
      Ax[k * S + j] = oracle_A(f, t);
      if (Ay) Ay[k * S + j] = oracle_Ay(f, t);
    }
  e->Ax_in = oracle_A(f, t_i);
  e->Ax_out = oracle_A(f, t_f);
  e->Ay_in = oracle_Ay(f, t_i);
  e->Ay_out = oracle_Ay(f, t_f);
}

/* A at the step boundary t_k = t_i + k dt (k = 0: A_in, k = N: A_out).  A table
   field gives A only at its sample times: between two steps it is taken as the
   mean of the last sample of step k-1 and the first sample of step k. */
static void boundary_A(const oracle_problem* f, long long k, const double* Ax, const double* Ay, const field_ends* e,
                       double* ax, double* ay) {
  long long N = f->n_steps;
  int S = stages_of(f);
  if (k <= 0) {
    *ax = e->Ax_in;
    *ay = e->Ay_in;
  } else if (k >= N) {
    *ax = e->Ax_out;
    *ay = e->Ay_out;
  } else if (f->field_kind == OR_FIELD_TABLE) {
    *ax = 0.5 * (Ax[k * S - 1] + Ax[k * S]);
    *ay = 0.5 * (Ay[k * S - 1] + Ay[k * S]);
  } else {
    double t_i, t_f;
    oracle_times(f, &t_i, &t_f);
    double t = t_i + (double)k * e->dt;
    *ax = oracle_A(f, t);
    *ay = oracle_Ay(f, t);
  }
}

/* ------------------------------------------------------------------------ */
/* Spinors (Sec. II, Eqs. (3)-(4)), divided by sqrt(2E) to unit norm.
   Returned as (re1, im1, re2, im2). */

void oracle_spinors(double Px, double Py, int valley, double u[4], double v[4]) {
  double E = sqrt(Px * Px + Py * Py);
  double d = sqrt(2.0) * E;
  if (valley >= 0) {
    /* u_K+ = (E, Px + i Py),  v_K+ = (-Px + i Py, E) */
    u[0] = E / d; u[1] = 0.0; u[2] = Px / d; u[3] = Py / d;
    v[0] = -Px / d; v[1] = Py / d; v[2] = E / d; v[3] = 0.0;
  } else {
    /* u_K- = (E, -Px - i Py),  v_K- = (Px - i Py, E) */
    u[0] = E / d; u[1] = 0.0; u[2] = -Px / d; u[3] = -Py / d;
    v[0] = Px / d; v[1] = -Py / d; v[2] = E / d; v[3] = 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* Elementary unitary factors acting on psi = (a1 + i b1, a2 + i b2).
   Each is written with h = cos(theta) - 1 = -2 sin^2(theta/2) and s = sin(theta):
   the small increment is formed first and added to the component last. */

/* exp(-i theta sigma_x) = [[c, -i s], [-i s, c]] */
static void apply_x(double psi[4], double theta) {
  double q = sin(0.5 * theta);
  double h = -2.0 * q * q, s = sin(theta);
  double a1 = psi[0], b1 = psi[1], a2 = psi[2], b2 = psi[3];
  psi[0] = a1 + (h * a1 + s * b2);
  psi[1] = b1 + (h * b1 - s * a2);
  psi[2] = a2 + (h * a2 + s * b1);
  psi[3] = b2 + (h * b2 - s * a1);
}

/* exp(-i theta sigma_y) = [[c, -s], [s, c]] */
static void apply_y(double psi[4], double theta) {
  double q = sin(0.5 * theta);
  double h = -2.0 * q * q, s = sin(theta);
  double a1 = psi[0], b1 = psi[1], a2 = psi[2], b2 = psi[3];
  psi[0] = a1 + (h * a1 - s * a2);
  psi[1] = b1 + (h * b1 - s * b2);
  psi[2] = a2 + (h * a2 + s * a1);
  psi[3] = b2 + (h * b2 + s * b1);
}

/* exp(-i g dt sigma.P), P = (Px, Py), g = valley sign: Eq. (13),
   cos(dt E) I - i g (sigma.P / E) sin(dt E), with sin(dt E)/E -> dt at E = 0. */
static void apply_midpoint(double psi[4], double dt, double Px, double Py, int g) {
  double E = sqrt(Px * Px + Py * Py);
  double th = dt * E;
  double q = sin(0.5 * th);
  double h = -2.0 * q * q;
  double sig = (E > 0.0) ? sin(th) / E : dt;
  double al = g * sig * Px, be = g * sig * Py;
  double a1 = psi[0], b1 = psi[1], a2 = psi[2], b2 = psi[3];
  /* psi1' = c psi1 + (-i al - be) psi2 ;  psi2' = c psi2 + (be - i al) psi1 */
  psi[0] = a1 + ((h * a1 - be * a2) + al * b2);
  psi[1] = b1 + ((h * b1 - be * b2) - al * a2);
  psi[2] = a2 + ((h * a2 + be * a1) + al * b1);
  psi[3] = b2 + ((h * b2 + be * b1) - al * a1);
}

/* One second-order step over an interval of length dt at momentum (px, py),
   with (Ax, Ay) the vector potential at the interval's midpoint. */
static void step(int scheme, int g, double psi[4], double dt, double px, double py, double Ax, double Ay) {
  double Px = px + Ax, Py = py + Ay;
  if (scheme == OR_SCHEME_MIDPOINT) {
    apply_midpoint(psi, dt, Px, Py, g);
  } else {
    apply_y(psi, g * 0.5 * dt * Py);
    apply_x(psi, g * dt * Px);
    apply_y(psi, g * 0.5 * dt * Py);
  }
}

/* Step k of the solve: every stage of the composition in turn. */
static void full_step(const oracle_problem* f, int g, double psi[4], const double* c, int S, double dt, double px,
                      double py, const double* Ax, const double* Ay, long long k) {
  for (int j = 0; j < S; ++j) step(f->scheme, g, psi, c[j] * dt, px, py, Ax[k * S + j], Ay[k * S + j]);
}

/* The 2x2 matrix of one step, column-major over the basis (e1, e2):
   U[0..3] = U e1 = (re, im, re, im), U[4..7] = U e2. */
void oracle_step_matrix(const oracle_problem* f, double px, double py, double dt, double A_k, double U[8]) {
  double e1[4] = {1.0, 0.0, 0.0, 0.0}, e2[4] = {0.0, 0.0, 1.0, 0.0};
  int g = f->valley >= 0 ? 1 : -1;
  step(f->scheme, g, e1, dt, px, py, A_k, 0.0);
  step(f->scheme, g, e2, dt, px, py, A_k, 0.0);
  memcpy(U, e1, sizeof e1);
  memcpy(U + 4, e2, sizeof e2);
}

/* The same with both components of A. */
void oracle_step_matrix_xy(const oracle_problem* f, double px, double py, double dt, double Ax, double Ay,
                           double U[8]) {
  double e1[4] = {1.0, 0.0, 0.0, 0.0}, e2[4] = {0.0, 0.0, 1.0, 0.0};
  int g = f->valley >= 0 ? 1 : -1;
  step(f->scheme, g, e1, dt, px, py, Ax, Ay);
  step(f->scheme, g, e2, dt, px, py, Ax, Ay);
  memcpy(U, e1, sizeof e1);
  memcpy(U + 4, e2, sizeof e2);
}

/* ------------------------------------------------------------------------ */

typedef struct {
  double* Ax;
  double* Ay;
  field_ends e;
  double c[5], sigma[5];
  int S;
} tables;

static int make_tables(const oracle_problem* f, tables* t) {
  t->S = oracle_composition(f->order, t->c, t->sigma);
  long long n = f->n_steps * t->S;
  t->Ax = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  t->Ay = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!t->Ax || !t->Ay) {
    free(t->Ax);
    free(t->Ay);
    return -1;
  }
  field_table(f, t->Ax, t->Ay, &t->e);
  return 0;
}

static void free_tables(tables* t) {
  free(t->Ax);
  free(t->Ay);
}

/* n = |u(P)^dagger psi|^2 with u the unit positive-energy spinor of the valley. */
static double project(int g, double Px, double Py, const double psi[4]) {
  double u[4], v[4];
  oracle_spinors(Px, Py, g, u, v);
  double re = (u[0] * psi[0] + u[1] * psi[1]) + (u[2] * psi[2] + u[3] * psi[3]);
  double im = (u[0] * psi[1] - u[1] * psi[0]) + (u[2] * psi[3] - u[3] * psi[2]);
  return re * re + im * im;
}

/* Propagate one momentum over the first k_stop steps and project on the
   positive-energy state at t_{k_stop}.  Returns 1 if the point is masked
   (|P| = 0 at t_i or at t_{k_stop}). */
static int solve_point(const oracle_problem* f, const tables* t, long long k_stop, double px, double py,
                       double* n_out, double* norm_dev, double psi_out[4]) {
  int g = f->valley >= 0 ? 1 : -1;
  double ax, ay;
  boundary_A(f, k_stop, t->Ax, t->Ay, &t->e, &ax, &ay);
  double Px_in = px + t->e.Ax_in, Py_in = py + t->e.Ay_in;
  double Px_out = px + ax, Py_out = py + ay;
  double E_in = sqrt(Px_in * Px_in + Py_in * Py_in);
  double E_out = sqrt(Px_out * Px_out + Py_out * Py_out);
  if (E_in == 0.0 || E_out == 0.0) {
    *n_out = 0.0;
    *norm_dev = 0.0;
    if (psi_out) memset(psi_out, 0, 4 * sizeof(double));
    return 1;
  }
  double u[4], v[4];
  oracle_spinors(Px_in, Py_in, g, u, v);
  double psi[4] = {v[0], v[1], v[2], v[3]};
  for (long long k = 0; k < k_stop; ++k) full_step(f, g, psi, t->c, t->S, t->e.dt, px, py, t->Ax, t->Ay, k);
  *n_out = project(g, Px_out, Py_out, psi);
  *norm_dev = (psi[0] * psi[0] + psi[1] * psi[1] + psi[2] * psi[2] + psi[3] * psi[3]) - 1.0;
  if (psi_out) memcpy(psi_out, psi, sizeof psi);
  return 0;
}

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  return nthreads;
#else
  (void)nthreads;
  return 1;
#endif
}

static long long solve_points_to(const oracle_problem* f, long long k_stop, long long count, const double* px,
                                  const double* py, double* n_out, double* norm_dev, int nthreads) {
  tables t;
  if (make_tables(f, &t) != 0) return -1;
  if (k_stop < 0) k_stop = 0;
  if (k_stop > f->n_steps) k_stop = f->n_steps;
  long long masked = 0;
  int nt = set_threads(nthreads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : masked) num_threads(nt)
  for (long long q = 0; q < count; ++q) {
    double nd;
    masked += solve_point(f, &t, k_stop, px[q], py[q], &n_out[q], &nd, NULL);
    if (norm_dev) norm_dev[q] = nd;
  }
  free_tables(&t);
  return masked;
}

/* n(p) at explicit momenta.  Returns the number of masked points, or -1 on
   allocation failure.  norm_dev (may be NULL) receives |psi_N|^2 - 1. */
long long oracle_solve_points(const oracle_problem* f, long long count, const double* px, const double* py,
                              double* n_out, double* norm_dev, int nthreads) {
  return solve_points_to(f, f->n_steps, count, px, py, n_out, norm_dev, nthreads);
}

/* Snapshot after the first k_steps steps: the occupation of the instantaneous
   positive-energy state of sigma.P(t_k), P(t_k) = p + A(t_i + k dt). */
long long oracle_snapshot_points(const oracle_problem* f, long long k_steps, long long count, const double* px,
                                 const double* py, double* n_out, int nthreads) {
  return solve_points_to(f, k_steps, count, px, py, n_out, NULL, nthreads);
}

/* Spinor after the first k_steps steps at one momentum (for continuum checks of
   the state itself).  Returns 1 if masked, -1 on allocation failure. */
int oracle_state_at(const oracle_problem* f, long long k_steps, double px, double py, double psi[4]) {
  tables t;
  if (make_tables(f, &t) != 0) return -1;
  double n, nd;
  int m = solve_point(f, &t, k_steps < f->n_steps ? k_steps : f->n_steps, px, py, &n, &nd, psi);
  free_tables(&t);
  return m;
}

/* Final spinor at one momentum. */
int oracle_final_state(const oracle_problem* f, double px, double py, double psi[4]) {
  return oracle_state_at(f, f->n_steps, px, py, psi);
}

/* Node grid: p_j = p_min + j (p_max - p_min) / n. */
double oracle_grid_p(double p_min, double p_max, int n, int j) {
  double d = (p_max - p_min) / (double)n;
  return p_min + (double)j * d;
}

/* n(p) on grid points given by linear index k = j*nx + i (idx == NULL: all,
   in index order).  Returns the masked count, or -1 on allocation failure. */
long long oracle_solve_grid(const oracle_problem* f, int nx, int ny, double px_min, double px_max, double py_min,
                            double py_max, const long long* idx, long long count, double* n_out, double* norm_dev,
                            int nthreads) {
  long long total = (long long)nx * (long long)ny;
  if (!idx) count = total;
  double* px = (double*)malloc((size_t)(count > 0 ? count : 1) * sizeof(double));
  double* py = (double*)malloc((size_t)(count > 0 ? count : 1) * sizeof(double));
  if (!px || !py) {
    free(px);
    free(py);
    return -1;
  }
  for (long long q = 0; q < count; ++q) {
    long long k = idx ? idx[q] : q;
    px[q] = oracle_grid_p(px_min, px_max, nx, (int)(k % nx));
    py[q] = oracle_grid_p(py_min, py_max, ny, (int)(k / nx));
  }
  long long m = oracle_solve_points(f, count, px, py, n_out, norm_dev, nthreads);
  free(px);
  free(py);
  return m;
}

/* rho = 4 dx dy / (2 pi)^2 * sum_k n_k over the full grid, summed in index
   order (kahan != 0: compensated summation). */
double oracle_density(int nx, int ny, double px_min, double px_max, double py_min, double py_max, const double* n,
                      int kahan) {
  double dx = (px_max - px_min) / (double)nx, dy = (py_max - py_min) / (double)ny;
  long long total = (long long)nx * (long long)ny;
  double s = 0.0, c = 0.0;
  for (long long k = 0; k < total; ++k) {
    if (kahan) {
      double y = n[k] - c;
      double t = s + y;
      c = (t - s) - y;
      s = t;
    } else {
      s += n[k];
    }
  }
  return 4.0 * dx * dy / (4.0 * M_PI * M_PI) * s;
}

/* A_x at the sample times (stages * N values, see field_table), A_x(t_i), A_x(t_f), dt. */
int oracle_field_table(const oracle_problem* f, double* A_mid, double* A_in, double* A_out, double* dt) {
  field_ends e;
  field_table(f, A_mid, NULL, &e);
  *A_in = e.Ax_in;
  *A_out = e.Ax_out;
  *dt = e.dt;
  return 0;
}

/* A_y at the sample times, A_y(t_i), A_y(t_f). */
int oracle_field_table_y(const oracle_problem* f, double* Ay_mid, double* Ay_in, double* Ay_out) {
  tables t;
  if (make_tables(f, &t) != 0) return -1;
  memcpy(Ay_mid, t.Ay, (size_t)(f->n_steps * t.S) * sizeof(double));
  *Ay_in = t.e.Ay_in;
  *Ay_out = t.e.Ay_out;
  free_tables(&t);
  return 0;
}

/* A at the step boundary t_i + k dt, both components (see boundary_A). */
int oracle_boundary_A(const oracle_problem* f, long long k, double* ax, double* ay) {
  tables t;
  if (make_tables(f, &t) != 0) return -1;
  boundary_A(f, k, t.Ax, t.Ay, &t.e, ax, ay);
  free_tables(&t);
  return 0;
}
