// Host side of the field: the vector potential A(t) of each supported field
// kind, sampled at the step midpoints, and the per-step rows the kernels read.
//
// Gauge A_0 = 0, E = -dA/dt, A(t) = -int_{t_i}^{t} E (Sec. II, after Eq. (2));
// A is sampled at t_i + (k + 1/2) dt (Sec. III, Eqs. (11)-(12)).
#include <cmath>
#include <cstring>

#include "pd_internal.h"

namespace pdx {
namespace {

constexpr double kPi = 3.14159265358979323846;

// 2 sin^2(x/2) = 1 - cos x without cancellation at small x.
double versine(double x) {
  double s = std::sin(0.5 * x);
  return 2.0 * s * s;
}

// sin^2-envelope pulse E0 sin^2(pi t / T) sin(w t) on [0, T]: with W = 2 pi / T,
// E = (E0/2) sin(w t) - (E0/4) sin((w + W) t) - (E0/4) sin((w - W) t), whose
// integral from 0 is a sum of versines.
struct Sin2Pulse {
  double E0, w, W, T;
  double A(double t) const {
    if (t <= 0.0) return 0.0;
    if (t > T) t = T;
    double I = versine(w * t) / (2.0 * w) - versine((w + W) * t) / (4.0 * (w + W)) -
               versine((w - W) * t) / (4.0 * (w - W));
    return -E0 * I;
  }
};

// The laser pulse of Sec. IV, Eq. (14): carrier cos(w t + phi) under an envelope
// that rises as sin^2(Wr t) over [0, tr], tr = pi/(2 Wr), is flat, and falls as
// cos^2(Wf (t - ta)) over [ta, D], ta = D - pi/(2 Wf).
struct LaserPulse {
  double E0, w, phi, Wr, Wf, D;
  double tr() const { return kPi / (2.0 * Wr); }
  double ta() const { return D - kPi / (2.0 * Wf); }
  // int_a^b cos(w t + phi) dt
  double carrier(double a, double b) const { return (std::sin(w * b + phi) - std::sin(w * a + phi)) / w; }
  // int_a^b cos(2 W (t - c)) cos(w t + phi) dt
  double beat(double W, double c, double a, double b) const {
    double w1 = w + 2.0 * W, q1 = phi - 2.0 * W * c;
    double w2 = w - 2.0 * W, q2 = phi + 2.0 * W * c;
    double i1 = (std::sin(w1 * b + q1) - std::sin(w1 * a + q1)) / w1;
    double i2 = (w2 != 0.0) ? (std::sin(w2 * b + q2) - std::sin(w2 * a + q2)) / w2 : (b - a) * std::cos(q2);
    return 0.5 * (i1 + i2);
  }
  double A(double t) const {
    if (t <= 0.0) return 0.0;
    if (t > D) t = D;
    double r = tr(), a = ta(), I = 0.0;
    double e1 = std::fmin(t, r);  // rise: sin^2 = (1 - cos 2 Wr t) / 2
    I += 0.5 * carrier(0.0, e1) - 0.5 * beat(Wr, 0.0, 0.0, e1);
    if (t > r) {
      double e2 = std::fmin(t, a);
      if (e2 > r) I += carrier(r, e2);
      if (t > a) I += 0.5 * carrier(a, t) + 0.5 * beat(Wf, a, a, t);  // fall: cos^2 = (1 + cos 2 Wf (t - a)) / 2
    }
    return -E0 * I;
  }
};

bool finite(double x) { return std::isfinite(x); }

}  // namespace

bool sample_field(const pd_field& f, long long n_steps, FieldTables* out, std::string* err) {
  if (n_steps < 1) {
    *err = "n_steps must be >= 1";
    return false;
  }
  if (n_steps > (1LL << 31)) {
    *err = "n_steps must be <= 2^31";
    return false;
  }
  FieldTables t;
  t.n_steps = n_steps;
  t.A_mid.resize((size_t)n_steps);
  auto sample = [&](auto&& A) {
    t.dt = (t.t_f - t.t_i) / (double)n_steps;
    for (long long k = 0; k < n_steps; ++k) t.A_mid[(size_t)k] = A(t.t_i + ((double)k + 0.5) * t.dt);
    t.A_in = A(t.t_i);
    t.A_out = A(t.t_f);
  };
  switch (f.kind) {
    case PD_FIELD_SIN2: {
      if (!finite(f.E0) || !finite(f.omega) || f.omega <= 0.0) {
        *err = "sin2 field needs finite E0 and omega > 0";
        return false;
      }
      if (f.cycles < 2) {
        *err = "sin2 field needs cycles >= 2";
        return false;
      }
      Sin2Pulse s{f.E0, f.omega, 0.0, f.cycles * 2.0 * kPi / f.omega};
      s.W = 2.0 * kPi / s.T;
      t.t_i = 0.0;
      t.t_f = s.T;
      sample([&](double x) { return s.A(x); });
      break;
    }
    case PD_FIELD_CONSTANT: {
      if (!finite(f.E0) || !finite(f.t_end) || f.t_end <= 0.0) {
        *err = "constant field needs finite E0 and t_end > 0";
        return false;
      }
      double E0 = f.E0, te = f.t_end;
      t.t_i = 0.0;
      t.t_f = te;
      sample([&](double x) { return x <= 0.0 ? 0.0 : -E0 * (x < te ? x : te); });
      break;
    }
    case PD_FIELD_PULSE: {
      LaserPulse p{f.E0, f.omega, f.phi, f.omega_rise, f.omega_fall, f.duration};
      if (!finite(f.E0) || !finite(f.omega) || !finite(f.phi) || f.omega <= 0.0 || !(f.omega_rise > 0.0) ||
          !(f.omega_fall > 0.0) || !finite(f.duration)) {
        *err = "pulse field needs finite E0, phi, duration and omega, omega_rise, omega_fall > 0";
        return false;
      }
      if (p.ta() < p.tr()) {
        *err = "pulse duration shorter than its rise plus fall windows";
        return false;
      }
      t.t_i = 0.0;
      t.t_f = f.duration;
      sample([&](double x) { return p.A(x); });
      break;
    }
    case PD_FIELD_TABLE: {
      if (!f.A_mid || f.n_table != n_steps) {
        *err = "table field needs A_mid with n_table == n_steps values";
        return false;
      }
      if (!finite(f.t_i) || !finite(f.t_f) || !(f.t_f > f.t_i) || !finite(f.A_in) || !finite(f.A_out)) {
        *err = "table field needs finite t_i < t_f, A_in, A_out";
        return false;
      }
      t.t_i = f.t_i;
      t.t_f = f.t_f;
      t.dt = (t.t_f - t.t_i) / (double)n_steps;
      std::memcpy(t.A_mid.data(), f.A_mid, (size_t)n_steps * sizeof(double));
      for (long long k = 0; k < n_steps; ++k)
        if (!finite(t.A_mid[(size_t)k])) {
          *err = "table field has a non-finite value";
          return false;
        }
      t.A_in = f.A_in;
      t.A_out = f.A_out;
      break;
    }
    default:
      *err = "unknown field kind";
      return false;
  }
  t.A_min = std::fmin(t.A_in, t.A_out);
  t.A_max = std::fmax(t.A_in, t.A_out);
  for (double a : t.A_mid) {
    t.A_min = std::fmin(t.A_min, a);
    t.A_max = std::fmax(t.A_max, a);
  }
  if (!finite(t.A_min) || !finite(t.A_max) || !(t.dt > 0.0)) {
    *err = "field sampling produced non-finite values";
    return false;
  }
  *out = std::move(t);
  return true;
}

void field_extent(const Grid& g, FieldTables* t) {
  // |p + A| is largest at a corner of the box [grid x range] x [A range].
  double x0 = g.px(0), x1 = g.px(g.nx - 1);
  double y = std::fmax(std::fabs(g.py(0)), std::fabs(g.py(g.ny - 1)));
  double X = std::fmax(std::fmax(std::fabs(x0 + t->A_min), std::fabs(x0 + t->A_max)),
                       std::fmax(std::fabs(x1 + t->A_min), std::fabs(x1 + t->A_max)));
  t->E_max = std::sqrt(X * X + y * y);
}

long long count_masked(const Grid& g, double A_in, double A_out) {
  // |P| = sqrt(Px^2 + py^2) is 0 only where py^2 == 0; scan those rows.
  long long m = 0;
  for (int j = 0; j < g.ny; ++j) {
    double py = g.py(j);
    if (py * py != 0.0) continue;
    for (int i = 0; i < g.nx; ++i) {
      double px = g.px(i);
      double Pi = px + A_in, Po = px + A_out;
      double Ei = std::sqrt(Pi * Pi + py * py), Eo = std::sqrt(Po * Po + py * py);
      if (Ei == 0.0 || Eo == 0.0) ++m;
    }
  }
  return m;
}

size_t table_row_bytes(int scheme, int precision) {
  if (scheme == PD_SCHEME_MIDPOINT) return sizeof(double);
  return precision == PD_FP32 ? 2 * sizeof(float) : 2 * sizeof(double);
}

void build_step_table(const FieldTables& t, int scheme, int precision, int form, std::vector<unsigned char>* rows) {
  size_t n = (size_t)t.n_steps;
  rows->resize(n * table_row_bytes(scheme, precision));
  if (scheme == PD_SCHEME_MIDPOINT) {
    double* d = reinterpret_cast<double*>(rows->data());
    for (size_t k = 0; k < n; ++k) d[k] = t.dt * t.A_mid[k];
    return;
  }
  // The sigma_x factor exp(-i dt A_k sigma_x) rotates the Bloch vector by
  // phi = 2a, a = dt A_k, about x: store (tan a, sin 2a) for the shear form or
  // (cos 2a - 1, sin 2a) = (-2 sin^2 a, 2 sin a cos a) for the versine form.
  for (size_t k = 0; k < n; ++k) {
    double a = t.dt * t.A_mid[k];
    double sa = std::sin(a), ca = std::cos(a);
    double c0 = form == kFormShear ? sa / ca : -2.0 * sa * sa, c1 = 2.0 * sa * ca;
    if (precision == PD_FP32) {
      float* r = reinterpret_cast<float*>(rows->data()) + 2 * k;
      r[0] = (float)c0;
      r[1] = (float)c1;
    } else {
      double* r = reinterpret_cast<double*>(rows->data()) + 2 * k;
      r[0] = c0;
      r[1] = c1;
    }
  }
}

namespace {

// Coefficients of the rotation by phi = 2 * half in the given form.
void rotation_coefficients(double half, int form, double* a, double* s) {
  double sh = std::sin(half), ch = std::cos(half);
  *s = 2.0 * sh * ch;
  *a = form == kFormShear ? sh / ch : -2.0 * sh * sh;
}

template <typename R>
void put(std::vector<unsigned char>* bytes, size_t offset, size_t index, double v) {
  reinterpret_cast<R*>(bytes->data() + offset)[index] = (R)v;
}

}  // namespace

void build_point_coefficients(const Grid& g, double dt, int precision, int form, std::vector<unsigned char>* bytes,
                              size_t* col_offset, size_t* row_offset) {
  const size_t v = precision == PD_FP32 ? sizeof(float) : sizeof(double);
  auto align = [](size_t n) { return (n + 255) / 256 * 256; };
  *col_offset = align(bytes->size());
  *row_offset = align(*col_offset + 2 * v * (size_t)g.nx);
  bytes->resize(align(*row_offset + 4 * v * (size_t)g.ny));
  auto store = [&](size_t off, size_t idx, double x) {
    if (precision == PD_FP32)
      put<float>(bytes, off, idx, x);
    else
      put<double>(bytes, off, idx, x);
  };
  double a, s;
  for (int i = 0; i < g.nx; ++i) {
    rotation_coefficients(dt * g.px(i), form, &a, &s);  // rotation by 2 dt px about x
    store(*col_offset, 2 * (size_t)i, a);
    store(*col_offset, 2 * (size_t)i + 1, s);
  }
  for (int j = 0; j < g.ny; ++j) {
    double py = g.py(j);
    rotation_coefficients(dt * py, form, &a, &s);  // rotation by 2 dt py about y
    store(*row_offset, 4 * (size_t)j, a);
    store(*row_offset, 4 * (size_t)j + 1, s);
    rotation_coefficients(0.5 * dt * py, form, &a, &s);  // half step: rotation by dt py
    store(*row_offset, 4 * (size_t)j + 2, a);
    store(*row_offset, 4 * (size_t)j + 3, s);
  }
}

int strang_form(const Grid& g, const FieldTables& t) {
  // Bloch rotation angles of a step: 2 dt A_k, 2 dt px and 2 dt py.
  double amax = std::fmax(std::fabs(t.A_min), std::fabs(t.A_max));
  double pxmax = std::fmax(std::fabs(g.px(0)), std::fabs(g.px(g.nx - 1)));
  double pymax = std::fmax(std::fabs(g.py(0)), std::fabs(g.py(g.ny - 1)));
  double phi = 2.0 * t.dt * std::fmax(amax, std::fmax(pxmax, pymax));
  return phi <= kShearMaxAngle ? kFormShear : kFormVersine;
}

int taylor_order(double x_max, int precision) {
  // Orders compiled into the midpoint kernels.
  static const int kOrders64[] = {5, 8, 14};
  static const int kOrders32[] = {3, 5, 9};
  const int* orders = precision == PD_FP32 ? kOrders32 : kOrders64;
  double tol = precision == PD_FP32 ? 0x1p-27 : 0x1p-56;
  for (int q = 0; q < 3; ++q) {
    int J = orders[q];
    // relative size of the first omitted terms: 2 x^J / (2J+2)! for cos - 1 and
    // x^(J+1) / (2J+3)! for sin(x)/x
    double f = 1.0;
    for (int m = 2; m <= 2 * J + 2; ++m) f *= m;
    double e1 = 2.0 * std::pow(x_max, J) / f;
    double e2 = std::pow(x_max, J + 1) / (f * (2 * J + 3));
    if (e1 <= tol && e2 <= tol) return J;
  }
  return -1;
}

}  // namespace pdx
