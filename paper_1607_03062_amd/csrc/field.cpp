// Host side of the field: the vector potential A(t) of each supported field
// kind (both components), sampled at the times the scheme uses, and the per-step
// rows and per-point rotation coefficients the kernels read.
//
// Gauge A_0 = 0, E = -dA/dt, A(t) = -int_{t_i}^{t} E (Sec. II, after Eq. (2));
// A is sampled at the step midpoints t_i + (k + 1/2) dt (Sec. III, Eqs. (11)-(12)),
// or for the fourth-order composition at the stage midpoints t_i + (k + sigma_j) dt.
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
// integral from 0 is a sum of versines.  Elliptic: E_y = e E0 sin^2(pi t/T) cos(w t)
// = (e E0/2) cos(w t) - (e E0/4)[cos((w + W) t) + cos((w - W) t)], integral a sum of sines.
struct Sin2Pulse {
  double E0, w, W, T, e;
  double A(double t) const {
    if (t <= 0.0) return 0.0;
    if (t > T) t = T;
    double I = versine(w * t) / (2.0 * w) - versine((w + W) * t) / (4.0 * (w + W)) -
               versine((w - W) * t) / (4.0 * (w - W));
    return -E0 * I;
  }
  double Ay(double t) const {
    if (t <= 0.0) return 0.0;
    if (t > T) t = T;
    double I = std::sin(w * t) / (2.0 * w) - std::sin((w + W) * t) / (4.0 * (w + W)) -
               std::sin((w - W) * t) / (4.0 * (w - W));
    return -e * E0 * I;
  }
};

// The laser pulse of Sec. IV, Eq. (14): carrier cos(w t + phi) under an envelope
// that rises as sin^2(Wr t) over [0, tr], tr = pi/(2 Wr), is flat, and falls as
// cos^2(Wf (t - ta)) over [ta, D], ta = D - pi/(2 Wf).  Its y component (elliptic)
// has the carrier sin(w t + phi) = cos(w t + phi - pi/2).
struct LaserPulse {
  double E0, w, phi, Wr, Wf, D;
  double tr() const { return kPi / (2.0 * Wr); }
  double ta() const { return D - kPi / (2.0 * Wf); }
  // int_a^b cos(w t + q) dt
  double carrier(double q, double a, double b) const { return (std::sin(w * b + q) - std::sin(w * a + q)) / w; }
  // int_a^b cos(2 W (t - c)) cos(w t + q) dt
  double beat(double q, double W, double c, double a, double b) const {
    double w1 = w + 2.0 * W, q1 = q - 2.0 * W * c;
    double w2 = w - 2.0 * W, q2 = q + 2.0 * W * c;
    double i1 = (std::sin(w1 * b + q1) - std::sin(w1 * a + q1)) / w1;
    double i2 = (w2 != 0.0) ? (std::sin(w2 * b + q2) - std::sin(w2 * a + q2)) / w2 : (b - a) * std::cos(q2);
    return 0.5 * (i1 + i2);
  }
  // -E0 int_0^t env(s) cos(w s + q) ds
  double A_phase(double q, double t) const {
    if (t <= 0.0) return 0.0;
    if (t > D) t = D;
    double r = tr(), a = ta(), I = 0.0;
    double e1 = std::fmin(t, r);  // rise: sin^2 = (1 - cos 2 Wr t) / 2
    I += 0.5 * carrier(q, 0.0, e1) - 0.5 * beat(q, Wr, 0.0, 0.0, e1);
    if (t > r) {
      double e2 = std::fmin(t, a);
      if (e2 > r) I += carrier(q, r, e2);
      if (t > a) I += 0.5 * carrier(q, a, t) + 0.5 * beat(q, Wf, a, a, t);  // fall: cos^2 = (1 + cos 2 Wf (t - a)) / 2
    }
    return -E0 * I;
  }
};

bool finite(double x) { return std::isfinite(x); }

// (A_x, A_y) of an analytic field kind at time t (the kind is validated).
void eval_A(const pd_field& f, double t, double* ax, double* ay) {
  switch (f.kind) {
    case PD_FIELD_SIN2: {
      double T = f.cycles * 2.0 * kPi / f.omega;
      Sin2Pulse s{f.E0, f.omega, 2.0 * kPi / T, T, f.ellipticity};
      *ax = s.A(t);
      *ay = f.ellipticity != 0.0 ? s.Ay(t) : 0.0;
      return;
    }
    case PD_FIELD_CONSTANT: {
      double u = t <= 0.0 ? 0.0 : (t < f.t_end ? t : f.t_end);
      *ax = -f.E0 * u;
      *ay = f.ellipticity != 0.0 ? -f.ellipticity * f.E0 * u : 0.0;
      return;
    }
    case PD_FIELD_PULSE: {
      LaserPulse p{f.E0, f.omega, f.phi, f.omega_rise, f.omega_fall, f.duration};
      *ax = p.A_phase(f.phi, t);
      *ay = f.ellipticity != 0.0 ? f.ellipticity * p.A_phase(f.phi - 0.5 * kPi, t) : 0.0;
      return;
    }
    default:
      *ax = 0.0;
      *ay = 0.0;
  }
}

}  // namespace

Composition composition_of(int scheme) {
  Composition c;
  if (scheme == PD_SCHEME_STRANG4 || scheme == PD_SCHEME_MIDPOINT4) {
    const double p = 1.0 / (4.0 - std::cbrt(4.0));
    c.stages = 5;
    const double v[5] = {p, p, 1.0 - 4.0 * p, p, p};
    double start = 0.0;
    c.cmax = 0.0;
    for (int j = 0; j < 5; ++j) {
      c.c[j] = v[j];
      c.sigma[j] = start + 0.5 * v[j];
      start += v[j];
      c.cmax = std::fmax(c.cmax, std::fabs(v[j]));
    }
  }
  return c;
}

bool sample_field(const pd_field& f, long long n_steps, const Composition& comp, FieldTables* out,
                  std::string* err) {
  if (n_steps < 1) {
    *err = "n_steps must be >= 1";
    return false;
  }
  if (n_steps > (1LL << 31)) {
    *err = "n_steps must be <= 2^31";
    return false;
  }
  const int S = comp.stages;
  const size_t n_samples = (size_t)n_steps * (size_t)S;
  FieldTables t;
  t.n_steps = n_steps;
  t.comp = comp;
  t.spec = f;
  t.spec.A_mid = nullptr;
  t.spec.Ay_mid = nullptr;
  if (f.kind != PD_FIELD_TABLE && !finite(f.ellipticity)) {
    *err = "ellipticity must be finite";
    return false;
  }
  switch (f.kind) {
    case PD_FIELD_SIN2:
      if (!finite(f.E0) || !finite(f.omega) || f.omega <= 0.0) {
        *err = "sin2 field needs finite E0 and omega > 0";
        return false;
      }
      if (f.cycles < 2) {
        *err = "sin2 field needs cycles >= 2";
        return false;
      }
      t.t_i = 0.0;
      t.t_f = f.cycles * 2.0 * kPi / f.omega;
      break;
    case PD_FIELD_CONSTANT:
      if (!finite(f.E0) || !finite(f.t_end) || f.t_end <= 0.0) {
        *err = "constant field needs finite E0 and t_end > 0";
        return false;
      }
      t.t_i = 0.0;
      t.t_f = f.t_end;
      break;
    case PD_FIELD_PULSE: {
      LaserPulse p{f.E0, f.omega, f.phi, f.omega_rise, f.omega_fall, f.duration};
      if (!finite(f.E0) || !finite(f.omega) || !finite(f.phi) || f.omega <= 0.0 || !(f.omega_rise > 0.0) ||
          !(f.omega_fall > 0.0) || !finite(f.duration)) {
        *err = "pulse field needs finite E0, phi, duration and omega, omega_rise, omega_fall > 0";
        return false;
      }
      // a pulse with no flat part (duration = rise + fall window) is valid: allow rounding
      if (p.ta() < p.tr() - 1e-12 * std::fabs(f.duration)) {
        *err = "pulse duration shorter than its rise plus fall windows";
        return false;
      }
      t.t_i = 0.0;
      t.t_f = f.duration;
      break;
    }
    case PD_FIELD_TABLE:
      if (!f.A_mid || f.n_table != (long long)n_samples) {
        *err = S == 1 ? "table field needs A_mid with n_table == n_steps values"
                      : "table field needs A_mid with n_table == 5 * n_steps values (one per stage)";
        return false;
      }
      if (!finite(f.t_i) || !finite(f.t_f) || !(f.t_f > f.t_i) || !finite(f.A_in) || !finite(f.A_out)) {
        *err = "table field needs finite t_i < t_f, A_in, A_out";
        return false;
      }
      if (f.Ay_mid && (!finite(f.Ay_in) || !finite(f.Ay_out))) {
        *err = "table field with Ay_mid needs finite Ay_in, Ay_out";
        return false;
      }
      t.t_i = f.t_i;
      t.t_f = f.t_f;
      break;
    default:
      *err = "unknown field kind";
      return false;
  }
  t.dt = (t.t_f - t.t_i) / (double)n_steps;
  t.elliptic = f.kind == PD_FIELD_TABLE ? f.Ay_mid != nullptr : f.ellipticity != 0.0;
  t.A_mid.resize(n_samples);
  if (t.elliptic) t.Ay_mid.resize(n_samples);
  if (f.kind == PD_FIELD_TABLE) {
    std::memcpy(t.A_mid.data(), f.A_mid, n_samples * sizeof(double));
    if (t.elliptic) std::memcpy(t.Ay_mid.data(), f.Ay_mid, n_samples * sizeof(double));
    t.A_in = f.A_in;
    t.A_out = f.A_out;
    t.Ay_in = t.elliptic ? f.Ay_in : 0.0;
    t.Ay_out = t.elliptic ? f.Ay_out : 0.0;
  } else {
    parallel_ranges(n_steps, 8192, [&](long long k0, long long k1) {
      double ax, ay;
      for (long long k = k0; k < k1; ++k)
        for (int j = 0; j < S; ++j) {
          eval_A(f, t.t_i + ((double)k + comp.sigma[j]) * t.dt, &ax, &ay);
          t.A_mid[(size_t)k * S + j] = ax;
          if (t.elliptic) t.Ay_mid[(size_t)k * S + j] = ay;
        }
    });
    eval_A(f, t.t_i, &t.A_in, &t.Ay_in);
    eval_A(f, t.t_f, &t.A_out, &t.Ay_out);
  }
  for (double a : t.A_mid)
    if (!finite(a)) {
      *err = "field has a non-finite value";
      return false;
    }
  for (double a : t.Ay_mid)
    if (!finite(a)) {
      *err = "field has a non-finite value";
      return false;
    }
  t.A_min = std::fmin(t.A_in, t.A_out);
  t.A_max = std::fmax(t.A_in, t.A_out);
  for (double a : t.A_mid) {
    t.A_min = std::fmin(t.A_min, a);
    t.A_max = std::fmax(t.A_max, a);
  }
  t.Ay_min = std::fmin(t.Ay_in, t.Ay_out);
  t.Ay_max = std::fmax(t.Ay_in, t.Ay_out);
  for (double a : t.Ay_mid) {
    t.Ay_min = std::fmin(t.Ay_min, a);
    t.Ay_max = std::fmax(t.Ay_max, a);
  }
  if (!finite(t.A_min) || !finite(t.A_max) || !finite(t.Ay_min) || !finite(t.Ay_max) || !(t.dt > 0.0)) {
    *err = "field sampling produced non-finite values";
    return false;
  }
  *out = std::move(t);
  return true;
}

void boundary_A(const FieldTables& t, long long k, double* ax, double* ay) {
  const long long S = t.comp.stages;
  if (k <= 0) {
    *ax = t.A_in;
    *ay = t.Ay_in;
  } else if (k >= t.n_steps) {
    *ax = t.A_out;
    *ay = t.Ay_out;
  } else if (t.spec.kind == PD_FIELD_TABLE) {
    *ax = 0.5 * (t.A_mid[(size_t)(k * S - 1)] + t.A_mid[(size_t)(k * S)]);
    *ay = t.elliptic ? 0.5 * (t.Ay_mid[(size_t)(k * S - 1)] + t.Ay_mid[(size_t)(k * S)]) : 0.0;
  } else {
    eval_A(t.spec, t.t_i + (double)k * t.dt, ax, ay);
    if (!t.elliptic) *ay = 0.0;
  }
}

void field_extent(const Grid& g, FieldTables* t) {
  // |p + A| is largest at a corner of the box [grid range] x [A range], per component.
  double x0 = g.px(0), x1 = g.px(g.nx - 1);
  double y0 = g.py(0), y1 = g.py(g.ny - 1);
  double X = std::fmax(std::fmax(std::fabs(x0 + t->A_min), std::fabs(x0 + t->A_max)),
                       std::fmax(std::fabs(x1 + t->A_min), std::fabs(x1 + t->A_max)));
  double Y = std::fmax(std::fmax(std::fabs(y0 + t->Ay_min), std::fabs(y0 + t->Ay_max)),
                       std::fmax(std::fabs(y1 + t->Ay_min), std::fabs(y1 + t->Ay_max)));
  t->E_max = std::sqrt(X * X + Y * Y);
}

long long count_masked(const Grid& g, const FieldTables& t) {
  // |P| = sqrt(Px^2 + Py^2) is 0 only where Py^2 == 0; scan those rows.
  long long m = 0;
  for (int j = 0; j < g.ny; ++j) {
    double py = g.py(j);
    double Pyi = py + t.Ay_in, Pyo = py + t.Ay_out;
    if (Pyi * Pyi != 0.0 && Pyo * Pyo != 0.0) continue;
    for (int i = 0; i < g.nx; ++i) {
      double px = g.px(i);
      double Pi = px + t.A_in, Po = px + t.A_out;
      double Ei = std::sqrt(Pi * Pi + Pyi * Pyi), Eo = std::sqrt(Po * Po + Pyo * Pyo);
      if (Ei == 0.0 || Eo == 0.0) ++m;
    }
  }
  return m;
}

size_t table_row_values(int scheme, int elliptic) {
  const size_t S = (size_t)composition_of(scheme).stages;
  const size_t per = base_scheme(scheme) == PD_SCHEME_MIDPOINT ? 1 : 2;
  return per * S * (elliptic ? 2 : 1);
}

size_t table_row_bytes(int scheme, int precision, int elliptic) {
  size_t v = (base_scheme(scheme) == PD_SCHEME_STRANG && is_fp32(precision)) ? sizeof(float) : sizeof(double);
  return table_row_values(scheme, elliptic) * v;
}

long long table_rows(int scheme, int elliptic, long long n_steps) {
  return (base_scheme(scheme) == PD_SCHEME_STRANG && elliptic) ? n_steps + 1 : n_steps;
}

void rotation_coefficients(double half, int form, double* a, double* s) {
  double sh = std::sin(half), ch = std::cos(half);
  *s = 2.0 * sh * ch;
  *a = form == kFormShear ? sh / ch : -2.0 * sh * sh;
}

namespace {

template <typename R>
void put(std::vector<unsigned char>* bytes, size_t offset, size_t index, double v) {
  reinterpret_cast<R*>(bytes->data() + offset)[index] = (R)v;
}

}  // namespace

void build_step_table(const FieldTables& t, int scheme, int precision, int form, double vsign,
                      std::vector<unsigned char>* rows) {
  const long long N = t.n_steps;
  const int S = t.comp.stages;
  const int ell = t.elliptic ? 1 : 0;
  const size_t W = table_row_values(scheme, ell);
  const long long R = table_rows(scheme, ell, N);
  rows->assign((size_t)R * table_row_bytes(scheme, precision, ell), 0);
  const double* c = t.comp.c;
  if (base_scheme(scheme) == PD_SCHEME_MIDPOINT) {
    // per stage the phase increment c_j dt A at the stage midpoint (then c_j dt A_y)
    double* d = reinterpret_cast<double*>(rows->data());
    for (long long k = 0; k < N; ++k)
      for (int j = 0; j < S; ++j) {
        d[(size_t)k * W + j] = vsign * (c[j] * t.dt) * t.A_mid[(size_t)k * S + j];
        if (ell) d[(size_t)k * W + S + j] = vsign * (c[j] * t.dt) * t.Ay_mid[(size_t)k * S + j];
      }
    return;
  }
  // Strang.  exp(-i h A sigma_x) rotates the Bloch vector by 2h A about x: store the
  // coefficients of the rotation by 2 * half, half = c_j dt A (valley sign included).
  auto store = [&](long long row, size_t slot, double half) {
    double a, s;
    rotation_coefficients(half, form, &a, &s);
    if (is_fp32(precision)) {
      put<float>(rows, 0, (size_t)row * W + 2 * slot, a);
      put<float>(rows, 0, (size_t)row * W + 2 * slot + 1, s);
    } else {
      put<double>(rows, 0, (size_t)row * W + 2 * slot, a);
      put<double>(rows, 0, (size_t)row * W + 2 * slot + 1, s);
    }
  };
  for (long long k = 0; k < N; ++k)
    for (int j = 0; j < S; ++j) store(k, (size_t)j, vsign * (c[j] * t.dt) * t.A_mid[(size_t)k * S + j]);
  if (!ell) return;
  // The y half steps of neighbouring stages (and of the last stage of a step and
  // the first of the next) are merged; the field part of the merged rotation
  // after stage j has half angle dt (c_j A_y,j + c_j+1 A_y,j+1) / 2.
  auto ay = [&](long long k, int j) { return t.Ay_mid[(size_t)k * S + j]; };
  for (long long k = 0; k < N; ++k)
    for (int j = 0; j < S; ++j) {
      double sum;
      if (j + 1 < S)
        sum = c[j] * ay(k, j) + c[j + 1] * ay(k, j + 1);
      else if (k + 1 < N)
        sum = c[j] * ay(k, j) + c[0] * ay(k + 1, 0);
      else
        sum = c[j] * ay(k, j);  // closing half step
      store(k, (size_t)(S + j), vsign * 0.5 * t.dt * sum);
    }
  store(N, (size_t)S, vsign * 0.5 * t.dt * (c[0] * ay(0, 0)));  // opening half step
}

size_t point_coefficient_pairs_x(int scheme, int precision) {
  return (composition_of(scheme).stages == 5 ? 2 : 1) * (size_t)coefficient_phases(precision);
}
size_t point_coefficient_pairs_y(int scheme, int precision) {
  return (composition_of(scheme).stages == 5 ? 2 : 1) * (size_t)coefficient_phases(precision) + 1;
}

namespace {

// The `phases` FP32 values of a coefficient x: the FP32 neighbours of |x| below
// and above it, the upper one in round(phases * f) of the phases, f being where |x|
// lies between them, with the sign of x (so that -x gives the negated values: the
// rotations of the K- valley are those of K+ with every angle negated); the phases
// that take the upper value are spread over the cycle (order 0, 2, 1, 3 for four
// phases), so that partial sums over the cycle stay close to x too.
void dither(double x, int phases, float* out) {
  if (x < 0.0) {
    dither(-x, phases, out);
    for (int h = 0; h < phases; ++h) out[h] = -out[h];
    return;
  }
  float lo = (float)x;
  if ((double)lo > x) lo = std::nextafter(lo, -INFINITY);
  const float hi = std::nextafter(lo, INFINITY);
  const double f = (x - (double)lo) / ((double)hi - (double)lo);
  const int up = (int)std::lround(f * phases);
  for (int h = 0; h < phases; ++h) {
    // rank of phase h in the bit-reversed order of the cycle
    int r = 0;
    for (int b = 1, v = h; b < phases; b <<= 1, v >>= 1) r = (r << 1) | (v & 1);
    out[h] = r < up ? hi : lo;
  }
}

}  // namespace

void build_point_coefficients(const Grid& g, const FieldTables& t, int scheme, int precision, int form, double vsign,
                              std::vector<unsigned char>* bytes, size_t* col_offset, size_t* row_offset) {
  const bool f32 = is_fp32(precision);
  const size_t v = f32 ? sizeof(float) : sizeof(double);
  const int H = coefficient_phases(precision);
  const size_t nxp = point_coefficient_pairs_x(scheme, precision), nyp = point_coefficient_pairs_y(scheme, precision);
  auto align = [](size_t n) { return (n + 255) / 256 * 256; };
  *col_offset = align(bytes->size());
  *row_offset = align(*col_offset + 2 * nxp * v * (size_t)g.nx);
  bytes->resize(align(*row_offset + 2 * nyp * v * (size_t)g.ny));
  // pair `pair` of `entry` (column or row) from the exact coefficients (a, s): one
  // value per phase in FP32 (dithered), the value itself in FP64
  auto store_pair = [&](size_t off, size_t entry, size_t per_entry, size_t pair, int phases, double a, double s) {
    float da[kDitherFP32], ds[kDitherFP32];
    if (f32 && phases > 1) {
      dither(a, phases, da);
      dither(s, phases, ds);
    }
    for (int h = 0; h < phases; ++h) {
      const size_t idx = 2 * (per_entry * entry + pair + (size_t)h);
      if (!f32) {
        put<double>(bytes, off, idx, a);
        put<double>(bytes, off, idx + 1, s);
      } else if (phases > 1) {
        put<float>(bytes, off, idx, da[h]);
        put<float>(bytes, off, idx + 1, ds[h]);
      } else {
        put<float>(bytes, off, idx, a);
        put<float>(bytes, off, idx + 1, s);
      }
    }
  };
  // Half-angle multipliers of dt px and dt py: x rotation of stage j: c_j; y
  // rotation after stage j: (c_j + c_j+1) / 2 (cyclic); opening / closing half: c_1 / 2.
  const double* c = t.comp.c;
  double mx[2], my[3];
  int nmx, nmy;  // distinct multipliers (the half step excluded)
  if (t.comp.stages == 5) {
    mx[0] = c[0];
    mx[1] = c[2];
    my[0] = 0.5 * (c[0] + c[1]);
    my[1] = 0.5 * (c[1] + c[2]);
    my[2] = 0.5 * c[0];
    nmx = nmy = 2;
  } else {
    mx[0] = 1.0;
    my[0] = 1.0;
    my[1] = 0.5;
    nmx = nmy = 1;
  }
  double a, s;
  for (int i = 0; i < g.nx; ++i)
    for (int q = 0; q < nmx; ++q) {
      rotation_coefficients(vsign * (mx[q] * t.dt) * g.px(i), form, &a, &s);
      store_pair(*col_offset, (size_t)i, nxp, (size_t)q * H, H, a, s);
    }
  for (int j = 0; j < g.ny; ++j) {
    for (int q = 0; q < nmy; ++q) {
      rotation_coefficients(vsign * (my[q] * t.dt) * g.py(j), form, &a, &s);
      store_pair(*row_offset, (size_t)j, nyp, (size_t)q * H, H, a, s);
    }
    // the opening / closing half step: applied twice per solve, one value
    rotation_coefficients(vsign * (my[nmy] * t.dt) * g.py(j), form, &a, &s);
    store_pair(*row_offset, (size_t)j, nyp, (size_t)nmy * H, 1, a, s);
  }
}

int strang_form(const Grid& g, const FieldTables& t) {
  // Bloch rotation angles of a stage: 2 c dt A_x, 2 c dt px, at most 2 c dt py and
  // 2 c dt A_y (merged halves), c <= cmax.
  double amax = std::fmax(std::fabs(t.A_min), std::fabs(t.A_max));
  double aymax = std::fmax(std::fabs(t.Ay_min), std::fabs(t.Ay_max));
  double pxmax = std::fmax(std::fabs(g.px(0)), std::fabs(g.px(g.nx - 1)));
  double pymax = std::fmax(std::fabs(g.py(0)), std::fabs(g.py(g.ny - 1)));
  double phi = 2.0 * t.comp.cmax * t.dt * std::fmax(std::fmax(amax, aymax), std::fmax(pxmax, pymax));
  return phi <= kShearMaxAngle ? kFormShear : kFormVersine;
}

int taylor_order(double x_max, int precision, int form) {
  // Orders compiled into the midpoint kernels.
  static const int kCos64[] = {5, 8, 14};
  static const int kCos32[] = {3, 5, 9};
  static const int kTan64[] = {5, 7, 10};
  static const int kTan32[] = {2, 3, 5};
  const bool f32 = is_fp32(precision);
  const int* orders = form == kMidTangent ? (f32 ? kTan32 : kTan64) : (f32 ? kCos32 : kCos64);
  double tol = f32 ? 0x1p-27 : 0x1p-56;
  for (int q = 0; q < 3; ++q) {
    int J = orders[q];
    if (form == kMidTangent) {
      // a_n > 0 and a_{n+1} / a_n < 4 / pi^2, so the omitted terms sum to at most
      // a_{J+1} x^J / (1 - 4 x / pi^2), relative to tan(x)/x >= 1
      double r = 4.0 * x_max / (kPi * kPi);
      if (r < 1.0 && tan_series_coef(J + 1) * std::pow(x_max, J) / (1.0 - r) <= tol) return J;
      continue;
    }
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

int midpoint_form(const FieldTables& t, int precision) {
  // every stage angle is at most theta = cmax dt E_max; a step of S stages grows
  // the state by at most (1 / cos theta)^S
  const double theta = t.comp.cmax * t.dt * t.E_max;
  if (!(theta < 0.5 * kPi)) return kMidCosine;
  const double growth_log2 = (double)kRenormEvery * t.comp.stages * -std::log2(std::cos(theta));
  if (growth_log2 > 32.0) return kMidCosine;
  return taylor_order(theta * theta, precision, kMidTangent) > 0 ? kMidTangent : kMidCosine;
}

}  // namespace pdx
