// C ABI of libpd (declared and documented in include/pd.h).
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pd.h"
#include "pd_internal.h"

using namespace pdx;

namespace {
thread_local std::string g_error;
constexpr double kPi = 3.14159265358979323846;
std::atomic<long long> g_versions{0};
// Versions come from one process-wide counter, so a handle created at the
// address of a destroyed one never matches the old handle's version.
long long next_version() { return ++g_versions; }

// The armed fault: its kind (-1: none) and how many events of that kind are left
// until it fires.
std::mutex g_fault_mu;
int g_fault_kind = -1;
long long g_fault_left = 0;
bool g_fault_read = false;

// "alloc@K" / "launch@K" (K >= 1), or empty / NULL for none; false if malformed.
bool parse_fault(const char* spec, int* kind, long long* left) {
  *kind = -1;
  *left = 0;
  if (!spec || !*spec) return true;
  const char* at = std::strchr(spec, '@');
  if (!at) return false;
  const std::string what(spec, (size_t)(at - spec));
  char* end = nullptr;
  const long long k = std::strtoll(at + 1, &end, 10);
  if (!end || end == at + 1 || *end != '\0' || k < 1) return false;
  if (what == "alloc")
    *kind = pdx::kFaultAlloc;
  else if (what == "launch")
    *kind = pdx::kFaultLaunch;
  else
    return false;
  *left = k;
  return true;
}
}  // namespace

namespace pdx {

pd_status set_error(pd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

bool fault_now(FaultKind kind) {
  std::lock_guard<std::mutex> lock(g_fault_mu);
  if (!g_fault_read) {
    g_fault_read = true;
    if (!parse_fault(std::getenv("PD_FAULT"), &g_fault_kind, &g_fault_left)) g_fault_kind = -1;
  }
  if (g_fault_kind != (int)kind) return false;
  if (--g_fault_left > 0) return false;
  g_fault_kind = -1;
  return true;
}

bool trace_on() {
  static const bool on = [] {
    const char* v = std::getenv("PD_TRACE");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void trace_line(const char* name, double ms) { std::fprintf(stderr, "pd_trace %s %.3f ms\n", name, ms); }

hipError_t device_malloc(void** p, size_t bytes) {
  if (fault_now(kFaultAlloc)) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

pd_status hip_error(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return set_error(PD_ERR_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_error(PD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

pd_status mark_use(pd_grid g, hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cs);
  if (e != hipSuccess) return hip_error(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) {
    g->wait_device = true;
    return PD_OK;
  }
  if (!g->last_use && (e = hipEventCreateWithFlags(&g->last_use, hipEventDisableTiming)) != hipSuccess)
    return hip_error(e, "hipEventCreate");
  if ((e = hipEventRecord(g->last_use, stream)) != hipSuccess) return hip_error(e, "hipEventRecord");
  return PD_OK;
}

pd_status grid_state_buffer(pd_grid g, void** out) {
  if (g->d_state_bound) {
    *out = g->d_state_bound;
    return PD_OK;
  }
  if (!g->d_state_own) {
    hipError_t e = device_malloc(&g->d_state_own, g->state_bytes());
    if (e != hipSuccess) return hip_error(e, "hipMalloc(state)");
  }
  *out = g->d_state_own;
  return PD_OK;
}

}  // namespace pdx

// rho = g dx dy / (2 pi)^2 sum n: g = 4 (2 spins x 2 valleys, the K- valley giving
// the same n as K+) unless one valley is solved explicitly (g = 2, spins only).
double pd_grid_s::density_scale() const {
  const double g = valley == PD_VALLEYS_BOTH ? 4.0 : 2.0;
  return g * grid.dx * grid.dy / (4.0 * kPi * kPi);
}

SolveParams pd_grid_s::solve_params(long long k_begin, long long k_end, void* state) const {
  SolveParams p{};
  p.npts = grid.points();
  p.nx = grid.nx;
  p.px_min = grid.px_min;
  p.dx = grid.dx;
  p.py_min = grid.py_min;
  p.dy = grid.dy;
  p.A_in = field.A_in;
  p.A_out = field.A_out;
  p.dt = field.dt;
  p.Ay_in = field.Ay_in;
  p.Ay_out = field.Ay_out;
  p.vsign = vsign();
  // midpoint: per-point phase multipliers vsign c dt of the distinct stage coefficients
  p.hx[0] = vsign() * (field.comp.c[0] * field.dt);
  p.hx[1] = vsign() * (field.comp.c[2] * field.dt);
  p.n_steps = field.n_steps;
  p.k_begin = k_begin;
  p.k_end = k_end;
  p.table = d_table;
  p.col_coef = static_cast<const unsigned char*>(d_table) + col_offset;
  p.row_coef = static_cast<const unsigned char*>(d_table) + row_offset;
  p.n_out = d_n;
  p.load_state = k_begin > 0;
  p.store_state = k_end < field.n_steps;
  p.state = (p.load_state || p.store_state) ? state : nullptr;
  // LDS staging holds chunk_steps rows in at most 64 KiB; larger rows use the scalar path
  const size_t row_bytes = table_row_bytes(scheme, precision, field.elliptic ? 1 : 0);
  p.stage = (table_stage == 1 && (size_t)chunk_steps * row_bytes <= 65536) ? 1 : 0;
  p.chunk_steps = chunk_steps;
  p.form = form;
  return p;
}

namespace {

pd_status fail(pd_status s, const char* msg) { return set_error(s, "%s", msg); }
template <typename... A>
pd_status fail(pd_status s, const char* fmt, A... a) {
  return set_error(s, fmt, a...);
}
pd_status ok() { return PD_OK; }
pd_status hip_fail(hipError_t e, const char* what) { return hip_error(e, what); }

// Wait for the handle's earlier work: its completion event, or the whole device if
// that work was enqueued under stream capture (no event could be recorded then).
pd_status wait_own_work(pd_grid g) {
  hipError_t e = hipSuccess;
  if (g->wait_device) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    g->wait_device = false;
  } else if (g->last_use) {
    e = hipEventSynchronize(g->last_use);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  return PD_OK;
}

void release(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T>
void release(T*& p) {
  void* v = p;
  release(v);
  p = nullptr;
}

pd_status prepare_field(pd_grid g, const pd_field* f, long long n_steps, FieldTables* t, long long* masked,
                        int* taylor, int* form) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!f) return fail(PD_ERR_INVALID, "null field");
  std::string err;
  if (!sample_field(*f, n_steps, composition_of(g->scheme), t, &err)) return fail(PD_ERR_INVALID, "%s", err.c_str());
  field_extent(g->grid, t);
  // Step-size condition of Sec. III (last paragraph): dt <= pi / max E.
  if (t->dt * t->E_max > kPi)
    return fail(PD_ERR_INVALID, "dt * E_max = %.6g exceeds pi (dt = %.6g, E_max = %.6g): use more steps",
                t->dt * t->E_max, t->dt, t->E_max);
  *masked = count_masked(g->grid, *t);
  *taylor = 0;
  if (base_scheme(g->scheme) == PD_SCHEME_MIDPOINT) {
    double xm = t->comp.cmax * t->dt * t->E_max;  // largest stage phase
    *form = midpoint_form(*t, g->precision);
    *taylor = taylor_order(xm * xm, g->precision, *form);
    if (*taylor < 0) return fail(PD_ERR_UNSUPPORTED, "midpoint step too large for the compiled Taylor orders");
  } else {
    *form = strang_form(g->grid, *t);
  }
  return ok();
}

void fill_info(pd_grid g, const FieldTables& t, long long masked, long long steps_done, pd_info* out) {
  std::memset(out, 0, sizeof *out);
  out->n_points = g->grid.points();
  out->n_steps = t.n_steps;
  out->steps_done = steps_done;
  out->n_masked = masked;
  out->dt = t.dt;
  out->t_i = t.t_i;
  out->t_f = t.t_f;
  out->A_in = t.A_in;
  out->A_out = t.A_out;
  out->E_max = t.E_max;
  out->A_min = t.A_min;
  out->A_max = t.A_max;
  out->precision = g->precision;
  out->scheme = g->scheme;
  out->points_per_lane = g->points_per_lane;
  out->block_threads = g->block_threads;
  out->table_stage = g->table_stage;
  out->chunk_steps = g->chunk_steps;
  out->rotation_form = t.n_steps > 0 ? strang_form(g->grid, t) : kFormShear;
  if (base_scheme(g->scheme) == PD_SCHEME_MIDPOINT && t.n_steps > 0) {
    double xm = t.comp.cmax * t.dt * t.E_max;
    out->rotation_form = midpoint_form(t, g->precision);
    out->taylor_order = taylor_order(xm * xm, g->precision, out->rotation_form);
  }
  out->device_bytes = g->device_bytes();
  if (t.n_steps > 0) out->solve_bytes = pd_solve_bytes(g, t.n_steps);
  out->valley = g->valley;
  out->stages = composition_of(g->scheme).stages;
  out->elliptic = t.elliptic ? 1 : 0;
  out->Ay_in = t.Ay_in;
  out->Ay_out = t.Ay_out;
}

}  // namespace

extern "C" {

const char* pd_last_error(void) { return g_error.c_str(); }

const char* pd_version(void) { return "libpd 0.1.0 gfx950"; }

pd_status pd_set_fault(const char* spec) {
  int kind = -1;
  long long left = 0;
  if (!parse_fault(spec, &kind, &left))
    return fail(PD_ERR_INVALID, "fault spec must be \"alloc@K\" or \"launch@K\" with K >= 1, got \"%s\"", spec);
  std::lock_guard<std::mutex> lock(g_fault_mu);
  g_fault_read = true;  // the call replaces whatever PD_FAULT armed
  g_fault_kind = kind;
  g_fault_left = left;
  return ok();
}

pd_status pd_create_grid(int nx, int ny, double px_min, double px_max, double py_min, double py_max, int precision,
                         int scheme, pd_grid* out) {
  if (!out) return fail(PD_ERR_INVALID, "null output handle pointer");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536) return fail(PD_ERR_INVALID, "nx, ny must be in [1, 65536]");
  if (!std::isfinite(px_min) || !std::isfinite(px_max) || !std::isfinite(py_min) || !std::isfinite(py_max) ||
      !(px_max > px_min) || !(py_max > py_min))
    return fail(PD_ERR_INVALID, "momentum ranges must be finite with max > min");
  if (precision != PD_FP64 && precision != PD_FP32 && precision != PD_FP32_FAST)
    return fail(PD_ERR_INVALID, "unknown precision %d", precision);
  if (scheme != PD_SCHEME_STRANG && scheme != PD_SCHEME_MIDPOINT && scheme != PD_SCHEME_STRANG4 &&
      scheme != PD_SCHEME_MIDPOINT4)
    return fail(PD_ERR_INVALID, "unknown scheme %d", scheme);
  pd_grid g = new (std::nothrow) pd_grid_s();
  if (!g) return fail(PD_ERR_NOMEM, "host allocation failed");
  g->grid.nx = nx;
  g->grid.ny = ny;
  g->grid.px_min = px_min;
  g->grid.px_max = px_max;
  g->grid.py_min = py_min;
  g->grid.py_max = py_max;
  g->grid.dx = (px_max - px_min) / (double)nx;
  g->grid.dy = (py_max - py_min) / (double)ny;
  g->precision = precision;
  g->scheme = scheme;
  // Default launch shape (fastest measured on MI355X for the 2048^2 x 80000
  // workload): field rows read by the scalar unit, 256-thread blocks; Strang: one
  // point per lane in FP32 and four in FP64; midpoint: four, which share their
  // column's FP64 phase.
  g->points_per_lane = (is_fp32(precision) && base_scheme(scheme) == PD_SCHEME_STRANG) ? 1 : 4;
  g->block_threads = 256;
  g->table_stage = 2;
  g->chunk_steps = 512;
  *out = g;
  return ok();
}

pd_status pd_check_field(pd_grid g, const pd_field* f, long long n_steps, pd_info* out) {
  FieldTables t;
  long long masked = 0;
  int taylor = 0, form = 0;
  pd_status s = prepare_field(g, f, n_steps, &t, &masked, &taylor, &form);
  if (out && g && (s == PD_OK || !t.A_mid.empty())) fill_info(g, t, masked, 0, out);
  return s;
}

pd_status pd_sample_field(const pd_field* f, long long n_steps, double* A_mid, double* t_i, double* t_f,
                          double* A_in, double* A_out) {
  if (!f) return fail(PD_ERR_INVALID, "null field");
  FieldTables t;
  std::string err;
  if (!sample_field(*f, n_steps, composition_of(PD_SCHEME_STRANG), &t, &err))
    return fail(PD_ERR_INVALID, "%s", err.c_str());
  if (A_mid) std::memcpy(A_mid, t.A_mid.data(), (size_t)n_steps * sizeof(double));
  if (t_i) *t_i = t.t_i;
  if (t_f) *t_f = t.t_f;
  if (A_in) *A_in = t.A_in;
  if (A_out) *A_out = t.A_out;
  return ok();
}

pd_status pd_sample_field_xy(const pd_field* f, long long n_steps, int scheme, double* Ax_mid, double* Ay_mid,
                             double* ends) {
  if (!f) return fail(PD_ERR_INVALID, "null field");
  if (scheme < PD_SCHEME_STRANG || scheme > PD_SCHEME_MIDPOINT4) return fail(PD_ERR_INVALID, "unknown scheme %d", scheme);
  FieldTables t;
  std::string err;
  if (!sample_field(*f, n_steps, composition_of(scheme), &t, &err)) return fail(PD_ERR_INVALID, "%s", err.c_str());
  const size_t n = t.A_mid.size();
  if (Ax_mid) std::memcpy(Ax_mid, t.A_mid.data(), n * sizeof(double));
  if (Ay_mid) {
    if (t.elliptic)
      std::memcpy(Ay_mid, t.Ay_mid.data(), n * sizeof(double));
    else
      std::memset(Ay_mid, 0, n * sizeof(double));
  }
  if (ends) {
    ends[0] = t.t_i;
    ends[1] = t.t_f;
    ends[2] = t.A_in;
    ends[3] = t.A_out;
    ends[4] = t.Ay_in;
    ends[5] = t.Ay_out;
  }
  return ok();
}

pd_status pd_set_valley(pd_grid g, int valley) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (valley != PD_VALLEYS_BOTH && valley != PD_VALLEY_KPLUS && valley != PD_VALLEY_KMINUS)
    return fail(PD_ERR_INVALID, "unknown valley %d", valley);
  if (g->field_set) return fail(PD_ERR_STATE, "pd_set_valley after pd_set_field");
  g->valley = valley;
  return ok();
}

pd_status pd_set_field(pd_grid g, const pd_field* f, long long n_steps) {
  TraceCall trace("pd_set_field");
  FieldTables t;
  long long masked = 0;
  int taylor = 0, form = 0;
  pd_status s = prepare_field(g, f, n_steps, &t, &masked, &taylor, &form);
  if (s != PD_OK) return s;
  std::vector<unsigned char> rows;
  build_step_table(t, g->scheme, g->precision, form, g->vsign(), &rows);
  size_t col_offset = 0, row_offset = 0;
  if (base_scheme(g->scheme) == PD_SCHEME_STRANG)
    build_point_coefficients(g->grid, t, g->scheme, g->precision, form, g->vsign(), &rows, &col_offset, &row_offset);

  if (g->device < 0) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    g->device = dev;
  }
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  hipError_t e;
  // Work of an earlier solve on this handle may still read the table or the state.
  if ((s = wait_own_work(g)) != PD_OK) return s;
  g->field_set = false;
  if (rows.size() > g->table_capacity) {
    release(g->d_table);
    g->table_bytes = g->table_capacity = 0;
    e = device_malloc(&g->d_table, rows.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(field table)");
    g->table_capacity = rows.size();
  }
  g->table_bytes = rows.size();
  e = hipMemcpy(g->d_table, rows.data(), rows.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(field table)");
  long long npts = g->grid.points();
  if (!g->d_n) {
    e = device_malloc(reinterpret_cast<void**>(&g->d_n), (size_t)npts * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(n)");
  }
  if (!g->d_partial) {
    e = device_malloc(reinterpret_cast<void**>(&g->d_partial), (size_t)density_partials(npts) * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(partials)");
    e = device_malloc(reinterpret_cast<void**>(&g->d_rho), sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(rho)");
  }
  g->field = std::move(t);
  g->n_masked = masked;
  g->taylor = taylor;
  g->form = form;
  g->col_offset = col_offset;
  g->row_offset = row_offset;
  g->steps_done = 0;
  g->field_set = true;
  g->version = next_version();
  return ok();
}

size_t pd_state_bytes(pd_grid g) { return g ? g->state_bytes() : 0; }

size_t pd_solve_bytes(pd_grid g, long long n_steps) {
  if (!g || n_steps < 1) return 0;
  auto align = [](size_t n) { return (n + 255) / 256 * 256; };
  size_t table = (size_t)table_rows(g->scheme, 0, n_steps) * table_row_bytes(g->scheme, g->precision, 0);
  if (base_scheme(g->scheme) == PD_SCHEME_STRANG) {
    const size_t v = is_fp32(g->precision) ? sizeof(float) : sizeof(double);
    size_t col = align(table);
    size_t row = align(col + 2 * point_coefficient_pairs_x(g->scheme, g->precision) * v * (size_t)g->grid.nx);
    table = align(row + 2 * point_coefficient_pairs_y(g->scheme, g->precision) * v * (size_t)g->grid.ny);
  }
  const size_t npts = (size_t)g->grid.points();
  return table + npts * sizeof(double) + (size_t)density_partials((long long)npts) * sizeof(double) +
         sizeof(double) + g->state_bytes();
}

pd_status pd_bind_state(pd_grid g, void* dev_ptr, size_t bytes) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (dev_ptr) {
    if (bytes < g->state_bytes())
      return fail(PD_ERR_INVALID, "state buffer of %zu bytes is smaller than the %zu needed", bytes,
                  g->state_bytes());
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return fail(PD_ERR_INVALID, "state buffer not 256-byte aligned");
  }
  if (g->field_set && g->steps_done > 0 && g->steps_done < g->field.n_steps)
    return fail(PD_ERR_STATE, "cannot rebind the state in the middle of a solve");
  g->d_state_bound = dev_ptr;
  g->state_bound_bytes = dev_ptr ? bytes : 0;
  return ok();
}

pd_status pd_resume(pd_grid g, long long steps_done) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!g->field_set) return fail(PD_ERR_STATE, "pd_resume before pd_set_field");
  if (!g->d_state_bound) return fail(PD_ERR_STATE, "pd_resume needs a state buffer bound with pd_bind_state");
  if (steps_done < 1 || steps_done >= g->field.n_steps)
    return fail(PD_ERR_INVALID, "steps_done = %lld outside 1 .. N - 1 (N = %lld)", steps_done, g->field.n_steps);
  g->steps_done = steps_done;
  return ok();
}

pd_status pd_save_state(pd_grid g, void* host, size_t bytes, long long* steps_done, void* stream) {
  TraceCall trace("pd_save_state");
  if (!g || !host) return fail(PD_ERR_INVALID, "null argument");
  if (!g->field_set || g->steps_done == 0 || g->steps_done == g->field.n_steps)
    return fail(PD_ERR_STATE, "pd_save_state: no solve in progress (%lld of %lld steps done)", g->steps_done,
                g->field_set ? g->field.n_steps : 0LL);
  if (bytes < g->state_bytes())
    return fail(PD_ERR_INVALID, "host buffer of %zu bytes is smaller than the %zu-byte state", bytes, g->state_bytes());
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  // 0 < steps done < N: the last propagation wrote the state buffer in use
  void* st = g->d_state_bound ? g->d_state_bound : g->d_state_own;
  if (!st) return fail(PD_ERR_STATE, "pd_save_state: the handle holds no state");
  pd_status s = wait_own_work(g);
  if (s != PD_OK) return s;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(host, st, g->state_bytes(), hipMemcpyDeviceToHost, hs);
  if (e != hipSuccess) return hip_fail(e, "copy of the state");
  if ((e = hipStreamSynchronize(hs)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (steps_done) *steps_done = g->steps_done;
  return ok();
}

pd_status pd_load_state(pd_grid g, const void* host, size_t bytes, long long steps_done, void* stream) {
  TraceCall trace("pd_load_state");
  if (!g || !host) return fail(PD_ERR_INVALID, "null argument");
  if (!g->field_set) return fail(PD_ERR_STATE, "pd_load_state before pd_set_field");
  if (steps_done < 1 || steps_done >= g->field.n_steps)
    return fail(PD_ERR_INVALID, "steps_done = %lld outside 1 .. N - 1 (N = %lld)", steps_done, g->field.n_steps);
  if (bytes != g->state_bytes())
    return fail(PD_ERR_INVALID, "state of %zu bytes, the handle's is %zu (another grid, precision or scheme?)", bytes,
                g->state_bytes());
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  // earlier work on the handle may still read or write the state buffer
  pd_status s = wait_own_work(g);
  if (s != PD_OK) return s;
  void* st = nullptr;
  if ((s = grid_state_buffer(g, &st)) != PD_OK) return s;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(st, host, bytes, hipMemcpyHostToDevice, hs);
  if (e != hipSuccess) return hip_fail(e, "copy of the state");
  if ((e = hipStreamSynchronize(hs)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  g->steps_done = steps_done;
  return ok();
}

pd_status pd_set_launch(pd_grid g, int points_per_lane, int block_threads, int table_stage, int chunk_steps) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (points_per_lane != 0 && points_per_lane != 1 && points_per_lane != 2 && points_per_lane != 4)
    return fail(PD_ERR_INVALID, "points_per_lane must be 1, 2 or 4");
  if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256)
    return fail(PD_ERR_INVALID, "block_threads must be 64, 128 or 256");
  if (table_stage != 0 && table_stage != 1 && table_stage != 2)
    return fail(PD_ERR_INVALID, "table_stage must be 1 (LDS) or 2 (scalar)");
  if (chunk_steps != 0) {
    int max_chunk = is_fp32(g->precision) ? 1024 : 4096;
    if (chunk_steps < 64 || chunk_steps > max_chunk || (chunk_steps & (chunk_steps - 1)) != 0)
      return fail(PD_ERR_INVALID, "chunk_steps must be a power of two in [64, %d]", max_chunk);
  }
  if (points_per_lane) g->points_per_lane = points_per_lane;
  if (block_threads) g->block_threads = block_threads;
  if (table_stage) g->table_stage = table_stage;
  if (chunk_steps) g->chunk_steps = chunk_steps;
  g->version = next_version();
  return ok();
}

pd_status pd_rewind(pd_grid g) {
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!g->field_set) return fail(PD_ERR_STATE, "pd_rewind before pd_set_field");
  g->steps_done = 0;
  return ok();
}

pd_status pd_propagate(pd_grid g, long long max_steps, void* stream) {
  TraceCall trace("pd_propagate");
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!g->field_set) return fail(PD_ERR_STATE, "pd_propagate before pd_set_field");
  const long long N = g->field.n_steps;
  long long left = N - g->steps_done;
  if (left == 0) return fail(PD_ERR_STATE, "solve already complete (%lld steps)", N);
  long long m = (max_steps < 0 || max_steps > left) ? left : max_steps;
  if (m == 0) return ok();
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);

  const long long k_begin = g->steps_done, k_end = g->steps_done + m;
  void* st = nullptr;
  if (k_begin > 0 || k_end < N) {
    pd_status s = grid_state_buffer(g, &st);
    if (s != PD_OK) return s;
  }
  const SolveParams p = g->solve_params(k_begin, k_end, st);
  if (fault_now(kFaultLaunch)) return fail(PD_ERR_DEVICE, "injected launch fault (PD_FAULT)");
  hipError_t e = launch_propagate(g->scheme, g->precision, g->points_per_lane, g->block_threads, g->taylor,
                                  g->field.elliptic ? 1 : 0, p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "propagate launch");
  g->steps_done = p.k_end;
  return mark_use(g, static_cast<hipStream_t>(stream));
}

namespace {

// Reduce the handle's n buffer into rho and copy the results out (pd_density, pd_snapshot).
pd_status reduce_and_copy(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, hipStream_t s) {
  const long long npts = g->grid.points();
  hipError_t e = launch_density(g->d_n, npts, g->density_scale(), g->d_partial, g->d_rho, s);
  if (e != hipSuccess) return hip_fail(e, "density launch");
  bool wait = false;
  if (n_out) {
    e = hipMemcpyAsync(n_out, g->d_n, (size_t)npts * sizeof(double),
                       n_out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy of n(p)");
    wait = !n_out_on_device;
  }
  pd_status m = mark_use(g, s);
  if (m != PD_OK) return m;
  double rho = 0.0;
  if (rho_out) {
    e = hipMemcpyAsync(&rho, g->d_rho, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy of rho");
    wait = true;
  }
  if (wait) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  if (rho_out) *rho_out = rho;
  return ok();
}

}  // namespace

pd_status pd_density(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream) {
  TraceCall trace("pd_density");
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!g->field_set || g->steps_done != g->field.n_steps)
    return fail(PD_ERR_STATE, "pd_density before the last step (%lld of %lld done)", g->steps_done,
                g->field_set ? g->field.n_steps : 0LL);
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  return reduce_and_copy(g, n_out, n_out_on_device, rho_out, static_cast<hipStream_t>(stream));
}

pd_status pd_density_static(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream) {
  TraceCall trace("pd_density_static");
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  const long long npts = g->grid.points();
  if (npts > kStaticMaxPoints)
    return fail(PD_ERR_INVALID, "pd_density_static: %lld points exceed the static scratch (at most %lld)", npts,
                kStaticMaxPoints);
  if (!g->field_set || g->steps_done != g->field.n_steps)
    return fail(PD_ERR_STATE, "pd_density_static before the last step (%lld of %lld done)", g->steps_done,
                g->field_set ? g->field.n_steps : 0LL);
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  double* sc = nullptr;
  hipError_t e = static_scratch(g->device, &sc);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // partials in sc[0 .. tiles), the sum in sc[kStaticPartials]; every partial is
  // written before it is read, so nothing needs clearing
  e = launch_density(g->d_n, npts, g->density_scale(), sc, sc + kStaticPartials, s);
  if (e != hipSuccess) return hip_fail(e, "density launch");
  bool wait = false;
  if (n_out) {
    e = hipMemcpyAsync(n_out, g->d_n, (size_t)npts * sizeof(double),
                       n_out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy of n(p)");
    wait = !n_out_on_device;
  }
  // the handle's completion event exists once a propagation was enqueued outside
  // capture; otherwise a later pd_set_field waits for the device (creating an event
  // here could allocate)
  if (g->last_use) {
    pd_status m = mark_use(g, s);
    if (m != PD_OK) return m;
  } else {
    g->wait_device = true;
  }
  double rho = 0.0;
  if (rho_out) {
    e = hipMemcpyAsync(&rho, sc + kStaticPartials, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy of rho");
    wait = true;
  }
  if (wait) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  if (rho_out) *rho_out = rho;
  return ok();
}

pd_status pd_snapshot(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream) {
  TraceCall trace("pd_snapshot");
  if (!g) return fail(PD_ERR_INVALID, "null handle");
  if (!g->field_set) return fail(PD_ERR_STATE, "pd_snapshot before pd_set_field");
  DeviceScope scope(g->device);
  if (!scope.ok) return fail(PD_ERR_DEVICE, "cannot select device %d", g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long k = g->steps_done, N = g->field.n_steps;
  if (k < N) {
    // k = 0: v_in is rebuilt in the kernel; 0 < k < N: the state buffer holds step k
    void* st = nullptr;
    if (k > 0) {
      pd_status r = grid_state_buffer(g, &st);
      if (r != PD_OK) return r;
    }
    SolveParams p = g->solve_params(k, k, st);
    p.load_state = k > 0;
    SnapshotParams q{};
    boundary_A(g->field, k, &q.Ax, &q.Ay);
    if (base_scheme(g->scheme) == PD_SCHEME_STRANG && g->field.elliptic && k > 0) {
      // the stored Bloch vector is ahead by the opening half step of step k; its
      // field part has half angle vsign c_1 dt A_y(k, stage 0) / 2
      const int S = g->field.comp.stages;
      double half = g->vsign() * 0.5 * g->field.dt * (g->field.comp.c[0] * g->field.Ay_mid[(size_t)(k * S)]);
      rotation_coefficients(-half, g->form, &q.undo_a, &q.undo_s);
    }
    hipError_t e = launch_snapshot(g->scheme, g->precision, g->field.elliptic ? 1 : 0, p, q, s);
    if (e != hipSuccess) return hip_fail(e, "snapshot launch");
  }
  return reduce_and_copy(g, n_out, n_out_on_device, rho_out, s);
}

pd_status pd_get_info(pd_grid g, pd_info* out) {
  if (!g || !out) return fail(PD_ERR_INVALID, "null argument");
  if (!g->field_set) {
    FieldTables empty;
    fill_info(g, empty, 0, 0, out);
    return ok();
  }
  fill_info(g, g->field, g->n_masked, g->steps_done, out);
  return ok();
}

void pd_destroy_grid(pd_grid g) {
  if (!g) return;
  if (g->device >= 0) {
    DeviceScope scope(g->device);
    release(g->d_table);
    release(g->d_n);
    release(g->d_partial);
    release(g->d_rho);
    release(g->d_state_own);
    if (g->last_use) (void)hipEventDestroy(g->last_use);
  }
  delete g;
}

}  // extern "C"
