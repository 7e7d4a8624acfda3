// Internal declarations shared by the host side of libpd and its HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <chrono>

#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "pd.h"

namespace pdx {

// Calls body(begin, end) on contiguous ranges that together cover [0, n): on up to
// 16 host threads when n is at least 2 * grain (the calling thread takes the first
// range), else once on the calling thread.  A range whose thread cannot be started
// runs on the calling thread.  body must not throw; the ranges write disjoint data.
template <typename F>
void parallel_ranges(long long n, long long grain, F&& body) {
  const unsigned hw = std::thread::hardware_concurrency();
  const long long nt = std::min<long long>(std::min<long long>(hw ? hw : 1, 16), n / std::max(grain, 1LL));
  if (nt <= 1) {
    if (n > 0) body(0LL, n);
    return;
  }
  const long long chunk = (n + nt - 1) / nt;
  std::vector<std::thread> pool;
  pool.reserve((size_t)nt);
  for (long long t = 1; t < nt; ++t) {
    const long long b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    try {
      pool.emplace_back([&body, b, e] { body(b, e); });
    } catch (...) {
      body(b, e);
    }
  }
  body(0LL, std::min(n, chunk));
  for (auto& th : pool) th.join();
}

// Stages of a step: 1 for the second-order schemes, 5 for Suzuki's fourth-order
// composition S(c1 dt) ... S(c5 dt), c = (p, p, 1 - 4p, p, p), p = 1/(4 - 4^(1/3));
// stage j samples the field at t_i + (k + sigma[j]) dt.
struct Composition {
  int stages = 1;
  double c[5] = {1, 0, 0, 0, 0};
  double sigma[5] = {0.5, 0, 0, 0, 0};
  double cmax = 1;  // max |c_j|
};
Composition composition_of(int scheme);
// FP32 state (PD_FP32 or PD_FP32_FAST)
inline bool is_fp32(int precision) { return precision == PD_FP32 || precision == PD_FP32_FAST; }
// PD_SCHEME_STRANG / STRANG4 -> PD_SCHEME_STRANG, MIDPOINT / MIDPOINT4 -> PD_SCHEME_MIDPOINT
inline int base_scheme(int scheme) { return scheme == PD_SCHEME_MIDPOINT || scheme == PD_SCHEME_MIDPOINT4 ? PD_SCHEME_MIDPOINT : PD_SCHEME_STRANG; }

// Host-side description of a field sampled for one solve.
struct FieldTables {
  double t_i = 0, t_f = 0, dt = 0;
  double A_in = 0, A_out = 0, A_min = 0, A_max = 0;      // x component
  double Ay_in = 0, Ay_out = 0, Ay_min = 0, Ay_max = 0;  // y component (0 when linear)
  bool elliptic = false;
  double E_max = 0;
  long long n_steps = 0;
  Composition comp;
  std::vector<double> A_mid;   // A_x at t_i + (k + sigma_j) dt, index k * stages + j
  std::vector<double> Ay_mid;  // A_y at the same times (empty when linear)
  pd_field spec{};             // the description (array pointers cleared), for A at other times
};

struct Grid {
  int nx = 0, ny = 0;
  double px_min = 0, px_max = 0, py_min = 0, py_max = 0;
  double dx = 0, dy = 0;
  // Node coordinates; the kernels evaluate the same expressions (no contraction).
  double px(int i) const { return px_min + (double)i * dx; }
  double py(int j) const { return py_min + (double)j * dy; }
  long long points() const { return (long long)nx * (long long)ny; }
};

// field.cpp
bool sample_field(const pd_field& f, long long n_steps, const Composition& comp, FieldTables* out,
                  std::string* err);
void field_extent(const Grid& g, FieldTables* t);  // E_max over the grid
long long count_masked(const Grid& g, const FieldTables& t);
// (A_x, A_y) at the step boundary t_i + k dt (k = 0: the start values, k = N: the
// end values; a table field between two steps: mean of the neighbouring samples).
void boundary_A(const FieldTables& t, long long k, double* ax, double* ay);

// Per-step rows of the field table, as the kernels read them (`stages` S).
//   Strang: per stage the two coefficients of the x rotation by 2 c_j dt A_x;
//           with a y component, then per stage the two coefficients of the y
//           rotation that follows it (its field part); in the solve's rotation
//           form, FP64 or rounded to FP32.  With a y component one more row
//           holds (in its first y slot) the opening half step's field part.
//   Midpoint: per stage c_j dt A_x, then (y component) per stage c_j dt A_y, FP64.
// All angles carry the valley sign.
size_t table_row_values(int scheme, int elliptic);
size_t table_row_bytes(int scheme, int precision, int elliptic);
long long table_rows(int scheme, int elliptic, long long n_steps);
void build_step_table(const FieldTables& t, int scheme, int precision, int form, double vsign,
                      std::vector<unsigned char>* rows);
// Rotation form of a Strang solve: shears when every rotation angle is small enough.
int strang_form(const Grid& g, const FieldTables& t);
// Phases of the per-point rotation coefficients of the FP32 Strang forms.  A
// coefficient rounded to FP32 changes the rotation angle (and its orthogonality)
// by a relative error of order 2^-24 that is the same at every step, so over a solve
// it acts as a constant perturbation of that point's Hamiltonian: the error in n
// grows with the total rotation angle 2 |p| (t_f - t_i), whatever N.  Each coefficient
// is therefore stored as kDitherFP32 FP32 values, each its lower or upper FP32
// neighbour, whose mean is the exact value to within 1/(2 kDitherFP32) of an ulp; step
// k uses value k mod kDitherFP32.  The per-step error then averages out over each
// cycle instead of adding up.  FP64 coefficients have one phase.
constexpr int kDitherFP32 = 4;
inline int coefficient_phases(int precision) { return is_fp32(precision) ? kDitherFP32 : 1; }

// Per-point rotation coefficients of a Strang solve, which depend on one grid
// coordinate each: per column i the x rotations by 2 c dt px_i for each distinct
// stage coefficient (1 pair, or 2 for the fourth-order composition), per row j
// the y rotations that follow the stages (1 or 2 pairs) and the opening / closing
// half step (1 pair), in the solve's form and precision, appended to `bytes`
// (each block 256-byte aligned).  Every pair except the half step is stored once
// per coefficient phase, phase-minor: pair q of phase h at index q * phases + h.
// Returns the byte offsets of the two blocks.
void build_point_coefficients(const Grid& g, const FieldTables& t, int scheme, int precision, int form, double vsign,
                              std::vector<unsigned char>* bytes, size_t* col_offset, size_t* row_offset);
size_t point_coefficient_pairs_x(int scheme, int precision);  // per column, phases included
size_t point_coefficient_pairs_y(int scheme, int precision);  // per row, phases and the half step included
// Coefficients (a, s) of the rotation by phi = 2 * half in a rotation form.
void rotation_coefficients(double half, int form, double* a, double* s);

// Strang rotation forms: three shears (tan(phi/2), sin phi) or versine (cos phi - 1, sin phi).
constexpr int kFormShear = 0;
constexpr int kFormVersine = 1;

// Midpoint step forms.  The step is U = cos(theta) I - i sin(theta) sigma.P / E with
// theta = c dt E (Sec. III, Eq. (13)).
//   Tangent: U / cos(theta) = I - i tan(theta) sigma.P / E, one series in x = theta^2;
//            the state then grows by 1 / cos(theta) per stage and is renormalised.
//   Cosine:  U itself, with the series of cos - 1 and sin(x)/x.
constexpr int kMidTangent = 0;
constexpr int kMidCosine = 1;

// Steps between renormalisations of the state (the FP32 forms and the midpoint
// tangent form); counted in absolute steps, so a chunked solve renormalises at the
// same steps as a single launch.
constexpr long long kRenormEvery = 1024;

// Coefficients of tan(sqrt x) / sqrt x = sum_{n >= 1} a_n x^(n-1).  From
// tan' = 1 + tan^2: a_1 = 1 and (2n - 1) a_n = sum_{k=1}^{n-1} a_k a_{n-k}.
constexpr double tan_series_coef(int n) {
  double a[24] = {};
  a[1] = 1.0;
  for (int m = 2; m <= n; ++m) {
    double s = 0.0;
    for (int k = 1; k < m; ++k) s += a[k] * a[m - k];
    a[m] = s / (2 * m - 1);
  }
  return a[n];
}

// Midpoint form of a solve: tangent when the state's growth over kRenormEvery
// steps stays below 2^32 and a compiled series order reaches the precision's
// rounding; cosine otherwise.
int midpoint_form(const FieldTables& t, int precision);

// Smallest compiled series order of a midpoint form (terms of tan(x)/x, or of
// cos - 1 and of sin(x)/x, in x = (c dt E)^2) whose truncation stays below the
// precision's rounding for x <= x_max; -1 if none does.
int taylor_order(double x_max, int precision, int form);
// The shear form is used when every rotation angle of a solve is at most this (|tan(phi/2)| <= 1).
constexpr double kShearMaxAngle = 1.5707963267948966;

// Parameters of one propagation launch (passed by value to the kernels).
struct SolveParams {
  long long npts;
  long long first;   // first point (Strang) or lane (midpoint: lanes cover bands of rows column
                     // by column) of this launch: a grid of more than 2^31 lanes runs as
                     // several launches over consecutive ranges
  int nx;
  double px_min, dx, py_min, dy;
  double A_in, A_out, dt;
  double Ay_in, Ay_out;
  double vsign;      // +1: valley K+, -1: K- (H = -sigma.P)
  double hx[2];      // midpoint: vsign * c dt for the distinct stage coefficients
  long long n_steps, k_begin, k_end;
  const void* table;
  const void* col_coef;  // Strang: per column the (a, s) pairs of the x rotations by 2 c dt px
  const void* row_coef;  // Strang: per row the (a, s) pairs of the y rotations, then the half step
  void* state;       // chunk state, structure of arrays; nullptr if not used
  double* n_out;     // written by the launch that reaches n_steps
  int load_state;    // 1: resume from state; 0: start from v_in
  int store_state;   // 1: keep the state after k_end
  int stage;         // Strang table path: 0 scalar-unit loads, 1 LDS chunks
  int form;          // Strang: kFormShear or kFormVersine; midpoint: kMidTangent or kMidCosine
  long long chunk_steps;  // LDS chunk length in steps (power of two; divides 1024 in FP32)
};

// Projection of a stored state at step k on the positive-energy state of
// sigma.(p + A(t_k)) (pd_snapshot).
struct SnapshotParams {
  double Ax, Ay;        // A(t_k)
  double undo_a, undo_s;  // Strang with a y component: the inverse of the field part of
                          // the half step the stored state is ahead by
};

// One solve of a batched launch (device descriptor).
struct BatchSolve {
  SolveParams p;
  int precision;
  int form;
};

// One work item of a batched launch: the tile of block_threads * points_per_lane
// points of solve `solve` starting at point `base`.
struct BatchItem {
  int solve;
  int pad;
  long long base;
};

// One density reduction of a batched launch: rho = scale * sum n, tiles
// [tile_begin, tile_begin + ceil(npts / 2048)) of the batched tile launch.
struct DensityJob {
  const double* n;
  long long npts;
  long long tile_begin;
  double* partial;
  double* rho;
  double* rho_copy;  // optional second destination (nullptr: none)
  double scale;
};

// kernels.hip
hipError_t launch_propagate(int scheme, int precision, int points_per_lane, int block_threads, int taylor,
                            int elliptic, const SolveParams& p, hipStream_t stream);
hipError_t launch_snapshot(int scheme, int precision, int elliptic, const SolveParams& p, const SnapshotParams& q,
                           hipStream_t stream);
hipError_t launch_density(const double* n, long long npts, double scale, double* partial, double* rho,
                          hipStream_t stream);
// Largest grid the static scratch of pd_density_static serves, and the tile
// partials it holds for it (the density reduction sums tiles of 2048 points).
constexpr long long kStaticMaxPoints = 1LL << 28;
constexpr long long kStaticPartials = kStaticMaxPoints / 2048;
// Device address of the static scratch on `device` (kStaticPartials partials, then
// one sum), looked up on the first call for that device.
hipError_t static_scratch(int device, double** out);
hipError_t launch_batch(int points_per_lane, int block_threads, int grid_blocks, const BatchSolve* solves,
                        const BatchItem* items, int n_items, unsigned int* counter, hipStream_t stream);
hipError_t launch_batch_density(const DensityJob* jobs, int n_jobs, long long total_tiles, hipStream_t stream);
int batch_blocks_per_cu(int points_per_lane, int block_threads);
long long density_partials(long long npts);
size_t state_values_per_point(int scheme);

}  // namespace pdx

// The solver handle behind pd_grid (pd_api.cpp; also used by the batch code).
struct pd_grid_s {
  pdx::Grid grid;
  int precision = PD_FP64;
  int scheme = PD_SCHEME_STRANG;
  int points_per_lane = 2;
  int block_threads = 256;
  int table_stage = 2;  // 1: LDS chunks, 2: scalar-unit reads
  int chunk_steps = 512;
  long long version = 0;  // bumped whenever the field or the launch shape changes

  bool field_set = false;
  pdx::FieldTables field;
  long long n_masked = 0;
  long long steps_done = 0;
  int taylor = 0;
  int form = pdx::kFormShear;  // Strang rotation form of the current field
  int valley = PD_VALLEYS_BOTH;
  double vsign() const { return valley == PD_VALLEY_KMINUS ? -1.0 : 1.0; }

  int device = -1;
  void* d_table = nullptr;
  size_t table_bytes = 0;     // step rows, then (Strang) the column and row coefficients
  size_t table_capacity = 0;  // bytes allocated at d_table: kept when a later table is smaller
  size_t col_offset = 0, row_offset = 0;
  double* d_n = nullptr;
  double* d_partial = nullptr;
  double* d_rho = nullptr;
  void* d_state_own = nullptr;
  void* d_state_bound = nullptr;
  size_t state_bound_bytes = 0;
  // Completion of the last work the library enqueued on this handle's buffers
  // (propagation, projection, copies, batch epochs); a new field waits for it
  // rather than for the whole device.  Work enqueued under stream capture has no
  // such event: then the whole device is waited for.
  hipEvent_t last_use = nullptr;
  bool wait_device = false;

  size_t device_bytes() const {
    size_t b = table_capacity;
    if (d_n) b += (size_t)grid.points() * sizeof(double);
    if (d_partial) b += (size_t)pdx::density_partials(grid.points()) * sizeof(double) + sizeof(double);
    if (d_state_own) b += state_bytes();
    return b;
  }
  size_t state_bytes() const {
    size_t v = pdx::is_fp32(precision) ? sizeof(float) : sizeof(double);
    return (size_t)grid.points() * pdx::state_values_per_point(scheme) * v;
  }
  double density_scale() const;
  // Launch parameters of steps [k_begin, k_end); `state` is the chunk state buffer (may be null).
  pdx::SolveParams solve_params(long long k_begin, long long k_end, void* state) const;
};

namespace pdx {
// Makes a device current for the lifetime of the scope.
struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (dev < 0) return;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Error reporting shared by the C entry points (pd_api.cpp).
pd_status set_error(pd_status s, const char* fmt, ...);
pd_status hip_error(hipError_t e, const char* what);

// Test hook for the error paths: PD_FAULT (read at the first query) or pd_set_fault
// arms one fault, "alloc@K" or "launch@K": the K-th device allocation, or the K-th
// launch sequence (pd_propagate, a batch run or epoch), counted from the arming, fails
// once, before anything is enqueued.
enum FaultKind { kFaultAlloc = 0, kFaultLaunch = 1 };
bool fault_now(FaultKind kind);
// hipMalloc, or hipErrorOutOfMemory when an allocation fault is due
hipError_t device_malloc(void** p, size_t bytes);

// PD_TRACE (set and not "0"): every traced entry point writes one line to stderr as it
// returns, "pd_trace <name> <ms> ms", with the host time spent in the call (launches
// are asynchronous: the time a call waits for the device is included only where it
// waits).  Read once per process.
bool trace_on();
void trace_line(const char* name, double ms);
struct TraceCall {
  const char* name;
  bool on;
  std::chrono::steady_clock::time_point t0;
  explicit TraceCall(const char* n) : name(n), on(trace_on()) {
    if (on) t0 = std::chrono::steady_clock::now();
  }
  ~TraceCall() {
    if (on) trace_line(name, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  }
};
// The chunk state buffer of a handle, allocated on first use.
pd_status grid_state_buffer(pd_grid g, void** out);
// Note work just enqueued on `stream` that uses g's device buffers (the handle's
// device must be current).
pd_status mark_use(pd_grid g, hipStream_t stream);
}  // namespace pdx
