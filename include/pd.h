/*
 * pd.h -- C ABI of libpd, the gfx950 (MI355X) solver for electron-hole pair
 * production in graphene by split-operator propagation of the massless 2D
 * Dirac equation in momentum space (Fillion-Gourdeau et al., arXiv:1607.03062).
 *
 * What a solve computes (Sec. II, Eq. (1); Sec. III, Eqs. (9)-(13)):
 *   for every point p of a uniform momentum grid, the negative-energy state
 *   v_in(p) of sigma.(p + A(t_i)) is advanced by N short-time steps of the
 *   equation i d/dt psi = sigma.(p + A(t)) psi (Sec. II, Eq. (2), valley K+
 *   unless pd_set_valley chooses K-, where H = -sigma.(p + A);
 *   hbar = v_F = e = 1), then projected on the positive-energy state
 *   u_out(p) of the Hamiltonian at t_f:  n(p) = |u_out^dagger psi(t_f)|^2
 *   (unit spinors, so 0 <= n <= 1), and the pair density is
 *   rho = 4 * dx * dy / (2 pi)^2 * sum_p n(p)  (rectangle rule on the grid;
 *   the factor 4 counts spin and valley; 2 when one valley is solved
 *   explicitly).
 *
 * Conventions shared by every entry point:
 *   - Grid: p_x[i] = px_min + i * (px_max - px_min) / nx, i < nx (same for y);
 *     point index k = j * nx + i (x fastest); n(p) is laid out [ny][nx].
 *   - Steps: dt = (t_f - t_i) / N; step k (0 <= k < N) uses the vector
 *     potential at its midpoint t_i + (k + 1/2) dt (Sec. III, Eqs. (11)-(12));
 *     a fourth-order step is five second-order stages, each with the potential
 *     at its own sub-interval midpoint (see pd_scheme).
 *   - A point where |p + A(t_i)| = 0 or |p + A(t_f)| = 0 has no defined
 *     adiabatic spinor; it gets n = 0 and is counted in pd_info.n_masked.
 *   - With a y component of the field (elliptic polarisation) P = p + A with
 *     both components everywhere: steps, spinors, masking, step condition.
 *   - Every call returns a pd_status; nothing crosses the ABI as an exception.
 *     The message of the last failure on the calling thread is returned by
 *     pd_last_error().
 *   - Device pointers are HIP device pointers of the device that was current
 *     when the field was first set; a stream is a hipStream_t passed as void*
 *     (NULL = the default stream).  All GPU work of a call is enqueued on its
 *     stream.
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef PD_H_
#define PD_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_grid_s* pd_grid;

typedef enum {
  PD_OK = 0,
  PD_ERR_INVALID = 1,     /* an argument is out of range, or dt * E_max > pi */
  PD_ERR_STATE = 2,       /* call out of order (e.g. pd_density before the last step) */
  PD_ERR_NOMEM = 3,       /* a device or host allocation failed */
  PD_ERR_DEVICE = 4,      /* a HIP call failed (no device, launch failure, ...) */
  PD_ERR_UNSUPPORTED = 5  /* a valid request the library does not implement */
} pd_status;

typedef enum {
  PD_FP64 = 0,     /* every step in FP64 */
  PD_FP32 = 1,     /* precision form: FP32 state and rotations; FP64 time, field table,
                      rotation angles, projection and density sum; the state is
                      renormalised every 1024 absolute steps (the exact step is unitary,
                      Sec. III); every rotation rounds each state component once */
  PD_FP32_FAST = 2 /* as PD_FP32, but the Strang rotations are plain shears (one
                      component rounded twice per rotation) whose orientation alternates
                      from one stage to the next, so that the doubly rounded component
                      alternates, and a stage's two rotations in one plane (field part
                      and per-point part) run as five shears: a quarter fewer
                      instructions.  On the 2048^2 benchmark solve every point is within
                      1e-5 of FP64 (worst 9.3e-6, PD_FP32 9.6e-6); over long solves on
                      wide grids its worst points reach up to about 1.8x PD_FP32's, so it
                      is not held to PD_FP32's bound (the midpoint schemes run as
                      PD_FP32) */
} pd_precision;

typedef enum {
  /* exp(-i dt Py sy/2) exp(-i dt Px sx) exp(-i dt Py sy/2), P = p + A(t_{k+1/2}):
     the midpoint Hamiltonian of Sec. III split into its sigma_y and sigma_x parts */
  PD_SCHEME_STRANG = 0,
  /* the paper's step, exp(-i dt sigma.P(t_{k+1/2})) in the closed 2x2 form of
     Sec. III, Eq. (13) */
  PD_SCHEME_MIDPOINT = 1,
  /* fourth order: each step is Suzuki's fractal composition of five steps of the
     second-order scheme, S(c1 dt) ... S(c5 dt), c = (p, p, 1 - 4p, p, p),
     p = 1/(4 - 4^(1/3)) (the higher-order decompositions Sec. III names after
     Eq. (12)); stage j samples A at its own sub-interval midpoint
     t_i + (k + sigma_j) dt, sigma_j = c1 + ... + c_{j-1} + c_j / 2 */
  PD_SCHEME_STRANG4 = 2,
  PD_SCHEME_MIDPOINT4 = 3
} pd_scheme;

typedef enum {
  /* valley K+ propagated; rho counts both valleys (identical n, Sec. II) and both
     spins: factor 4 */
  PD_VALLEYS_BOTH = 0,
  /* one valley explicitly (K+: H = +sigma.P, K-: H = -sigma.P with the spinors
     of Sec. II, Eqs. (3)-(4)); rho counts the two spins only: factor 2 */
  PD_VALLEY_KPLUS = 1,
  PD_VALLEY_KMINUS = 2
} pd_valley;

typedef enum {
  PD_FIELD_SIN2 = 0,     /* E(t) = E0 sin^2(pi t/T) sin(omega t), T = cycles 2 pi/omega, t in [0, T] */
  PD_FIELD_CONSTANT = 1, /* E(t) = E0 on [0, t_end] */
  PD_FIELD_TABLE = 2,    /* caller's A at the N step midpoints, with t_i, t_f, A_in, A_out */
  PD_FIELD_PULSE = 3     /* the rise / flat / fall laser pulse of Sec. IV, Eq. (14), on [0, duration]:
                            E0 sin^2(omega_rise t) cos(omega t + phi) for t < pi/(2 omega_rise),
                            E0 cos^2(omega_fall (t - duration + pi/(2 omega_fall))) cos(omega t + phi)
                            over the last pi/(2 omega_fall), E0 cos(omega t + phi) between */
} pd_field_kind;

/* A homogeneous field in the gauge A_0 = 0, E = -dA/dt (Sec. II, after
   Eq. (2)); A(t) = -int_{t_i}^{t} E.  Linear along x unless a y component is
   given (elliptic polarisation, Sec. V): `ellipticity` e adds
     SIN2:     E_y = e E0 sin^2(pi t/T) cos(omega t)
     PULSE:    E_y = e E0 env(t) sin(omega t + phi)  (the x carrier a quarter period later)
     CONSTANT: E_y = e E0
   and a TABLE field may carry A_y samples.  A TABLE gives A at the sample times
   the scheme uses: stages * N values (index k * stages + j) at
   t_i + (k + sigma_j) dt, i.e. the N step midpoints for the second-order
   schemes and 5 N stage midpoints for the fourth-order ones.  Only the members
   of the chosen kind are read.  The struct and the arrays are copied during the
   call. */
typedef struct {
  int kind;                 /* pd_field_kind */
  double E0, omega;         /* SIN2, PULSE */
  int cycles;               /* SIN2: >= 2 */
  double t_end;             /* CONSTANT: > 0 */
  const double* A_mid;      /* TABLE: host array of n_table = N values A(t_i + (k + 1/2) dt) */
  long long n_table;        /* TABLE */
  double t_i, t_f;          /* TABLE: t_f > t_i */
  double A_in, A_out;       /* TABLE: A(t_i), A(t_f) */
  double phi;               /* PULSE: carrier phase */
  double omega_rise;        /* PULSE: > 0 */
  double omega_fall;        /* PULSE: > 0 */
  double duration;          /* PULSE: >= pi/(2 omega_rise) + pi/(2 omega_fall) (equality up to rounding
                               allowed: no flat part) */
  double ellipticity;       /* SIN2, PULSE, CONSTANT: E_y amplitude / E0 (0: linear) */
  const double* Ay_mid;     /* TABLE: NULL (A_y = 0) or n_table values of A_y */
  double Ay_in, Ay_out;     /* TABLE with Ay_mid: A_y(t_i), A_y(t_f) */
} pd_field;

typedef struct {
  long long n_points;       /* nx * ny */
  long long n_steps;        /* N */
  long long steps_done;     /* steps applied so far */
  long long n_masked;       /* points with |p + A_in| = 0 or |p + A_out| = 0 */
  double dt, t_i, t_f, A_in, A_out;
  double E_max;             /* max over grid and step midpoints of |p + A| (also A_in, A_out) */
  double A_min, A_max;      /* range of A over the midpoints and the end points */
  int precision;            /* pd_precision */
  int scheme;               /* pd_scheme */
  int points_per_lane;      /* launch shape in use */
  int block_threads;
  int table_stage;          /* 1 = LDS chunks, 2 = scalar-unit reads */
  int chunk_steps;
  int rotation_form;        /* Strang: 0 = three shears per rotation (every rotation angle of the
                               solve <= pi/2), 1 = versine form (h = cos - 1, s = sin).
                               Midpoint: 0 = tangent form (the step divided by cos(dt E), one
                               series; chosen when the state's growth over 1024 steps stays
                               below 2^32), 1 = cosine form (cos - 1 and sin(x)/x) */
  int taylor_order;         /* midpoint: terms J of the series (tan(x)/x, or cos - 1 and
                               sin(x)/x) in x = (c dt E)^2 */
  size_t device_bytes;      /* device memory the handle owns (its table allocation may exceed the current table) */
  size_t solve_bytes;       /* device memory a solve of this field needs, chunk state included:
                               tables + n(p) + density partials + state (for admission control) */
  int valley;               /* pd_valley */
  int stages;               /* second-order steps per step: 1, or 5 for the fourth-order schemes */
  int elliptic;             /* 1 if the field has a y component */
  double Ay_in, Ay_out;     /* A_y(t_i), A_y(t_f) */
} pd_info;

/* Create a solver on an nx x ny node grid (1 <= nx, ny <= 65536; finite ranges
   with max > min).  Allocates nothing on the device.  *out receives the handle;
   it is NULL on failure. */
pd_status pd_create_grid(int nx, int ny, double px_min, double px_max, double py_min, double py_max,
                         int precision, int scheme, pd_grid* out);

/* Validate a field and step count without touching the device: fills *out
   (dt, E_max, A range, n_masked ...) and returns PD_ERR_INVALID if the step
   would violate dt * E_max <= pi (Sec. III, last paragraph) or an argument is
   out of range.  out may be NULL. */
pd_status pd_check_field(pd_grid g, const pd_field* f, long long n_steps, pd_info* out);

/* Host-only query of the field sampling used by a second-order solve: writes
   the n_steps values A_x(t_i + (k + 1/2) dt) to the host array A_mid (may be
   NULL) and the end values to *t_i, *t_f, *A_in, *A_out (each may be NULL).
   No device work. */
pd_status pd_sample_field(const pd_field* f, long long n_steps, double* A_mid, double* t_i, double* t_f,
                          double* A_in, double* A_out);

/* The same for any scheme and both components: stages * n_steps samples of A_x
   and of A_y at t_i + (k + sigma_j) dt (host arrays, each may be NULL), and
   ends[6] = {t_i, t_f, A_x(t_i), A_x(t_f), A_y(t_i), A_y(t_f)} (may be NULL). */
pd_status pd_sample_field_xy(const pd_field* f, long long n_steps, int scheme, double* Ax_mid, double* Ay_mid,
                             double* ends);

/* Choose the valley (pd_valley) before pd_set_field; PD_ERR_STATE once a
   field is set on the handle, PD_ERR_INVALID for an unknown value.  The default
   is PD_VALLEYS_BOTH. */
pd_status pd_set_valley(pd_grid g, int valley);

/* Set the field and the number of steps N >= 1: builds the per-step FP64
   table of the field on the host (A at the step midpoints, Sec. III,
   Eqs. (11)-(12)), uploads it with a blocking copy, allocates the handle's
   device buffers on first use and resets the solve to t_i (steps_done = 0).
   Same validation as pd_check_field.  For long solves (16384 steps or more) the
   sampling of an analytic field runs on up to 16 short-lived host threads,
   joined before the call returns.
   On a handle already used, the call first waits for the work the library last
   enqueued on its buffers (propagation, density, snapshot, batch epoch), not
   for other work on the device; if that work was enqueued under stream
   capture, it waits for the whole device.  The device table is reallocated
   only when the new one is larger (freeing the old one waits for the whole
   device), so a handle reused for solves of up to the longest it has seen
   frees and allocates nothing. */
pd_status pd_set_field(pd_grid g, const pd_field* f, long long n_steps);

/* Restart the solve at t_i (steps_done = 0) with the field already set; the
   device table is kept.  PD_ERR_STATE before pd_set_field. */
pd_status pd_rewind(pd_grid g);

/* Advance up to max_steps steps (max_steps < 0: all remaining).  Enqueued on
   stream, returns without waiting.  A call that starts at step 0 and runs to N
   keeps every spinor in registers; otherwise the state is kept in device
   memory between calls (the handle's own buffer, or the one given to
   pd_bind_state).  The call that reaches step N also projects on u_out and
   stores n(p) in the handle's device buffer.  The work is one kernel launch,
   or several over consecutive point ranges when the grid needs more than 2^31
   lanes (above 2^31 points at one point per lane), all on `stream`.
   PD_ERR_STATE before pd_set_field or after the last step. */
pd_status pd_propagate(pd_grid g, long long max_steps, void* stream);

/* After the last step: sums n(p) into rho with a fixed-order reduction (the
   result does not depend on the launch shape), optionally copies n(p) to
   n_out (n_points doubles; device memory if n_out_on_device, else host
   memory, pageable or, for a copy at the full host-link rate, page-locked), and
   writes rho to the host double *rho_out (may be NULL).  When rho_out or a host
   n_out is given the call waits for stream. */
pd_status pd_density(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): pd_density with the
   reduction's scratch -- the per-tile partial sums and the device-side rho -- in
   a static device array of the library (1 MiB per device, held until the process
   ends) instead of the handle's buffers.  Same arguments, result (bit for bit)
   and waiting as pd_density; the call itself allocates nothing and creates
   nothing.  Grids of at most 2^28 points (16384 x 16384); larger ones return
   PD_ERR_INVALID before any device work.  Every call on a device shares that
   device's scratch, so calls that overlap on one device (on different streams or
   threads) race; calls ordered on one stream do not. */
pd_status pd_density_static(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream);

/* Time-resolved occupation after the steps done so far (0 <= steps_done <= N,
   e.g. between chunked pd_propagate calls): the state is projected on the
   positive-energy eigenvector of the Hamiltonian at the step boundary
   t_k = t_i + k dt, k = steps_done, n_k(p) = |u(p + A(t_k))^dagger psi_k|^2
   (the instantaneous adiabatic occupation; equal to n(p) at k = N).  A(t_k)
   is the field's own value there; for a TABLE field, between two steps, the
   mean of the last sample of step k - 1 and the first of step k.  Points with
   |p + A(t_i)| = 0 or |p + A(t_k)| = 0 get 0.  Writes n_k to the handle's n
   buffer (a later pd_density is only valid after the solve completes again),
   sums it into rho with the factor of pd_density, copies n_k to n_out and rho
   to *rho_out like pd_density.  Does not advance the solve.  PD_ERR_STATE
   before pd_set_field. */
pd_status pd_snapshot(pd_grid g, double* n_out, int n_out_on_device, double* rho_out, void* stream);

/* Bytes of device state a chunked solve keeps between pd_propagate calls
   (3 FP64 or FP32 values per point for the Strang schemes, 4 for the midpoint
   schemes). */
size_t pd_state_bytes(pd_grid g);

/* Device memory a solve of n_steps steps on g needs, chunk state included
   (field table and rotation tables, n(p), density partials, state), for a field
   without a y component (a y component doubles the step table); closed form,
   no field sampling, no device work (0 for a null handle or n_steps < 1).  Used
   for admission control. */
size_t pd_solve_bytes(pd_grid g, long long n_steps);

/* Use caller-owned device memory (at least pd_state_bytes, 256-byte aligned)
   for the chunked state instead of the handle's own buffer.  The caller keeps
   it alive until the handle is destroyed or another buffer is bound.
   dev_ptr = NULL returns to the handle's own buffer. */
pd_status pd_bind_state(pd_grid g, void* dev_ptr, size_t bytes);

/* Checkpoint and restart: declare that the buffer bound with pd_bind_state holds
   the state after steps_done steps of this same solve (the same grid, field,
   step count, precision, scheme and valley), as a chunked pd_propagate that
   stopped there left it (for example saved to a file and copied back), so that
   the next pd_propagate continues from it.  The continuation is bit-identical to
   the uninterrupted solve.  1 <= steps_done <= N - 1.  PD_ERR_STATE before
   pd_set_field or with no buffer bound; PD_ERR_INVALID for steps_done out of
   range.  The content of the buffer is the caller's responsibility: another
   solve's state gives that solve's continuation, not this one's. */
pd_status pd_resume(pd_grid g, long long steps_done);

/* Checkpoint to host memory: copy the state of a solve in progress (0 < steps
   done < N, as a chunked pd_propagate left it) into the caller's host buffer of
   `bytes` >= pd_state_bytes(g) bytes, and the number of steps it belongs to into
   *steps_done (may be NULL).  The layout is the library's own, point index fastest
   within each state component; it is valid only for a handle with the same grid,
   field, step count, precision, scheme and valley.  The call waits for the
   handle's earlier work, copies on `stream`, and returns when the copy is done.
   PD_ERR_STATE if no solve is in progress; PD_ERR_INVALID for a null pointer or a
   short buffer. */
pd_status pd_save_state(pd_grid g, void* host, size_t bytes, long long* steps_done, void* stream);

/* Restart from a checkpoint: after pd_set_field with the saved solve's field and
   step count, copy the state saved by pd_save_state (exactly pd_state_bytes(g)
   bytes) into the handle's state buffer (the bound one, else its own, allocated
   here if needed) and continue as after steps_done steps: the rest of the solve is
   bit-identical to the uninterrupted one (the state evolves step by step,
   Sec. III, with every per-step choice keyed to the absolute step index).  The call
   waits for the handle's earlier work, copies on `stream`, and returns when the
   copy is done.  1 <= steps_done <= N - 1.  PD_ERR_STATE before pd_set_field;
   PD_ERR_INVALID for a null pointer, a size other than the handle's state size or
   steps_done out of range; PD_ERR_NOMEM if the state buffer cannot be allocated.
   As with pd_resume, the content is the caller's responsibility. */
pd_status pd_load_state(pd_grid g, const void* host, size_t bytes, long long steps_done, void* stream);

/* Override the launch shape of the propagation kernel: points_per_lane in
   {1, 2, 4}; block_threads in {64, 128, 256}; table_stage 1 = the per-step
   field rows are staged through LDS in time chunks (read from VGPRs), 2 = read
   directly by the scalar unit (SGPR operands); chunk_steps = LDS chunk length,
   a power of two in [64, 4096] (at most 1024 in the FP32 form, whose
   renormalisation period it must divide); a solve whose chunk of rows would
   exceed 64 KiB of LDS (long rows: fourth order, y component) reads them with the
   scalar unit instead.  0 keeps the current value.  Results do not depend on the
   launch shape (bit for bit). */
pd_status pd_set_launch(pd_grid g, int points_per_lane, int block_threads, int table_stage, int chunk_steps);

pd_status pd_get_info(pd_grid g, pd_info* out);

/* Release the handle and the device memory it owns.  NULL is a no-op. */
void pd_destroy_grid(pd_grid g);

/* Choose the launch shape of g by timing candidates on the first
   min(trial_steps, N) steps of g's own solve on `stream`: points_per_lane
   {1, 2, 4} x block_threads {64, 256} x (scalar-unit rows, LDS chunks of 256 or
   1024 steps for Strang).  The fastest is applied as by pd_set_launch; the solve
   is left rewound (steps_done = 0).  With use_cache != 0 and the environment
   variable PD_AUTOTUNE_CACHE naming a file, a shape stored there for the same
   (GPU architecture, precision, scheme, rotation form, floor(log2 points)) is
   applied without timing, and a newly timed one is appended. */
pd_status pd_autotune(pd_grid g, long long trial_steps, int use_cache, void* stream);

/* ---- Batches: many solves in one launch sequence ---------------------------

   A batch holds grids (any sizes, schemes, fields, step counts, precisions and
   valleys, each with its field set).  Its second-order Strang members with
   fields along x and fewer tiles than the persistent kernel has resident blocks
   share that kernel: each block takes the next work item -- one tile of
   block_threads * points_per_lane points of one grid -- from a device counter
   until none is left; the items of the grids with the most steps come first.
   Every item does the same arithmetic as the single-grid kernel with the
   scalar-unit table path.  The other members (those that fill the device by
   themselves, fourth-order or midpoint schemes, fields with a y component) run
   their own single-solve launches, with their own launch shapes, concurrently
   with it on a stream of the batch's own (default priority) that is forked from
   the caller's stream by an event and joined back into it before the densities,
   so the sequence stays ordered on the caller's stream.  Each grid's n(p) and rho are therefore
   bit-identical to its solve alone.  Densities of the grids that finish
   are reduced in the same launch sequence (per grid, same fixed order as
   pd_density).  Grids must stay alive while they are members and must not be
   used with pd_propagate while a batch call on them is in flight. */
typedef struct pd_batch_s* pd_batch;

typedef struct {
  int n_grids;
  int points_per_lane;
  int block_threads;
  int graph_captured;     /* 1 if the whole-solve launch is captured and current */
  int work_items;         /* items of the last launch */
  int separate_launches;  /* members of the last launch run by their own kernel */
  long long n_points;     /* sum over members */
  double point_steps;     /* sum over members of points x N */
} pd_batch_info;

pd_status pd_batch_create(pd_batch* out);
/* Add a grid (any scheme); PD_ERR_INVALID if it is already a member. */
pd_status pd_batch_add(pd_batch b, pd_grid g);
/* Remove one member (PD_ERR_INVALID if it is not one); remove a grid from every
   batch before destroying it.  Neither call touches the grids themselves. */
pd_status pd_batch_remove(pd_batch b, pd_grid g);
/* Remove every member. */
pd_status pd_batch_clear(pd_batch b);
int pd_batch_size(pd_batch b);
/* Members in the order they were added; capacity >= pd_batch_size(b). */
pd_status pd_batch_members(pd_batch b, pd_grid* out, int capacity);
/* Launch shape of the persistent kernel: points_per_lane {1, 2, 4},
   block_threads {64, 128, 256}; 0 keeps the current value. */
pd_status pd_batch_set_launch(pd_batch b, int points_per_lane, int block_threads);
/* Run every member's whole solve from t_i: counter reset, the persistent
   kernel (and the other members' launches beside it) and the batched density,
   captured into a HIP graph on the first call and replayed while the membership,
   the members' fields and the launch shape are unchanged (the graph holds kernel
   nodes only).  The graph reads descriptors of its own, which epochs
   (pd_batch_step, pd_batch_step_each, pd_batch_autotune) between two calls do not
   touch; a new capture waits for the last replay first.  Members end with
   steps_done = N and n(p) in their buffers (pd_density works on them).
   rho_out: host array of pd_batch_size(b) doubles, in member order (may be
   NULL; if given, the call waits for stream). */
pd_status pd_batch_run(pd_batch b, double* rho_out, void* stream);
/* One epoch of continuous batching: advance every member that is not complete
   by up to max_steps steps from where it stands (state kept in each grid's
   device state buffer between calls), in one launch sequence as in
   pd_batch_run but not captured, and reduce the densities of the members that
   complete.  rho_out[i] (host, may be NULL) is
   written for members that complete in this call; finished_out[i] (host, may
   be NULL) is 1 for every complete member.  Waits for stream if rho_out is
   given. */
pd_status pd_batch_step(pd_batch b, long long max_steps, double* rho_out, int* finished_out, void* stream);
/* As pd_batch_step with a step limit per member: member i advances by up to
   max_steps[i] steps (host array of pd_batch_size(b) values, each >= 0; 0 leaves
   the member where it stands), so a scheduler can give members different shares
   of an epoch.  The items of the persistent launch are ordered by their step
   counts, longest first.  Each member's arithmetic, and so its n(p) and rho, is
   the same as alone, whatever the limits.  PD_ERR_INVALID if max_steps is NULL
   or a limit is negative. */
pd_status pd_batch_step_each(pd_batch b, const long long* max_steps, double* rho_out, int* finished_out,
                             void* stream);
pd_status pd_batch_get_info(pd_batch b, pd_batch_info* out);
/* Time points_per_lane {1, 2, 4} x block_threads {64, 128, 256} over the first
   trial_steps steps of every member, keep the fastest; members are left
   rewound. */
pd_status pd_batch_autotune(pd_batch b, long long trial_steps, void* stream);
/* Release the batch (not its grids).  NULL is a no-op. */
void pd_batch_destroy(pd_batch b);

/* Message of the last failed call on this thread ("" if none). */
const char* pd_last_error(void);

/* Library version string. */
const char* pd_version(void);

/* Test hook for callers' error handling, for tests only: arm one fault.  "alloc@K":
   the K-th device allocation of the library from now on fails (PD_ERR_NOMEM from
   the call that needed it); "launch@K": the K-th launch sequence (pd_propagate,
   pd_batch_run, pd_batch_step, pd_batch_step_each) fails with PD_ERR_DEVICE
   before it enqueues anything, leaving every grid where it stood.  The fault fires
   once, then disarms; NULL or "" disarms.  The environment variable PD_FAULT with
   the same syntax arms a fault at the library's first allocation or launch.
   PD_ERR_INVALID for any other text.  Process-wide. */
pd_status pd_set_fault(const char* spec);

/* Environment: PD_TRACE (set and not "0") makes pd_set_field, pd_propagate,
   pd_density, pd_density_static, pd_snapshot, pd_autotune and the batch run, step
   and autotune calls each write "pd_trace <name> <ms> ms" to stderr as they return:
   the host time of the call (launches are asynchronous; a call that waits for the
   device includes the wait).  PD_AUTOTUNE_CACHE names the autotuner's cache file
   (pd_autotune). */

#ifdef __cplusplus
}
#endif

#endif /* PD_H_ */
