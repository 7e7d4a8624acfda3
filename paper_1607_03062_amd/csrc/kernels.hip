// gfx950 kernels of libpd: split-operator propagation of one state per momentum
// point, projection on the final positive-energy state, and the density sum.
//
// One lane per momentum point (points_per_lane of them, strided by the block
// size so loads and stores stay coalesced).  The per-step field row is the same
// for every lane: it is either staged through LDS in time chunks (every lane then
// reads it into VGPRs) or read by the scalar unit into SGPRs.
//
// Strang scheme (Sec. III, Eqs. (11)-(12), with the midpoint Hamiltonian
// sigma_x P_x + sigma_y p_y split into its two parts):
//   U_k = exp(-i dt py sy / 2) exp(-i dt (px + A_k) sx) exp(-i dt py sy / 2).
// The kernel propagates the Bloch vector r of the pure state, psi psi^dagger =
// (1 + r.sigma) / 2, which carries everything n(p) depends on (the global
// phase of psi is unobservable): exp(-i a sx) rotates r by 2a about x and
// exp(-i b sy) by 2b about y.  Since exp(-i dt (px + A_k) sx) =
// exp(-i dt px sx) exp(-i dt A_k sx), every step is three plane rotations:
// by 2 dt A_k about x (table row, the same for all lanes), by 2 dt px about x
// and by 2 dt py about y (per-point constants computed once); the half steps of
// neighbouring steps are merged.
//
// A plane rotation by phi is applied either as three shears (Paeth's
// decomposition; one FMA each, coefficients tan(phi/2) and sin(phi)), or, when
// some angle of the solve is too large for the shears to stay well conditioned,
// in versine form with h = cos(phi) - 1 and s = sin(phi).  The fast FP32 form runs
// two successive rotations in one plane (a stage's field and per-point parts) as
// five shears, the two adjacent shears of the same component merged.
// The projection on u_out is n = |u_out^dagger psi|^2 = (1 + r.r_u) / 2 with
// r_u = P_out / |P_out| the Bloch vector of u_out (Sec. II, Eqs. (1), (3)); r
// is normalised first (the exact steps are unitary, Sec. III).
//
// Midpoint scheme (Sec. III, Eq. (13)): per step the closed 2x2 form
//   U = cos(dt E) I - i sigma.P sin(dt E) / E,  P = p + A_k,
// acting on the spinor (a1 + i b1, a2 + i b2).  For the small step angles of
// most solves the kernel applies U / cos(dt E) = I - i tan(dt E) sigma.P / E, one
// even series (tan(x)/x) instead of two and one rounding per component; the
// state's norm then grows by 1 / cos(dt E) per step and is renormalised every
// kRenormEvery steps (n divides it out).  Otherwise cos - 1 and sin(x)/x are
// evaluated.  The series are Taylor series in x = (dt E)^2 of an order chosen
// by the host.
//
// Both kernels are templated on the composition (NS = 1 second-order step, or
// NS = 5 stages of Suzuki's fourth-order composition, each a second-order step
// over c_j dt with the field at its own sub-interval midpoint) and on a y
// component of the field (POL: sigma_y (p_y + A_y) in place of sigma_y p_y; the
// Strang kernel then adds the field part of each y rotation from the table).
// The K- valley (H = -sigma.P) arrives as negated table and coefficient angles
// plus the sign vsign of the initial state and of the projection.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pd_internal.h"

namespace pdx {
namespace {

// Rotation of (u, v) by phi: u' = u cos - v sin, v' = u sin + v cos.
// Shear form, t = tan(phi/2), s = sin(phi): u -= t v; v += s u; u -= t v.
template <typename R>
__device__ __forceinline__ void rotate_shear(R& u, R& v, R t, R s) {
  u = fma(-t, v, u);
  v = fma(s, u, v);
  u = fma(-t, v, u);
}

// Versine form, h = cos - 1: u' = u + h u - s v,  v' = v + h v + s u.
__device__ __forceinline__ void rotate_versine(double& u, double& v, double h, double s) {
  double nu = fma(h, u, fma(-s, v, u));
  double nv = fma(h, v, fma(s, u, v));
  u = nu;
  v = nv;
}

// FP32 versine form: the small increment is formed first and added once, so the
// state sees a single rounding per component per rotation.
__device__ __forceinline__ void rotate_versine(float& u, float& v, float h, float s) {
  float du = fmaf(h, u, -(s * v));
  float dv = fmaf(h, v, s * u);
  u = u + du;
  v = v + dv;
}

template <int FORM, typename R>
__device__ __forceinline__ void rotate(R& u, R& v, R a, R s) {
  if (FORM == kFormShear)
    rotate_shear(u, v, a, s);
  else
    rotate_versine(u, v, a, s);
}


// Shear form with every component rounded once per rotation: the two u shears
// add up to u - t (v + v'), so u is updated from its value before the rotation
// (3 FMA + 1 add).  In FP32 the state's rounding errors are the whole error of a
// solve, and the second rounding of u per rotation dominates them (its increments
// are small, and the roundings of a slowly varying state accumulate); rounding each
// component once halves the worst-point error of the FP32 form on the benchmark
// workloads, for a quarter more instructions.
__device__ __forceinline__ void rotate_shear_once(float& u, float& v, float t, float s) {
  float u1 = fmaf(-t, v, u);
  float v1 = fmaf(s, u1, v);
  float w = v + v1;
  u = fmaf(-t, w, u);
  v = v1;
}

// The same shear rotation with the roles of u and v exchanged: v += t u; u -= s v;
// v += t u.  Now v is the component rounded twice.
template <typename R>
__device__ __forceinline__ void rotate_shear_vu(R& u, R& v, R t, R s) {
  v = fma(t, u, v);
  u = fma(-s, v, u);
  v = fma(t, u, v);
}

// Two rotations in one plane, by a and then by b, as five shears: the last shear of
// the first triple and the first of the second act on the same component, so they
// merge into one with the summed coefficient (one add).  Both orientations.
template <typename R>
__device__ __forceinline__ void rotate_two_shear(R& u, R& v, R ta, R sa, R tb, R sb) {
  u = fma(-ta, v, u);
  v = fma(sa, u, v);
  u = fma(-(ta + tb), v, u);
  v = fma(sb, u, v);
  u = fma(-tb, v, u);
}

template <typename R>
__device__ __forceinline__ void rotate_two_shear_vu(R& u, R& v, R ta, R sa, R tb, R sb) {
  v = fma(ta, u, v);
  u = fma(-sa, v, u);
  v = fma(ta + tb, u, v);
  u = fma(-sb, v, u);
  v = fma(tb, u, v);
}

// Shear variants (FP32 forms):
//   kShearPlain  u -= t v; v += s u; u -= t v (u rounded twice per rotation);
//   kShearOnce   each component rounded once (rotate_shear_once, 4 instructions);
//   kShearAlt    plain shears with the orientation alternating from one stage to the
//                next (u-v-u, then v-u-v; the parity of the absolute stage index), so
//                that the doubly rounded component alternates and the systematic part
//                of the roundings largely cancels between neighbouring stages; the
//                stage's two rotations in one plane (field and per-point parts) run as
//                five shears (rotate_two_shear), which rounds less for the same count:
//                3 instructions per rotation.
constexpr int kShearPlain = 0;
constexpr int kShearOnce = 1;
constexpr int kShearAlt = 2;

// A rotation in the solve's form and shear variant SH; odd: the stage's parity
// (kShearAlt only; a compile-time constant wherever the steps are unrolled).
template <int FORM, int SH, typename R>
__device__ __forceinline__ void rot(R& u, R& v, R a, R s, bool odd = false) {
  if constexpr (FORM == kFormShear && SH == kShearOnce && sizeof(R) == 4) {
    rotate_shear_once(u, v, a, s);
  } else if constexpr (FORM == kFormShear && SH == kShearAlt) {
    if (odd)
      rotate_shear_vu(u, v, a, s);
    else
      rotate_shear(u, v, a, s);
  } else {
    rotate<FORM>(u, v, a, s);
  }
}

struct PointCoords {
  int i, j;
  double px, py;
};

__device__ __forceinline__ PointCoords coords(const SolveParams& p, long long idx) {
  long long j = idx / p.nx;
  long long i = idx - j * p.nx;
  PointCoords c;
  c.i = (int)i;
  c.j = (int)j;
  c.px = p.px_min + (double)i * p.dx;
  c.py = p.py_min + (double)j * p.dy;
  return c;
}

// Rotation layout of one step of a composition with NS stages.  Stage j applies
// the x rotation by its field part (table) and by its per-point part (class
// xcls(j) of the column coefficients), then the y rotation that follows it: its
// per-point part (class ycls(j) of the row coefficients) and, with a y component
// of the field (POL), its field part (table).  The y rotations of neighbouring
// stages, and of the last stage of a step and the first of the next, are merged;
// the solve opens and closes with a half step (the last row class).
template <int NS>
struct Layout;
template <>
struct Layout<1> {
  static constexpr int NX = 1, NY = 2;  // y classes: full, half
  __device__ static constexpr int xcls(int) { return 0; }
  __device__ static constexpr int ycls(int) { return 0; }
};
template <>
struct Layout<5> {
  // c = (p, p, q, p, p): x classes {p, q}; y classes {(p + p)/2, (p + q)/2, half}
  static constexpr int NX = 2, NY = 3;
  __device__ static constexpr int xcls(int j) { return j == 2 ? 1 : 0; }
  __device__ static constexpr int ycls(int j) { return (j == 1 || j == 2) ? 1 : 0; }
};

// Coefficient phases of the per-point rotations (host: coefficient_phases): the
// FP32 forms cycle through kDitherFP32 values of each coefficient, step k using
// value k mod kDitherFP32.
template <typename R>
constexpr int phases_of() {
  return sizeof(R) == 4 ? kDitherFP32 : 1;
}

// Period of a solve's step pattern: the coefficient phases and, for alternating
// shears, the orientation parity.  Steps run in groups that start at multiples of
// it, so inside a group every step's pattern is a compile-time constant.
template <typename R, int SH>
constexpr int step_period() {
  return (SH == kShearAlt && phases_of<R>() % 2 != 0) ? 2 * phases_of<R>() : phases_of<R>();
}

// The Bloch vectors of a lane's points and their per-point rotations.
template <typename R, int PPL, int FORM, int NS, int POL, int SH>
struct BlochLanes {
  using L = Layout<NS>;
  static constexpr int kRow = 2 * NS * (1 + POL);  // table values per step
  static constexpr int D = phases_of<R>();
  static constexpr int P = step_period<R, SH>();
  R x[PPL], y[PPL], z[PPL];
  R aX[L::NX][D][PPL], sX[L::NX][D][PPL];          // x rotations by 2 c dt px, per phase
  R aY[L::NY - 1][D][PPL], sY[L::NY - 1][D][PPL];  // y rotations after the stages, by (c_j + c_j+1) dt py

  // One step; row = the step's table values; PH = the step's absolute index modulo
  // P (phase PH % D of the coefficients; with alternating shears stage j of step k
  // has parity k + j, NS odd).  LAST: the y rotation after the last stage is the
  // closing half step (ha, hs per point).
  template <bool LAST, int PH>
  __device__ __forceinline__ void step(const R* row, const R* ha, const R* hs) {
    constexpr int h = PH % D;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const bool o = ((PH & 1) != 0) != ((j & 1) != 0);
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        const R ya = (LAST && j == NS - 1) ? ha[q] : aY[L::ycls(j)][h][q];
        const R ys = (LAST && j == NS - 1) ? hs[q] : sY[L::ycls(j)][h][q];
        if constexpr (FORM == kFormShear && SH == kShearAlt) {
          // the x rotations by the field part and the point's part, then the y rotation
          // by the point's part and (POL) the field part, each pair as five shears
          if (o)
            rotate_two_shear_vu(y[q], z[q], row[2 * j], row[2 * j + 1], aX[L::xcls(j)][h][q], sX[L::xcls(j)][h][q]);
          else
            rotate_two_shear(y[q], z[q], row[2 * j], row[2 * j + 1], aX[L::xcls(j)][h][q], sX[L::xcls(j)][h][q]);
          if constexpr (POL) {
            if (o)
              rotate_two_shear_vu(z[q], x[q], ya, ys, row[2 * NS + 2 * j], row[2 * NS + 2 * j + 1]);
            else
              rotate_two_shear(z[q], x[q], ya, ys, row[2 * NS + 2 * j], row[2 * NS + 2 * j + 1]);
          } else {
            rot<FORM, SH>(z[q], x[q], ya, ys, o);
          }
        } else {
          rot<FORM, SH>(y[q], z[q], row[2 * j], row[2 * j + 1], o);
          rot<FORM, SH>(y[q], z[q], aX[L::xcls(j)][h][q], sX[L::xcls(j)][h][q], o);
          rot<FORM, SH>(z[q], x[q], ya, ys, o);
          if (POL) rot<FORM, SH>(z[q], x[q], row[2 * NS + 2 * j], row[2 * NS + 2 * j + 1], o);
        }
      }
    }
  }

  // A step whose pattern index k mod P is known only at run time (uniform over the wave).
  template <bool LAST>
  __device__ __forceinline__ void step_at(const R* row, long long k, const R* ha = nullptr, const R* hs = nullptr) {
    switch ((int)(k % P)) {
      case 0: step<LAST, 0>(row, ha, hs); break;
      case 1: if constexpr (P > 1) step<LAST, 1 % P>(row, ha, hs); break;
      case 2: if constexpr (P > 2) step<LAST, 2 % P>(row, ha, hs); break;
      case 3: if constexpr (P > 3) step<LAST, 3 % P>(row, ha, hs); break;
      case 4: if constexpr (P > 4) step<LAST, 4 % P>(row, ha, hs); break;
      case 5: if constexpr (P > 5) step<LAST, 5 % P>(row, ha, hs); break;
      case 6: if constexpr (P > 6) step<LAST, 6 % P>(row, ha, hs); break;
      default: if constexpr (P > 7) step<LAST, 7 % P>(row, ha, hs); break;
    }
  }

  __device__ __forceinline__ void renormalise() {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      double X = x[q], Y = y[q], Z = z[q];
      double nr = sqrt(X * X + Y * Y + Z * Z);
      if (nr > 0.0) {
        x[q] = (R)(X / nr);
        y[q] = (R)(Y / nr);
        z[q] = (R)(Z / nr);
      }
    }
  }
};

template <typename R, int W>
struct RowN {
  R v[W];
};

// Steps U of a group that starts at a multiple of the step period, with the
// pattern index of each known at compile time.
template <typename Lanes, typename Row, int U, int G>
__device__ __forceinline__ void group_steps(Lanes& L, const Row* r) {
  if constexpr (U < G) {
    L.template step<false, U % Lanes::P>(r[U].v, nullptr, nullptr);
    group_steps<Lanes, Row, U + 1, G>(L, r);
  }
}

// Steps U of a group whose rows are long (fourth order, y component), each row loaded
// one step ahead: row U + 1 (or the next group's first, `after`) is requested before step
// U's arithmetic, so two rows are live instead of two groups of them.
template <typename Lanes, typename Row, int U, int G>
__device__ __forceinline__ void group_steps_ahead(Lanes& L, const Row* __restrict__ g, const Row* __restrict__ after,
                                                  Row& cur) {
  if constexpr (U < G) {
    const Row nxt = (U + 1 < G) ? g[U + 1] : after[0];
    __builtin_amdgcn_sched_barrier(0);
    L.template step<false, U % Lanes::P>(cur.v, nullptr, nullptr);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
    group_steps_ahead<Lanes, Row, U + 1, G>(L, g, after, cur);
  }
}

// Steps [k, k_full) with the table rows read by the scalar unit (SGPR operands).
template <typename R, int PPL, int FORM, int NS, int POL, int SH>
__device__ __forceinline__ void steps_scalar(BlochLanes<R, PPL, FORM, NS, POL, SH>& L, const R* __restrict__ table,
                                             long long k, long long k_full) {
  using Lanes = BlochLanes<R, PPL, FORM, NS, POL, SH>;
  using Row = RowN<R, Lanes::kRow>;
  constexpr int P = Lanes::P;
  const Row* __restrict__ tab = reinterpret_cast<const Row*>(table);
  constexpr int kRows = Lanes::kRow >= 8 ? 1 : 8 / (Lanes::kRow / 2);  // rows fetched together
  constexpr int kGroup = (kRows + P - 1) / P * P;                     // whole periods
  // two sets of a group's rows fit the scalar registers for short rows, or groups of one
  // row; the long rows of the FP32 forms (groups of a whole coefficient period) go one
  // row ahead instead
  constexpr bool kTwoSets = kGroup == 1 || kGroup * Lanes::kRow * (int)sizeof(R) <= 32 * 4;
  while (k < k_full) {
    long long seg = k_full;
    if (sizeof(R) == 4) {
      long long next = (k / kRenormEvery + 1) * kRenormEvery;
      seg = next < k_full ? next : k_full;
    }
    // up to the first multiple of the period (renormalisation steps are multiples of it)
    for (; (k % P) != 0 && k < seg; ++k) {
      const Row r = tab[k];
      L.template step_at<false>(r.v, k);
    }
    // whole groups: a 32-bit trip count, so the loop test stays on the scalar unit, and
    // two row sets in turn.  Each set is loaded right after the other set's first step
    // (scalar loads complete out of order, so the wait before a set's first use covers
    // every load in flight) and its latency is hidden behind that set's other steps; the
    // scheduling barriers keep the loads there.  The clamped index re-reads the last
    // group instead of branching.
    if constexpr (!kTwoSets) {
      // long rows: one row ahead.  Rows k .. k + n kGroup are read; the last of them is
      // at most seg <= the last step's row, so every read is inside the table.
      while (k + kGroup <= seg) {
        const long long left = (seg - k) / kGroup;
        const int n = left < (1 << 30) ? (int)left : (1 << 30);
        const Row* __restrict__ g = tab + k;
        Row cur = g[0];
        for (int i = 0; i < n; ++i) {
          const Row* __restrict__ gi = g + (long long)i * kGroup;
          group_steps_ahead<Lanes, Row, 0, kGroup>(L, gi, gi + kGroup, cur);
        }
        k += (long long)n * kGroup;
      }
    }
    while (kTwoSets && k + kGroup <= seg) {
      const long long left = (seg - k) / kGroup;
      const int n = left < (1 << 30) ? (int)left : (1 << 30);
      const Row* __restrict__ g = tab + k;
      Row a[kGroup], b[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) a[u] = g[u];
      int i = 0;
      for (; i + 1 < n; i += 2) {
        group_steps<Lanes, Row, 0, 1>(L, a);
        __builtin_amdgcn_sched_barrier(0);
        const Row* __restrict__ gb = g + (long long)(i + 1) * kGroup;
#pragma unroll
        for (int u = 0; u < kGroup; ++u) b[u] = gb[u];
        __builtin_amdgcn_sched_barrier(0);
        group_steps<Lanes, Row, 1, kGroup>(L, a);
        group_steps<Lanes, Row, 0, 1>(L, b);
        __builtin_amdgcn_sched_barrier(0);
        const Row* __restrict__ ga = g + (long long)(i + 2 < n ? i + 2 : n - 1) * kGroup;
#pragma unroll
        for (int u = 0; u < kGroup; ++u) a[u] = ga[u];
        __builtin_amdgcn_sched_barrier(0);
        group_steps<Lanes, Row, 1, kGroup>(L, b);
      }
      if (i < n) group_steps<Lanes, Row, 0, kGroup>(L, a);
      k += (long long)n * kGroup;
    }
    for (; k < seg; ++k) {
      const Row r = tab[k];
      L.template step_at<false>(r.v, k);
    }
    if (sizeof(R) == 4 && (k % kRenormEvery) == 0) L.renormalise();
  }
}

// Steps [k, k_full) with the table staged through LDS in chunks of `chunk` rows
// (absolute chunk boundaries; a power of two dividing the renormalisation period
// in the FP32 form, and a multiple of the step period), so every lane reads its
// rotation from VGPRs.
template <typename R, int PPL, int FORM, int NS, int POL, int SH>
__device__ __forceinline__ void steps_lds(BlochLanes<R, PPL, FORM, NS, POL, SH>& L, const R* __restrict__ table,
                                          long long k, long long k_full, long long chunk) {
  using Lanes = BlochLanes<R, PPL, FORM, NS, POL, SH>;
  using Row = RowN<R, Lanes::kRow>;
  constexpr int P = Lanes::P;
  const Row* __restrict__ tab = reinterpret_cast<const Row*>(table);
  extern __shared__ unsigned char pd_lds[];
  Row* rows = reinterpret_cast<Row*>(pd_lds);
  while (k < k_full) {
    long long cend = (k / chunk + 1) * chunk;
    if (cend > k_full) cend = k_full;
    const int cnt = (int)(cend - k);
    __syncthreads();  // every wave has finished with the previous chunk
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) rows[t] = tab[k + t];
    __syncthreads();
    int t = 0;
    for (; ((k + t) % P) != 0 && t < cnt; ++t) {
      const Row r = rows[t];
      L.template step_at<false>(r.v, k + t);
    }
    if constexpr (P == 1) {
#pragma unroll 8
      for (; t < cnt; ++t) {
        const Row r = rows[t];
        L.template step<false, 0>(r.v, nullptr, nullptr);
      }
    } else {
#pragma unroll 2
      for (; t + P <= cnt; t += P) {
        Row r[P];
#pragma unroll
        for (int u = 0; u < P; ++u) r[u] = rows[t + u];
        group_steps<Lanes, Row, 0, P>(L, r);
      }
      for (; t < cnt; ++t) {
        const Row r = rows[t];
        L.template step_at<false>(r.v, k + t);
      }
    }
    k = cend;
    if (sizeof(R) == 4 && (k % kRenormEvery) == 0) L.renormalise();
  }
}

// One tile of a Strang solve: the block's lanes own points base + q * blockDim.x,
// q < PPL; steps [p.k_begin, p.k_end).
template <typename R, int PPL, int STAGE, int FORM, int NS, int POL, int SH>
__device__ __forceinline__ void strang_tile(const SolveParams& p, const long long base) {
  using Lanes = BlochLanes<R, PPL, FORM, NS, POL, SH>;
  using LY = Layout<NS>;
  constexpr int D = Lanes::D;
  constexpr int CX = 2 * LY::NX * D;                // coefficient values per column
  constexpr int CY = 2 * ((LY::NY - 1) * D + 1);    // per row: the phased pairs, then the half step
  constexpr int HALF = 2 * (LY::NY - 1) * D;        // offset of the half-step pair in a row
  const R* __restrict__ colc = static_cast<const R*>(p.col_coef);
  const R* __restrict__ rowc = static_cast<const R*>(p.row_coef);
  const R* __restrict__ table = static_cast<const R*>(p.table);
  Lanes L;

#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    long long idx = base + (long long)q * blockDim.x;
    if (idx >= p.npts) idx = p.npts - 1;  // tail lanes recompute a valid point and store nothing
    PointCoords c = coords(p, idx);
#pragma unroll
    for (int m = 0; m < LY::NX; ++m)
#pragma unroll
      for (int h = 0; h < D; ++h) {
        L.aX[m][h][q] = colc[CX * c.i + 2 * (m * D + h)];
        L.sX[m][h][q] = colc[CX * c.i + 2 * (m * D + h) + 1];
      }
#pragma unroll
    for (int m = 0; m < LY::NY - 1; ++m)
#pragma unroll
      for (int h = 0; h < D; ++h) {
        L.aY[m][h][q] = rowc[CY * c.j + 2 * (m * D + h)];
        L.sY[m][h][q] = rowc[CY * c.j + 2 * (m * D + h) + 1];
      }
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      L.x[q] = st[idx];
      L.y[q] = st[p.npts + idx];
      L.z[q] = st[2 * p.npts + idx];
    } else {
      // v_in: negative-energy eigenvector of the valley Hamiltonian vsign sigma.P_in,
      // Bloch vector -vsign P_in/|P_in|
      double Px = c.px + p.A_in, Py = c.py + p.Ay_in;
      double E = sqrt(Px * Px + Py * Py);
      double rx = 0.0, ry = 0.0;
      if (E > 0.0) {
        rx = -p.vsign * Px / E;
        ry = -p.vsign * Py / E;
      }
      L.x[q] = (R)rx;
      L.y[q] = (R)ry;
      L.z[q] = (R)0;
      // opening half step about y: per-point part, then (POL) the field part
      rot<FORM, SH>(L.z[q], L.x[q], rowc[CY * c.j + HALF], rowc[CY * c.j + HALF + 1]);
      if (POL) {
        const R* open = table + (size_t)p.n_steps * Lanes::kRow + 2 * NS;
        rot<FORM, SH>(L.z[q], L.x[q], open[0], open[1]);
      }
    }
  }

  const long long k_full = p.k_end < p.n_steps ? p.k_end : p.n_steps - 1;
  if (STAGE == 1)
    steps_lds(L, table, p.k_begin, k_full, p.chunk_steps);
  else
    steps_scalar(L, table, p.k_begin, k_full);

  if (p.k_end == p.n_steps) {
    // last step: its y rotation after the last stage is the closing half step
    R ha[PPL], hs[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      long long idx = base + (long long)q * blockDim.x;
      if (idx >= p.npts) idx = p.npts - 1;
      PointCoords c = coords(p, idx);
      ha[q] = rowc[CY * c.j + HALF];
      hs[q] = rowc[CY * c.j + HALF + 1];
    }
    const R* last = table + (size_t)(p.n_steps - 1) * Lanes::kRow;
    L.template step_at<true>(last, p.n_steps - 1, ha, hs);
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      long long idx = base + (long long)q * blockDim.x;
      bool valid = idx < p.npts;
      if (!valid) idx = p.npts - 1;
      PointCoords c = coords(p, idx);
      // projection on u_out: n = (1 + vsign r.P_out / |P_out|) / 2 with r normalised
      double Pxi = c.px + p.A_in, Pyi = c.py + p.Ay_in;
      double Pxo = c.px + p.A_out, Pyo = c.py + p.Ay_out;
      double Ei = sqrt(Pxi * Pxi + Pyi * Pyi), Eo = sqrt(Pxo * Pxo + Pyo * Pyo);
      double X = L.x[q], Y = L.y[q], Z = L.z[q];
      double nr = sqrt(X * X + Y * Y + Z * Z);
      double n = 0.0;
      if (Ei > 0.0 && Eo > 0.0 && nr > 0.0) {
        double dot = (Pxo * X + Pyo * Y) / nr;
        n = (Eo + p.vsign * dot) / (2.0 * Eo);
      }
      if (valid) p.n_out[idx] = n;
    }
  } else if (p.store_state) {
    R* st = static_cast<R*>(p.state);
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      long long idx = base + (long long)q * blockDim.x;
      if (idx < p.npts) {
        st[idx] = L.x[q];
        st[p.npts + idx] = L.y[q];
        st[2 * p.npts + idx] = L.z[q];
      }
    }
  }
}

template <typename R, int PPL, int STAGE, int FORM, int NS, int POL, int SH>
__global__ void __launch_bounds__(256) strang_kernel(const SolveParams p) {
  strang_tile<R, PPL, STAGE, FORM, NS, POL, SH>(p, p.first + (long long)blockIdx.x * blockDim.x * PPL + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched Strang solves in one persistent launch.  Every block takes the next
// work item (one tile of one solve) from a global counter until none is left;
// the host orders the items longest first.  An item's arithmetic is the same as
// in the single-solve kernel, so each solve's result does not depend on the
// batch it runs in.

__global__ void batch_reset(unsigned int* counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
}

template <int PPL>
__global__ void __launch_bounds__(256) batch_kernel(const BatchSolve* __restrict__ solves,
                                                    const BatchItem* __restrict__ items, int n_items,
                                                    unsigned int* counter) {
  __shared__ int next;
  for (;;) {
    __syncthreads();  // every lane has read the previous item index
    if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = next;
    if (it >= n_items) return;  // uniform over the block
    const BatchItem w = items[it];
    const BatchSolve& s = solves[w.solve];
    const long long base = w.base + threadIdx.x;
    if (s.precision == PD_FP32) {
      if (s.form == kFormShear)
        strang_tile<float, PPL, 0, kFormShear, 1, 0, kShearOnce>(s.p, base);
      else
        strang_tile<float, PPL, 0, kFormVersine, 1, 0, kShearPlain>(s.p, base);
    } else if (s.precision == PD_FP32_FAST) {
      if (s.form == kFormShear)
        strang_tile<float, PPL, 0, kFormShear, 1, 0, kShearAlt>(s.p, base);
      else
        strang_tile<float, PPL, 0, kFormVersine, 1, 0, kShearPlain>(s.p, base);
    } else {
      if (s.form == kFormShear)
        strang_tile<double, PPL, 0, kFormShear, 1, 0, kShearPlain>(s.p, base);
      else
        strang_tile<double, PPL, 0, kFormVersine, 1, 0, kShearPlain>(s.p, base);
    }
  }
}

// ---------------------------------------------------------------------------
// Midpoint scheme: spinor state, series coefficients per point and step.

template <int J>
struct Taylor {
  // cos(sqrt x) - 1 = sum_{j>=1} (-x)^j / (2j)!;  sin(sqrt x)/sqrt x = sum_{j>=0} (-x)^j / (2j+1)!
  __device__ __forceinline__ static double h(double x) {
    double acc = coef_h(J);
#pragma unroll
    for (int j = J - 1; j >= 1; --j) acc = fma(acc, x, coef_h(j));
    return acc * x;
  }
  __device__ __forceinline__ static double s(double x) {
    double acc = coef_s(J);
#pragma unroll
    for (int j = J - 1; j >= 0; --j) acc = fma(acc, x, coef_s(j));
    return acc;
  }
  __device__ __forceinline__ static float h(float x) {
    float acc = (float)coef_h(J);
#pragma unroll
    for (int j = J - 1; j >= 1; --j) acc = fmaf(acc, x, (float)coef_h(j));
    return acc * x;
  }
  __device__ __forceinline__ static float s(float x) {
    float acc = (float)coef_s(J);
#pragma unroll
    for (int j = J - 1; j >= 0; --j) acc = fmaf(acc, x, (float)coef_s(j));
    return acc;
  }
  // (-1)^j / (2j)!  and  (-1)^j / (2j+1)!, folded by the compiler
  __device__ __forceinline__ static constexpr double coef_h(int j) {
    double f = 1.0;
    for (int m = 2; m <= 2 * j; ++m) f *= m;
    return (j % 2 ? -1.0 : 1.0) / f;
  }
  __device__ __forceinline__ static constexpr double coef_s(int j) {
    double f = 1.0;
    for (int m = 2; m <= 2 * j + 1; ++m) f *= m;
    return (j % 2 ? -1.0 : 1.0) / f;
  }
};

// psi1' = c psi1 + (-i al - be) psi2 ;  psi2' = c psi2 + (be - i al) psi1, with c = 1 + h.
__device__ __forceinline__ void midpoint_update(double& a1, double& b1, double& a2, double& b2, double h, double al,
                                                double be) {
  double na1 = fma(h, a1, fma(-be, a2, fma(al, b2, a1)));
  double nb1 = fma(h, b1, fma(-be, b2, fma(-al, a2, b1)));
  double na2 = fma(h, a2, fma(be, a1, fma(al, b1, a2)));
  double nb2 = fma(h, b2, fma(be, b1, fma(-al, a1, b2)));
  a1 = na1;
  b1 = nb1;
  a2 = na2;
  b2 = nb2;
}

__device__ __forceinline__ void midpoint_update(float& a1, float& b1, float& a2, float& b2, float h, float al,
                                                float be) {
  float da1 = fmaf(h, a1, fmaf(-be, a2, al * b2));
  float db1 = fmaf(h, b1, fmaf(-be, b2, -(al * a2)));
  float da2 = fmaf(h, a2, fmaf(be, a1, al * b1));
  float db2 = fmaf(h, b2, fmaf(be, b1, -(al * a1)));
  a1 += da1;
  b1 += db1;
  a2 += da2;
  b2 += db2;
}

// tan(sqrt x) / sqrt x - 1 = sum_{n=2}^{J} a_n x^(n-1) (coefficients from tan' = 1 + tan^2).
// The 1 is left out so that the rounding of the sum is relative to its own small
// size; the caller adds it exactly, as (al, be) = fma(tau - 1, (X, Y), (X, Y)).
template <int J>
struct TanSeries {
  template <typename R>
  __device__ __forceinline__ static R minus1(R x) {
    R acc = (R)tan_series_coef(J);
#pragma unroll
    for (int n = J - 1; n >= 2; --n) acc = fma(acc, x, (R)tan_series_coef(n));
    return acc * x;
  }
};

// Tangent form: psi += (-i al sigma_x - i be sigma_y) psi with (al, be) = tan(theta) (X, Y) / theta,
// i.e. U / cos(theta).  FP32: each component rounded once (the increment is formed
// first).  FP64: two chained FMAs per component (two roundings at 2^-53 stay far below
// the 1e-12 target and save a third of the update's instructions).
__device__ __forceinline__ void midpoint_update_tan(float& a1, float& b1, float& a2, float& b2, float al, float be) {
  float da1 = fmaf(-be, a2, al * b2);
  float db1 = fmaf(-be, b2, -(al * a2));
  float da2 = fmaf(be, a1, al * b1);
  float db2 = fmaf(be, b1, -(al * a1));
  a1 += da1;
  b1 += db1;
  a2 += da2;
  b2 += db2;
}

__device__ __forceinline__ void midpoint_update_tan(double& a1, double& b1, double& a2, double& b2, double al,
                                                    double be) {
  double na1 = fma(-be, a2, fma(al, b2, a1));
  double nb1 = fma(-be, b2, fma(-al, a2, b1));
  double na2 = fma(be, a1, fma(al, b1, a2));
  double nb2 = fma(be, b1, fma(-al, a1, b2));
  a1 = na1;
  b1 = nb1;
  a2 = na2;
  b2 = nb2;
}

// Stage layout of the midpoint kernel: stage j of a step of the NS-stage
// composition uses the per-point phase of class mcls(j) (c = p or q).
template <int NS>
__device__ __forceinline__ constexpr int mcls(int j) {
  return NS == 5 && j == 2 ? 1 : 0;
}

// Point q of a lane of the midpoint kernel: the lane owns column i of the band of
// PPL consecutive rows band * PPL .. band * PPL + PPL - 1, so all its points share
// p_x and with it the FP64 phase c dt (p_x + A_k) of every step (and its FP32
// rounding), computed once per lane.  Consecutive lanes take consecutive columns,
// so loads and stores stay coalesced.  Rows past the last one recompute a valid
// point (the last row) and store nothing.
struct BandPoint {
  long long idx;
  bool valid;
};

__device__ __forceinline__ BandPoint band_point(const SolveParams& p, long long band, int i, int ppl, int q) {
  const long long ny = p.npts / p.nx;
  long long j = band * ppl + q;
  BandPoint b;
  b.valid = j < ny;
  if (!b.valid) j = ny - 1;
  b.idx = j * p.nx + i;
  return b;
}

// TAN: the tangent form (U / cos(theta), one series); otherwise the cosine form.
template <typename R, int J, int PPL, int NS, int POL, int TAN>
__global__ void __launch_bounds__(256) midpoint_kernel(const SolveParams p) {
  constexpr int NC = NS == 5 ? 2 : 1;  // distinct stage coefficients
  constexpr int W = NS * (1 + POL);    // table values per step
  constexpr bool kRenorm = sizeof(R) == 4 || TAN;  // renormalise every kRenormEvery steps
  constexpr int kUnroll = NS == 1 ? 4 : 1;
  // p.first counts lanes here: lane -> (band of rows, column)
  long long lane = p.first + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long bands = (p.npts / p.nx + PPL - 1) / PPL;
  if (lane >= bands * p.nx) lane = bands * p.nx - 1;  // tail lanes recompute a valid lane's points
  const long long band = lane / p.nx;
  const int col = (int)(lane - band * p.nx);
  const bool lane_valid = p.first + (long long)blockIdx.x * blockDim.x + threadIdx.x < bands * p.nx;
  const double px = p.px_min + (double)col * p.dx;
  R a1[PPL], b1[PPL], a2[PPL], b2[PPL];
  double X0[NC], Y0[NC][PPL], Y2[NC][PPL];
#pragma unroll
  for (int m = 0; m < NC; ++m) X0[m] = p.hx[m] * px;  // vsign c dt px, shared by the lane's points
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    const long long idx = band_point(p, band, col, PPL, q).idx;
    const double py = p.py_min + (double)(idx / p.nx) * p.dy;
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      Y0[m][q] = p.hx[m] * py;
      Y2[m][q] = Y0[m][q] * Y0[m][q];
    }
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      a1[q] = st[idx];
      b1[q] = st[p.npts + idx];
      a2[q] = st[2 * p.npts + idx];
      b2[q] = st[3 * p.npts + idx];
    } else {
      // v_in = (-Px + i Py, E) / (sqrt(2) E) (Sec. II, Eq. (3), unit norm); the K-
      // spinor of Eq. (4) is the same with P -> -P
      double Px = p.vsign * (px + p.A_in), Py = p.vsign * (py + p.Ay_in);
      double E = sqrt(Px * Px + Py * Py);
      double d = 1.4142135623730951 * E;
      bool ok = E > 0.0;
      a1[q] = ok ? (R)(-Px / d) : (R)0;
      b1[q] = ok ? (R)(Py / d) : (R)0;
      a2[q] = ok ? (R)(E / d) : (R)0;
      b2[q] = (R)0;
    }
  }
  const double* __restrict__ tab = static_cast<const double*>(p.table);
  long long k = p.k_begin;
  while (k < p.k_end) {
    long long seg = p.k_end;
    if (kRenorm) {
      long long next = (k / kRenormEvery + 1) * kRenormEvery;
      seg = next < p.k_end ? next : p.k_end;
    }
    // one step: the stages of table row `row` (W values)
    auto one_step = [&](const double* row) {
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const double d = row[j];
        const double dy = POL ? row[NS + j] : 0.0;
        const double X = X0[mcls<NS>(j)] + d;  // vsign c dt (px + A_x), FP64 in both forms, once per lane
        const float Xs = (float)X;              // its FP32 rounding (FP32 tangent form)
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          double Y = POL ? Y0[mcls<NS>(j)][q] + dy : Y0[mcls<NS>(j)][q];
          if constexpr (TAN && sizeof(R) == 4) {
            // the series is evaluated in FP32, so (c dt E)^2 is formed from the rounded
            // phases (a relative error of the size of the coefficient's own rounding)
            float Xr = Xs, Yr = (float)Y;
            float x = POL ? fmaf(Xr, Xr, Yr * Yr) : fmaf(Xr, Xr, (float)Y2[mcls<NS>(j)][q]);
            float t1 = TanSeries<J>::minus1(x);  // tan(c dt E) / (c dt E) - 1
            midpoint_update_tan(a1[q], b1[q], a2[q], b2[q], fmaf(t1, Xr, Xr), fmaf(t1, Yr, Yr));
          } else if constexpr (TAN) {
            double x = POL ? fma(X, X, Y * Y) : fma(X, X, Y2[mcls<NS>(j)][q]);
            double t1 = TanSeries<J>::minus1(x);
            midpoint_update_tan(a1[q], b1[q], a2[q], b2[q], fma(t1, X, X), fma(t1, Y, Y));
          } else {
            double x = POL ? fma(X, X, Y * Y) : fma(X, X, Y2[mcls<NS>(j)][q]);  // (c dt E)^2
            R xr = (R)x;
            R h = Taylor<J>::h(xr);
            R sp = Taylor<J>::s(xr);  // sin(c dt E) / (c dt E)
            R al = sp * (R)X, be = sp * (R)Y;
            midpoint_update(a1[q], b1[q], a2[q], b2[q], h, al, be);
          }
        }
      }
    };
    if constexpr (NS == 1) {
      // groups of kUnroll steps as in the Strang kernel: a 32-bit trip count (a scalar
      // loop test) and two row sets in turn, each loaded right after the other set's
      // first step and pinned there, so its latency is hidden behind that set's other
      // steps; the clamped index re-reads the last group instead of branching
      constexpr int kG = kUnroll, kV = kUnroll * W;
      while (k + kG <= seg) {
        const long long left = (seg - k) / kG;
        const int n = left < (1 << 30) ? (int)left : (1 << 30);
        const double* __restrict__ g = tab + k * W;
        double ra[kV], rb[kV];
#pragma unroll
        for (int u = 0; u < kV; ++u) ra[u] = g[u];
        int i = 0;
        for (; i + 1 < n; i += 2) {
          one_step(ra);
          __builtin_amdgcn_sched_barrier(0);
          const double* __restrict__ gb = g + (long long)(i + 1) * kV;
#pragma unroll
          for (int u = 0; u < kV; ++u) rb[u] = gb[u];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 1; u < kG; ++u) one_step(ra + u * W);
          one_step(rb);
          __builtin_amdgcn_sched_barrier(0);
          const double* __restrict__ ga = g + (long long)(i + 2 < n ? i + 2 : n - 1) * kV;
#pragma unroll
          for (int u = 0; u < kV; ++u) ra[u] = ga[u];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 1; u < kG; ++u) one_step(rb + u * W);
        }
        if (i < n) {
#pragma unroll
          for (int u = 0; u < kG; ++u) one_step(ra + u * W);
        }
        k += (long long)n * kG;
      }
    }
#pragma unroll kUnroll
    for (; k < seg; ++k) one_step(tab + k * W);
    if (kRenorm && (k % kRenormEvery) == 0 && k < p.n_steps) {
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        double A1 = a1[q], B1 = b1[q], A2 = a2[q], B2 = b2[q];
        double nr = sqrt(A1 * A1 + B1 * B1 + A2 * A2 + B2 * B2);
        if (nr > 0.0) {
          a1[q] = (R)(A1 / nr);
          b1[q] = (R)(B1 / nr);
          a2[q] = (R)(A2 / nr);
          b2[q] = (R)(B2 / nr);
        }
      }
    }
  }
  if (p.k_end == p.n_steps) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      const BandPoint b = band_point(p, band, col, PPL, q);
      PointCoords c = coords(p, b.idx);
      double Pxi = c.px + p.A_in, Pyi = c.py + p.Ay_in;
      double Pxo = p.vsign * (c.px + p.A_out), Pyo = p.vsign * (c.py + p.Ay_out);
      double Ei = sqrt(Pxi * Pxi + Pyi * Pyi), Eo = sqrt(Pxo * Pxo + Pyo * Pyo);
      double A1 = a1[q], B1 = b1[q], A2 = a2[q], B2 = b2[q];
      double n = 0.0;
      if (Ei > 0.0 && Eo > 0.0) {
        // u_out = (E, Px + i Py) / (sqrt(2) E):  sqrt(2) E amp = (E a1 + Px a2 + Py b2) + i (E b1 + Px b2 - Py a2)
        double re = (Eo * A1 + Pxo * A2) + Pyo * B2;
        double im = (Eo * B1 + Pxo * B2) - Pyo * A2;
        n = (re * re + im * im) / (2.0 * Eo * Eo);
        if (kRenorm) n = n / (A1 * A1 + B1 * B1 + A2 * A2 + B2 * B2);
      }
      if (lane_valid && b.valid) p.n_out[b.idx] = n;
    }
  } else if (p.store_state) {
    R* st = static_cast<R*>(p.state);
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      const BandPoint b = band_point(p, band, col, PPL, q);
      if (lane_valid && b.valid) {
        st[b.idx] = a1[q];
        st[p.npts + b.idx] = b1[q];
        st[2 * p.npts + b.idx] = a2[q];
        st[3 * p.npts + b.idx] = b2[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Snapshots: the state after k steps (in the state buffer, or v_in at k = 0)
// projected on the positive-energy state of sigma.(p + A(t_k)).

template <typename R, int POL>
__global__ void __launch_bounds__(256) strang_snapshot_kernel(const SolveParams p, const SnapshotParams s,
                                                              int half_offset, int row_stride) {
  const long long idx = p.first + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.npts) return;
  PointCoords c = coords(p, idx);
  double Pxi = c.px + p.A_in, Pyi = c.py + p.Ay_in;
  double Px = c.px + s.Ax, Py = c.py + s.Ay;
  double Ei = sqrt(Pxi * Pxi + Pyi * Pyi), E = sqrt(Px * Px + Py * Py);
  double n = 0.0;
  if (Ei > 0.0 && E > 0.0) {
    double X, Y, Z;
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      R x = st[idx], y = st[p.npts + idx], z = st[2 * p.npts + idx];
      // the stored state is ahead by the opening half step of step k: undo it
      // (field part first, then the per-point part, each by its inverse rotation)
      const R* rowc = static_cast<const R*>(p.row_coef);
      R ha = rowc[(size_t)row_stride * c.j + half_offset], hs = rowc[(size_t)row_stride * c.j + half_offset + 1];
      if (POL) {
        if (p.form == kFormShear)
          rotate_shear(z, x, (R)s.undo_a, (R)s.undo_s);
        else
          rotate_versine(z, x, (R)s.undo_a, (R)s.undo_s);
      }
      if (p.form == kFormShear)
        rotate_shear(z, x, -ha, -hs);
      else
        rotate_versine(z, x, ha, -hs);
      X = x;
      Y = y;
      Z = z;
    } else {
      X = -p.vsign * Pxi / Ei;
      Y = -p.vsign * Pyi / Ei;
      Z = 0.0;
    }
    double nr = sqrt(X * X + Y * Y + Z * Z);
    if (nr > 0.0) n = (E + p.vsign * (Px * X + Py * Y) / nr) / (2.0 * E);
  }
  p.n_out[idx] = n;
}

template <typename R>
__global__ void __launch_bounds__(256) midpoint_snapshot_kernel(const SolveParams p, const SnapshotParams s) {
  const long long idx = p.first + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.npts) return;
  PointCoords c = coords(p, idx);
  double Pxi = p.vsign * (c.px + p.A_in), Pyi = p.vsign * (c.py + p.Ay_in);
  double Px = p.vsign * (c.px + s.Ax), Py = p.vsign * (c.py + s.Ay);
  double Ei = sqrt(Pxi * Pxi + Pyi * Pyi), E = sqrt(Px * Px + Py * Py);
  double n = 0.0;
  if (Ei > 0.0 && E > 0.0) {
    double A1, B1, A2, B2;
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      A1 = st[idx];
      B1 = st[p.npts + idx];
      A2 = st[2 * p.npts + idx];
      B2 = st[3 * p.npts + idx];
    } else {
      double d = 1.4142135623730951 * Ei;
      A1 = -Pxi / d;
      B1 = Pyi / d;
      A2 = Ei / d;
      B2 = 0.0;
    }
    double re = (E * A1 + Px * A2) + Py * B2;
    double im = (E * B1 + Px * B2) - Py * A2;
    n = (re * re + im * im) / (2.0 * E * E) / (A1 * A1 + B1 * B1 + A2 * A2 + B2 * B2);
  }
  p.n_out[idx] = n;
}

// ---------------------------------------------------------------------------
// Density: rho = scale * sum n, in a fixed order that depends only on npts.

constexpr int kRedThreads = 256;
constexpr int kRedPerThread = 8;
constexpr long long kRedTile = (long long)kRedThreads * kRedPerThread;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wave_part[kRedThreads / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wave_part[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kRedThreads / 64; ++w) s += wave_part[w];
  }
  return s;
}

// Sum of tile `tile` of n (2048 points), valid in thread 0.
__device__ __forceinline__ double tile_sum(const double* __restrict__ n, long long npts, long long tile) {
  const long long base = tile * kRedTile + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kRedPerThread; ++q) {
    long long i = base + (long long)q * kRedThreads;
    if (i < npts) s += n[i];
  }
  return block_sum(s);
}

// Sum of the tile partials, valid in thread 0.
__device__ __forceinline__ double partials_sum(const double* __restrict__ partial, long long count) {
  double s = 0.0;
  for (long long i = threadIdx.x; i < count; i += kRedThreads) s += partial[i];
  return block_sum(s);
}

__global__ void __launch_bounds__(kRedThreads) density_tiles(const double* __restrict__ n, long long npts,
                                                             double* __restrict__ partial) {
  double s = tile_sum(n, npts, blockIdx.x);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) density_finish(const double* __restrict__ partial, long long count,
                                                              double scale, double* __restrict__ rho) {
  double s = partials_sum(partial, count);
  if (threadIdx.x == 0) *rho = scale * s;
}

// Batched densities: the tiles of every job in one launch (block -> job by
// binary search over the jobs' first tiles), then one block per job.
__global__ void __launch_bounds__(kRedThreads) batch_density_tiles(const DensityJob* __restrict__ jobs, int n_jobs) {
  const long long b = blockIdx.x;
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (jobs[mid].tile_begin <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const DensityJob& j = jobs[lo];
  const long long tile = b - j.tile_begin;
  double s = tile_sum(j.n, j.npts, tile);
  if (threadIdx.x == 0) j.partial[tile] = s;
}

__global__ void __launch_bounds__(kRedThreads) batch_density_finish(const DensityJob* __restrict__ jobs) {
  const DensityJob& j = jobs[blockIdx.x];
  double s = partials_sum(j.partial, (j.npts + kRedTile - 1) / kRedTile);
  if (threadIdx.x == 0) {
    *j.rho = j.scale * s;
    if (j.rho_copy) *j.rho_copy = j.scale * s;
  }
}

// A dispatch packet holds a grid's size in work-items in 32 bits, so one launch
// covers at most kMaxLanes lanes; a larger grid (up to 65536 x 65536 points at one
// point per lane) runs as consecutive launches over point ranges, each starting at
// a multiple of the block's span, so every point sees the same tile as in one launch.
constexpr long long kMaxLanes = 1LL << 31;

// Launch `launch(q, blocks)` over the grid in slices of at most kMaxLanes lanes,
// q.first being the slice's first point.
template <typename F>
hipError_t sliced_launch(const SolveParams& p, int block, int ppl, F launch) {
  const long long span = (long long)block * ppl;
  const long long blocks = (p.npts + span - 1) / span;
  const long long max_blocks = kMaxLanes / block;
  SolveParams q = p;
  for (long long b0 = 0; b0 < blocks; b0 += max_blocks) {
    q.first = b0 * span;
    launch(q, (unsigned)(blocks - b0 < max_blocks ? blocks - b0 : max_blocks));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename R, int PPL, int FORM, int NS, int POL, int SH>
hipError_t launch_strang(int block, const SolveParams& p, hipStream_t stream) {
  if (p.stage == 1) {
    const size_t lds = (size_t)p.chunk_steps * BlochLanes<R, PPL, FORM, NS, POL, SH>::kRow * sizeof(R);
    return sliced_launch(p, block, PPL, [&](const SolveParams& q, unsigned nb) {
      hipLaunchKernelGGL((strang_kernel<R, PPL, 1, FORM, NS, POL, SH>), dim3(nb), dim3(block), lds, stream, q);
    });
  }
  return sliced_launch(p, block, PPL, [&](const SolveParams& q, unsigned nb) {
    hipLaunchKernelGGL((strang_kernel<R, PPL, 0, FORM, NS, POL, SH>), dim3(nb), dim3(block), 0, stream, q);
  });
}

template <typename R, int FORM, int NS, int POL, int SH>
hipError_t strang_ppl(int ppl, int block, const SolveParams& p, hipStream_t stream) {
  switch (ppl) {
    case 1: return launch_strang<R, 1, FORM, NS, POL, SH>(block, p, stream);
    case 2: return launch_strang<R, 2, FORM, NS, POL, SH>(block, p, stream);
    default: return launch_strang<R, 4, FORM, NS, POL, SH>(block, p, stream);
  }
}

template <typename R, int FORM, int SH>
hipError_t strang_variant(int stages, int elliptic, int ppl, int block, const SolveParams& p, hipStream_t stream) {
  if (stages == 5)
    return elliptic ? strang_ppl<R, FORM, 5, 1, SH>(ppl, block, p, stream)
                    : strang_ppl<R, FORM, 5, 0, SH>(ppl, block, p, stream);
  return elliptic ? strang_ppl<R, FORM, 1, 1, SH>(ppl, block, p, stream)
                  : strang_ppl<R, FORM, 1, 0, SH>(ppl, block, p, stream);
}

// The midpoint kernel's lanes cover bands of PPL rows column by column (band_point):
// ceil(ny / PPL) * nx lanes, launched in slices of at most kMaxLanes, q.first being
// the slice's first lane.
template <typename R, int J, int PPL, int NS, int POL, int TAN>
hipError_t launch_midpoint(int block, const SolveParams& p, hipStream_t stream) {
  const long long lanes = (p.npts / p.nx + PPL - 1) / PPL * p.nx;
  const long long blocks = (lanes + block - 1) / block;
  const long long max_blocks = kMaxLanes / block;
  SolveParams q = p;
  for (long long b0 = 0; b0 < blocks; b0 += max_blocks) {
    q.first = b0 * block;
    const unsigned nb = (unsigned)(blocks - b0 < max_blocks ? blocks - b0 : max_blocks);
    hipLaunchKernelGGL((midpoint_kernel<R, J, PPL, NS, POL, TAN>), dim3(nb), dim3(block), 0, stream, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename R, int J, int NS, int POL, int TAN>
hipError_t midpoint_ppl(int ppl, int block, const SolveParams& p, hipStream_t stream) {
  switch (ppl) {
    case 1: return launch_midpoint<R, J, 1, NS, POL, TAN>(block, p, stream);
    case 2: return launch_midpoint<R, J, 2, NS, POL, TAN>(block, p, stream);
    default: return launch_midpoint<R, J, 4, NS, POL, TAN>(block, p, stream);
  }
}

template <typename R, int J, int TAN>
hipError_t midpoint_variant(int stages, int elliptic, int ppl, int block, const SolveParams& p, hipStream_t stream) {
  if (stages == 5)
    return elliptic ? midpoint_ppl<R, J, 5, 1, TAN>(ppl, block, p, stream)
                    : midpoint_ppl<R, J, 5, 0, TAN>(ppl, block, p, stream);
  return elliptic ? midpoint_ppl<R, J, 1, 1, TAN>(ppl, block, p, stream)
                  : midpoint_ppl<R, J, 1, 0, TAN>(ppl, block, p, stream);
}

}  // namespace

size_t state_values_per_point(int scheme) { return base_scheme(scheme) == PD_SCHEME_MIDPOINT ? 4 : 3; }

long long density_partials(long long npts) { return (npts + kRedTile - 1) / kRedTile; }

hipError_t launch_propagate(int scheme, int precision, int ppl, int block, int taylor, int elliptic,
                            const SolveParams& p, hipStream_t stream) {
  const int S = (scheme == PD_SCHEME_STRANG4 || scheme == PD_SCHEME_MIDPOINT4) ? 5 : 1;
  if (base_scheme(scheme) == PD_SCHEME_STRANG) {
    if (precision == PD_FP32)
      return p.form == kFormShear ? strang_variant<float, kFormShear, kShearOnce>(S, elliptic, ppl, block, p, stream)
                                  : strang_variant<float, kFormVersine, kShearPlain>(S, elliptic, ppl, block, p, stream);
    if (precision == PD_FP32_FAST)
      return p.form == kFormShear ? strang_variant<float, kFormShear, kShearAlt>(S, elliptic, ppl, block, p, stream)
                                  : strang_variant<float, kFormVersine, kShearPlain>(S, elliptic, ppl, block, p, stream);
    return p.form == kFormShear ? strang_variant<double, kFormShear, kShearPlain>(S, elliptic, ppl, block, p, stream)
                                : strang_variant<double, kFormVersine, kShearPlain>(S, elliptic, ppl, block, p, stream);
  }
  // series orders: those taylor_order() chooses from
  if (p.form == kMidTangent) {
    if (is_fp32(precision)) {
      switch (taylor) {
        case 2: return midpoint_variant<float, 2, 1>(S, elliptic, ppl, block, p, stream);
        case 3: return midpoint_variant<float, 3, 1>(S, elliptic, ppl, block, p, stream);
        default: return midpoint_variant<float, 5, 1>(S, elliptic, ppl, block, p, stream);
      }
    }
    switch (taylor) {
      case 5: return midpoint_variant<double, 5, 1>(S, elliptic, ppl, block, p, stream);
      case 7: return midpoint_variant<double, 7, 1>(S, elliptic, ppl, block, p, stream);
      default: return midpoint_variant<double, 10, 1>(S, elliptic, ppl, block, p, stream);
    }
  }
  if (is_fp32(precision)) {
    switch (taylor) {
      case 3: return midpoint_variant<float, 3, 0>(S, elliptic, ppl, block, p, stream);
      case 5: return midpoint_variant<float, 5, 0>(S, elliptic, ppl, block, p, stream);
      default: return midpoint_variant<float, 9, 0>(S, elliptic, ppl, block, p, stream);
    }
  }
  switch (taylor) {
    case 5: return midpoint_variant<double, 5, 0>(S, elliptic, ppl, block, p, stream);
    case 8: return midpoint_variant<double, 8, 0>(S, elliptic, ppl, block, p, stream);
    default: return midpoint_variant<double, 14, 0>(S, elliptic, ppl, block, p, stream);
  }
}

hipError_t launch_snapshot(int scheme, int precision, int elliptic, const SolveParams& p, const SnapshotParams& q,
                           hipStream_t stream) {
  return sliced_launch(p, 256, 1, [&](const SolveParams& ps, unsigned nb) {
    if (base_scheme(scheme) == PD_SCHEME_STRANG) {
      // per row: (stage classes) x (coefficient phases) pairs, then the half-step pair
      const int classes = scheme == PD_SCHEME_STRANG4 ? 2 : 1;
      const int half_offset = 2 * classes * coefficient_phases(precision), row_stride = half_offset + 2;
      if (is_fp32(precision)) {
        if (elliptic)
          hipLaunchKernelGGL((strang_snapshot_kernel<float, 1>), dim3(nb), dim3(256), 0, stream, ps, q, half_offset,
                             row_stride);
        else
          hipLaunchKernelGGL((strang_snapshot_kernel<float, 0>), dim3(nb), dim3(256), 0, stream, ps, q, half_offset,
                             row_stride);
      } else {
        if (elliptic)
          hipLaunchKernelGGL((strang_snapshot_kernel<double, 1>), dim3(nb), dim3(256), 0, stream, ps, q, half_offset,
                             row_stride);
        else
          hipLaunchKernelGGL((strang_snapshot_kernel<double, 0>), dim3(nb), dim3(256), 0, stream, ps, q, half_offset,
                             row_stride);
      }
    } else if (is_fp32(precision)) {
      hipLaunchKernelGGL((midpoint_snapshot_kernel<float>), dim3(nb), dim3(256), 0, stream, ps, q);
    } else {
      hipLaunchKernelGGL((midpoint_snapshot_kernel<double>), dim3(nb), dim3(256), 0, stream, ps, q);
    }
  });
}

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation density (pd_density_static): the tile partials
// of one reduction, then its sum.  Each device holds its own copy until the process
// ends; every call on a device shares it.

static_assert(kRedTile * kStaticPartials == kStaticMaxPoints, "static scratch sized for the reduction's tiles");
static __device__ __align__(256) double scratch[kStaticPartials + 1];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    // the array's device address, looked up once per device with that device current
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_density(const double* n, long long npts, double scale, double* partial, double* rho,
                          hipStream_t stream) {
  long long tiles = density_partials(npts);
  hipLaunchKernelGGL(density_tiles, dim3((unsigned)tiles), dim3(kRedThreads), 0, stream, n, npts, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(density_finish, dim3(1), dim3(kRedThreads), 0, stream, partial, tiles, scale, rho);
  return hipGetLastError();
}

hipError_t launch_batch_density(const DensityJob* jobs, int n_jobs, long long total_tiles, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_density_tiles, dim3((unsigned)total_tiles), dim3(kRedThreads), 0, stream, jobs, n_jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_density_finish, dim3((unsigned)n_jobs), dim3(kRedThreads), 0, stream, jobs);
  return hipGetLastError();
}

hipError_t launch_batch(int ppl, int block, int grid_blocks, const BatchSolve* solves, const BatchItem* items,
                        int n_items, unsigned int* counter, hipStream_t stream) {
  hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (ppl) {
    case 1:
      hipLaunchKernelGGL(batch_kernel<1>, dim3(grid_blocks), dim3(block), 0, stream, solves, items, n_items, counter);
      break;
    case 2:
      hipLaunchKernelGGL(batch_kernel<2>, dim3(grid_blocks), dim3(block), 0, stream, solves, items, n_items, counter);
      break;
    default:
      hipLaunchKernelGGL(batch_kernel<4>, dim3(grid_blocks), dim3(block), 0, stream, solves, items, n_items, counter);
      break;
  }
  return hipGetLastError();
}

int batch_blocks_per_cu(int ppl, int block) {
  int n = 0;
  hipError_t e;
  switch (ppl) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<1>, block, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<2>, block, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<4>, block, 0); break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace pdx
