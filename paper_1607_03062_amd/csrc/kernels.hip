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
// in versine form with h = cos(phi) - 1 and s = sin(phi).
// The projection on u_out is n = |u_out^dagger psi|^2 = (1 + r.r_u) / 2 with
// r_u = P_out / |P_out| the Bloch vector of u_out (Sec. II, Eqs. (1), (3)); r
// is normalised first (the exact steps are unitary, Sec. III).
//
// Midpoint scheme (Sec. III, Eq. (13)): per step the closed 2x2 form
//   U = cos(dt E) I - i sigma.P sin(dt E) / E,  P = p + A_k,
// acting on the spinor (a1 + i b1, a2 + i b2); cos - 1 and sin(x)/x are even
// Taylor series in x = (dt E)^2 of an order chosen by the host.
#include <hip/hip_runtime.h>

#include "pd_internal.h"

namespace pdx {
namespace {

constexpr long long kRenormEvery = 1024;  // FP32 form: renormalise after every 1024th step

// Two coefficients of a plane rotation: (tan(phi/2), sin(phi)) in the shear
// form, (cos(phi) - 1, sin(phi)) in the versine form.
template <typename R>
struct Row {
  R a, s;
};

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

// The Bloch vectors of a lane's points and their per-point rotations.
template <typename R, int PPL, int FORM>
struct BlochLanes {
  R x[PPL], y[PPL], z[PPL];
  R aX[PPL], sX[PPL], aY[PPL], sY[PPL];  // rotations by 2 dt px about x and 2 dt py about y

  // one merged Strang step: rotation by 2 dt A_k about x (table row), by
  // 2 dt px about x, and by 2 dt py about y
  __device__ __forceinline__ void step(R a, R s) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      rotate<FORM>(y[q], z[q], a, s);
      rotate<FORM>(y[q], z[q], aX[q], sX[q]);
      rotate<FORM>(z[q], x[q], aY[q], sY[q]);
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

// Steps [k, k_full) with the table rows read by the scalar unit (SGPR operands).
template <typename R, int PPL, int FORM>
__device__ __forceinline__ void steps_scalar(BlochLanes<R, PPL, FORM>& L, const Row<R>* __restrict__ tab,
                                             long long k, long long k_full) {
  while (k < k_full) {
    long long seg = k_full;
    if (sizeof(R) == 4) {
      long long next = (k / kRenormEvery + 1) * kRenormEvery;
      seg = next < k_full ? next : k_full;
    }
    constexpr int kGroup = 8;  // rows fetched together by one scalar load
    for (; k + kGroup <= seg; k += kGroup) {
      Row<R> r[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) r[u] = tab[k + u];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) L.step(r[u].a, r[u].s);
    }
    for (; k < seg; ++k) {
      const Row<R> r = tab[k];
      L.step(r.a, r.s);
    }
    if (sizeof(R) == 4 && (k % kRenormEvery) == 0) L.renormalise();
  }
}

// Steps [k, k_full) with the table staged through LDS in chunks of `chunk` rows
// (absolute chunk boundaries; a power of two dividing the renormalisation period
// in the FP32 form), so every lane reads its rotation from VGPRs.
template <typename R, int PPL, int FORM>
__device__ __forceinline__ void steps_lds(BlochLanes<R, PPL, FORM>& L, const Row<R>* __restrict__ tab, long long k,
                                          long long k_full, long long chunk) {
  extern __shared__ unsigned char pd_lds[];
  Row<R>* rows = reinterpret_cast<Row<R>*>(pd_lds);
  while (k < k_full) {
    long long cend = (k / chunk + 1) * chunk;
    if (cend > k_full) cend = k_full;
    const int cnt = (int)(cend - k);
    __syncthreads();  // every wave has finished with the previous chunk
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) rows[t] = tab[k + t];
    __syncthreads();
#pragma unroll 8
    for (int t = 0; t < cnt; ++t) {
      const Row<R> r = rows[t];
      L.step(r.a, r.s);
    }
    k = cend;
    if (sizeof(R) == 4 && (k % kRenormEvery) == 0) L.renormalise();
  }
}

// One tile of a Strang solve: the block's lanes own points base + q * blockDim.x,
// q < PPL; steps [p.k_begin, p.k_end).
template <typename R, int PPL, int STAGE, int FORM>
__device__ __forceinline__ void strang_tile(const SolveParams& p, const long long base) {
  const R* __restrict__ colc = static_cast<const R*>(p.col_coef);
  const R* __restrict__ rowc = static_cast<const R*>(p.row_coef);
  BlochLanes<R, PPL, FORM> L;

#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    long long idx = base + (long long)q * blockDim.x;
    if (idx >= p.npts) idx = p.npts - 1;  // tail lanes recompute a valid point and store nothing
    PointCoords c = coords(p, idx);
    L.aX[q] = colc[2 * c.i];
    L.sX[q] = colc[2 * c.i + 1];
    L.aY[q] = rowc[4 * c.j];
    L.sY[q] = rowc[4 * c.j + 1];
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      L.x[q] = st[idx];
      L.y[q] = st[p.npts + idx];
      L.z[q] = st[2 * p.npts + idx];
    } else {
      // v_in: negative-energy eigenvector of sigma.P_in, Bloch vector -P_in/|P_in|
      double Px = c.px + p.A_in;
      double E = sqrt(Px * Px + c.py * c.py);
      double rx = 0.0, ry = 0.0;
      if (E > 0.0) {
        rx = -Px / E;
        ry = -c.py / E;
      }
      L.x[q] = (R)rx;
      L.y[q] = (R)ry;
      L.z[q] = (R)0;
      // first half step exp(-i dt py sy / 2): rotation by dt py about y
      rotate<FORM>(L.z[q], L.x[q], rowc[4 * c.j + 2], rowc[4 * c.j + 3]);
    }
  }

  const Row<R>* __restrict__ tab = static_cast<const Row<R>*>(p.table);
  const long long k_full = p.k_end < p.n_steps ? p.k_end : p.n_steps - 1;
  if (STAGE == 1)
    steps_lds(L, tab, p.k_begin, k_full, p.chunk_steps);
  else
    steps_scalar(L, tab, p.k_begin, k_full);

  if (p.k_end == p.n_steps) {
    // last step: full sigma_x factor, then the closing half step about y
    const Row<R> r = tab[p.n_steps - 1];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      long long idx = base + (long long)q * blockDim.x;
      bool valid = idx < p.npts;
      if (!valid) idx = p.npts - 1;
      PointCoords c = coords(p, idx);
      rotate<FORM>(L.y[q], L.z[q], r.a, r.s);
      rotate<FORM>(L.y[q], L.z[q], L.aX[q], L.sX[q]);
      rotate<FORM>(L.z[q], L.x[q], rowc[4 * c.j + 2], rowc[4 * c.j + 3]);
      // projection on u_out: n = (1 + r.P_out / |P_out|) / 2 with r normalised
      double Pxi = c.px + p.A_in, Pxo = c.px + p.A_out;
      double Ei = sqrt(Pxi * Pxi + c.py * c.py), Eo = sqrt(Pxo * Pxo + c.py * c.py);
      double X = L.x[q], Y = L.y[q], Z = L.z[q];
      double nr = sqrt(X * X + Y * Y + Z * Z);
      double n = 0.0;
      if (Ei > 0.0 && Eo > 0.0 && nr > 0.0) {
        double dot = (Pxo * X + c.py * Y) / nr;
        n = (Eo + dot) / (2.0 * Eo);
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

template <typename R, int PPL, int STAGE, int FORM>
__global__ void __launch_bounds__(256) strang_kernel(const SolveParams p) {
  strang_tile<R, PPL, STAGE, FORM>(p, (long long)blockIdx.x * blockDim.x * PPL + threadIdx.x);
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
        strang_tile<float, PPL, 0, kFormShear>(s.p, base);
      else
        strang_tile<float, PPL, 0, kFormVersine>(s.p, base);
    } else {
      if (s.form == kFormShear)
        strang_tile<double, PPL, 0, kFormShear>(s.p, base);
      else
        strang_tile<double, PPL, 0, kFormVersine>(s.p, base);
    }
  }
}

// ---------------------------------------------------------------------------
// Midpoint scheme: spinor state, Taylor coefficients per point and step.

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

template <typename R, int J, int PPL>
__global__ void __launch_bounds__(256) midpoint_kernel(const SolveParams p) {
  const long long base = (long long)blockIdx.x * blockDim.x * PPL + threadIdx.x;
  R a1[PPL], b1[PPL], a2[PPL], b2[PPL];
  double X0[PPL], Y[PPL], Y2[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    long long idx = base + (long long)q * blockDim.x;
    if (idx >= p.npts) idx = p.npts - 1;
    PointCoords c = coords(p, idx);
    X0[q] = p.dt * c.px;
    Y[q] = p.dt * c.py;
    Y2[q] = Y[q] * Y[q];
    if (p.load_state) {
      const R* st = static_cast<const R*>(p.state);
      a1[q] = st[idx];
      b1[q] = st[p.npts + idx];
      a2[q] = st[2 * p.npts + idx];
      b2[q] = st[3 * p.npts + idx];
    } else {
      // v_in = (-Px + i py, E) / (sqrt(2) E)   (Sec. II, Eq. (3), unit norm)
      double Px = c.px + p.A_in;
      double E = sqrt(Px * Px + c.py * c.py);
      double d = 1.4142135623730951 * E;
      bool ok = E > 0.0;
      a1[q] = ok ? (R)(-Px / d) : (R)0;
      b1[q] = ok ? (R)(c.py / d) : (R)0;
      a2[q] = ok ? (R)(E / d) : (R)0;
      b2[q] = (R)0;
    }
  }
  const double* __restrict__ tab = static_cast<const double*>(p.table);
  long long k = p.k_begin;
  while (k < p.k_end) {
    long long seg = p.k_end;
    if (sizeof(R) == 4) {
      long long next = (k / kRenormEvery + 1) * kRenormEvery;
      seg = next < p.k_end ? next : p.k_end;
    }
#pragma unroll 4
    for (; k < seg; ++k) {
      const double d = tab[k];
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        double X = X0[q] + d;           // dt (px + A_k), FP64 in both forms
        double x = fma(X, X, Y2[q]);    // (dt E)^2
        R xr = (R)x;
        R h = Taylor<J>::h(xr);
        R sp = Taylor<J>::s(xr);        // sin(dt E) / (dt E)
        R al = sp * (R)X, be = sp * (R)Y[q];
        midpoint_update(a1[q], b1[q], a2[q], b2[q], h, al, be);
      }
    }
    if (sizeof(R) == 4 && (k % kRenormEvery) == 0 && k < p.n_steps) {
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
      long long idx = base + (long long)q * blockDim.x;
      bool valid = idx < p.npts;
      if (!valid) idx = p.npts - 1;
      PointCoords c = coords(p, idx);
      double Pxi = c.px + p.A_in, Pxo = c.px + p.A_out;
      double Ei = sqrt(Pxi * Pxi + c.py * c.py), Eo = sqrt(Pxo * Pxo + c.py * c.py);
      double A1 = a1[q], B1 = b1[q], A2 = a2[q], B2 = b2[q];
      double n = 0.0;
      if (Ei > 0.0 && Eo > 0.0) {
        // u_out = (E, Px + i py) / (sqrt(2) E):  sqrt(2) E amp = (E a1 + Px a2 + py b2) + i (E b1 + Px b2 - py a2)
        double re = (Eo * A1 + Pxo * A2) + c.py * B2;
        double im = (Eo * B1 + Pxo * B2) - c.py * A2;
        n = (re * re + im * im) / (2.0 * Eo * Eo);
        if (sizeof(R) == 4) n = n / (A1 * A1 + B1 * B1 + A2 * A2 + B2 * B2);
      }
      if (valid) p.n_out[idx] = n;
    }
  } else if (p.store_state) {
    R* st = static_cast<R*>(p.state);
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      long long idx = base + (long long)q * blockDim.x;
      if (idx < p.npts) {
        st[idx] = a1[q];
        st[p.npts + idx] = b1[q];
        st[2 * p.npts + idx] = a2[q];
        st[3 * p.npts + idx] = b2[q];
      }
    }
  }
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

template <typename R, int PPL, int FORM>
hipError_t launch_strang(int block, const SolveParams& p, hipStream_t stream) {
  long long per_block = (long long)block * PPL;
  long long blocks = (p.npts + per_block - 1) / per_block;
  if (p.stage == 1) {
    size_t lds = (size_t)p.chunk_steps * sizeof(Row<R>);
    hipLaunchKernelGGL((strang_kernel<R, PPL, 1, FORM>), dim3((unsigned)blocks), dim3(block), lds, stream, p);
  } else {
    hipLaunchKernelGGL((strang_kernel<R, PPL, 0, FORM>), dim3((unsigned)blocks), dim3(block), 0, stream, p);
  }
  return hipGetLastError();
}

template <typename R, int FORM>
hipError_t strang_ppl(int ppl, int block, const SolveParams& p, hipStream_t stream) {
  switch (ppl) {
    case 1: return launch_strang<R, 1, FORM>(block, p, stream);
    case 2: return launch_strang<R, 2, FORM>(block, p, stream);
    default: return launch_strang<R, 4, FORM>(block, p, stream);
  }
}

template <typename R, int J, int PPL>
hipError_t launch_midpoint(int block, const SolveParams& p, hipStream_t stream) {
  long long per_block = (long long)block * PPL;
  long long blocks = (p.npts + per_block - 1) / per_block;
  hipLaunchKernelGGL((midpoint_kernel<R, J, PPL>), dim3((unsigned)blocks), dim3(block), 0, stream, p);
  return hipGetLastError();
}

template <typename R, int J>
hipError_t midpoint_ppl(int ppl, int block, const SolveParams& p, hipStream_t stream) {
  switch (ppl) {
    case 1: return launch_midpoint<R, J, 1>(block, p, stream);
    case 2: return launch_midpoint<R, J, 2>(block, p, stream);
    default: return launch_midpoint<R, J, 4>(block, p, stream);
  }
}

}  // namespace

size_t state_values_per_point(int scheme) { return scheme == PD_SCHEME_MIDPOINT ? 4 : 3; }

long long density_partials(long long npts) { return (npts + kRedTile - 1) / kRedTile; }

hipError_t launch_propagate(int scheme, int precision, int ppl, int block, int taylor, const SolveParams& p,
                            hipStream_t stream) {
  if (scheme == PD_SCHEME_STRANG) {
    if (precision == PD_FP32)
      return p.form == kFormShear ? strang_ppl<float, kFormShear>(ppl, block, p, stream)
                                  : strang_ppl<float, kFormVersine>(ppl, block, p, stream);
    return p.form == kFormShear ? strang_ppl<double, kFormShear>(ppl, block, p, stream)
                                : strang_ppl<double, kFormVersine>(ppl, block, p, stream);
  }
  if (precision == PD_FP32) {
    switch (taylor) {
      case 3: return midpoint_ppl<float, 3>(ppl, block, p, stream);
      case 5: return midpoint_ppl<float, 5>(ppl, block, p, stream);
      default: return midpoint_ppl<float, 9>(ppl, block, p, stream);
    }
  }
  switch (taylor) {
    case 5: return midpoint_ppl<double, 5>(ppl, block, p, stream);
    case 8: return midpoint_ppl<double, 8>(ppl, block, p, stream);
    default: return midpoint_ppl<double, 14>(ppl, block, p, stream);
  }
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
