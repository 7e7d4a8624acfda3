"""Precision-budget model of the FP32 form (test infrastructure, CPU only).

The FP32 form of the Strang scheme evolves each point's Bloch vector r = psi^dagger sigma psi
by plane rotations (the split steps of Sec. III, Eqs. (11)-(12): rotation by 2 dt P_x
about x, and dt p_y per half step about y, P = p + A(t_k+1/2)), with the state and the
rotation coefficients in FP32 and everything else in FP64.  This module emulates that
arithmetic in numpy float32, so that the error of the FP32 form against the FP64 oracle
can be predicted on the CPU before the kernels run:

  * coefficients t = tan(theta/2), s = sin(theta) computed in FP64 and rounded to FP32;
    the per-point ones take four FP32 values in turn (step k uses value k mod 4) whose
    mean is within 1/8 ulp of the FP64 value;
  * arrangement "once" (PD_FP32): every rotation as three shears, each state component
    rounded once per rotation (u1 = u - t v; v' = v + s u1; u' = u - t (v + v'));
    arrangement "fast" (PD_FP32_FAST): plain shears whose orientation alternates from
    step to step (u-v-u, then v-u-v), the step's two rotations about x (field part,
    then the point's part) as five shears, the middle two merged into one with the
    summed coefficient; a fused multiply-add is one rounding, emulated as an exact FP64
    product and sum rounded to FP32;
  * the state renormalised in FP64 every 1024 steps; the initial state and the
    projection n = (1 + r.P_out/|P_out|) / 2 (Sec. II, Eqs. (1), (3)) in FP64.

With arithmetic=np.float64 the same steps are evaluated in FP64 and must reproduce the
oracle to rounding; that pins the rotation sequence, angles and signs of the model.  It
imports nothing from the library; the field samples and grid nodes come from the oracle.
"""
from __future__ import annotations

import numpy as np

import oracle

F32 = np.float32
RENORM_EVERY = 1024
PHASES = 4


def _coefficients(theta):
    """(t, s) = (tan(theta/2), sin(theta)) of a rotation by theta, FP64."""
    return np.tan(0.5 * theta), np.sin(theta)


def _phases(c):
    """PHASES FP32 values per FP64 coefficient whose mean is within 1/8 ulp of it."""
    hi = c.astype(F32)
    ulp = np.spacing(np.abs(hi)).astype(np.float64)
    m = np.rint(PHASES * (c - hi.astype(np.float64)) / np.where(ulp > 0, ulp, 1.0))
    return np.stack([(hi + np.where(j < np.abs(m), np.sign(m), 0.0) * ulp).astype(F32) for j in range(PHASES)])


def _rotate(u, v, t, s, arithmetic):
    """Rotation of (u, v) by theta (u' = u cos - v sin, v' = u sin + v cos) as three shears,
    each component rounded once."""
    if arithmetic is np.float64:
        u1 = u - t * v
        v1 = v + s * u1
        return u - t * (v + v1), v1
    d = np.float64
    u1 = (d(u) - d(t) * d(v)).astype(F32)
    v1 = (d(v) + d(s) * d(u1)).astype(F32)
    w = (d(v) + d(v1)).astype(F32)
    return (d(u) - d(t) * d(w)).astype(F32), v1


def _fma(a, b, c, arithmetic):
    """a * b + c with one rounding in the given arithmetic."""
    if arithmetic is np.float64:
        return a * b + c
    return (np.float64(a) * np.float64(b) + np.float64(c)).astype(F32)


def _shears(u, v, coefs, odd, arithmetic):
    """Rotations in the (u, v) plane by the angles whose (t, s) are listed, in order, as
    plain shears; odd: v-u-v orientation.  Adjacent shears of the same component merge
    (coefficients summed, one rounding of the sum)."""
    seq = []  # (component moved: 0 = u, 1 = v, coefficient)
    for t, s in coefs:
        trip = [(1, t), (0, -s), (1, t)] if odd else [(0, -t), (1, s), (0, -t)]
        for c, k in trip:
            if seq and seq[-1][0] == c:
                summed = seq[-1][1] + k
                seq[-1] = (c, summed if arithmetic is np.float64 else summed.astype(F32))
            else:
                seq.append((c, k))
    for c, k in seq:
        if c == 0:
            u = _fma(k, v, u, arithmetic)
        else:
            v = _fma(k, u, v, arithmetic)
    return u, v


def solve_grid(field, grid, n_steps, arithmetic=F32, arrangement="once"):
    """n(p) on the grid (row-major, y rows) after n_steps second-order Strang steps in the
    given arithmetic and arrangement of the roundings; NaN where |p + A(t_i)| or
    |p + A(t_f)| is 0 (masked points)."""
    if arrangement not in ("once", "fast"):
        raise ValueError("arrangement must be 'once' or 'fast'")
    A, a_in, a_out, dt = oracle.field_table(field, n_steps)
    px = np.array([oracle.grid_p(grid["px"][0], grid["px"][1], grid["nx"], i) for i in range(grid["nx"])])
    py = np.array([oracle.grid_p(grid["py"][0], grid["py"][1], grid["ny"], j) for j in range(grid["ny"])])
    PX, PY = (a.ravel() for a in np.meshgrid(px, py))
    with np.errstate(invalid="ignore", divide="ignore"):
        e_in = np.hypot(PX + a_in, PY)
        x = (-(PX + a_in) / e_in).astype(arithmetic)  # v_in: r = -P_in / |P_in|
        y = (-PY / e_in).astype(arithmetic)
    z = np.zeros_like(x)

    def per_point(theta):
        t, s = _coefficients(theta)
        if arithmetic is np.float64:
            return np.stack([t] * PHASES), np.stack([s] * PHASES)
        return _phases(t), _phases(s)

    tx, sx = per_point(2.0 * dt * PX)  # x rotation by the point's part of 2 dt P_x
    ty, sy = per_point(2.0 * dt * PY)  # two merged half steps about y
    th, sh = (c.astype(arithmetic) for c in _coefficients(dt * PY))  # opening and closing half steps
    tf, sf = (c.astype(arithmetic) for c in _coefficients(2.0 * dt * A))  # field part, per step
    if arrangement == "fast":  # the opening half step about y
        z, x = _shears(z, x, [(th, sh)], False, arithmetic)
    else:
        z, x = _rotate(z, x, th, sh, arithmetic)
    for k in range(int(n_steps)):
        if arithmetic is not np.float64 and k > 0 and k % RENORM_EVERY == 0:
            X, Y, Z = (c.astype(np.float64) for c in (x, y, z))
            nr = np.sqrt(X * X + Y * Y + Z * Z)
            x, y, z = ((c / nr).astype(F32) for c in (X, Y, Z))
        h = k % PHASES
        yt, ys = (th, sh) if k == n_steps - 1 else (ty[h], sy[h])
        if arrangement == "fast":
            y, z = _shears(y, z, [(tf[k], sf[k]), (tx[h], sx[h])], k % 2 == 1, arithmetic)
            z, x = _shears(z, x, [(yt, ys)], k % 2 == 1, arithmetic)
            continue
        y, z = _rotate(y, z, tf[k], sf[k], arithmetic)
        y, z = _rotate(y, z, tx[h], sx[h], arithmetic)
        z, x = _rotate(z, x, yt, ys, arithmetic)
    X, Y, Z = (c.astype(np.float64) for c in (x, y, z))
    with np.errstate(invalid="ignore", divide="ignore"):
        return 0.5 * (1.0 + (X * (PX + a_out) + Y * PY) / (np.sqrt(X * X + Y * Y + Z * Z) * np.hypot(PX + a_out, PY)))


def error_stats(n, n_ref):
    """(max |dn|, rms |dn|) over the points both define."""
    ok = np.isfinite(n) & np.isfinite(n_ref)
    e = np.abs(n[ok] - n_ref[ok])
    return float(e.max()), float(np.sqrt(np.mean(e * e)))
