"""ctypes wrapper over ``liboracle.so`` (the plain FP64 C oracle).

Test infrastructure only.  Field and grid descriptions are plain dicts:

  field: {"kind": "sin2", "E0", "omega", "cycles"}
         {"kind": "constant", "E0", "t_end"}
         {"kind": "table", "A_mid" (array, stages * n_steps values), "t_i", "t_f", "A_in", "A_out"}
         {"kind": "pulse", "E0", "omega", "phi", "omega_rise", "omega_fall", "duration"}
         optional y component: "ellipticity" (sin2, pulse, constant), or
         "Ay_mid", "Ay_in", "Ay_out" (table)
  grid:  {"nx", "ny", "px": (min, max), "py": (min, max)}
  scheme: "strang", "midpoint" (second order) or "strang4", "midpoint4"
          (Suzuki's fourth-order composition of the same step; 5 stages)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_KINDS = {"sin2": 0, "constant": 1, "table": 2, "pulse": 3}
_SCHEMES = {"strang": (0, 2), "midpoint": (1, 2), "strang4": (0, 4), "midpoint4": (1, 4)}

_dp = ctypes.POINTER(ctypes.c_double)
_llp = ctypes.POINTER(ctypes.c_longlong)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("field_kind", ctypes.c_int),
        ("E0", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("cycles", ctypes.c_int),
        ("t_end", ctypes.c_double),
        ("A_mid", _dp),
        ("t_i", ctypes.c_double),
        ("t_f", ctypes.c_double),
        ("A_in", ctypes.c_double),
        ("A_out", ctypes.c_double),
        ("phi", ctypes.c_double),
        ("omega_rise", ctypes.c_double),
        ("omega_fall", ctypes.c_double),
        ("duration", ctypes.c_double),
        ("n_steps", ctypes.c_longlong),
        ("scheme", ctypes.c_int),
        ("valley", ctypes.c_int),
        ("order", ctypes.c_int),
        ("ellipticity", ctypes.c_double),
        ("Ay_mid", _dp),
        ("Ay_in", ctypes.c_double),
        ("Ay_out", ctypes.c_double),
    ]


def lib_path() -> str:
    return _LIB_PATH


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _configure(lib):
    P = ctypes.POINTER(_Problem)
    lib.oracle_solve_points.argtypes = [P, ctypes.c_longlong, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_solve_points.restype = ctypes.c_longlong
    lib.oracle_solve_grid.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _llp, ctypes.c_longlong, _dp, _dp,
                                      ctypes.c_int]
    lib.oracle_solve_grid.restype = ctypes.c_longlong
    lib.oracle_density.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int]
    lib.oracle_density.restype = ctypes.c_double
    lib.oracle_A.argtypes = [P, ctypes.c_double]
    lib.oracle_A.restype = ctypes.c_double
    lib.oracle_E.argtypes = [P, ctypes.c_double]
    lib.oracle_E.restype = ctypes.c_double
    lib.oracle_times.argtypes = [P, _dp, _dp]
    lib.oracle_times.restype = None
    lib.oracle_step_matrix.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp]
    lib.oracle_step_matrix.restype = None
    lib.oracle_spinors.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.oracle_spinors.restype = None
    lib.oracle_final_state.argtypes = [P, ctypes.c_double, ctypes.c_double, _dp]
    lib.oracle_final_state.restype = ctypes.c_int
    lib.oracle_grid_p.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.oracle_grid_p.restype = ctypes.c_double
    lib.oracle_field_table.argtypes = [P, _dp, _dp, _dp, _dp]
    lib.oracle_field_table.restype = ctypes.c_int
    lib.oracle_field_table_y.argtypes = [P, _dp, _dp, _dp]
    lib.oracle_field_table_y.restype = ctypes.c_int
    lib.oracle_Ay.argtypes = [P, ctypes.c_double]
    lib.oracle_Ay.restype = ctypes.c_double
    lib.oracle_Ey.argtypes = [P, ctypes.c_double]
    lib.oracle_Ey.restype = ctypes.c_double
    lib.oracle_composition.argtypes = [ctypes.c_int, _dp, _dp]
    lib.oracle_composition.restype = ctypes.c_int
    lib.oracle_step_matrix_xy.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _dp]
    lib.oracle_step_matrix_xy.restype = None
    lib.oracle_snapshot_points.argtypes = [P, ctypes.c_longlong, ctypes.c_longlong, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_snapshot_points.restype = ctypes.c_longlong
    lib.oracle_state_at.argtypes = [P, ctypes.c_longlong, ctypes.c_double, ctypes.c_double, _dp]
    lib.oracle_state_at.restype = ctypes.c_int
    lib.oracle_boundary_A.argtypes = [P, ctypes.c_longlong, _dp, _dp]
    lib.oracle_boundary_A.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


class use_library:
    """Context manager: route every call of this module to another build of the
    oracle source (used by the tests that plant a mistake in a copy of oracle.c)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _load()
        _lib = _configure(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def compile_source(src_text: str, out_path: str) -> str:
    """Compile a (possibly modified) copy of the oracle source to a shared library."""
    c_path = out_path + ".c"
    with open(c_path, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", "-o", out_path, c_path, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _problem(field: dict, n_steps: int = 1, scheme: str = "strang", valley: int = 1):
    """Build the C problem struct; returns (struct, keep-alive list)."""
    p = _Problem()
    keep = []
    kind = field["kind"]
    p.field_kind = _KINDS[kind]
    p.E0 = float(field.get("E0", 0.0))
    p.omega = float(field.get("omega", 0.0))
    p.cycles = int(field.get("cycles", 0))
    p.t_end = float(field.get("t_end", 0.0))
    sch, order = _SCHEMES[scheme]
    stages = 5 if order == 4 else 1
    if kind == "table":
        A = np.ascontiguousarray(field["A_mid"], dtype=np.float64)
        if A.shape[0] != stages * n_steps:
            raise ValueError("table field needs exactly stages * n_steps sample values")
        keep.append(A)
        p.A_mid = _ptr(A)
        p.t_i, p.t_f = float(field["t_i"]), float(field["t_f"])
        p.A_in, p.A_out = float(field["A_in"]), float(field["A_out"])
        if field.get("Ay_mid") is not None:
            Ay = np.ascontiguousarray(field["Ay_mid"], dtype=np.float64)
            if Ay.shape[0] != stages * n_steps:
                raise ValueError("table field needs exactly stages * n_steps A_y values")
            keep.append(Ay)
            p.Ay_mid = _ptr(Ay)
            p.Ay_in, p.Ay_out = float(field["Ay_in"]), float(field["Ay_out"])
    p.ellipticity = float(field.get("ellipticity", 0.0))
    p.phi = float(field.get("phi", 0.0))
    p.omega_rise = float(field.get("omega_rise", 0.0))
    p.omega_fall = float(field.get("omega_fall", 0.0))
    p.duration = float(field.get("duration", 0.0))
    p.n_steps = int(n_steps)
    p.scheme = sch
    p.order = order
    p.valley = 1 if valley >= 0 else -1
    return p, keep


def solve_points(field, px, py, n_steps, scheme="strang", valley=1, threads=0):
    """n(p) at explicit momenta.  Returns (n, |psi|^2 - 1, masked count)."""
    lib = _load()
    px = np.ascontiguousarray(px, dtype=np.float64).ravel()
    py = np.ascontiguousarray(py, dtype=np.float64).ravel()
    if px.shape != py.shape:
        raise ValueError("px and py must have the same length")
    n = np.zeros(px.shape[0])
    nd = np.zeros(px.shape[0])
    p, keep = _problem(field, n_steps, scheme, valley)
    m = lib.oracle_solve_points(ctypes.byref(p), px.shape[0], _ptr(px), _ptr(py), _ptr(n), _ptr(nd), int(threads))
    if m < 0:
        raise MemoryError("oracle allocation failed")
    return n, nd, int(m)


def solve_grid(field, grid, n_steps, scheme="strang", valley=1, idx=None, threads=0):
    """n(p) on the node grid; idx = linear indices j*nx + i (None: all, in index order)."""
    lib = _load()
    nx, ny = int(grid["nx"]), int(grid["ny"])
    (x0, x1), (y0, y1) = grid["px"], grid["py"]
    if idx is None:
        count = nx * ny
        idx_p = None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
        count = idx.shape[0]
        idx_p = idx.ctypes.data_as(_llp)
    n = np.zeros(count)
    nd = np.zeros(count)
    p, keep = _problem(field, n_steps, scheme, valley)
    m = lib.oracle_solve_grid(ctypes.byref(p), nx, ny, x0, x1, y0, y1, idx_p, count, _ptr(n), _ptr(nd),
                              int(threads))
    if m < 0:
        raise MemoryError("oracle allocation failed")
    return n, nd, int(m)


def density(grid, n, kahan=False) -> float:
    """rho = 4 dx dy / (2 pi)^2 * sum n over the full grid (index order)."""
    lib = _load()
    n = np.ascontiguousarray(n, dtype=np.float64).ravel()
    nx, ny = int(grid["nx"]), int(grid["ny"])
    if n.shape[0] != nx * ny:
        raise ValueError("density needs n on the full grid")
    (x0, x1), (y0, y1) = grid["px"], grid["py"]
    return float(lib.oracle_density(nx, ny, x0, x1, y0, y1, _ptr(n), 1 if kahan else 0))


def field_A(field, t):
    lib = _load()
    p, keep = _problem(field)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([lib.oracle_A(ctypes.byref(p), float(x)) for x in t])


def field_E(field, t):
    lib = _load()
    p, keep = _problem(field)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([lib.oracle_E(ctypes.byref(p), float(x)) for x in t])


def times(field):
    lib = _load()
    p, keep = _problem(field)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.oracle_times(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def field_Ay(field, t):
    lib = _load()
    p, keep = _problem(field)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([lib.oracle_Ay(ctypes.byref(p), float(x)) for x in t])


def field_Ey(field, t):
    lib = _load()
    p, keep = _problem(field)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([lib.oracle_Ey(ctypes.byref(p), float(x)) for x in t])


def composition(order):
    """(stage coefficients c, stage midpoints sigma) of the oracle's composition."""
    c = np.zeros(5)
    sg = np.zeros(5)
    S = _load().oracle_composition(int(order), _ptr(c), _ptr(sg))
    return c[:S].copy(), sg[:S].copy()


def field_table(field, n_steps, scheme="strang"):
    """(A_x at the sample times (stages * n_steps values), A_x(t_i), A_x(t_f), dt)."""
    lib = _load()
    p, keep = _problem(field, n_steps, scheme)
    A = np.zeros(int(n_steps) * (5 if _SCHEMES[scheme][1] == 4 else 1))
    a_in, a_out, dt = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.oracle_field_table(ctypes.byref(p), _ptr(A), ctypes.byref(a_in), ctypes.byref(a_out), ctypes.byref(dt))
    return A, a_in.value, a_out.value, dt.value


def field_table_y(field, n_steps, scheme="strang"):
    """(A_y at the sample times, A_y(t_i), A_y(t_f))."""
    lib = _load()
    p, keep = _problem(field, n_steps, scheme)
    A = np.zeros(int(n_steps) * (5 if _SCHEMES[scheme][1] == 4 else 1))
    a_in, a_out = ctypes.c_double(), ctypes.c_double()
    if lib.oracle_field_table_y(ctypes.byref(p), _ptr(A), ctypes.byref(a_in), ctypes.byref(a_out)) != 0:
        raise MemoryError("oracle allocation failed")
    return A, a_in.value, a_out.value


def boundary_A(field, n_steps, k, scheme="strang"):
    """(A_x, A_y) at the step boundary t_i + k dt."""
    lib = _load()
    p, keep = _problem(field, n_steps, scheme)
    ax, ay = ctypes.c_double(), ctypes.c_double()
    if lib.oracle_boundary_A(ctypes.byref(p), int(k), ctypes.byref(ax), ctypes.byref(ay)) != 0:
        raise MemoryError("oracle allocation failed")
    return ax.value, ay.value


def snapshot_points(field, px, py, n_steps, k_steps, scheme="strang", valley=1, threads=0):
    """Occupation of the instantaneous positive-energy state after k_steps of n_steps steps."""
    lib = _load()
    px = np.ascontiguousarray(px, dtype=np.float64).ravel()
    py = np.ascontiguousarray(py, dtype=np.float64).ravel()
    n = np.zeros(px.shape[0])
    p, keep = _problem(field, n_steps, scheme, valley)
    m = lib.oracle_snapshot_points(ctypes.byref(p), int(k_steps), px.shape[0], _ptr(px), _ptr(py), _ptr(n),
                                   int(threads))
    if m < 0:
        raise MemoryError("oracle allocation failed")
    return n, int(m)


def snapshot_grid(field, grid, n_steps, k_steps, scheme="strang", valley=1, idx=None, threads=0):
    """snapshot_points on grid points (idx = linear indices j*nx + i; None: all)."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    if idx is None:
        idx = np.arange(nx * ny, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    px = np.array([grid_p(grid["px"][0], grid["px"][1], nx, int(k % nx)) for k in idx])
    py = np.array([grid_p(grid["py"][0], grid["py"][1], ny, int(k // nx)) for k in idx])
    return snapshot_points(field, px, py, n_steps, k_steps, scheme, valley, threads)


def state_at(field, px, py, n_steps, k_steps, scheme="strang", valley=1):
    """psi after k_steps steps at one momentum (None if masked)."""
    lib = _load()
    p, keep = _problem(field, n_steps, scheme, valley)
    psi = np.zeros(4)
    m = lib.oracle_state_at(ctypes.byref(p), int(k_steps), float(px), float(py), _ptr(psi))
    if m < 0:
        raise MemoryError("oracle allocation failed")
    if m:
        return None
    return np.array([psi[0] + 1j * psi[1], psi[2] + 1j * psi[3]])


def step_matrix_xy(px, py, dt, Ax, Ay, scheme="strang", valley=1):
    """Complex 2x2 matrix of one second-order step with both components of A."""
    lib = _load()
    p, keep = _problem({"kind": "constant"}, 1, scheme, valley)
    U = np.zeros(8)
    lib.oracle_step_matrix_xy(ctypes.byref(p), float(px), float(py), float(dt), float(Ax), float(Ay), _ptr(U))
    return np.array([[U[0] + 1j * U[1], U[4] + 1j * U[5]],
                     [U[2] + 1j * U[3], U[6] + 1j * U[7]]])


def step_matrix(px, py, dt, A_k, scheme="strang", valley=1):
    """Complex 2x2 matrix of one oracle step at momentum (px, py), midpoint potential A_k."""
    lib = _load()
    p, keep = _problem({"kind": "constant"}, 1, scheme, valley)
    U = np.zeros(8)
    lib.oracle_step_matrix(ctypes.byref(p), float(px), float(py), float(dt), float(A_k), _ptr(U))
    c1 = U[0:4]
    c2 = U[4:8]
    return np.array([[c1[0] + 1j * c1[1], c2[0] + 1j * c2[1]],
                     [c1[2] + 1j * c1[3], c2[2] + 1j * c2[3]]])


def spinors(Px, Py, valley=1):
    """Unit spinors (u, v) of the oracle as complex 2-vectors."""
    lib = _load()
    u = np.zeros(4)
    v = np.zeros(4)
    lib.oracle_spinors(float(Px), float(Py), 1 if valley >= 0 else -1, _ptr(u), _ptr(v))
    return (np.array([u[0] + 1j * u[1], u[2] + 1j * u[3]]), np.array([v[0] + 1j * v[1], v[2] + 1j * v[3]]))


def final_state(field, px, py, n_steps, scheme="strang", valley=1):
    """psi(t_f) at one momentum as a complex 2-vector (None if masked)."""
    lib = _load()
    p, keep = _problem(field, n_steps, scheme, valley)
    psi = np.zeros(4)
    m = lib.oracle_final_state(ctypes.byref(p), float(px), float(py), _ptr(psi))
    if m < 0:
        raise MemoryError("oracle allocation failed")
    if m:
        return None
    return np.array([psi[0] + 1j * psi[1], psi[2] + 1j * psi[3]])


def grid_p(p_min, p_max, n, j):
    return float(_load().oracle_grid_p(float(p_min), float(p_max), int(n), int(j)))
