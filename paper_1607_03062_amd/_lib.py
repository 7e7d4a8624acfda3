"""ctypes binding of libpd (argument marshalling only: every step of a solve
runs in the library's HIP kernels).  Names follow include/pd.h."""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpd.so")

PD_OK, PD_ERR_INVALID, PD_ERR_STATE, PD_ERR_NOMEM, PD_ERR_DEVICE, PD_ERR_UNSUPPORTED = range(6)
PD_FP64, PD_FP32, PD_FP32_FAST = 0, 1, 2
PD_SCHEME_STRANG, PD_SCHEME_MIDPOINT, PD_SCHEME_STRANG4, PD_SCHEME_MIDPOINT4 = 0, 1, 2, 3
PD_VALLEYS_BOTH, PD_VALLEY_KPLUS, PD_VALLEY_KMINUS = 0, 1, 2
PD_FIELD_SIN2, PD_FIELD_CONSTANT, PD_FIELD_TABLE, PD_FIELD_PULSE = 0, 1, 2, 3

PRECISIONS = {"fp64": PD_FP64, "fp32": PD_FP32, "fp32fast": PD_FP32_FAST}
SCHEMES = {"strang": PD_SCHEME_STRANG, "midpoint": PD_SCHEME_MIDPOINT, "strang4": PD_SCHEME_STRANG4,
           "midpoint4": PD_SCHEME_MIDPOINT4}
STAGES = {"strang": 1, "midpoint": 1, "strang4": 5, "midpoint4": 5}
VALLEYS = {"both": PD_VALLEYS_BOTH, "K+": PD_VALLEY_KPLUS, "K-": PD_VALLEY_KMINUS}
FIELD_KINDS = {"sin2": PD_FIELD_SIN2, "constant": PD_FIELD_CONSTANT, "table": PD_FIELD_TABLE,
               "pulse": PD_FIELD_PULSE}
STATUS_NAMES = {0: "PD_OK", 1: "PD_ERR_INVALID", 2: "PD_ERR_STATE", 3: "PD_ERR_NOMEM", 4: "PD_ERR_DEVICE",
                5: "PD_ERR_UNSUPPORTED"}

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class pd_field(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("E0", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("cycles", ctypes.c_int),
        ("t_end", ctypes.c_double),
        ("A_mid", _dp),
        ("n_table", ctypes.c_longlong),
        ("t_i", ctypes.c_double),
        ("t_f", ctypes.c_double),
        ("A_in", ctypes.c_double),
        ("A_out", ctypes.c_double),
        ("phi", ctypes.c_double),
        ("omega_rise", ctypes.c_double),
        ("omega_fall", ctypes.c_double),
        ("duration", ctypes.c_double),
        ("ellipticity", ctypes.c_double),
        ("Ay_mid", _dp),
        ("Ay_in", ctypes.c_double),
        ("Ay_out", ctypes.c_double),
    ]


class pd_info(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_longlong),
        ("n_steps", ctypes.c_longlong),
        ("steps_done", ctypes.c_longlong),
        ("n_masked", ctypes.c_longlong),
        ("dt", ctypes.c_double),
        ("t_i", ctypes.c_double),
        ("t_f", ctypes.c_double),
        ("A_in", ctypes.c_double),
        ("A_out", ctypes.c_double),
        ("E_max", ctypes.c_double),
        ("A_min", ctypes.c_double),
        ("A_max", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("scheme", ctypes.c_int),
        ("points_per_lane", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("table_stage", ctypes.c_int),
        ("chunk_steps", ctypes.c_int),
        ("rotation_form", ctypes.c_int),
        ("taylor_order", ctypes.c_int),
        ("device_bytes", ctypes.c_size_t),
        ("solve_bytes", ctypes.c_size_t),
        ("valley", ctypes.c_int),
        ("stages", ctypes.c_int),
        ("elliptic", ctypes.c_int),
        ("Ay_in", ctypes.c_double),
        ("Ay_out", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PDError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        self.message = message
        super().__init__("%s failed with %s: %s" % (where, STATUS_NAMES.get(status, status), message))


_lib = None

# (name, restype, argtypes) of every exported entry point of include/pd.h
SIGNATURES = [
    ("pd_create_grid", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(_vp)]),
    ("pd_check_field", ctypes.c_int, [_vp, ctypes.POINTER(pd_field), ctypes.c_longlong, ctypes.POINTER(pd_info)]),
    ("pd_sample_field", ctypes.c_int, [ctypes.POINTER(pd_field), ctypes.c_longlong, _dp, _dp, _dp, _dp, _dp]),
    ("pd_sample_field_xy", ctypes.c_int, [ctypes.POINTER(pd_field), ctypes.c_longlong, ctypes.c_int, _dp, _dp,
                                          _dp]),
    ("pd_set_valley", ctypes.c_int, [_vp, ctypes.c_int]),
    ("pd_set_field", ctypes.c_int, [_vp, ctypes.POINTER(pd_field), ctypes.c_longlong]),
    ("pd_rewind", ctypes.c_int, [_vp]),
    ("pd_resume", ctypes.c_int, [_vp, ctypes.c_longlong]),
    ("pd_propagate", ctypes.c_int, [_vp, ctypes.c_longlong, _vp]),
    ("pd_density", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _vp]),
    ("pd_snapshot", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _vp]),
    ("pd_density_static", ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _vp]),
    ("pd_state_bytes", ctypes.c_size_t, [_vp]),
    ("pd_solve_bytes", ctypes.c_size_t, [_vp, ctypes.c_longlong]),
    ("pd_bind_state", ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    ("pd_save_state", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_longlong), _vp]),
    ("pd_load_state", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_longlong, _vp]),
    ("pd_set_launch", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("pd_get_info", ctypes.c_int, [_vp, ctypes.POINTER(pd_info)]),
    ("pd_destroy_grid", None, [_vp]),
    ("pd_last_error", ctypes.c_char_p, []),
    ("pd_version", ctypes.c_char_p, []),
    ("pd_set_fault", ctypes.c_int, [ctypes.c_char_p]),
    ("pd_autotune", ctypes.c_int, [_vp, ctypes.c_longlong, ctypes.c_int, _vp]),
    ("pd_batch_create", ctypes.c_int, [ctypes.POINTER(_vp)]),
    ("pd_batch_add", ctypes.c_int, [_vp, _vp]),
    ("pd_batch_remove", ctypes.c_int, [_vp, _vp]),
    ("pd_batch_clear", ctypes.c_int, [_vp]),
    ("pd_batch_size", ctypes.c_int, [_vp]),
    ("pd_batch_members", ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int]),
    ("pd_batch_set_launch", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    ("pd_batch_run", ctypes.c_int, [_vp, _dp, _vp]),
    ("pd_batch_step", ctypes.c_int, [_vp, ctypes.c_longlong, _dp, ctypes.POINTER(ctypes.c_int), _vp]),
    ("pd_batch_step_each", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_longlong), _dp, ctypes.POINTER(ctypes.c_int),
                                          _vp]),
    ("pd_batch_get_info", ctypes.c_int, [_vp, ctypes.c_void_p]),
    ("pd_batch_autotune", ctypes.c_int, [_vp, ctypes.c_longlong, _vp]),
    ("pd_batch_destroy", None, [_vp]),
]


class pd_batch_info(ctypes.Structure):
    _fields_ = [
        ("n_grids", ctypes.c_int),
        ("points_per_lane", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("graph_captured", ctypes.c_int),
        ("work_items", ctypes.c_int),
        ("separate_launches", ctypes.c_int),
        ("n_points", ctypes.c_longlong),
        ("point_steps", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def load() -> ctypes.CDLL:
    """Load the in-tree libpd.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpd.so is not built (%s); run `python -m paper_1607_03062_amd.build` "
                              "or __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str):
    if status != PD_OK:
        raise PDError(status, where, load().pd_last_error().decode())


def stream_handle(stream) -> int | None:
    """hipStream_t of a torch stream, an int handle, or None (default stream)."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def version_string() -> str:
    return load().pd_version().decode()


def set_fault(spec: str | None):
    """Arm one injected fault for tests of error handling ("alloc@K" or "launch@K";
    None disarms); see pd_set_fault."""
    check(load().pd_set_fault(spec.encode() if spec else None), "pd_set_fault")


def make_field(field: dict, n_steps: int):
    """pd_field from a field dict; returns (struct, keep-alive)."""
    f = pd_field()
    keep = []
    kind = field["kind"]
    f.kind = FIELD_KINDS[kind]
    f.E0 = float(field.get("E0", 0.0))
    f.omega = float(field.get("omega", 0.0))
    f.cycles = int(field.get("cycles", 0))
    f.t_end = float(field.get("t_end", 0.0))
    if kind == "table":
        A = np.ascontiguousarray(field["A_mid"], dtype=np.float64)
        keep.append(A)
        f.A_mid = A.ctypes.data_as(_dp)
        f.n_table = A.shape[0]
        f.t_i, f.t_f = float(field["t_i"]), float(field["t_f"])
        f.A_in, f.A_out = float(field["A_in"]), float(field["A_out"])
        if field.get("Ay_mid") is not None:
            Ay = np.ascontiguousarray(field["Ay_mid"], dtype=np.float64)
            if Ay.shape != A.shape:
                raise ValueError("Ay_mid must have as many values as A_mid")
            keep.append(Ay)
            f.Ay_mid = Ay.ctypes.data_as(_dp)
            f.Ay_in, f.Ay_out = float(field["Ay_in"]), float(field["Ay_out"])
    f.ellipticity = float(field.get("ellipticity", 0.0))
    f.phi = float(field.get("phi", 0.0))
    f.omega_rise = float(field.get("omega_rise", 0.0))
    f.omega_fall = float(field.get("omega_fall", 0.0))
    f.duration = float(field.get("duration", 0.0))
    return f, keep


def sample_field(field: dict, n_steps: int):
    """Host-side field sampling of the library: (A at the step midpoints, t_i, t_f, A_in, A_out)."""
    f, keep = make_field(field, n_steps)
    A = np.zeros(int(n_steps))
    vals = [ctypes.c_double() for _ in range(4)]
    check(load().pd_sample_field(ctypes.byref(f), int(n_steps), A.ctypes.data_as(_dp),
                                 *[ctypes.byref(v) for v in vals]), "pd_sample_field")
    return (A,) + tuple(v.value for v in vals)


def sample_field_xy(field: dict, n_steps: int, scheme: str = "strang"):
    """Library sampling for any scheme: (A_x samples, A_y samples, (t_i, t_f, Ax_in, Ax_out, Ay_in, Ay_out))."""
    f, keep = make_field(field, n_steps)
    m = STAGES[scheme] * int(n_steps)
    Ax, Ay, ends = np.zeros(m), np.zeros(m), np.zeros(6)
    check(load().pd_sample_field_xy(ctypes.byref(f), int(n_steps), SCHEMES[scheme], Ax.ctypes.data_as(_dp),
                                    Ay.ctypes.data_as(_dp), ends.ctypes.data_as(_dp)), "pd_sample_field_xy")
    return Ax, Ay, tuple(ends)


def _ptr_of(buf):
    """(address, on_device) of a torch tensor or numpy array."""
    if hasattr(buf, "data_ptr"):
        return int(buf.data_ptr()), 1 if buf.is_cuda else 0
    return int(buf.ctypes.data), 0


class Solver:
    """One momentum grid and its solve (pd_grid handle)."""

    def __init__(self, nx, ny, px, py, precision="fp64", scheme="strang", valley="both"):
        lib = load()
        h = _vp()
        check(lib.pd_create_grid(int(nx), int(ny), float(px[0]), float(px[1]), float(py[0]), float(py[1]),
                                 PRECISIONS[precision], SCHEMES[scheme], ctypes.byref(h)), "pd_create_grid")
        self._h = h
        self.nx, self.ny = int(nx), int(ny)
        self.px, self.py = (float(px[0]), float(px[1])), (float(py[0]), float(py[1]))
        self.precision, self.scheme, self.valley = precision, scheme, "both"
        self.field, self.n_steps = None, None
        if valley != "both":
            self.set_valley(valley)

    @classmethod
    def for_grid(cls, grid: dict, precision="fp64", scheme="strang", valley="both"):
        return cls(grid["nx"], grid["ny"], grid["px"], grid["py"], precision, scheme, valley)

    def set_valley(self, valley: str):
        check(load().pd_set_valley(self._h, VALLEYS[valley]), "pd_set_valley")
        self.valley = valley
        return self

    @property
    def handle(self):
        return self._h

    def check_field(self, field: dict, n_steps: int) -> dict:
        f, keep = make_field(field, n_steps)
        info = pd_info()
        check(load().pd_check_field(self._h, ctypes.byref(f), int(n_steps), ctypes.byref(info)), "pd_check_field")
        return info.as_dict()

    def set_field(self, field: dict, n_steps: int):
        f, keep = make_field(field, n_steps)
        check(load().pd_set_field(self._h, ctypes.byref(f), int(n_steps)), "pd_set_field")
        self.field, self.n_steps = field, int(n_steps)
        return self

    def rewind(self):
        check(load().pd_rewind(self._h), "pd_rewind")
        return self

    def resume(self, steps_done: int):
        """Continue from the state in the bound buffer (bind_state), which holds this solve's
        state after steps_done steps (e.g. a checkpoint copied back)."""
        check(load().pd_resume(self._h, int(steps_done)), "pd_resume")
        return self

    def propagate(self, max_steps: int = -1, stream=None):
        check(load().pd_propagate(self._h, int(max_steps), stream_handle(stream)), "pd_propagate")
        return self

    def density(self, n_out=None, want_rho: bool = True, stream=None):
        """Returns rho (float) or None; fills n_out (torch device tensor or numpy array) if given."""
        ptr, dev = (None, 0) if n_out is None else _ptr_of(n_out)
        rho = ctypes.c_double()
        check(load().pd_density(self._h, ptr, dev, ctypes.byref(rho) if want_rho else None,
                                stream_handle(stream)), "pd_density")
        return rho.value if want_rho else None

    def density_static(self, n_out=None, want_rho: bool = True, stream=None):
        """As density(), through pd_density_static (the reduction's scratch in the
        library's static device array: the call allocates nothing)."""
        ptr, dev = (None, 0) if n_out is None else _ptr_of(n_out)
        rho = ctypes.c_double()
        check(load().pd_density_static(self._h, ptr, dev, ctypes.byref(rho) if want_rho else None,
                                       stream_handle(stream)), "pd_density_static")
        return rho.value if want_rho else None

    def snapshot(self, n_out=None, want_rho: bool = True, stream=None):
        """Instantaneous occupation after the steps done so far; rho (float) or None, n_out filled if given."""
        ptr, dev = (None, 0) if n_out is None else _ptr_of(n_out)
        rho = ctypes.c_double()
        check(load().pd_snapshot(self._h, ptr, dev, ctypes.byref(rho) if want_rho else None,
                                 stream_handle(stream)), "pd_snapshot")
        return rho.value if want_rho else None

    def solve(self, stream=None, n_out=None):
        self.propagate(-1, stream)
        return self.density(n_out, True, stream)

    def state_bytes(self) -> int:
        return int(load().pd_state_bytes(self._h))

    def save_state(self, stream=None):
        """(state bytes as a uint8 array, steps done) of the solve in progress (pd_save_state)."""
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        done = ctypes.c_longlong()
        check(load().pd_save_state(self._h, buf.ctypes.data, buf.nbytes, ctypes.byref(done), stream_handle(stream)),
              "pd_save_state")
        return buf, done.value

    def load_state(self, state, steps_done: int, stream=None):
        """Continue as after steps_done steps from a state saved by save_state (pd_load_state)."""
        buf = np.ascontiguousarray(state, dtype=np.uint8)
        check(load().pd_load_state(self._h, buf.ctypes.data, buf.nbytes, int(steps_done), stream_handle(stream)),
              "pd_load_state")
        return self

    def _checkpoint_meta(self) -> dict:
        return {"grid": {"nx": self.nx, "ny": self.ny, "px": list(self.px), "py": list(self.py)},
                "precision": self.precision, "scheme": self.scheme, "valley": self.valley}

    def save_checkpoint(self, path, stream=None):
        """Write the solve in progress to `path` (.npz, no pickled objects): its state after
        the steps done so far, with the grid, precision, scheme, valley, field and step count
        it belongs to.  Restart it with Solver.from_checkpoint or load_checkpoint."""
        if self.field is None:
            raise PDError(PD_ERR_STATE, "save_checkpoint", "no field set")
        state, done = self.save_state(stream)
        scalars = {k: v for k, v in self.field.items() if k not in ("A_mid", "Ay_mid")}
        meta = dict(self._checkpoint_meta(), field=scalars, n_steps=self.n_steps, steps_done=done,
                    library=version_string())
        arrays = {"state": state, "meta": np.array(json.dumps(meta, default=float))}
        for k in ("A_mid", "Ay_mid"):
            if self.field.get(k) is not None:
                arrays[k] = np.ascontiguousarray(self.field[k], dtype=np.float64)
        with open(path, "wb") as fh:
            np.savez(fh, **arrays)
        return done

    @staticmethod
    def _read_checkpoint(path):
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            field = dict(meta["field"])
            for k in ("A_mid", "Ay_mid"):
                if k in z.files:
                    field[k] = z[k]
            return meta, field, z["state"]

    def load_checkpoint(self, path, stream=None):
        """Set the checkpoint's field on this handle (same grid, precision, scheme and valley
        as the saved solve, else PDError) and continue from its state."""
        meta, field, state = self._read_checkpoint(path)
        mine = self._checkpoint_meta()
        for key in mine:
            if meta[key] != mine[key]:
                raise PDError(PD_ERR_INVALID, "load_checkpoint",
                              "checkpoint %s %r does not match the handle's %r" % (key, meta[key], mine[key]))
        self.set_field(field, meta["n_steps"])
        return self.load_state(state, meta["steps_done"], stream)

    @classmethod
    def from_checkpoint(cls, path, stream=None):
        """A new handle that continues the solve saved in `path`."""
        meta = cls._read_checkpoint(path)[0]
        return cls.for_grid(meta["grid"], meta["precision"], meta["scheme"], meta["valley"]).load_checkpoint(
            path, stream)

    def solve_bytes(self, n_steps: int) -> int:
        return int(load().pd_solve_bytes(self._h, int(n_steps)))

    def bind_state(self, buf=None):
        if buf is None:
            check(load().pd_bind_state(self._h, None, 0), "pd_bind_state")
        else:
            ptr, dev = _ptr_of(buf)
            nbytes = buf.numel() * buf.element_size() if hasattr(buf, "numel") else buf.nbytes
            check(load().pd_bind_state(self._h, ptr, nbytes), "pd_bind_state")
        return self

    def set_launch(self, points_per_lane: int = 0, block_threads: int = 0, table_stage: int = 0,
                   chunk_steps: int = 0):
        check(load().pd_set_launch(self._h, int(points_per_lane), int(block_threads), int(table_stage),
                                   int(chunk_steps)), "pd_set_launch")
        return self

    def autotune(self, trial_steps: int = 2048, use_cache: bool = False, stream=None):
        check(load().pd_autotune(self._h, int(trial_steps), 1 if use_cache else 0, stream_handle(stream)),
              "pd_autotune")
        return self

    def info(self) -> dict:
        info = pd_info()
        check(load().pd_get_info(self._h, ctypes.byref(info)), "pd_get_info")
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().pd_destroy_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


class Batch:
    """Many solves in one launch sequence (pd_batch handle): second-order Strang
    members share a persistent kernel, the others run their own launches.  Member
    Solvers must stay alive while they are in the batch."""

    def __init__(self, solvers=()):
        h = _vp()
        check(load().pd_batch_create(ctypes.byref(h)), "pd_batch_create")
        self._h = h
        self.members = []
        for s in solvers:
            self.add(s)

    def add(self, solver: Solver):
        check(load().pd_batch_add(self._h, solver.handle), "pd_batch_add")
        self.members.append(solver)
        return self

    def remove(self, solver: Solver):
        check(load().pd_batch_remove(self._h, solver.handle), "pd_batch_remove")
        self.members.remove(solver)
        return self

    def clear(self):
        check(load().pd_batch_clear(self._h), "pd_batch_clear")
        self.members = []
        return self

    def __len__(self):
        return int(load().pd_batch_size(self._h))

    def set_launch(self, points_per_lane: int = 0, block_threads: int = 0):
        check(load().pd_batch_set_launch(self._h, int(points_per_lane), int(block_threads)), "pd_batch_set_launch")
        return self

    def run(self, stream=None, want_rho: bool = True):
        """Every member's whole solve; returns the members' rho (numpy array) or None."""
        rho = np.zeros(len(self.members)) if want_rho else None
        check(load().pd_batch_run(self._h, rho.ctypes.data_as(_dp) if want_rho else None, stream_handle(stream)),
              "pd_batch_run")
        return rho

    def step(self, max_steps: int, stream=None, want_rho: bool = True):
        """One epoch; returns (rho array with NaN for members not completing now, finished flags)."""
        n = len(self.members)
        rho = np.full(n, np.nan)
        fin = (ctypes.c_int * max(n, 1))()
        check(load().pd_batch_step(self._h, int(max_steps), rho.ctypes.data_as(_dp) if want_rho else None, fin,
                                   stream_handle(stream)), "pd_batch_step")
        return (rho if want_rho else None), np.array(fin[:n], dtype=bool)

    def step_each(self, max_steps, stream=None, want_rho: bool = True):
        """One epoch with a step limit per member (sequence in member order, 0 = stays);
        returns (rho array with NaN for members not completing now, finished flags)."""
        n = len(self.members)
        if len(max_steps) != n:
            raise ValueError("max_steps has %d values for %d members" % (len(max_steps), n))
        lim = (ctypes.c_longlong * max(n, 1))(*[int(m) for m in max_steps])
        rho = np.full(n, np.nan)
        fin = (ctypes.c_int * max(n, 1))()
        check(load().pd_batch_step_each(self._h, lim, rho.ctypes.data_as(_dp) if want_rho else None, fin,
                                        stream_handle(stream)), "pd_batch_step_each")
        return (rho if want_rho else None), np.array(fin[:n], dtype=bool)

    def autotune(self, trial_steps: int = 1024, stream=None):
        check(load().pd_batch_autotune(self._h, int(trial_steps), stream_handle(stream)), "pd_batch_autotune")
        return self

    def info(self) -> dict:
        info = pd_batch_info()
        check(load().pd_batch_get_info(self._h, ctypes.byref(info)), "pd_batch_get_info")
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().pd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
