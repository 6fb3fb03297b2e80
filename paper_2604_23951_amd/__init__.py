"""Python binding of the MI355X restarted-PDHG LP solver (include/lp.h).

Argument marshalling only: every step of the solve runs in the HIP library
`_lib/liblpgpu.so`. Importing this package does not need a GPU; calling the solver
does, and a missing library is an error (there is no CPU path).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LPGPU_CHECKED=1 loads the bounds-checked build (include/lp.h, lp_check_word)
LIB_PATH = os.environ.get("LPGPU_LIB_OVERRIDE", os.path.join(
    _HERE, "_lib", "liblpgpu_checked.so" if os.environ.get("LPGPU_CHECKED") == "1" else "liblpgpu.so"))

LP_OK = 0
ERRORS = {1: "LP_ERR_INVALID_ARG", 2: "LP_ERR_INVALID_MATRIX", 3: "LP_ERR_INCONSISTENT_BOUNDS",
          4: "LP_ERR_NAN_INPUT", 5: "LP_ERR_OUT_OF_MEMORY", 6: "LP_ERR_DEVICE", 7: "LP_ERR_NOT_SOLVED",
          8: "LP_ERR_INTERNAL"}
STATUS = {0: "optimal", 1: "iteration_limit", 2: "time_limit", 3: "numerical_error", 4: "primal_infeasible",
          5: "dual_infeasible", 6: "cancelled"}
LP_METHOD_AVERAGED = 0
LP_METHOD_HALPERN = 1
LP_PW_DEFAULT = 0
LP_PW_SMOOTH = 1
LP_PW_PID = 2
LP_LAYOUT_PANELS = 0
LP_LAYOUT_TILES = 1
LP_LAYOUT_TUNED = 2
LP_PRESET_DEFAULT = 0
LP_PRESET_SMALL = 1
LP_PRESET_LARGE = 2
LP_PRESET_LARGE_FP32 = 3
LP_PRESET_BATCH = 4
LP_PRESET_SERVING = 5
PRESETS = {"default": LP_PRESET_DEFAULT, "small": LP_PRESET_SMALL, "large": LP_PRESET_LARGE,
           "large_fp32": LP_PRESET_LARGE_FP32, "batch": LP_PRESET_BATCH, "serving": LP_PRESET_SERVING}
LP_PREC_FP64 = 0
LP_PREC_FP32_REFINED = 1
TRACE_WIDTH = 12
LP_STATIC_BATCH_MAX = 4096  # include/lp.h

# names of every function include/lp.h declares
EXPORTS = (
    "lp_default_options", "lp_preset_options", "lp_create", "lp_update_options", "lp_solve", "lp_polish", "lp_solve_until", "lp_resume",
    "lp_export_state", "lp_import_state", "lp_solve_batch", "lp_solve_batch_static", "lp_get_solution", "lp_destroy", "lp_check_word", "lp_error_string",
    "lp_last_error", "lp_get_iterates", "lp_get_scaled", "lp_get_trace", "lp_set_kernel_timing",
    "lp_get_kernel_times", "lp_get_layout", "lp_server_create", "lp_server_submit", "lp_server_poll",
    "lp_server_ticket_times", "lp_server_result", "lp_server_cancel", "lp_server_wait", "lp_server_stats_get", "lp_server_destroy",
    "lp_presolve_default_options", "lp_presolve", "lp_presolve_get_info", "lp_presolve_get_reduced",
    "lp_presolve_get_maps", "lp_postsolve", "lp_presolve_destroy",
)


class LpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lp_options(C.Structure):
    _fields_ = [
        ("eps_rel", C.c_double), ("max_iters", C.c_int64), ("time_limit_s", C.c_double),
        ("eval_every", C.c_int32), ("precision", C.c_int32), ("scaling", C.c_int32), ("ruiz_passes", C.c_int32),
        ("pow_iters", C.c_int32), ("restarts", C.c_int32), ("step_size", C.c_double), ("omega0", C.c_double),
        ("seed", C.c_uint64), ("hip_stream", C.c_void_p), ("device", C.c_int32), ("trace_cap", C.c_int32),
        ("spmv_layout", C.c_int32), ("long_row_len", C.c_int32), ("units_per_cu", C.c_int32),
        ("batch_wg_per_cu", C.c_int32),
        ("panel_slice_bytes", C.c_int64), ("batch_split_nnz", C.c_int64), ("deferred", C.c_int32),
        ("small_lp_lds", C.c_int32), ("x0", C.c_void_p), ("y0", C.c_void_p), ("eps_infeas", C.c_double),
        ("method", C.c_int32), ("restart_metric", C.c_int32), ("reflection", C.c_double),
        ("omega_steps", C.c_int32), ("pad3", C.c_int32), ("pw_rule", C.c_int32), ("pad4", C.c_int32),
        ("pid_kp", C.c_double), ("pid_ki", C.c_double), ("pid_kd", C.c_double),
        ("tile_nnz", C.c_int32), ("pad5", C.c_int32),
    ]


class lp_presolve_options(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("dual_reductions", C.c_int32), ("substitute", C.c_int32),
                ("doubletons", C.c_int32), ("feas_tol", C.c_double), ("pivot_tol", C.c_double)]


class lp_presolve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("m", C.c_int32), ("n", C.c_int32), ("pad", C.c_int32), ("nnz", C.c_int64),
                ("rounds", C.c_int32), ("pad2", C.c_int32)] + \
               [(k, C.c_int64) for k in ("empty_rows", "singleton_rows", "redundant_rows", "dropped_sides",
                                         "empty_cols", "fixed_cols", "lock_fixed_cols", "substituted_cols")] + \
               [("seconds", C.c_double), ("doubleton_cols", C.c_int64), ("cancelled_entries", C.c_int64)]


class lp_server_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "admitted", "completed", "queued", "running", "rounds",
                                           "bytes_in_use", "peak_bytes", "hbm_budget", "lp_iterations")]
    _fields_ += [("nnz_iterations", C.c_double)]


class lp_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("output_is_avg", C.c_int32), ("iterations", C.c_int64), ("restarts", C.c_int64),
        ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("rel_primal_res", C.c_double),
        ("rel_dual_res", C.c_double), ("rel_gap", C.c_double), ("rel_kkt", C.c_double), ("sigma_max", C.c_double),
        ("step_size", C.c_double), ("omega", C.c_double), ("setup_seconds", C.c_double),
        ("solve_seconds", C.c_double), ("done_clock", C.c_int64), ("clock_hz", C.c_double),
        ("polish_primal_iterations", C.c_int64), ("polish_dual_iterations", C.c_int64),
        ("polish_seconds", C.c_double), ("ray_source", C.c_int32), ("solve_path", C.c_int32),
    ]


_lib = None


def library_loaded() -> bool:
    return _lib is not None


def _share_torch_runtime():
    """PyTorch-ROCm ships its own libamdhip64 with the same soname as the system one. Loading
    torch first makes the dynamic loader bind this library to torch's copy, so a process
    that uses both has one HIP runtime (and torch streams and device pointers are valid
    here). Without torch the system runtime is used."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load the HIP library; raise if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP solver library missing: {LIB_PATH} (run __graft_entry__.build())")
        _share_torch_runtime()
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.lp_default_options.argtypes = [P]
        L.lp_default_options.restype = None
        L.lp_preset_options.argtypes = [P, I32]
        L.lp_preset_options.restype = I32
        L.lp_create.argtypes = [P, I32, I32, I64, P, P, P, P, D, P, P, P, P, P]
        L.lp_create.restype = I32
        L.lp_update_options.argtypes = [P, P]
        L.lp_update_options.restype = I32
        L.lp_solve.argtypes = [P]
        L.lp_solve.restype = I32
        L.lp_solve_batch.argtypes = [P, I32, P]
        L.lp_solve_batch.restype = I32
        L.lp_polish.argtypes = [P, D, I64]
        L.lp_polish.restype = I32
        L.lp_solve_until.argtypes = [P, I64]
        L.lp_solve_until.restype = I32
        L.lp_resume.argtypes = [P, I64]
        L.lp_resume.restype = I32
        L.lp_export_state.argtypes = [P, P, I64, P]
        L.lp_export_state.restype = I32
        L.lp_import_state.argtypes = [P, P, I64]
        L.lp_import_state.restype = I32
        L.lp_solve_batch_static.argtypes = [P, I32, P]
        L.lp_solve_batch_static.restype = I32
        L.lp_get_solution.argtypes = [P, P, P, P, P]
        L.lp_get_solution.restype = I32
        L.lp_destroy.argtypes = [P]
        L.lp_destroy.restype = None
        L.lp_check_word.argtypes = [I32, P, P]
        L.lp_check_word.restype = I32
        L.lp_error_string.argtypes = [I32]
        L.lp_error_string.restype = C.c_char_p
        L.lp_last_error.argtypes = [P]
        L.lp_last_error.restype = C.c_char_p
        L.lp_get_iterates.argtypes = [P, P, P, P, P]
        L.lp_get_iterates.restype = I32
        L.lp_get_scaled.argtypes = [P, P, P, P, P, P, P]
        L.lp_get_scaled.restype = I32
        L.lp_get_trace.argtypes = [P, P, I32, P]
        L.lp_get_trace.restype = I32
        L.lp_set_kernel_timing.argtypes = [P, I32]
        L.lp_set_kernel_timing.restype = I32
        L.lp_get_kernel_times.argtypes = [P, P, P, P]
        L.lp_get_kernel_times.restype = I32
        L.lp_get_layout.argtypes = [P, P, I32]
        L.lp_get_layout.restype = I32
        L.lp_server_create.argtypes = [P, I32, I64, I32, P]
        L.lp_server_create.restype = I32
        L.lp_server_submit.argtypes = [P, P, P]
        L.lp_server_submit.restype = I32
        L.lp_server_poll.argtypes = [P, P, I32, P]
        L.lp_server_poll.restype = I32
        L.lp_server_ticket_times.argtypes = [P, C.c_uint64, P]
        L.lp_server_ticket_times.restype = I32
        L.lp_server_result.argtypes = [P, C.c_uint64, P, P, P, P]
        L.lp_server_result.restype = I32
        L.lp_server_cancel.argtypes = [P, C.c_uint64]
        L.lp_server_cancel.restype = I32
        L.lp_server_wait.argtypes = [P, D]
        L.lp_server_wait.restype = I32
        L.lp_server_stats_get.argtypes = [P, P]
        L.lp_server_stats_get.restype = I32
        L.lp_server_destroy.argtypes = [P]
        L.lp_server_destroy.restype = None
        L.lp_presolve_default_options.argtypes = [P]
        L.lp_presolve_default_options.restype = None
        L.lp_presolve.argtypes = [P, I32, I32, I64, P, P, P, P, D, P, P, P, P, P, P]
        L.lp_presolve.restype = I32
        L.lp_presolve_get_info.argtypes = [P, P]
        L.lp_presolve_get_info.restype = I32
        L.lp_presolve_get_reduced.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.lp_presolve_get_reduced.restype = I32
        L.lp_presolve_get_maps.argtypes = [P, P, P]
        L.lp_presolve_get_maps.restype = I32
        L.lp_postsolve.argtypes = [P, P, P, P, P, P, P]
        L.lp_postsolve.restype = I32
        L.lp_presolve_destroy.argtypes = [P]
        L.lp_presolve_destroy.restype = None
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(rc: int, handle=None):
    if rc != LP_OK:
        msg = lib().lp_last_error(handle).decode(errors="replace")
        raise LpError(rc, msg)


# ---- raw C-ABI names ----------------------------------------------------------------

def lp_default_options() -> lp_options:
    o = lp_options()
    lib().lp_default_options(C.byref(o))
    return o


def lp_preset_options(preset) -> lp_options:
    """Options of a preset (an LP_PRESET_* value or its name in PRESETS)."""
    o = lp_options()
    _check(lib().lp_preset_options(C.byref(o), PRESETS.get(preset, preset) if isinstance(preset, str) else preset))
    return o


def lp_create(m, n, nnz, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi, opt: Optional[lp_options] = None):
    """Host numpy arrays in, opaque handle (c_void_p) out."""
    h = C.c_void_p()
    rc = lib().lp_create(C.byref(h), m, n, nnz, _p(row_ptr), _p(col_idx), _p(vals), _p(c), float(c0), _p(b_lo),
                         _p(b_hi), _p(x_lo), _p(x_hi), None if opt is None else C.byref(opt))
    _check(rc)
    return h


def lp_update_options(h, opt: lp_options):
    _check(lib().lp_update_options(h, C.byref(opt)), h)


def lp_solve(h):
    _check(lib().lp_solve(h), h)


def lp_solve_until(h, k_pause: int):
    _check(lib().lp_solve_until(h, int(k_pause)), h)


def lp_resume(h, k_pause: int = 0):
    _check(lib().lp_resume(h, int(k_pause)), h)


def lp_export_state(h) -> bytes:
    size = C.c_int64()
    _check(lib().lp_export_state(h, None, 0, C.byref(size)), h)
    buf = C.create_string_buffer(max(size.value, 1))
    _check(lib().lp_export_state(h, buf, size.value, C.byref(size)), h)
    return buf.raw[: size.value]


def lp_import_state(h, state: bytes):
    buf = C.create_string_buffer(bytes(state), len(state))
    _check(lib().lp_import_state(h, buf, len(state)), h)


def lp_solve_batch(handles, opt: Optional[lp_options] = None):
    arr = (C.c_void_p * max(len(handles), 1))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    rc = lib().lp_solve_batch(arr, len(handles), None if opt is None else C.byref(opt))
    _check(rc)


def lp_solve_batch_static(handles, opt: Optional[lp_options] = None):
    arr = (C.c_void_p * max(len(handles), 1))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    rc = lib().lp_solve_batch_static(arr, len(handles), None if opt is None else C.byref(opt))
    _check(rc)


def lp_get_solution(h, x=None, y=None, z=None) -> lp_info:
    info = lp_info()
    _check(lib().lp_get_solution(h, _p(x), _p(y), _p(z), C.byref(info)), h)
    return info


def lp_destroy(h):
    if h:
        lib().lp_destroy(h)


def lp_check_word(device: int = 0):
    """(word, checked): the device check word (read and cleared) and whether this library is
    the checked build."""
    w, c = C.c_uint32(), C.c_int32()
    _check(lib().lp_check_word(int(device), C.byref(w), C.byref(c)))
    return w.value, bool(c.value)


def lp_error_string(code: int) -> str:
    return lib().lp_error_string(code).decode()


def lp_last_error(h=None) -> str:
    return lib().lp_last_error(h).decode(errors="replace")


def lp_get_iterates(h, x=None, y=None, x_avg=None, y_avg=None):
    _check(lib().lp_get_iterates(h, _p(x), _p(y), _p(x_avg), _p(y_avg)), h)


def lp_get_scaled(h, vals=None, R=None, Cc=None, t_row_ptr=None, t_col_idx=None, t_vals=None):
    _check(lib().lp_get_scaled(h, _p(vals), _p(R), _p(Cc), _p(t_row_ptr), _p(t_col_idx), _p(t_vals)), h)


def lp_get_trace(h, cap: int = 4096) -> np.ndarray:
    out = np.zeros((max(cap, 1), TRACE_WIDTH))
    n = C.c_int32()
    _check(lib().lp_get_trace(h, _p(out), cap, C.byref(n)), h)
    return out[: min(n.value, cap)].copy()


def lp_set_kernel_timing(h, enable: bool):
    _check(lib().lp_set_kernel_timing(h, int(enable)), h)


def lp_get_kernel_times(h):
    p, d, k = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().lp_get_kernel_times(h, C.byref(p), C.byref(d), C.byref(k)), h)
    return p.value, d.value, k.value


def lp_get_layout(h):
    out = np.zeros(13, np.int64)
    _check(lib().lp_get_layout(h, _p(out), 13), h)
    keys = ("tiles_a", "tiles_at", "long_rows_a", "long_rows_at", "device_bytes", "units_a", "units_at",
            "panels_a", "panels_at", "layout", "trial_ns_panels", "trial_ns_tiles", "tile_nnz")
    return {k: int(v) for k, v in zip(keys, out)}


# ---- convenience wrapper ---------------------------------------------------------------

@dataclass
class Solution:
    status: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    info: lp_info
    trace: np.ndarray = field(default_factory=lambda: np.zeros((0, TRACE_WIDTH)))

    def __getattr__(self, k):
        info = self.__dict__.get("info")
        if info is not None and k in dict(lp_info._fields_):
            return getattr(info, k)
        raise AttributeError(k)


_OPT_KEYS = {f[0] for f in lp_options._fields_} - {"x0", "y0", "hip_stream"}


def make_options(preset=None, **kw) -> lp_options:
    """Options from the defaults (or a preset, see lp_preset_options) with fields replaced."""
    o = lp_default_options() if preset is None else lp_preset_options(preset)
    for k, v in kw.items():
        if k not in _OPT_KEYS:
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Solver:
    """Owns one lp_handle. `lp` is any object with the fields of eq. (1):
    m, n, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi."""

    def __init__(self, lp, *, x0=None, y0=None, stream=None, **options):
        self._keep = []
        o = make_options(**options)

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        if x0 is not None:
            o.x0 = arr(x0, np.float64).ctypes.data
        if y0 is not None:
            o.y0 = arr(y0, np.float64).ctypes.data
        if stream is not None:  # a torch.cuda.Stream or a raw hipStream_t integer
            o.hip_stream = getattr(stream, "cuda_stream", stream)
        self.m, self.n = int(lp.m), int(lp.n)
        rp = arr(lp.row_ptr, np.int32)
        self.nnz = int(rp[self.m])
        ci = arr(lp.col_idx if self.nnz else np.zeros(1), np.int32)
        v = arr(lp.vals if self.nnz else np.zeros(1), np.float64)
        bl = arr(lp.b_lo, np.float64) if self.m else None
        bu = arr(lp.b_hi, np.float64) if self.m else None
        self.h = lp_create(self.m, self.n, self.nnz, rp, ci, v, arr(lp.c, np.float64), float(getattr(lp, "c0", 0.0)),
                           bl, bu, arr(lp.x_lo, np.float64), arr(lp.x_hi, np.float64), o)
        self.trace_cap = o.trace_cap
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def update(self, **options):
        """Change solve-time options (eps_rel, max_iters, time_limit_s, eval_every, restarts,
        eps_infeas, method, reflection, omega_steps, pw_rule, pid_kp, pid_ki, pid_kd); the ones
        not given take their defaults."""
        lp_update_options(self.h, make_options(**options))

    def solve(self, with_trace: bool = False) -> Solution:
        lp_solve(self.h)
        x = np.empty(self.n)
        y = np.empty(max(self.m, 1))
        z = np.empty(self.n)
        info = lp_get_solution(self.h, x, y, z)
        tr = lp_get_trace(self.h, self.trace_cap) if with_trace else np.zeros((0, TRACE_WIDTH))
        return Solution(STATUS.get(info.status, str(info.status)), x, y[: self.m], z, info, tr)

    def _result(self, with_trace: bool = False) -> Solution:
        x = np.empty(self.n)
        y = np.empty(max(self.m, 1))
        z = np.empty(self.n)
        info = lp_get_solution(self.h, x, y, z)
        tr = lp_get_trace(self.h, self.trace_cap) if with_trace else np.zeros((0, TRACE_WIDTH))
        return Solution(STATUS.get(info.status, str(info.status)), x, y[: self.m], z, info, tr)

    def solve_until(self, k_pause: int, with_trace: bool = False) -> Solution:
        """lp_solve_until: run until the first evaluation at or beyond k_pause, then pause."""
        lp_solve_until(self.h, k_pause)
        return self._result(with_trace)

    def resume(self, k_pause: int = 0, with_trace: bool = False) -> Solution:
        """lp_resume: continue a paused run (pausing again at k_pause > 0)."""
        lp_resume(self.h, k_pause)
        return self._result(with_trace)

    def export_state(self) -> bytes:
        return lp_export_state(self.h)

    def import_state(self, state: bytes) -> Solution:
        lp_import_state(self.h, state)
        return self._result()

    def polish(self, eps: float = 1e-8, max_iters: int = 100000) -> Solution:
        """Feasibility polishing of the last solve's point (lp_polish); returns the polished point."""
        _check(lib().lp_polish(self.h, float(eps), int(max_iters)), self.h)
        x = np.empty(self.n)
        y = np.empty(max(self.m, 1))
        z = np.empty(self.n)
        info = lp_get_solution(self.h, x, y, z)
        return Solution(STATUS.get(info.status, str(info.status)), x, y[: self.m], z, info)

    def iterates(self):
        x, xa = np.empty(self.n), np.empty(self.n)
        y, ya = np.empty(max(self.m, 1)), np.empty(max(self.m, 1))
        lp_get_iterates(self.h, x, y, xa, ya)
        return x, y[: self.m], xa, ya[: self.m]

    def scaled(self):
        nz = max(self.nnz, 1)
        v, R, Cc = np.empty(nz), np.empty(max(self.m, 1)), np.empty(self.n)
        trp, tci, tv = np.empty(self.n + 1, np.int32), np.empty(nz, np.int32), np.empty(nz)
        lp_get_scaled(self.h, v, R, Cc, trp, tci, tv)
        return v[: self.nnz], R[: self.m], Cc, trp, tci[: self.nnz], tv[: self.nnz]

    def layout(self):
        return lp_get_layout(self.h)


def solve_batch(solvers, **options):
    """Solve several Solver objects in one persistent launch; returns their Solutions."""
    opt = make_options(**options) if options else None
    lp_solve_batch([s.h for s in solvers], opt)
    out = []
    for s in solvers:
        x = np.empty(s.n)
        y = np.empty(max(s.m, 1))
        z = np.empty(s.n)
        info = lp_get_solution(s.h, x, y, z)
        out.append(Solution(STATUS.get(info.status, str(info.status)), x, y[: s.m], z, info))
    return out


class Server:
    """Serving form: continuous batching of deferred LPs (see include/lp.h, lp_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, device: int = 0, **options):
        self.h = C.c_void_p()
        o = make_options(**options) if options else None
        _check(lib().lp_server_create(C.byref(self.h), device, int(hbm_budget_bytes), int(max_slots),
                                      None if o is None else C.byref(o)))
        self._dims = {}

    def submit(self, solver: "Solver") -> int:
        """Queue a request for the solver's LP (a deferred Solver; may be submitted repeatedly)."""
        t = C.c_uint64()
        _check(lib().lp_server_submit(self.h, solver.h, C.byref(t)), solver.h)
        self._dims[t.value] = (solver.n, solver.m)
        return t.value

    def poll(self, cap: int = 4096):
        buf = (C.c_uint64 * max(cap, 1))()
        n = C.c_int32()
        _check(lib().lp_server_poll(self.h, buf, cap, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def times(self, ticket: int):
        t = (C.c_double * 3)()
        _check(lib().lp_server_ticket_times(self.h, C.c_uint64(ticket), t))
        return tuple(t)

    def cancel(self, ticket: int):
        """lp_server_cancel: a queued request completes at once, a running one after the round."""
        _check(lib().lp_server_cancel(self.h, C.c_uint64(ticket)))

    def wait(self, timeout_s: float = 0.0):
        _check(lib().lp_server_wait(self.h, float(timeout_s)))

    def stats(self) -> dict:
        st = lp_server_stats()
        _check(lib().lp_server_stats_get(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in lp_server_stats._fields_}

    def result(self, ticket: int) -> Solution:
        n, m = self._dims.pop(ticket)
        x = np.empty(n)
        y = np.empty(max(m, 1))
        z = np.empty(n)
        info = lp_info()
        _check(lib().lp_server_result(self.h, C.c_uint64(ticket), _p(x), _p(y), _p(z), C.byref(info)))
        return Solution(STATUS.get(info.status, str(info.status)), x, y[:m], z, info)

    def close(self):
        if getattr(self, "h", None):
            lib().lp_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(lp, **options) -> Solution:
    with Solver(lp, **options) as s:
        return s.solve()


# ---- presolve / postsolve (host) -----------------------------------------------------

PRESOLVE_STATUS = {0: "reduced", 1: "solved", 2: "infeasible", 3: "unbounded"}


class ReducedLP:
    """The reduced LP of a presolve, with the fields Solver expects."""

    def __init__(self, m, n, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi):
        self.m, self.n = m, n
        self.row_ptr, self.col_idx, self.vals = row_ptr, col_idx, vals
        self.c, self.c0 = c, c0
        self.b_lo, self.b_hi, self.x_lo, self.x_hi = b_lo, b_hi, x_lo, x_hi

    @property
    def nnz(self):
        return int(self.row_ptr[self.m])


class Presolve:
    """Owns one lp_presolver: `Presolve(lp, **options)` runs the presolve; `.reduced` is the
    reduced LP, `.postsolve(x, y, z)` maps its solution back to the original LP."""

    def __init__(self, lp, **options):
        o = lp_presolve_options()
        lib().lp_presolve_default_options(C.byref(o))
        for k, v in options.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown presolve option {k}")
            setattr(o, k, v)
        self.m0, self.n0 = int(lp.m), int(lp.n)
        rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int32)
        nnz = int(rp[self.m0])
        ci = np.ascontiguousarray(lp.col_idx if nnz else np.zeros(1), dtype=np.int32)
        v = np.ascontiguousarray(lp.vals if nnz else np.zeros(1), dtype=np.float64)
        c = np.ascontiguousarray(lp.c, dtype=np.float64)
        bl = np.ascontiguousarray(lp.b_lo, dtype=np.float64) if self.m0 else None
        bu = np.ascontiguousarray(lp.b_hi, dtype=np.float64) if self.m0 else None
        xl = np.ascontiguousarray(lp.x_lo, dtype=np.float64)
        xu = np.ascontiguousarray(lp.x_hi, dtype=np.float64)
        h = C.c_void_p()
        info = lp_presolve_info()
        _check(lib().lp_presolve(C.byref(h), self.m0, self.n0, nnz, _p(rp), _p(ci), _p(v), _p(c),
                                 float(getattr(lp, "c0", 0.0)), _p(bl), _p(bu), _p(xl), _p(xu), C.byref(o),
                                 C.byref(info)))
        self.h = h
        self.info = info
        self.status = PRESOLVE_STATUS.get(info.status, str(info.status))
        self.reduced = None
        if info.status in (0, 1):
            m, n, k = info.m, info.n, info.nnz
            r = ReducedLP(m, n, np.zeros(m + 1, np.int32), np.zeros(max(k, 1), np.int32), np.zeros(max(k, 1)),
                          np.zeros(max(n, 1)), 0.0, np.zeros(max(m, 1)), np.zeros(max(m, 1)), np.zeros(max(n, 1)),
                          np.zeros(max(n, 1)))
            c0 = C.c_double()
            _check(lib().lp_presolve_get_reduced(self.h, _p(r.row_ptr), _p(r.col_idx), _p(r.vals), _p(r.c),
                                                 C.byref(c0), _p(r.b_lo), _p(r.b_hi), _p(r.x_lo), _p(r.x_hi)))
            r.c0 = c0.value
            r.col_idx, r.vals = r.col_idx[:k], r.vals[:k]
            r.c, r.x_lo, r.x_hi = r.c[:n], r.x_lo[:n], r.x_hi[:n]
            r.b_lo, r.b_hi = r.b_lo[:m], r.b_hi[:m]
            self.reduced = r

    def stats(self) -> dict:
        return {k: getattr(self.info, k) for k, _ in lp_presolve_info._fields_ if not k.startswith("pad")}

    def maps(self):
        rm = np.zeros(max(self.info.m, 1), np.int32)
        cm = np.zeros(max(self.info.n, 1), np.int32)
        _check(lib().lp_presolve_get_maps(self.h, _p(rm), _p(cm)))
        return rm[: self.info.m], cm[: self.info.n]

    def postsolve(self, x=None, y=None, z=None):
        def arr(a, size):
            if size == 0:
                return None
            return np.ascontiguousarray(a, dtype=np.float64)

        xo, yo, zo = np.empty(self.n0), np.empty(max(self.m0, 1)), np.empty(self.n0)
        _check(lib().lp_postsolve(self.h, _p(arr(x, self.info.n)), _p(arr(y, self.info.m)), _p(arr(z, self.info.n)),
                                  _p(xo), _p(yo), _p(zo)))
        return xo, yo[: self.m0], zo

    def close(self):
        if getattr(self, "h", None):
            lib().lp_presolve_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PresolvedSolution:
    """Result of solve_presolved: the original LP's (x, y, z), the presolve record and the
    reduced solve (None when presolve decided the LP on its own)."""

    def __init__(self, status, x, y, z, presolve_stats, reduced, times):
        self.status, self.x, self.y, self.z = status, x, y, z
        self.presolve = presolve_stats
        self.reduced = reduced
        self.times = times


def solve_presolved(lp, presolve_options=None, **options) -> PresolvedSolution:
    """Presolve on the host, solve the reduced LP with the GPU solver, postsolve on the host."""
    import time

    t0 = time.perf_counter()
    with Presolve(lp, **(presolve_options or {})) as P:
        t1 = time.perf_counter()
        stats = P.stats()
        if P.status in ("infeasible", "unbounded"):
            return PresolvedSolution(P.status, None, None, None, stats, None,
                                     {"presolve_s": t1 - t0, "solve_s": 0.0, "postsolve_s": 0.0})
        red = None
        if P.info.n > 0:
            with Solver(P.reduced, **options) as s:
                red = s.solve()
            t2 = time.perf_counter()
            x, y, z = P.postsolve(red.x, red.y, red.z)
            status = red.status
        else:
            t2 = time.perf_counter()
            x, y, z = P.postsolve()
            status = "optimal"
        t3 = time.perf_counter()
    return PresolvedSolution(status, x, y, z, stats, red,
                             {"presolve_s": t1 - t0, "solve_s": t2 - t1, "postsolve_s": t3 - t2})


def evaluate(lp, x, y, **options) -> lp_info:
    """E_rel and its terms of the point (x, y) on `lp`, computed by the solver's own evaluation
    (a handle warm-started at the point and run for zero iterations)."""
    with Solver(lp, x0=x, y0=y, max_iters=0, eps_rel=0.0, **options) as s:
        return s.solve().info
