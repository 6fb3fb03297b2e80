"""FP64 CPU oracle for restarted averaged PDHG (ctypes binding of pdhg_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the benchmark's
CPU-baseline leg use this module. The GPU solver never imports or links it, and
it shares no code with the solver.

Parity notes: the problem form, the dual sign rules and the reduced-cost identity follow
the paper's Section 2 (eq. 1, eq. 2) and Section 2.1. The PDHG iteration, restart rules,
step size, primal weight and scaling are the published PDLP-family method the paper
names without detail; the restart constants (0.2, 0.8, 0.36) and the evaluation period are
readings with parity unpinned, while the restart cycle itself is pinned by
tests/test_oracle_restarts.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# The mutation tests point this module at a deliberately broken copy of the oracle.
_LOAD_PATH = os.environ.get("ORACLE_LIB_OVERRIDE", _LIB_PATH)

TRACE_W = 12
STATUS = {0: "optimal", 1: "iteration_limit", 2: "numerical_error", 3: "primal_infeasible", 4: "dual_infeasible"}


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source with gcc (no contraction of multiply-add, portable -O2)."""
    tmp = out + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-ffp-contract=off", "-fno-fast-math",
         "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, src, "-lm"]
    )
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


class _LPStruct(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
        ("vals", C.c_void_p), ("c", C.c_void_p), ("c0", C.c_double),
        ("b_lo", C.c_void_p), ("b_hi", C.c_void_p), ("x_lo", C.c_void_p), ("x_hi", C.c_void_p),
    ]


class _OptsStruct(C.Structure):
    _fields_ = [
        ("eps_rel", C.c_double), ("max_iters", C.c_int64), ("eval_every", C.c_int32),
        ("scaling", C.c_int32), ("ruiz_passes", C.c_int32), ("pow_iters", C.c_int32),
        ("restarts", C.c_int32), ("pad0", C.c_int32), ("eta", C.c_double), ("omega0", C.c_double),
        ("seed", C.c_uint64), ("x0", C.c_void_p), ("y0", C.c_void_p),
        ("n_snap", C.c_int32), ("pad1", C.c_int32), ("snap_k", C.c_void_p), ("snap_out", C.c_void_p),
        ("trace_cap", C.c_int32), ("pad2", C.c_int32), ("trace", C.c_void_p), ("eps_infeas", C.c_double),
        ("method", C.c_int32), ("restart_metric", C.c_int32), ("reflection", C.c_double),
        ("omega_steps", C.c_int32), ("pad4", C.c_int32), ("pw_rule", C.c_int32), ("pad5", C.c_int32),
        ("pid_kp", C.c_double), ("pid_ki", C.c_double), ("pid_kd", C.c_double),
        ("term_mode", C.c_int32), ("ray_candidates", C.c_int32),
    ]


class _InfoStruct(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("output_is_avg", C.c_int32), ("iters", C.c_int64),
        ("restarts", C.c_int64), ("n_trace", C.c_int64), ("pobj", C.c_double), ("dobj", C.c_double),
        ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double), ("erel", C.c_double),
        ("sigma_max", C.c_double), ("eta", C.c_double), ("omega", C.c_double),
        ("setup_s", C.c_double), ("iter_s", C.c_double), ("ray_source", C.c_int32), ("pad", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LOAD_PATH):
            build()
        L = C.CDLL(_LOAD_PATH)
        P = C.c_void_p
        L.ora_validate.argtypes = [P]
        L.ora_validate.restype = C.c_int
        L.ora_transpose.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P]
        L.ora_transpose.restype = None
        L.ora_scale.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.c_int32, P, P]
        L.ora_scale.restype = None
        L.ora_power_norm.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P, C.c_int32, C.c_uint64]
        L.ora_power_norm.restype = C.c_double
        L.ora_scaled_problem.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P, P]
        L.ora_scaled_problem.restype = C.c_int
        L.ora_kkt.argtypes = [P, P, P, P, P]
        L.ora_kkt.restype = C.c_int
        L.ora_default_opts.argtypes = [P]
        L.ora_default_opts.restype = None
        L.ora_solve.argtypes = [P, P, P, P, P, P]
        L.ora_solve.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Bound:
    """Keeps the contiguous copies alive while the C struct points at them."""

    def __init__(self, lp):
        self.rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int32)
        self.ci = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
        self.v = np.ascontiguousarray(lp.vals, dtype=np.float64)
        self.c = np.ascontiguousarray(lp.c, dtype=np.float64)
        self.bl = np.ascontiguousarray(lp.b_lo, dtype=np.float64)
        self.bh = np.ascontiguousarray(lp.b_hi, dtype=np.float64)
        self.xl = np.ascontiguousarray(lp.x_lo, dtype=np.float64)
        self.xh = np.ascontiguousarray(lp.x_hi, dtype=np.float64)
        self.s = _LPStruct(lp.m, lp.n, int(self.rp[-1]) if len(self.rp) else 0, _ptr(self.rp), _ptr(self.ci),
                           _ptr(self.v), _ptr(self.c), float(lp.c0), _ptr(self.bl), _ptr(self.bh),
                           _ptr(self.xl), _ptr(self.xh))


def validate(lp) -> int:
    b = _Bound(lp)
    return lib().ora_validate(C.byref(b.s))


def transpose(m: int, n: int, row_ptr, col_idx, vals):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    nnz = int(rp[m])
    rpT = np.empty(n + 1, np.int32)
    ciT = np.empty(max(nnz, 1), np.int32)
    vT = np.empty(max(nnz, 1), np.float64)
    lib().ora_transpose(m, n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(rpT), _ptr(ciT), _ptr(vT))
    return rpT, ciT[:nnz], vT[:nnz]


def scale(m: int, n: int, row_ptr, col_idx, vals, ruiz: int = 10, pock_chambolle: bool = True):
    """Return (A~ values, R, C) of the power-of-two Ruiz + Pock-Chambolle scaling."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    av = np.array(vals, dtype=np.float64, copy=True)
    R = np.empty(max(m, 1))
    Cc = np.empty(n)
    lib().ora_scale(m, n, _ptr(rp), _ptr(ci), _ptr(av), ruiz, int(pock_chambolle), _ptr(R), _ptr(Cc))
    return av, R[:m], Cc


def power_norm(m, n, row_ptr, col_idx, vals, iters: int = 200, seed: int = 0x5EED0C0FFEE) -> float:
    rpT, ciT, vT = transpose(m, n, row_ptr, col_idx, vals)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    return lib().ora_power_norm(m, n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(rpT), _ptr(ciT), _ptr(vT), iters,
                                C.c_uint64(seed))


def scaled_problem(lp, scaling: bool = True, ruiz: int = 10):
    """(A~ values in CSR order, R, C, A~^T row_ptr, col_idx, values)."""
    b = _Bound(lp)
    nnz = b.s.nnz
    av = np.empty(max(nnz, 1))
    R = np.empty(max(lp.m, 1))
    Cc = np.empty(lp.n)
    rpT = np.empty(lp.n + 1, np.int32)
    ciT = np.empty(max(nnz, 1), np.int32)
    avT = np.empty(max(nnz, 1))
    rc = lib().ora_scaled_problem(C.byref(b.s), int(scaling), ruiz, _ptr(av), _ptr(R), _ptr(Cc), _ptr(rpT),
                                  _ptr(ciT), _ptr(avT))
    if rc:
        raise ValueError(f"oracle rejected the LP (code {rc})")
    return av[:nnz], R[: lp.m], Cc, rpT, ciT[:nnz], avT[:nnz]


def kkt(lp, x, y):
    """KKT check on the original data: dict(rel_p, rel_d, rel_gap, erel, pobj, dobj, z)."""
    b = _Bound(lp)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64) if lp.m else np.zeros(1)
    out = np.empty(6)
    z = np.empty(lp.n)
    rc = lib().ora_kkt(C.byref(b.s), _ptr(x), _ptr(y), _ptr(out), _ptr(z))
    if rc:
        raise ValueError(f"oracle rejected the LP (code {rc})")
    return dict(rel_p=out[0], rel_d=out[1], rel_gap=out[2], erel=out[3], pobj=out[4], dobj=out[5], z=z)


@dataclass
class Result:
    status: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    iters: int
    restarts: int
    pobj: float
    dobj: float
    rel_p: float
    rel_d: float
    rel_gap: float
    erel: float
    sigma_max: float
    eta: float
    omega: float
    setup_s: float
    iter_s: float
    output_is_avg: bool
    trace: np.ndarray = field(default_factory=lambda: np.zeros((0, TRACE_W)))
    snaps: Optional[np.ndarray] = None
    ray_source: int = 0  # candidate that gave a certificate: 1 displacement, 2 anchored average


def solve(lp, *, eps_rel: float = 1e-4, max_iters: int = 100000, eval_every: int = 64, scaling: bool = True,
          ruiz_passes: int = 10, pow_iters: int = 200, restarts: bool = True, eta: float = 0.0,
          omega0: float = 0.0, seed: int = 0x5EED0C0FFEE, x0=None, y0=None,
          snap_k: Sequence[int] = (), trace_cap: int = 4096, eps_infeas: float = 1e-8, method: int = 0,
          reflection: float = 1.0, omega_steps: int = 0, pw_rule: int = 0, pid_kp: Optional[float] = None,
          pid_ki: Optional[float] = None, pid_kd: Optional[float] = None, term_mode: int = 0,
          ray_candidates: int = 0, restart_metric: int = 0) -> Result:
    """Run the oracle. `snap_k` lists iterations whose scaled-space state
    (x~, y~, x~avg, y~avg) is recorded right after the update of that iteration.
    `ray_candidates`: 0 both candidate rays, 1 the displacement since the previous evaluation
    only, 2 the averaged point's displacement from the restart anchor only.
    `restart_metric` (Halpern form): 0 the restart tests compare KKT_omega values, 1 they
    compare fixed-point residuals ||z - T(z)|| in the PDHG norm."""
    b = _Bound(lp)
    o = _OptsStruct()
    lib().ora_default_opts(C.byref(o))
    o.eps_rel = eps_rel
    o.max_iters = max_iters
    o.eval_every = eval_every
    o.scaling = int(scaling)
    o.ruiz_passes = ruiz_passes
    o.pow_iters = pow_iters
    o.restarts = int(restarts)
    o.eta = eta
    o.omega0 = omega0
    o.seed = seed
    o.eps_infeas = eps_infeas
    o.method = method
    o.reflection = reflection
    o.omega_steps = omega_steps
    o.pw_rule = pw_rule
    o.term_mode = term_mode
    o.ray_candidates = ray_candidates
    o.restart_metric = restart_metric
    if pid_kp is not None:
        o.pid_kp = pid_kp
    if pid_ki is not None:
        o.pid_ki = pid_ki
    if pid_kd is not None:
        o.pid_kd = pid_kd
    keep = []
    if x0 is not None:
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        keep.append(x0)
        o.x0 = _ptr(x0)
    if y0 is not None:
        y0 = np.ascontiguousarray(y0, dtype=np.float64)
        keep.append(y0)
        o.y0 = _ptr(y0)
    sk = np.ascontiguousarray(sorted(snap_k), dtype=np.int64)
    snaps = np.zeros((len(sk), 2 * lp.n + 2 * lp.m)) if len(sk) else None
    if len(sk):
        o.n_snap = len(sk)
        o.snap_k = _ptr(sk)
        o.snap_out = _ptr(snaps)
    trace = np.zeros((trace_cap, TRACE_W))
    o.trace_cap = trace_cap
    o.trace = _ptr(trace)
    x = np.empty(lp.n)
    y = np.empty(max(lp.m, 1))
    z = np.empty(lp.n)
    info = _InfoStruct()
    rc = lib().ora_solve(C.byref(b.s), C.byref(o), _ptr(x), _ptr(y), _ptr(z), C.byref(info))
    if rc:
        raise ValueError(f"oracle rejected the LP (code {rc})")
    ntr = min(int(info.n_trace), trace_cap)
    return Result(STATUS.get(info.status, str(info.status)), x, y[: lp.m], z, int(info.iters), int(info.restarts),
                  info.pobj, info.dobj, info.rel_p, info.rel_d, info.rel_gap, info.erel, info.sigma_max, info.eta,
                  info.omega, info.setup_s, info.iter_s, bool(info.output_is_avg), trace[:ntr].copy(), snaps,
                  int(info.ray_source))


def split_snap(snap: np.ndarray, n: int, m: int):
    """(x~, y~, x~avg, y~avg) views of one snapshot row."""
    return snap[:n], snap[n : n + m], snap[n + m : 2 * n + m], snap[2 * n + m :]


@dataclass
class Polished:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    primal_iters: int
    dual_iters: int
    primal_status: str
    dual_status: str
    kkt: dict


def polish(lp, x, y, *, eps: float = 1e-8, max_iters: int = 100000, method: int = 0, **kw) -> Polished:
    """Feasibility polishing of an approximate solution (x, y) (original scale): two more
    restarted-PDHG solves warm-started at it, each stopped on one residual alone.

    Primal: the same constraints with the objective removed (c = 0), started at (x, 0) and run
    until the relative primal residual is at most eps: its iterate is a point that satisfies
    the constraints to eps near x. Dual: the same matrix and costs with every finite row and
    variable bound set to 0 (the recession cone of the feasible set, whose dual constraints
    are those of the LP), started at (0, y) and run until the relative dual residual is at
    most eps: its y is dual feasible to eps near y. Reading (the paper names the PDLP family;
    this is that family's polishing): the polished point is (x_primal, y_dual), z its projected
    reduced cost, and its KKT record on the original data is returned. Both solves take the
    modified LP's own primal weight (1: one of ||c|| and ||q|| vanishes) and the same step."""
    import dataclasses

    zero_c = dataclasses.replace(lp, c=np.zeros(lp.n)) if dataclasses.is_dataclass(lp) else _with(lp, c=np.zeros(lp.n))
    cone = dict(b_lo=np.where(np.isfinite(lp.b_lo), 0.0, lp.b_lo), b_hi=np.where(np.isfinite(lp.b_hi), 0.0, lp.b_hi),
                x_lo=np.where(np.isfinite(lp.x_lo), 0.0, lp.x_lo), x_hi=np.where(np.isfinite(lp.x_hi), 0.0, lp.x_hi))
    homog = dataclasses.replace(lp, **cone) if dataclasses.is_dataclass(lp) else _with(lp, **cone)
    rp = solve(zero_c, eps_rel=eps, max_iters=max_iters, x0=x, y0=np.zeros(lp.m), eps_infeas=0.0, method=method,
               term_mode=1, **kw)
    rd = solve(homog, eps_rel=eps, max_iters=max_iters, x0=np.zeros(lp.n), y0=y, eps_infeas=0.0, method=method,
               term_mode=2, **kw)
    k = kkt(lp, rp.x, rd.y)
    return Polished(rp.x, rd.y, k["z"], rp.iters, rd.iters, rp.status, rd.status, k)


def _with(lp, **fields):
    import copy

    out = copy.copy(lp)
    for key, v in fields.items():
        setattr(out, key, v)
    return out
