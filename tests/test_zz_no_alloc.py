"""Allocation-free batched solve (lp_solve_batch_static) against lp_solve_batch.

Every LP of lp_solve_batch_static runs in the persistent one-workgroup-per-LP launch with its
job table in the library's static device array; lp_solve_batch with a split above every LP's
size sends the same LPs to the same launch with a per-call allocation. The results must be
bit-identical, on two calls in a row (the second with fewer and smaller LPs, so the static
table holds stale entries past the new count), and the limits must be rejected cleanly."""
import ctypes as C

import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu

FP32 = lpg.LP_PREC_FP32_REFINED


def _lps(count, m_max):
    out = [synth.cfg3_lp(j, m_max=m_max) for j in range(count - 2)]
    out += [synth.cfg0(0), synth.transportation(min(m_max, 120), np.random.default_rng(5))]
    return out


def _solve(fn, lps, precisions, **opts):
    solvers = [lpg.Solver(lp, spmv_layout=1, precision=p) for lp, p in zip(lps, precisions)]
    try:
        o = lpg.make_options(**opts)
        fn([s.h for s in solvers], o)
        out = []
        for s in solvers:
            x, y, z = np.empty(s.n), np.empty(max(s.m, 1)), np.empty(s.n)
            info = lpg.lp_get_solution(s.h, x, y, z)
            out.append((info.status, info.iterations, info.restarts, info.rel_kkt, x, y[: s.m], z))
        return out
    finally:
        for s in solvers:
            s.close()


def _compare(lps, precisions, **opts):
    print(f"no-alloc batch: {len(lps)} LPs, opts {opts}", flush=True)
    split = 1 << 40
    ref = _solve(lpg.lp_solve_batch, lps, precisions, batch_split_nnz=split, **opts)
    got = _solve(lpg.lp_solve_batch_static, lps, precisions, batch_split_nnz=split, **opts)
    for lp, a, b in zip(lps, ref, got):
        assert a[:3] == b[:3], (lp.name, a[:3], b[:3])
        assert a[3] == b[3], lp.name
        for u, v in zip(a[4:], b[4:]):
            assert np.array_equal(u, v), lp.name
    return got


def test_static_batch_equals_batch_twice():
    lps = _lps(24, 400)
    prec = [FP32 if j % 3 == 0 else lpg.LP_PREC_FP64 for j in range(len(lps))]
    first = _compare(lps, prec, eps_rel=1e-4, max_iters=200000)
    assert all(r[0] == 0 for r in first)
    # second call: fewer, smaller LPs, other form
    small = _lps(8, 120)
    _compare(small, [lpg.LP_PREC_FP64] * len(small), eps_rel=1e-5, max_iters=200000, method=lpg.LP_METHOD_HALPERN)


def test_static_batch_limits():
    with lpg.Solver(synth.cfg0(0), spmv_layout=1) as s:
        too_many = lpg.LP_STATIC_BATCH_MAX + 1
        arr = (C.c_void_p * too_many)(*([s.h.value] * too_many))
        rc = lpg.lib().lp_solve_batch_static(arr, too_many, None)
        assert rc == 1  # LP_ERR_INVALID_ARG
        assert lpg.lib().lp_solve_batch_static(arr, 0, None) == 0
    with lpg.Solver(synth.cfg0(1), spmv_layout=1, deferred=1) as d:
        arr = (C.c_void_p * 1)(d.h.value)
        assert lpg.lib().lp_solve_batch_static(arr, 1, None) == 1  # not on the device yet
