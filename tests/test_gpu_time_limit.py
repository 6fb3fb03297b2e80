"""time_limit_s in the batched and served solves, checked on the device at every evaluation.

A limit far below one evaluation period stops every LP at its first evaluation (iteration 64,
with eval_every 64) with LP_TIME_LIMIT. In the Halpern form the point returned there is the
PDHG output, which is also what a solve stopped by max_iters = 64 returns, so the stopped
batch must equal 64-iteration single solves bit for bit: in the persistent launch, in the
block-diagonal launches, in the allocation-free form and in a server. A limit of a fraction
of a second on LPs that would run far longer must end the call soon after it."""
import time

import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu
HALPERN = dict(method=lpg.LP_METHOD_HALPERN, spmv_layout=1)
TINY = 1e-7  # seconds: shorter than any evaluation period


def _lps():
    rng = np.random.default_rng(17)
    return [synth.cfg0(0), synth.transportation(60, rng), synth.cfg3_lp(3, m_max=300), synth.cfg4_lp(2, m_hi=500)]


def _single_64(lp):
    with lpg.Solver(lp, eps_rel=1e-14, max_iters=64, **HALPERN) as s:
        return s.solve()


def _check_stopped(lps, sols):
    for lp, sol in zip(lps, sols):
        ref = _single_64(lp)
        assert sol.status == "time_limit", (lp.name, sol.status)
        assert sol.info.iterations == 64, (lp.name, sol.info.iterations)
        assert ref.status == "iteration_limit"
        np.testing.assert_array_equal(sol.x, ref.x)
        np.testing.assert_array_equal(sol.y, ref.y)
        assert sol.info.rel_kkt == ref.info.rel_kkt


@pytest.mark.parametrize("split", [1 << 40, 0], ids=["persistent", "block_diagonal"])
def test_batch_stops_at_first_evaluation(split):
    lps = _lps()
    print(f"time limit batch split={split}", flush=True)
    solvers = [lpg.Solver(lp, **HALPERN) for lp in lps]
    try:
        sols = lpg.solve_batch(solvers, eps_rel=1e-14, max_iters=10**7, time_limit_s=TINY,
                               batch_split_nnz=split, **HALPERN)
    finally:
        for s in solvers:
            s.close()
    _check_stopped(lps, sols)


def test_static_batch_stops_at_first_evaluation():
    lps = _lps()
    print("time limit static batch", flush=True)
    solvers = [lpg.Solver(lp, **HALPERN) for lp in lps]
    try:
        lpg.lp_solve_batch_static([s.h for s in solvers],
                                  lpg.make_options(eps_rel=1e-14, max_iters=10**7, time_limit_s=TINY, **HALPERN))
        sols = []
        for s in solvers:
            x, y, z = np.empty(s.n), np.empty(max(s.m, 1)), np.empty(s.n)
            info = lpg.lp_get_solution(s.h, x, y, z)
            sols.append(lpg.Solution(lpg.STATUS[info.status], x, y[: s.m], z, info))
    finally:
        for s in solvers:
            s.close()
    _check_stopped(lps, sols)


def test_server_requests_stop_at_first_evaluation():
    lps = _lps()
    print("time limit server", flush=True)
    tmpls = [lpg.Solver(lp, deferred=1, **HALPERN) for lp in lps]
    try:
        with lpg.Server(1 << 34, 8, eps_rel=1e-14, max_iters=10**7, time_limit_s=TINY, **HALPERN) as srv:
            tickets = [srv.submit(t) for t in tmpls]
            srv.wait(60.0)
            sols = [srv.result(t) for t in tickets]
    finally:
        for t in tmpls:
            t.close()
    _check_stopped(lps, sols)


@pytest.mark.parametrize("split", [1 << 40, 0], ids=["persistent", "block_diagonal"])
def test_batch_limit_bounds_the_call(split):
    """LPs asked for 1e-14 within 10^7 iterations, with a 0.4 s limit."""
    lps = [synth.cfg4_lp(j, m_lo=400, m_hi=900) for j in range(6)]
    limit = 0.4
    solvers = [lpg.Solver(lp, spmv_layout=1) for lp in lps]
    try:
        t = time.perf_counter()
        sols = lpg.solve_batch(solvers, eps_rel=1e-14, max_iters=10**7, time_limit_s=limit, batch_split_nnz=split,
                               spmv_layout=1)
        wall = time.perf_counter() - t
    finally:
        for s in solvers:
            s.close()
    its = [s.info.iterations for s in sols]
    print(f"split={split}: call {wall:.3f} s, iterations {its}", flush=True)
    # an LP may still reach 1e-14 before the limit; the others stop at an evaluation
    assert all(s.status in ("time_limit", "optimal") for s in sols)
    assert any(s.status == "time_limit" for s in sols)
    assert all(k > 64 and k % 64 == 0 for s, k in zip(sols, its) if s.status == "time_limit")
    assert wall < limit + 1.0
    for s in sols:
        assert np.isfinite(s.info.rel_kkt) and np.all(np.isfinite(s.x))
