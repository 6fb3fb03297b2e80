"""Serving form: continuous batching of LPs that arrive while others run.

Bars: every served LP's result is bit-identical to the same LP solved alone (lp_solve with
the row-tile layout and the same solve-time options); the admitted device footprint never
exceeds the HBM budget; an LP that cannot converge leaves the others' results unchanged;
FP32 LPs reach the tolerance (checked in FP64 by the oracle)."""
import time

import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
from test_oracle_infeasible import check_primal_ray
import synth
from conftest import golden_lps

pytestmark = pytest.mark.gpu

OPTS = dict(eps_rel=1e-5, max_iters=200000)


def _pool():
    lps = [synth.cfg4_lp(j, m_hi=3000) for j in range(6)]
    lps += [synth.cfg0(2), synth.transportation(200, np.random.default_rng(8)), synth.cfg1(1, m=800, n=1600, nnz=9000)]
    lps += [synth.cfg3_lp(j, m_max=600) for j in range(3)]
    return lps


def _solo(lp, **kw):
    with lpg.Solver(lp, spmv_layout=1, **OPTS, **kw) as s:
        return s.solve()


def _serve(lps, budget, slots, stagger=0.0, srv_kw=None, **kw):
    solvers = [lpg.Solver(lp, spmv_layout=1, deferred=1, **kw) for lp in lps]
    with lpg.Server(budget, slots, **OPTS, **(srv_kw or {})) as srv:
        tickets = []
        for s in solvers:
            tickets.append(srv.submit(s))
            if stagger:
                time.sleep(stagger)
        srv.wait(120.0)
        done = set()
        for _ in range(100):
            done |= set(srv.poll())
            if len(done) == len(tickets):
                break
            time.sleep(0.01)
        assert done == set(tickets)
        sols = [srv.result(t) for t in tickets]
        times = [srv.times(t) for t in tickets]
        st = srv.stats()
    return solvers, sols, times, st


@pytest.mark.parametrize("method", [lpg.LP_METHOD_AVERAGED, lpg.LP_METHOD_HALPERN])
def test_served_results_equal_solo(method):
    lps = _pool()
    solvers, sols, times, st = _serve(lps, budget=1 << 34, slots=64, stagger=0.002, srv_kw=dict(method=method))
    for lp, sol in zip(lps, sols):
        ref = _solo(lp, method=method)
        assert sol.status == ref.status and sol.info.iterations == ref.info.iterations, lp.name
        assert np.array_equal(sol.x, ref.x) and np.array_equal(sol.y, ref.y) and np.array_equal(sol.z, ref.z)
    assert st["completed"] == len(lps) and st["bytes_in_use"] == 0
    for t in times:
        assert t[0] <= t[1] <= t[2]
    for s in solvers:
        s.close()


def test_same_template_submitted_many_times():
    lp = synth.cfg4_lp(3, m_hi=2000)
    with lpg.Solver(lp, spmv_layout=1, deferred=1) as tmpl, lpg.Server(1 << 34, 8, **OPTS) as srv:
        tickets = [srv.submit(tmpl) for _ in range(12)]
        srv.wait(120.0)
        sols = [srv.result(t) for t in tickets]
    ref = _solo(lp)
    for sol in sols:
        assert sol.info.iterations == ref.info.iterations and np.array_equal(sol.x, ref.x)


def test_admission_respects_hbm_budget():
    lps = _pool()
    fps = [lpg.Solver(lp, spmv_layout=1, deferred=1).layout()["device_bytes"] for lp in lps]
    budget = int(2.5 * max(fps))
    solvers, sols, times, st = _serve(lps, budget=budget, slots=3)
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(lps)
    # later requests waited for memory: some admission happened after an earlier completion
    assert any(t[1] > min(tt[2] for tt in times) for t in times)
    for lp, sol in zip(lps, sols):
        ref = _solo(lp)
        assert np.array_equal(sol.x, ref.x), lp.name
    for s in solvers:
        s.close()


@pytest.mark.parametrize("eps_infeas", [1e-8, 0.0])
def test_failure_is_isolated(eps_infeas):
    """An unbounded request among feasible ones: with certificates on it ends with a primal
    ray, with them off at the iteration limit; the others get their solo results either way."""
    lps = _pool()[:5]
    bad, _ = golden_lps()["T3"]
    bad.x_hi = np.array([np.inf, 4.0])  # unbounded
    mix = lps[:2] + [bad] + lps[2:]
    solvers = [lpg.Solver(lp, spmv_layout=1, deferred=1) for lp in mix]
    with lpg.Server(1 << 34, 16, eps_rel=1e-5, max_iters=20000, eps_infeas=eps_infeas) as srv:
        tickets = [srv.submit(s) for s in solvers]
        srv.wait(120.0)
        sols = [srv.result(t) for t in tickets]
    if eps_infeas > 0:
        assert sols[2].status == "dual_infeasible"
        check_primal_ray(bad, sols[2].x, 2 * eps_infeas)
    else:
        assert sols[2].status == "iteration_limit"
    for lp, sol in zip(lps, sols[:2] + sols[3:]):
        with lpg.Solver(lp, spmv_layout=1, eps_rel=1e-5, max_iters=20000) as s1:
            ref = s1.solve()
        assert np.array_equal(sol.x, ref.x), lp.name
    for s in solvers:
        s.close()


def test_fp32_served_and_handle_reuse(oracle_lib):
    lps = _pool()[:6]
    fp32 = lpg.LP_PREC_FP32_REFINED
    solvers, sols, times, st = _serve(lps, budget=1 << 34, slots=8, precision=fp32)
    n_opt = 0
    for lp, sol in zip(lps, sols):
        ref = _solo(lp, precision=fp32)
        assert sol.status == ref.status and np.array_equal(sol.x, ref.x), lp.name
        if sol.status == "optimal":
            n_opt += 1
            assert oracle.kkt(lp, sol.x, sol.y)["erel"] <= 1e-5 * (1 + 1e-9)
    assert n_opt >= 4
    # a released handle is placed on the device again by lp_solve and gives the same result
    solvers[0].update(**OPTS)
    again = solvers[0].solve()
    assert np.array_equal(again.x, sols[0].x)
    for s in solvers:
        s.close()
