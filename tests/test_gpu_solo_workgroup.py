"""lp_solve of a small LP on one workgroup from LDS (the default when its iteration arrays fit
small_lp_lds) against the kernel-per-phase loop with the same row tiles (small_lp_lds = 0,
spmv_layout = row tiles): same iterations, restarts, trace, iterates and returned point, bit
for bit, in both iteration forms and both precisions, with warm starts, certificates, time
limits and iteration limits; larger LPs keep the kernel-per-phase loop."""
import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth
from conftest import golden_lps
from test_oracle_infeasible import CASES as INFEASIBLE

pytestmark = pytest.mark.gpu
TILES = dict(spmv_layout=lpg.LP_LAYOUT_TILES)


def _pair(lp, **opts):
    out = []
    for extra in ({}, {"small_lp_lds": 0}):
        with lpg.Solver(lp, **TILES, **opts, **extra) as s:
            sol = s.solve(with_trace=True)
            out.append((sol, s.iterates()))
    return out


def _same(a, b):
    (sa, ia), (sb, ib) = a, b
    assert sa.info.solve_path == 1 and sb.info.solve_path == 0
    assert (sa.status, sa.info.iterations, sa.info.restarts) == (sb.status, sb.info.iterations, sb.info.restarts)
    assert sa.info.ray_source == sb.info.ray_source
    np.testing.assert_array_equal(sa.trace, sb.trace)
    for u, v in zip((sa.x, sa.y, sa.z), (sb.x, sb.y, sb.z)):
        np.testing.assert_array_equal(u, v)
    for u, v in zip(ia, ib):
        np.testing.assert_array_equal(u, v)
    assert sa.info.rel_kkt == sb.info.rel_kkt and sa.info.primal_obj == sb.info.primal_obj


@pytest.mark.parametrize("precision", [lpg.LP_PREC_FP64, lpg.LP_PREC_FP32_REFINED])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["cfg0", "cfg0b", "transport", "batch_small"])
def test_one_workgroup_equals_kernel_loop(name, method, precision):
    lp = {"cfg0": lambda: synth.cfg0(0), "cfg0b": lambda: synth.cfg0(1),
          "transport": lambda: synth.transportation(120, np.random.default_rng(3)),
          "batch_small": lambda: synth.cfg3_lp(2688)}[name]()
    print(f"{name} method {method} precision {precision}", flush=True)
    _same(*_pair(lp, eps_rel=1e-6, max_iters=200000, method=method, precision=precision))


@pytest.mark.parametrize("k", [0, 1, 63, 64, 65, 200])
def test_iteration_limits_and_iterates(k):
    a, b = _pair(synth.cfg0(0), eps_rel=0.0, max_iters=k)
    _same(a, b)
    assert a[0].info.iterations == k


def test_worked_examples_and_warm_start():
    for name, (lp, _) in golden_lps().items():
        _same(*_pair(lp, eps_rel=1e-8, max_iters=50000))
    lp = synth.cfg0(0)
    x0 = np.linspace(0.0, 1.0, lp.n)
    y0 = np.linspace(-1.0, 1.0, lp.m)
    _same(*_pair(lp, eps_rel=1e-6, max_iters=200000, x0=x0, y0=y0))


@pytest.mark.parametrize("name", ["I1", "U1", "pinf2", "unb0"])
def test_certificates(name):
    lp = INFEASIBLE[name]
    a, b = _pair(lp, eps_rel=1e-8, max_iters=100000)
    assert a[0].status in ("primal_infeasible", "dual_infeasible")
    _same(a, b)


def test_time_limit_stops_at_an_evaluation():
    with lpg.Solver(synth.cfg0(0), **TILES, eps_rel=1e-14, max_iters=10**7, time_limit_s=1e-7) as s:
        sol = s.solve()
    assert sol.info.solve_path == 1
    assert sol.status == "time_limit" and sol.info.iterations == 64


def test_larger_lps_and_kernel_timing_keep_the_kernel_loop():
    big = synth.cfg1(0, m=3000, n=6000, nnz=36000)
    with lpg.Solver(big, eps_rel=0.0, max_iters=128) as s:
        assert s.solve().info.solve_path == 0
    with lpg.Solver(synth.cfg0(0), eps_rel=0.0, max_iters=128) as s:
        assert s.solve().info.solve_path == 1
        lpg.lp_set_kernel_timing(s.h, True)
        assert s.solve().info.solve_path == 0
