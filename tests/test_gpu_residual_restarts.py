"""Restarts on the fixed-point residual (Halpern form, restart_metric 1) on the GPU against the
oracle: iterates of the first 200 iterations and the decision trace (the residual of the last
iterate and of the anchor in the trace's KKT columns), solves to 1e-4 with the oracle's
iteration and restart counts, every batched path equal to the solo solve bit for bit, the
FP32 form, a run split by a pause, and the option switched on an existing handle."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from test_gpu_parity import CASES, ITER_TOL, _case, _close

pytestmark = pytest.mark.gpu
R = dict(method=lpg.LP_METHOD_HALPERN, restart_metric=1)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_iterates_and_trace_first_200(oracle_lib, name, layout):
    lp = _case(name)
    ks = list(range(1, 201))
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=200, snap_k=ks, **R)
    print(f"{name} layout {layout}", flush=True)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, spmv_layout=layout, small_lp_lds=0, **R) as s:
        for k in ks:
            s.update(eps_rel=0.0, max_iters=k, **R)
            sol = s.solve()
            assert sol.info.iterations == k
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[k - 1], lp.n, lp.m)):
                assert _close(a, b) <= ITER_TOL, (name, k)
        tr = lpg.lp_get_trace(s.h)
    ot = ref.trace
    assert len(tr) == len(ot)
    np.testing.assert_array_equal(tr[:, [0, 1, 6, 7]], ot[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(tr[:, [2, 3, 4, 5, 8, 9]], ot[:, [2, 3, 4, 5, 8, 9]], rtol=1e-9)


@pytest.mark.parametrize("name", CASES)
def test_solve_parity(oracle_lib, name):
    lp = _case(name)
    ref = oracle.solve(lp, eps_rel=1e-4, max_iters=200000, **R)
    kkt = oracle.solve(lp, eps_rel=1e-4, max_iters=200000, method=1)
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=200000, **R) as s:
        sol = s.solve(with_trace=True)
    print(f"{name}: residual restarts {sol.info.iterations} iterations (oracle {ref.iters}), KKT restarts "
          f"{kkt.iters}", flush=True)
    assert sol.status == ref.status == "optimal"
    assert (sol.info.iterations, sol.info.restarts) == (ref.iters, ref.restarts)
    np.testing.assert_array_equal(sol.trace[:, [0, 1, 7]], ref.trace[:, [0, 1, 7]])
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert chk["erel"] <= 1e-4
    assert abs(sol.info.primal_obj - ref.pobj) <= 1e-6 * max(1.0, abs(ref.pobj))


def test_pid_weight_parity(oracle_lib):
    lp = _case("cfg0")
    kw = dict(pw_rule=lpg.LP_PW_PID, **R)
    ref = oracle.solve(lp, eps_rel=1e-6, max_iters=200000, **kw)
    with lpg.Solver(lp, eps_rel=1e-6, max_iters=200000, **kw) as s:
        sol = s.solve(with_trace=True)
    print(f"PID: {sol.info.iterations} iterations (oracle {ref.iters})", flush=True)
    assert (sol.status, sol.info.iterations, sol.info.restarts) == (ref.status, ref.iters, ref.restarts)
    np.testing.assert_allclose(sol.trace[:, 8], ref.trace[:, 8], rtol=1e-9)


@pytest.mark.parametrize("split", [10**9, 0], ids=["persistent", "block_diagonal"])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single(split, precision):
    lps = [synth.cfg0(0), synth.transportation(80, np.random.default_rng(2)), synth.cfg4_lp(4, m_hi=600),
           synth.cfg3_lp(9, m_max=300)]
    opts = dict(eps_rel=1e-5, max_iters=200000, spmv_layout=1, precision=precision, **R)
    print(f"batch split {split} precision {precision}", flush=True)
    solo = []
    for lp in lps:
        with lpg.Solver(lp, small_lp_lds=0, **opts) as s:
            solo.append(s.solve(with_trace=True))
    solvers = [lpg.Solver(lp, **opts) for lp in lps]
    try:
        mix = lpg.solve_batch(solvers, batch_split_nnz=split, **opts)
        traces = [lpg.lp_get_trace(s.h) for s in solvers]
    finally:
        for s in solvers:
            s.close()
    for a, b, tb in zip(solo, mix, traces):
        assert a.status == b.status == "optimal"
        assert (a.info.iterations, a.info.restarts) == (b.info.iterations, b.info.restarts)
        np.testing.assert_array_equal(a.x, b.x)
        np.testing.assert_array_equal(a.y, b.y)
        np.testing.assert_array_equal(a.trace, tb)


@pytest.mark.parametrize("precision", [0, 1])
def test_one_workgroup_solve_equals_kernel_loop(precision):
    """lp_solve of a small LP on one workgroup from LDS against the kernel-per-phase loop."""
    lp = synth.cfg0(1)
    opts = dict(eps_rel=1e-6, max_iters=200000, spmv_layout=1, precision=precision, **R)
    out = []
    for extra in ({}, {"small_lp_lds": 0}):
        with lpg.Solver(lp, **opts, **extra) as s:
            out.append(s.solve(with_trace=True))
    a, b = out
    assert a.info.solve_path == 1 and b.info.solve_path == 0
    assert (a.status, a.info.iterations, a.info.restarts) == (b.status, b.info.iterations, b.info.restarts)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.x, b.x)


@pytest.mark.parametrize("name", ["cfg0", "serving_recipe_small"])
def test_fp32_form_to_1e8(oracle_lib, name):
    lp = _case(name)
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=400000, precision=lpg.LP_PREC_FP32_REFINED, **R) as s:
        sol = s.solve()
    chk = oracle.kkt(lp, sol.x, sol.y)
    print(f"{name} FP32 residual restarts to 1e-8: {sol.status} {sol.info.iterations} it, "
          f"E_rel {chk['erel']:.2e}", flush=True)
    assert sol.status == "optimal" and chk["erel"] <= 1e-8 * (1 + 1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_paused_run_equals_straight_run(precision):
    """The anchor's residual is part of the state a pause keeps: a run split twice (and moved to
    a second handle through lp_export_state) equals the uninterrupted one."""
    lp = synth.transportation(120, np.random.default_rng(3))
    opts = dict(eps_rel=1e-7, max_iters=200000, spmv_layout=1, small_lp_lds=0, precision=precision, **R)
    with lpg.Solver(lp, **opts) as s:
        ref = s.solve(with_trace=True)
    total = ref.info.iterations
    assert total >= 256
    with lpg.Solver(lp, **opts) as a:
        a.solve_until(total // 3 - 7)
        state = a.export_state()
    with lpg.Solver(lp, **opts) as b:
        b.import_state(state)
        b.resume((2 * total) // 3)
        out = b.resume(with_trace=True)
    assert (out.status, out.info.iterations, out.info.restarts) == (ref.status, ref.info.iterations, ref.info.restarts)
    np.testing.assert_array_equal(out.trace, ref.trace)
    np.testing.assert_array_equal(out.x, ref.x)


def test_option_switched_on_a_handle():
    """lp_update_options turning the residual restarts on and off gives the runs of handles
    created with those options (the captured iteration bundle is rebuilt)."""
    lp = synth.cfg0(0)
    base = dict(eps_rel=1e-5, max_iters=200000, spmv_layout=1, small_lp_lds=0, method=lpg.LP_METHOD_HALPERN)
    fresh = {}
    for rm in (0, 1):
        with lpg.Solver(lp, restart_metric=rm, **base) as s:
            fresh[rm] = s.solve(with_trace=True)
    assert fresh[0].info.iterations != fresh[1].info.iterations or not np.array_equal(fresh[0].trace, fresh[1].trace)
    with lpg.Solver(lp, **base) as s:
        for rm in (0, 1, 0):
            s.update(restart_metric=rm, **base)
            sol = s.solve(with_trace=True)
            np.testing.assert_array_equal(sol.trace, fresh[rm].trace)
            np.testing.assert_array_equal(sol.x, fresh[rm].x)
