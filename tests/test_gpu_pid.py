"""The PID rule of the primal weight (pw_rule = LP_PW_PID) on the GPU against the oracle:
iterates of the first 200 iterations in both iteration forms (the weight changes at the
restarts of iterations 64, 128, ...), identical decision sequences with the weight after each
decision, solves with the oracle's iteration and restart counts, the batched paths equal to
single solves, and the FP32 form reaching the tolerance."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from test_gpu_parity import ITER_TOL, _case, _close

pytestmark = pytest.mark.gpu
GAINS = dict(pid_kp=0.7, pid_ki=0.05, pid_kd=0.2)
PID = dict(pw_rule=lpg.LP_PW_PID, **GAINS)
ORA_PID = dict(pw_rule=2, **GAINS)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["cfg0", "large_recipe_small", "serving_recipe_small"])
def test_iterates_first_200(oracle_lib, name, method, layout):
    lp = _case(name)
    ks = [1, 2, 63, 64, 65, 66, 127, 128, 129, 191, 192, 193, 200]
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=200, snap_k=ks, method=method, **ORA_PID)
    print(f"{name} method {method} layout {layout}", flush=True)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, spmv_layout=layout, method=method, **PID) as s:
        for i, k in enumerate(ks):
            s.update(eps_rel=0.0, max_iters=k, method=method, **PID)
            sol = s.solve()
            assert sol.info.iterations == k
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                assert _close(a, b) <= ITER_TOL, (name, k, _close(a, b))
        tr = lpg.lp_get_trace(s.h)
    ot = ref.trace
    assert len(tr) == len(ot)
    np.testing.assert_array_equal(tr[:, [0, 1, 6, 7]], ot[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(tr[:, 8], ot[:, 8], rtol=1e-12)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["cfg0", "cfg0b", "transport", "serving_recipe_small"])
def test_solve_parity(oracle_lib, name, method):
    lp = _case(name)
    ref = oracle.solve(lp, eps_rel=1e-4, max_iters=200000, method=method, **ORA_PID)
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=200000, method=method, **PID) as s:
        sol = s.solve(with_trace=True)
    print(f"{name} method {method}: PID {sol.info.iterations} iterations (oracle {ref.iters})")
    assert sol.status == ref.status == "optimal"
    assert sol.info.iterations == ref.iters and sol.info.restarts == ref.restarts
    np.testing.assert_array_equal(sol.trace[:, [0, 1, 6, 7]], ref.trace[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(sol.trace[:, 8], ref.trace[:, 8], rtol=1e-9)
    assert abs(sol.info.primal_obj - ref.pobj) <= 1e-6 * max(1.0, abs(ref.pobj))
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert chk["erel"] <= 1e-4


@pytest.mark.parametrize("split", [10**9, 0])
def test_batch_equals_single(split):
    lps = [synth.cfg0(0), synth.transportation(80, np.random.default_rng(2)), synth.cfg4_lp(4, m_hi=600)]
    opts = dict(eps_rel=1e-5, max_iters=200000, spmv_layout=1, method=lpg.LP_METHOD_HALPERN, **PID)
    solo = []
    for lp in lps:
        with lpg.Solver(lp, **opts) as s:
            solo.append(s.solve())
    solvers = [lpg.Solver(lp, **opts) for lp in lps]
    try:
        mix = lpg.solve_batch(solvers, batch_split_nnz=split, **opts)
    finally:
        for s in solvers:
            s.close()
    for a, b in zip(solo, mix):
        assert a.status == b.status == "optimal" and a.info.iterations == b.info.iterations
        np.testing.assert_array_equal(a.x, b.x)
        np.testing.assert_array_equal(a.y, b.y)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_fp32_form(oracle_lib, eps):
    lp = _case("serving_recipe_small")
    with lpg.Solver(lp, eps_rel=eps, max_iters=400000, precision=lpg.LP_PREC_FP32_REFINED,
                    method=lpg.LP_METHOD_HALPERN, **PID) as s:
        sol = s.solve()
    chk = oracle.kkt(lp, sol.x, sol.y)
    print(f"FP32 Halpern PID to {eps}: {sol.status} {sol.info.iterations} it, E_rel {chk['erel']:.2e}")
    assert sol.status == "optimal"
    assert chk["erel"] <= eps * (1 + 1e-9)
