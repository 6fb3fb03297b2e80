"""The reflected Halpern form (method 1) on the GPU against the oracle: iterates of the first
200 iterations (Halpern iterate and PDHG output), restart decisions, solves, layouts, the
FP32 form, the batched paths and the certificates."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from test_gpu_parity import CASES, ITER_TOL, _case, _close
from test_oracle_infeasible import EPS, check_dual_ray, check_primal_ray, infeasible_lps

pytestmark = pytest.mark.gpu
H = dict(method=lpg.LP_METHOD_HALPERN)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_iterates_first_200(oracle_lib, name, layout):
    lp = _case(name)
    ks = list(range(1, 201))
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=200, snap_k=ks, method=1)
    worst = 0.0
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, spmv_layout=layout, **H) as s:
        for k in ks:
            s.update(eps_rel=0.0, max_iters=k, **H)
            sol = s.solve()
            assert sol.info.iterations == k
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[k - 1], lp.n, lp.m)):
                d = _close(a, b)
                worst = max(worst, d)
                assert d <= ITER_TOL, (name, k, d)
        tr = lpg.lp_get_trace(s.h)
    ot = ref.trace
    assert len(tr) == len(ot)
    np.testing.assert_array_equal(tr[:, [0, 1, 6, 7]], ot[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(tr[:, [2, 3, 4, 5, 8]], ot[:, [2, 3, 4, 5, 8]], rtol=1e-10)
    print(f"{name} layout {layout}: worst relative iterate difference {worst:.3e}")


@pytest.mark.parametrize("name", CASES)
def test_solve_parity(oracle_lib, name):
    lp = _case(name)
    ref = oracle.solve(lp, eps_rel=1e-4, max_iters=200000, method=1)
    avg = oracle.solve(lp, eps_rel=1e-4, max_iters=200000)
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=200000, **H) as s:
        sol = s.solve()
    print(f"{name}: Halpern {sol.info.iterations} iterations (oracle {ref.iters}), averaged form {avg.iters}")
    assert sol.status == ref.status == "optimal"
    assert sol.info.iterations == ref.iters
    assert sol.info.restarts == ref.restarts
    assert abs(sol.info.primal_obj - ref.pobj) <= 1e-6 * max(1.0, abs(ref.pobj))
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert chk["erel"] <= 1e-4
    assert abs(chk["erel"] - sol.info.rel_kkt) <= 1e-9 * max(chk["erel"], 1e-12) + 1e-15
    assert np.all(sol.x >= lp.x_lo) and np.all(sol.x <= lp.x_hi)  # the returned point is T(z)


@pytest.mark.parametrize("name", ["cfg0", "serving_recipe_small"])
@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_fp32_form(oracle_lib, name, eps):
    lp = _case(name)
    with lpg.Solver(lp, eps_rel=eps, max_iters=400000, precision=lpg.LP_PREC_FP32_REFINED, **H) as s:
        sol = s.solve()
    chk = oracle.kkt(lp, sol.x, sol.y)
    print(f"{name} FP32 Halpern to {eps}: {sol.status} {sol.info.iterations} it, E_rel {chk['erel']:.2e}")
    assert sol.status == "optimal"
    assert chk["erel"] <= eps * (1 + 1e-9)


@pytest.mark.parametrize("split", [10**9, 0])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single(split, precision):
    lps = [synth.cfg0(0), synth.transportation(80, np.random.default_rng(2)), synth.cfg4_lp(4, m_hi=600),
           synth.cfg3_lp(9, m_max=300)]
    opts = dict(eps_rel=1e-5, max_iters=200000, spmv_layout=1, precision=precision, **H)
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


@pytest.mark.parametrize("name", ["I1", "I2", "U1", "U2"])
def test_certificates(oracle_lib, name):
    lp, spec = infeasible_lps()[name]
    ref = oracle.solve(lp, eps_rel=1e-8, max_iters=20000, eps_infeas=EPS, method=1)
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=20000, eps_infeas=EPS, **H) as s:
        sol = s.solve()
    assert sol.status == ref.status == spec["status"]
    assert sol.info.iterations == ref.iters
    if sol.status == "primal_infeasible":
        check_dual_ray(lp, sol.y, sol.z, 2 * EPS)
    else:
        check_primal_ray(lp, sol.x, 2 * EPS)


def test_time_limit_returns_pdhg_output():
    lp = synth.cfg0(0)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=10**7, time_limit_s=0.05, **H) as s:
        sol = s.solve()
    assert sol.status == "time_limit"
    assert np.all(sol.x >= lp.x_lo) and np.all(sol.x <= lp.x_hi)
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert abs(chk["erel"] - sol.info.rel_kkt) <= 1e-9 * max(chk["erel"], 1e-12)


def test_update_switches_form():
    """lp_update_options changes the form of a handle (and drops its captured bundle)."""
    lp = _case("cfg0")
    opts = dict(eps_rel=1e-4, max_iters=200000)
    with lpg.Solver(lp, **opts) as s:
        a = s.solve()
        s.update(**opts, **H)
        h = s.solve()
        s.update(**opts)
        a2 = s.solve()
    with lpg.Solver(lp, **opts, **H) as s2:
        h2 = s2.solve()
    assert h.info.iterations == h2.info.iterations != a.info.iterations
    assert np.array_equal(h.x, h2.x)
    assert a.info.iterations == a2.info.iterations and np.array_equal(a.x, a2.x)


@pytest.mark.parametrize("layout", [0, 1])
def test_close_gap_lp_step_condition(oracle_lib, layout):
    """A 90-row LP of the batched recipe whose two largest singular values are 0.4% apart:
    the power iteration goes past its first chunk on the device as in the oracle (same
    estimate to 1e-12), eta ||A~|| stays below 1, and the reflected Halpern form solves it
    with the oracle's iteration count."""
    lp = synth.cfg3_lp(2564)
    ref = oracle_lib.solve(lp, eps_rel=1e-4, max_iters=20000, method=1)
    assert ref.status == "optimal"
    with lpg.Solver(lp, spmv_layout=layout, eps_rel=1e-4, max_iters=20000, method=1) as s:
        sol = s.solve()
    assert abs(sol.info.sigma_max - ref.sigma_max) <= 1e-12 * ref.sigma_max
    assert sol.status == "optimal" and sol.info.iterations == ref.iters
    # the batched FP32 form reaches the tolerance too (it hit the iteration limit before)
    with lpg.Solver(lp, spmv_layout=1, precision=lpg.LP_PREC_FP32_REFINED, method=1) as s:
        (b,) = lpg.solve_batch([s], eps_rel=1e-4, max_iters=20000, method=1)
    assert b.status == "optimal"
