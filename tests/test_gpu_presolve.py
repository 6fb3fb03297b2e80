"""Presolve (host) + restarted PDHG on the GPU + postsolve, end to end (Section 3 with the
solver of Section 4). The postsolved point is checked on the original LP by the oracle's KKT
routine and against the planted optimum."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from conftest import golden_lps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def planted():
    return synth.presolve_lp(1, m=1500, n=3000, density=0.004)


def test_presolved_solve_matches_planted_optimum(oracle_lib, planted):
    lp = planted
    r = lpg.solve_presolved(lp, eps_rel=1e-7, max_iters=400000)
    print(f"presolve {r.presolve['m']}x{r.presolve['n']} from {lp.m}x{lp.n}; reduced solve: {r.reduced.status} "
          f"{r.reduced.info.iterations} it, E_rel {r.reduced.info.rel_kkt:.2e}; times {r.times}")
    assert r.status == "optimal"
    chk = oracle.kkt(lp, r.x, r.y)
    print(f"postsolved E_rel on the original: {chk['erel']:.3e}; p = {chk['pobj']:.12g} vs p* = {lp.p_star:.12g}")
    assert chk["erel"] <= 1e-5
    assert abs(chk["pobj"] - lp.p_star) <= 1e-5 * (1 + abs(lp.p_star))
    # the solver's own evaluation of the postsolved point agrees with the oracle; the handle
    # clamps the warm start into the variable bounds first, and a substituted variable can sit
    # outside its bounds by the reduced row's residual, so the two agree to about 1e-3
    info = lpg.evaluate(lp, r.x, r.y)
    assert info.rel_kkt == pytest.approx(chk["erel"], rel=1e-2, abs=1e-14)
    # z is the reduced cost of the original LP at y up to the dual residual (the solver returns
    # the reduced cost projected onto the sign pattern of eq. 2 for the columns it kept)
    zc = lp.c - lp.dense().T @ r.y
    assert np.max(np.abs(r.z - zc)) <= 10 * chk["erel"] * (1 + np.linalg.norm(lp.c))


def test_presolve_reduces_work(planted):
    lp = planted
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=400000) as s:
        direct = s.solve()
    r = lpg.solve_presolved(lp, eps_rel=1e-4, max_iters=400000)
    print(f"direct: {direct.info.iterations} it {direct.info.solve_seconds:.3f}s; presolved: "
          f"{r.reduced.info.iterations} it {r.times}")
    assert direct.status == "optimal" and r.status == "optimal"
    assert r.presolve["nnz"] < lp.nnz


def test_presolve_decides_small_lp_alone():
    lp, spec = golden_lps()["T1"]
    r = lpg.solve_presolved(lp, eps_rel=1e-6)
    assert r.status == "optimal" and r.reduced is None
    np.testing.assert_allclose(r.x, [1.0, 2.0])
    info = lpg.evaluate(lp, r.x, r.y)
    assert info.rel_kkt <= 1e-15


def test_presolved_fp32_form(oracle_lib, planted):
    lp = planted
    r = lpg.solve_presolved(lp, eps_rel=1e-6, max_iters=400000, precision=lpg.LP_PREC_FP32_REFINED)
    assert r.status == "optimal"
    chk = oracle.kkt(lp, r.x, r.y)
    print(f"FP32 form, postsolved E_rel {chk['erel']:.3e}")
    assert chk["erel"] <= 1e-4
    assert abs(chk["pobj"] - lp.p_star) <= 1e-4 * (1 + abs(lp.p_star))
