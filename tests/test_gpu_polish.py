"""Feasibility polishing (lp_polish) on the GPU against the oracle's polishing: the same
numbers of primal and dual polishing iterations, polished points within 1e-8 (both start
from solves that agree to ~1e-13), residuals of the polished pair at most eps on the original
data (the oracle's KKT routine), the handle's data restored afterwards, and the FP32 form."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu


def _lp(name):
    return {"cfg0": lambda: synth.cfg0(0), "large_recipe": lambda: synth.cfg1(0, m=3000, n=6000, nnz=36000),
            "serving": lambda: synth.cfg4_lp(1, m_hi=2000)}[name]()


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["cfg0", "large_recipe", "serving"])
def test_polish_matches_oracle(oracle_lib, name, method):
    lp = _lp(name)
    eps = 1e-9
    ref = oracle.solve(lp, eps_rel=1e-4, max_iters=200000, method=method)
    pol = oracle.polish(lp, ref.x, ref.y, eps=eps, method=method)
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=200000, method=method) as s:
        sol = s.solve()
        assert sol.info.iterations == ref.iters
        p = s.polish(eps=eps, max_iters=100000)
        again = s.solve()
    print(f"{name} method {method}: polish {p.info.polish_primal_iterations}/{p.info.polish_dual_iterations} "
          f"iterations (oracle {pol.primal_iters}/{pol.dual_iters}), rel_p {p.info.rel_primal_res:.2e}, "
          f"rel_d {p.info.rel_dual_res:.2e}, gap {p.info.rel_gap:.2e} (before {sol.info.rel_gap:.2e})")
    assert p.info.polish_primal_iterations == pol.primal_iters
    assert p.info.polish_dual_iterations == pol.dual_iters
    for a, b in ((p.x, pol.x), (p.y, pol.y), (p.z, pol.z)):
        assert float(np.max(np.abs(a - b), initial=0.0)) <= 1e-8 * max(1.0, float(np.max(np.abs(b), initial=0.0)))
    chk = oracle.kkt(lp, p.x, p.y)
    assert chk["rel_p"] <= eps * (1 + 1e-6) and chk["rel_d"] <= eps * (1 + 1e-6)
    assert abs(chk["erel"] - p.info.rel_kkt) <= 1e-8 * max(chk["erel"], 1e-12)
    # the handle's data were restored: a new solve repeats the first one bit for bit
    assert again.info.iterations == sol.info.iterations and np.array_equal(again.x, sol.x)


def test_polish_fp32_form(oracle_lib):
    lp = _lp("large_recipe")
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=200000, method=1, precision=lpg.LP_PREC_FP32_REFINED) as s:
        s.solve()
        p = s.polish(eps=1e-9)
    chk = oracle.kkt(lp, p.x, p.y)
    assert chk["rel_p"] <= 1e-9 * (1 + 1e-6) and chk["rel_d"] <= 1e-9 * (1 + 1e-6)


def test_polish_errors():
    lp = _lp("cfg0")
    with lpg.Solver(lp) as s:
        with pytest.raises(lpg.LpError):
            s.polish()  # before a solve
        s.solve()
        with pytest.raises(lpg.LpError):
            s.polish(eps=0.0)


def test_polish_refused_after_a_certificate():
    from test_oracle_infeasible import infeasible_lps

    lp, _ = infeasible_lps()["I1"]
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=10000) as s:
        assert s.solve().status == "primal_infeasible"
        with pytest.raises(lpg.LpError):
            s.polish()
