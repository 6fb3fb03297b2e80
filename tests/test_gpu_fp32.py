"""FP32 storage form (matrix and iterates in FP32 around an FP64 master, FP64 evaluation,
restart decisions and refinement) against the FP64 oracle.

Bars: before the first restart the FP32 iterates follow the oracle's FP64 iterates to
FP32 rounding; solves reach the requested E_rel, re-checked in FP64 by the oracle's KKT
function on the original data, and the objective error against the FP64 oracle and
against the known optimum is reported per result."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu

FP32 = lpg.LP_PREC_FP32_REFINED


def _cases():
    return {
        "cfg0": synth.cfg0(0),
        "large_recipe_small": synth.cfg1(0, m=3000, n=6000, nnz=36000),
        "transport": synth.transportation(300, np.random.default_rng(3)),
        "serving_recipe_small": synth.cfg4_lp(1, m_hi=2000),
    }


@pytest.mark.parametrize("name", ["cfg0", "large_recipe_small", "transport"])
def test_fp32_iterates_track_fp64_before_first_restart(oracle_lib, name):
    lp = _cases()[name]
    ks = [1, 2, 10, 40, 63]
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=63, snap_k=ks)
    with lpg.Solver(lp, precision=FP32, eps_rel=0.0, max_iters=1) as s:
        for i, k in enumerate(ks):
            s.update(eps_rel=0.0, max_iters=k)
            s.solve()
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                scale = max(1.0, float(np.max(np.abs(b))))
                err = float(np.max(np.abs(a - b))) / scale
                assert err <= 2e-5 * k, (name, k, err)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
@pytest.mark.parametrize("name", ["cfg0", "large_recipe_small", "transport", "serving_recipe_small"])
def test_fp32_solve_reaches_tolerance(oracle_lib, name, eps):
    lp = _cases()[name]
    ref = oracle.solve(lp, eps_rel=eps, max_iters=2_000_000)
    with lpg.Solver(lp, precision=FP32, eps_rel=eps, max_iters=2_000_000) as s:
        sol = s.solve()
    assert sol.status == "optimal", (sol.status, sol.info.rel_kkt)
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert chk["erel"] <= eps * (1 + 1e-9)
    err_ora = abs(sol.info.primal_obj - ref.pobj) / (1 + abs(ref.pobj))
    msg = (f"{name} eps={eps:g}: FP32 form {sol.info.iterations} it (FP64 oracle {ref.iters}), "
           f"E_rel {chk['erel']:.2e}, |p - p_oracle|/(1+|p_oracle|) = {err_ora:.2e}")
    if lp.p_star is not None:
        err_star = abs(sol.info.primal_obj - lp.p_star) / (1 + abs(lp.p_star))
        msg += f", |p - p*|/(1+|p*|) = {err_star:.2e}"
        assert err_star <= 100 * eps
    print(msg)
    assert err_ora <= 100 * eps
