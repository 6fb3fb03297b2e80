"""Infeasibility and unboundedness certificates on the GPU against the oracle (same
evaluation, same status, same normalised ray), checked against their definitions."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from test_oracle_infeasible import CASES as ORACLE_CASES
from test_oracle_infeasible import (EPS, _contradicting_rows, _free_descent_column, check_dual_ray,
                                    check_primal_ray, infeasible_lps)

pytestmark = pytest.mark.gpu


def cases():
    out = dict((k, v[0]) for k, v in infeasible_lps().items())
    for j in range(2):
        rng = np.random.default_rng([synth.SEED_ROOT, 6, j])
        base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.5)
        out[f"rand_infeasible_{j}"] = _contradicting_rows(base, rng, 1 + j)
        rng = np.random.default_rng([synth.SEED_ROOT, 7, j])
        base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.3)
        out[f"rand_unbounded_{j}"] = _free_descent_column(base, rng)
    return out


CASES = cases()


def rel(a, b):
    return float(np.max(np.abs(a - b))) / max(1e-300, float(np.max(np.abs(b))))


@pytest.mark.parametrize("name", sorted(CASES))
def test_certificate_matches_oracle(oracle_lib, name):
    lp = CASES[name]
    ref = oracle.solve(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS)
    assert ref.status in ("primal_infeasible", "dual_infeasible")
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS) as s:
        sol = s.solve()
    print(f"{name}: oracle {ref.status} at {ref.iters}, gpu {sol.status} at {sol.info.iterations}")
    assert sol.status == ref.status
    assert sol.info.iterations == ref.iters
    assert sol.info.ray_source == ref.ray_source
    if sol.status == "primal_infeasible":
        check_dual_ray(lp, sol.y, sol.z, 2 * EPS)
        assert rel(sol.y, ref.y) <= 1e-7 and rel(sol.z, ref.z) <= 1e-7
    else:
        check_primal_ray(lp, sol.x, 2 * EPS)
        assert rel(sol.x, ref.x) <= 1e-7


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["pinf0", "pinf1", "pinf2", "unb0", "unb1", "unb2"])
def test_both_candidate_rays_match_oracle(oracle_lib, name, method):
    """The two candidate rays (displacement, then anchored average) in both iteration forms:
    same detecting evaluation, same candidate, same normalised ray as the oracle; on these
    LPs the anchored candidate certifies first in the averaged form on pinf2 and in the
    Halpern form on pinf1."""
    lp = ORACLE_CASES[name]
    ref = oracle.solve(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method)
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method) as s:
        sol = s.solve()
    print(f"{name} method {method}: oracle {ref.status} at {ref.iters} (ray {ref.ray_source}), "
          f"gpu {sol.status} at {sol.info.iterations} (ray {sol.info.ray_source})", flush=True)
    assert (sol.status, sol.info.iterations, sol.info.ray_source) == (ref.status, ref.iters, ref.ray_source)
    if (name, method) in (("pinf2", 0), ("pinf1", 1)):
        assert ref.ray_source == 2
    if sol.status == "primal_infeasible":
        check_dual_ray(lp, sol.y, sol.z, 2 * EPS)
        assert rel(sol.y, ref.y) <= 1e-7 and rel(sol.z, ref.z) <= 1e-7
    else:
        check_primal_ray(lp, sol.x, 2 * EPS)
        assert rel(sol.x, ref.x) <= 1e-7


@pytest.mark.parametrize("name", ["I1", "U2", "rand_infeasible_0", "rand_unbounded_1"])
def test_certificate_fp32_form(name):
    lp = CASES[name]
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS,
                    precision=lpg.LP_PREC_FP32_REFINED) as s:
        sol = s.solve()
    print(f"{name} FP32: {sol.status} at {sol.info.iterations}")
    if sol.status == "primal_infeasible":
        check_dual_ray(lp, sol.y, sol.z, 2 * EPS)
    else:
        assert sol.status == "dual_infeasible"
        check_primal_ray(lp, sol.x, 2 * EPS)


def test_detection_off_and_feasible_unaffected():
    lp = CASES["U1"]
    with lpg.Solver(lp, eps_rel=1e-8, max_iters=5000, eps_infeas=0.0) as s:
        assert s.solve().status == "iteration_limit"
    lp = synth.cfg0(0)
    with lpg.Solver(lp, eps_rel=1e-5, max_iters=200000) as s:
        assert s.solve().status == "optimal"


@pytest.mark.parametrize("layout", [0, 1])
def test_batch_mix_equals_solo(layout):
    """Feasible and infeasible LPs solved together: each LP's outcome is its solo outcome
    (persistent launch for the small ones, block-diagonal launches above batch_split_nnz)."""
    lps = [CASES["I2"], synth.cfg0(1), CASES["rand_unbounded_0"], CASES["rand_infeasible_1"],
           synth.transportation(50, np.random.default_rng(5)), ORACLE_CASES["pinf2"]]
    opts = dict(eps_rel=1e-6, max_iters=100000, eps_infeas=EPS, spmv_layout=1)
    solo = []
    for lp in lps:
        with lpg.Solver(lp, **opts) as s:
            solo.append(s.solve())
    solvers = [lpg.Solver(lp, **opts) for lp in lps]
    try:
        mix = lpg.solve_batch(solvers, batch_split_nnz=0 if layout else 10**9, **opts)
    finally:
        for s in solvers:
            s.close()
    assert solo[-1].info.ray_source == 2  # certified by the anchored-average candidate
    for a, b in zip(solo, mix):
        assert a.status == b.status and a.info.iterations == b.info.iterations
        assert a.info.ray_source == b.info.ray_source
        np.testing.assert_array_equal(a.x, b.x)
        np.testing.assert_array_equal(a.y, b.y)
