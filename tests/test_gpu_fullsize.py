"""Parity at the full size of the large workload (m = 1e6, n = 2e6, nnz = 1.2e7), in the
launch configuration the benchmark times: the scaled matrix and its transpose bit-exact,
the iterates over the first 200 iterations (crossing the first three evaluations and the
first restart) element by element against the oracle, converged points checked by the
oracle's KKT function on the original data against the known optimum, and a run paused,
carried to another handle and resumed equal to the straight run bit for bit."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    return synth.cfg1(0)


def test_full_size_structure_and_iterates(oracle_lib, big):
    lp = big
    ks = [1, 2, 64, 65, 66, 128, 129, 192, 193, 200]
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=max(ks), pow_iters=20, snap_k=ks)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, pow_iters=20) as s:
        lay = s.layout()
        assert lay["long_rows_at"] >= 1  # power-law columns longer than one LDS tile
        # the panel units never exceed their target (4 per CU), so every workgroup of two
        # units is resident in one round
        import torch
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert 0.9 * 4 * cus <= lay["units_a"] <= 4 * cus and 0.9 * 4 * cus <= lay["units_at"] <= 4 * cus
        gv, gR, gC, grp, gci, gvt = s.scaled()
        av, R, Cc, rpT, ciT, avT = oracle.scaled_problem(lp)
        assert np.array_equal(grp, rpT) and np.array_equal(gci, ciT)
        assert np.array_equal(gv.view(np.uint64), av.view(np.uint64))
        assert np.array_equal(gvt.view(np.uint64), avT.view(np.uint64))
        assert np.array_equal(gR, R) and np.array_equal(gC, Cc)
        del gv, gvt, av, avT
        for i, k in enumerate(ks):
            s.update(eps_rel=0.0, max_iters=k)
            sol = s.solve()
            assert sol.info.iterations == k
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                d = float(np.max(np.abs(a - b))) / max(1.0, float(np.max(np.abs(b))))
                assert d <= 1e-12, (k, d)
            print(f"full-size iterates at k={k}: within 1e-12", flush=True)
        assert abs(sol.info.sigma_max - ref.sigma_max) <= 1e-12 * ref.sigma_max


def test_full_size_solve_properties(oracle_lib, big):
    """Properties that hold at any size, on a bounded run of the full-size LP in the
    benchmark's configuration: the E_rel the solver reports for its returned point equals
    the oracle's KKT check of that point on the original data, the residuals shrink from the
    start, and the objective approaches the known optimum."""
    lp = big
    with lpg.Solver(lp, eps_rel=1e-4, max_iters=6400) as s:
        sol = s.solve()
    print(f"full-size: {sol.status}, {sol.info.iterations} iterations, {sol.info.solve_seconds:.2f}s, "
          f"E_rel {sol.info.rel_kkt:.2e}, p {sol.info.primal_obj:.10g} vs p* {lp.p_star:.10g}")
    assert sol.status in ("optimal", "iteration_limit")
    chk = oracle.kkt(lp, sol.x, sol.y)
    assert abs(chk["erel"] - sol.info.rel_kkt) <= 1e-8 * chk["erel"]
    x0 = np.clip(np.zeros(lp.n), lp.x_lo, lp.x_hi)
    start = oracle.kkt(lp, x0, np.zeros(lp.m))
    # This LP needs about 2e5 iterations to reach E_rel 1e-3; after 6400 it sits near 0.18.
    assert chk["erel"] < 0.25 * start["erel"]
    assert abs(sol.info.primal_obj - lp.p_star) <= 1e-2 * (1 + abs(lp.p_star))


def test_full_size_fp32_halpern_to_tolerance(oracle_lib, big):
    """The FP32 storage form (FP64 evaluation and refinement) with the reflected Halpern
    iteration solves the full-size LP to E_rel 1e-4 (about 1.26e5 iterations, ~30 s). Error
    against the FP64 oracle: its KKT check of the returned point on the original data gives
    the same E_rel (to 1e-8) below the tolerance, and the objective is within 1e-5 of the
    known optimum (the construction's p*)."""
    lp = big
    with lpg.Solver(lp, precision=lpg.LP_PREC_FP32_REFINED, method=lpg.LP_METHOD_HALPERN, eps_rel=1e-4,
                    max_iters=300000, time_limit_s=150.0) as s:
        sol = s.solve()
    chk = oracle.kkt(lp, sol.x, sol.y)
    rel_obj = abs(sol.info.primal_obj - lp.p_star) / (1 + abs(lp.p_star))
    print(f"full-size FP32 Halpern: {sol.status}, {sol.info.iterations} iterations, {sol.info.solve_seconds:.1f}s, "
          f"E_rel {sol.info.rel_kkt:.3e} (oracle {chk['erel']:.3e}), objective error {rel_obj:.2e}")
    assert sol.status == "optimal"
    assert chk["erel"] <= 1e-4 * (1 + 1e-9)
    assert abs(chk["erel"] - sol.info.rel_kkt) <= 1e-8 * chk["erel"]
    assert rel_obj <= 1e-5


def test_full_size_fp64_halpern_to_tolerance(oracle_lib, big):
    """The FP64 reflected Halpern form solves the full-size LP to E_rel 1e-4 in the
    benchmark's launch configuration (about 7e4 iterations, ~20 s). The oracle's KKT check of
    the returned point on the original data gives the same E_rel (to 1e-8), below the
    tolerance; the objective error against the construction's optimum p* is reported and
    bounded by the tolerance's scale."""
    lp = big
    with lpg.Solver(lp, method=lpg.LP_METHOD_HALPERN, eps_rel=1e-4, max_iters=300000, time_limit_s=150.0) as s:
        sol = s.solve()
    chk = oracle.kkt(lp, sol.x, sol.y)
    rel_obj = abs(sol.info.primal_obj - lp.p_star) / (1 + abs(lp.p_star))
    print(f"full-size FP64 Halpern: {sol.status}, {sol.info.iterations} iterations, {sol.info.solve_seconds:.1f}s, "
          f"E_rel {sol.info.rel_kkt:.3e} (oracle {chk['erel']:.3e}), |p - p*| / (1 + |p*|) = {rel_obj:.2e}")
    assert sol.status == "optimal"
    assert chk["erel"] <= 1e-4 * (1 + 1e-9)
    assert abs(chk["erel"] - sol.info.rel_kkt) <= 1e-8 * chk["erel"]
    assert rel_obj <= 1e-4


@pytest.mark.parametrize("precision", [lpg.LP_PREC_FP64, lpg.LP_PREC_FP32_REFINED])
def test_full_size_pause_export_resume(big, precision):
    """Checkpoint and resume at full size, in the benchmark's launch configuration: 384
    iterations straight against a pause after 128, the state carried through a host buffer
    to a second handle and resumed there; iterates, returned point and trace bit-identical."""
    lp = big
    opts = dict(eps_rel=0.0, max_iters=384, pow_iters=20, precision=precision)
    print(f"full-size checkpoint, precision {precision}", flush=True)
    with lpg.Solver(lp, **opts) as s:
        ref = s.solve(with_trace=True)
        ref_it = s.iterates()
    with lpg.Solver(lp, **opts) as a:
        paused = a.solve_until(100)
        assert paused.status == "iteration_limit" and paused.info.iterations == 128
        state = a.export_state()
    with lpg.Solver(lp, **opts) as b:
        b.import_state(state)
        del state
        out = b.resume(with_trace=True)
        out_it = b.iterates()
    assert (out.status, out.info.iterations, out.info.restarts) == (ref.status, ref.info.iterations, ref.info.restarts)
    np.testing.assert_array_equal(out.trace, ref.trace)
    for u, v in zip((out.x, out.y, out.z), (ref.x, ref.y, ref.z)):
        np.testing.assert_array_equal(u, v)
    for u, v in zip(out_it, ref_it):
        np.testing.assert_array_equal(u, v)


def test_full_size_residual_restarts_first_200(oracle_lib, big):
    """The Halpern form with residual restarts at full size against the oracle: iterates
    (Halpern iterate and T(z)) at iterations around the first three evaluations within 1e-12,
    and the decision trace (restart reasons, the residuals of the last iterate and of the
    anchor)."""
    lp = big
    ks = [1, 64, 65, 128, 129, 192, 200]
    kw = dict(method=1, restart_metric=1)
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=max(ks), pow_iters=20, snap_k=ks, **kw)
    print("full-size residual restarts: oracle done", flush=True)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, pow_iters=20, **kw) as s:
        for i, k in enumerate(ks):
            s.update(eps_rel=0.0, max_iters=k, **kw)
            sol = s.solve(with_trace=True)
            assert sol.info.iterations == k
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                d = float(np.max(np.abs(a - b))) / max(1.0, float(np.max(np.abs(b))))
                assert d <= 1e-12, (k, d)
        tr = sol.trace
    ot = ref.trace
    assert len(tr) == len(ot)
    np.testing.assert_array_equal(tr[:, [0, 1, 6, 7]], ot[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(tr[:, [2, 3, 8, 9]], ot[:, [2, 3, 8, 9]], rtol=1e-9)
