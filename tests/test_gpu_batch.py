"""Batched form: many LPs in one persistent launch, one workgroup per LP at a time.

Bars: FP64 iterates of every LP in the batch match the oracle to 1e-12 relative; each
LP's result in a batch is bit-identical to the same LP solved alone in a batch of one;
FP32 and mixed-precision batches reach the requested E_rel (checked in FP64 by the oracle
on the original data)."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu

FP32 = lpg.LP_PREC_FP32_REFINED


def _lps():
    out = [synth.cfg0(0), synth.cfg0(1), synth.transportation(120, np.random.default_rng(5)),
           synth.cfg1(0, m=400, n=800, nnz=4000), synth.cfg4_lp(2, m_hi=600)]
    out += [synth.cfg3_lp(j, m_max=400) for j in range(4)]
    return out


def _solvers(lps, **kw):
    return [lpg.Solver(lp, spmv_layout=1, **kw) for lp in lps]


def test_batch_iterates_match_oracle(oracle_lib):
    lps = _lps()
    ks = [1, 2, 64, 65, 130]
    refs = [oracle.solve(lp, eps_rel=0.0, max_iters=max(ks), snap_k=ks) for lp in lps]
    solvers = _solvers(lps, eps_rel=0.0)
    try:
        for i, k in enumerate(ks):
            lpg.solve_batch(solvers, eps_rel=0.0, max_iters=k)
            for s, lp, ref in zip(solvers, lps, refs):
                for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                    scale = max(1.0, float(np.max(np.abs(b)))) if b.size else 1.0
                    assert float(np.max(np.abs(a - b), initial=0.0)) / scale <= 1e-12, (lp.name, k)
    finally:
        for s in solvers:
            s.close()


def test_batch_solve_matches_oracle_and_single_path(oracle_lib):
    lps = _lps()
    solvers = _solvers(lps)
    try:
        sols = lpg.solve_batch(solvers, eps_rel=1e-4, max_iters=400000)
    finally:
        for s in solvers:
            s.close()
    for lp, sol in zip(lps, sols):
        ref = oracle.solve(lp, eps_rel=1e-4, max_iters=400000)
        assert sol.status == ref.status == "optimal", lp.name
        assert sol.info.iterations == ref.iters, lp.name
        assert abs(sol.info.primal_obj - ref.pobj) <= 1e-6 * max(1.0, abs(ref.pobj)), lp.name
        chk = oracle.kkt(lp, sol.x, sol.y)
        assert chk["erel"] <= 1e-4


def test_batch_alone_equals_in_mix():
    lps = _lps()
    mix = _solvers(lps)
    try:
        in_mix = lpg.solve_batch(mix, eps_rel=1e-5, max_iters=400000)
    finally:
        for s in mix:
            s.close()
    for j in (0, 3, len(lps) - 1):
        with lpg.Solver(lps[j], spmv_layout=1) as s:
            alone = lpg.solve_batch([s], eps_rel=1e-5, max_iters=400000)[0]
        a, b = alone, in_mix[j]
        assert a.info.iterations == b.info.iterations
        assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y) and np.array_equal(a.z, b.z)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_batch_fp32_and_mixed_precision(oracle_lib, eps):
    lps = _lps()
    solvers = [lpg.Solver(lp, spmv_layout=1, precision=(FP32 if i % 3 else lpg.LP_PREC_FP64))
               for i, lp in enumerate(lps)]
    try:
        sols = lpg.solve_batch(solvers, eps_rel=eps, max_iters=1_000_000)
    finally:
        for s in solvers:
            s.close()
    for lp, sol in zip(lps, sols):
        assert sol.status == "optimal", (lp.name, sol.info.rel_kkt)
        chk = oracle.kkt(lp, sol.x, sol.y)
        assert chk["erel"] <= eps * (1 + 1e-9), lp.name


def test_batched_workload_sample(oracle_lib):
    """A stratified sample of the batched workload (random-sparse and transportation LPs,
    rows capped for test time), FP32 form to 1e-4."""
    lps = [synth.cfg3_lp(j, m_max=1500) for j in range(24)]
    solvers = [lpg.Solver(lp, spmv_layout=1, precision=FP32) for lp in lps]
    try:
        sols = lpg.solve_batch(solvers, eps_rel=1e-4, max_iters=1_000_000)
    finally:
        for s in solvers:
            s.close()
    for lp, sol in zip(lps, sols):
        assert sol.status == "optimal", (lp.name, sol.info.rel_kkt, sol.info.iterations)
        assert oracle.kkt(lp, sol.x, sol.y)["erel"] <= 1e-4


@pytest.mark.parametrize("precision", [lpg.LP_PREC_FP64, FP32])
def test_block_diagonal_equals_single_lp_solve(precision):
    """LPs in the block-diagonal group follow their own lp_solve trajectory exactly."""
    lps = _lps()
    with_batch = [lpg.Solver(lp, spmv_layout=1, precision=precision) for lp in lps]
    try:
        sols = lpg.solve_batch(with_batch, eps_rel=1e-6, max_iters=400000, batch_split_nnz=0)
    finally:
        for s in with_batch:
            s.close()
    for lp, sb in zip(lps, sols):
        with lpg.Solver(lp, spmv_layout=1, precision=precision, eps_rel=1e-6, max_iters=400000) as s1:
            ss = s1.solve()
        assert sb.status == ss.status and sb.info.iterations == ss.info.iterations, lp.name
        assert np.array_equal(sb.x, ss.x) and np.array_equal(sb.y, ss.y) and np.array_equal(sb.z, ss.z), lp.name


def test_block_diagonal_alone_equals_in_mix_and_split(oracle_lib):
    lps = _lps()
    mix = [lpg.Solver(lp, spmv_layout=1) for lp in lps]
    try:
        # a split that sends part of the batch to each path
        split = int(np.median([lp.nnz for lp in lps]))
        in_mix = lpg.solve_batch(mix, eps_rel=1e-5, max_iters=400000, batch_split_nnz=split)
    finally:
        for s in mix:
            s.close()
    for j, lp in enumerate(lps):
        with lpg.Solver(lp, spmv_layout=1) as s:
            alone = lpg.solve_batch([s], eps_rel=1e-5, max_iters=400000, batch_split_nnz=split)[0]
        assert alone.info.iterations == in_mix[j].info.iterations, lp.name
        assert np.array_equal(alone.x, in_mix[j].x) and np.array_equal(alone.y, in_mix[j].y), lp.name
        assert oracle.kkt(lp, alone.x, alone.y)["erel"] <= 1e-5


def test_full_4096_batch_sample_equals_solo():
    """The whole 4096-LP batch of the batched workload in one lp_solve_batch (FP32 storage,
    Halpern form, persistent and block-diagonal paths side by side): every LP reaches 1e-4,
    and 16 LPs drawn across the batch (both paths) give bit-identical results solved alone."""
    lps = [synth.cfg3_lp(j) for j in range(4096)]
    kw = dict(spmv_layout=1, precision=lpg.LP_PREC_FP32_REFINED, method=lpg.LP_METHOD_HALPERN)
    solvers = [lpg.Solver(lp, **kw) for lp in lps]
    try:
        sols = lpg.solve_batch(solvers, eps_rel=1e-4, max_iters=400000, method=lpg.LP_METHOD_HALPERN)
    finally:
        for s in solvers:
            s.close()
    assert all(s.status == "optimal" for s in sols)
    rng = np.random.default_rng(4096)
    pick = sorted(rng.choice(4096, 16, replace=False).tolist())
    nnz = np.array([lps[j].nnz for j in pick])
    assert (nnz > 20000).any() and (nnz <= 20000).any()  # both paths represented
    for j in pick:
        with lpg.Solver(lps[j], **kw) as s:
            (alone,) = lpg.solve_batch([s], eps_rel=1e-4, max_iters=400000, method=lpg.LP_METHOD_HALPERN)
        assert alone.info.iterations == sols[j].info.iterations, j
        assert np.array_equal(alone.x, sols[j].x) and np.array_equal(alone.y, sols[j].y), j


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("method", [0, 1])
def test_small_lps_from_lds_equal_global(precision, method):
    """LPs of the persistent launch whose arrays fit the small-LP LDS budget are solved from
    LDS (a launch of their own): their iterates after a fixed count and their solves equal,
    bit for bit, the same LPs solved from global memory (small_lp_lds = 0)."""
    lps = [synth.cfg0(0), synth.cfg3_lp(576), synth.cfg3_lp(3568), synth.transportation(60, np.random.default_rng(4)),
           synth.cfg3_lp(1, m_max=900)]
    opts = dict(spmv_layout=1, precision=precision, method=method)
    out = {}
    for budget in (0, 112 * 1024):
        solvers = [lpg.Solver(lp, **opts) for lp in lps]
        try:
            lpg.solve_batch(solvers, eps_rel=0.0, max_iters=130, small_lp_lds=budget, **opts)
            its = [s.iterates() for s in solvers]
            sols = lpg.solve_batch(solvers, eps_rel=1e-5, max_iters=100000, small_lp_lds=budget, **opts)
        finally:
            for s in solvers:
                s.close()
        out[budget] = (its, sols)
    (ia, sa), (ib, sb) = out[0], out[112 * 1024]
    for j, lp in enumerate(lps):
        for u, v in zip(ia[j], ib[j]):
            assert np.array_equal(u, v), (lp.name, "iterates")
        assert sa[j].status == sb[j].status and sa[j].info.iterations == sb[j].info.iterations, lp.name
        assert np.array_equal(sa[j].x, sb[j].x) and np.array_equal(sa[j].y, sb[j].y) and np.array_equal(sa[j].z, sb[j].z)
