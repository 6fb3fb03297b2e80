"""Presolve and postsolve (the paper's Section 3; reductions of Section 2.1, explorers of
Sections 2.2, 2.3 and Table 1). Host code: these tests run without a GPU.

A presolved LP is not unique, so the tests compare what is: the optimal value (scipy HiGHS
on the original LP vs. on the reduced LP plus its offset, and vs. the planted optimum), and
check that postsolve maps an exact solution of the reduced LP to a point that the oracle's KKT
routine accepts on the original data (eq. 2), with z equal to the reduced cost c - A^T y.
"""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from conftest import golden_lps, load_golden
from exact_lp import highs


def reduced_cost(lp, y):
    return lp.c - lp.dense().T @ y if lp.m else lp.c.copy()


def exact_roundtrip(lp, P, tol=1e-9):
    """Solve the reduced LP exactly, postsolve, and check the result on the original LP."""
    if P.info.n > 0:
        r = highs(P.reduced)
        assert r["status"] == "optimal", r.get("message")
        x, y, z = P.postsolve(r["x"], r["y"], r["z"])
        red_obj = r["obj"]
    else:
        x, y, z = P.postsolve()
        red_obj = P.reduced.c0
    k = oracle.kkt(lp, x, y)
    assert k["erel"] <= tol, k
    assert np.all(x >= lp.x_lo - 1e-9) and np.all(x <= lp.x_hi + 1e-9)
    zc = reduced_cost(lp, y)
    assert np.max(np.abs(z - zc), initial=0.0) <= 1e-9 * (1 + np.max(np.abs(lp.c)))
    return x, y, z, k, red_obj


@pytest.mark.parametrize("name", ["T1", "T2", "T3"])
def test_paper_examples(name):
    exp = {e["name"]: e for e in load_golden("presolve_expect.json")["paper"]}[name]
    lp, spec = golden_lps()[name]
    with lpg.Presolve(lp) as P:
        assert P.status == exp["status"]
        st = P.stats()
        for key, lo in exp["at_least"].items():
            assert st[key] >= lo, (key, st)
        x, y, z, k, _ = exact_roundtrip(lp, P)
        assert k["pobj"] == pytest.approx(spec["p_star"], abs=1e-12)
        if "x" in exp:
            np.testing.assert_allclose(x, exp["x"], atol=1e-12)
        if "x1" in exp:
            assert x[0] == pytest.approx(exp["x1"], abs=1e-12)


@pytest.mark.parametrize("name", ["T4", "T5"])
def test_sign_remark_examples(name):
    lp, spec = golden_lps()[name]
    with lpg.Presolve(lp) as P:
        assert P.status in ("reduced", "solved")
        _, _, _, k, _ = exact_roundtrip(lp, P)
        assert k["pobj"] == pytest.approx(spec["p_star"], abs=1e-12)


@pytest.mark.parametrize("idx", [0, 1])
def test_hand_solved_dual_recovery(idx):
    exp = load_golden("presolve_expect.json")["hand"][idx]
    lp = synth.tiny_lp(exp)
    with lpg.Presolve(lp) as P:
        assert P.status == "solved"
        x, y, z = P.postsolve()
        np.testing.assert_allclose(x, exp["x"], atol=1e-14)
        np.testing.assert_allclose(y, exp["y"], atol=1e-14)
        np.testing.assert_allclose(z, exp["z"], atol=1e-14)
        assert oracle.kkt(lp, x, y)["erel"] <= 1e-15


@pytest.mark.parametrize("j", range(6))
def test_planted_reductions(j):
    lp = synth.presolve_lp(j, m=300 + 100 * j, n=600 + 200 * j, density=0.01)
    ref = highs(lp)
    assert ref["obj"] == pytest.approx(lp.p_star, rel=1e-9, abs=1e-9)
    with lpg.Presolve(lp) as P:
        assert P.status == "reduced"
        st = P.stats()
        for key in ("empty_rows", "singleton_rows", "redundant_rows", "empty_cols", "fixed_cols",
                    "lock_fixed_cols", "substituted_cols"):
            assert st[key] > 0, (key, st)
        assert P.info.m < lp.m and P.info.n < lp.n and P.info.nnz <= lp.nnz
        _, _, _, k, red_obj = exact_roundtrip(lp, P, tol=1e-8)
        assert red_obj == pytest.approx(lp.p_star, rel=1e-9, abs=1e-9)
        assert k["pobj"] == pytest.approx(lp.p_star, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("case", ["cfg0", "transport", "serving_recipe"])
def test_workload_lps(case):
    if case == "cfg0":
        lp = synth.cfg0(1)
    elif case == "transport":
        lp = synth.transportation(60, np.random.default_rng(11))
    else:
        lp = synth.cfg4_lp(2, m_hi=400)
    ref = highs(lp)
    with lpg.Presolve(lp) as P:
        assert P.status in ("reduced", "solved")
        _, _, _, k, red_obj = exact_roundtrip(lp, P, tol=1e-8)
        assert red_obj == pytest.approx(ref["obj"], rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("opts", [dict(dual_reductions=0), dict(substitute=0), dict(dual_reductions=0, substitute=0),
                                  dict(max_rounds=1), dict(doubletons=0)])
def test_option_subsets(opts):
    lp = synth.presolve_lp(3, m=400, n=800, density=0.01)
    with lpg.Presolve(lp, **opts) as P:
        st = P.stats()
        if opts.get("dual_reductions") == 0:
            assert st["lock_fixed_cols"] == 0
        if opts.get("substitute") == 0:
            assert st["substituted_cols"] == 0
        if opts.get("max_rounds") == 1:
            assert st["rounds"] == 1
        if opts.get("doubletons") == 0:
            assert st["doubleton_cols"] == 0
        _, _, _, k, red_obj = exact_roundtrip(lp, P, tol=1e-8)
        assert red_obj == pytest.approx(lp.p_star, rel=1e-9, abs=1e-9)


def test_reduced_structure_and_maps():
    lp = synth.presolve_lp(4, m=400, n=800, density=0.01)
    # doubleton substitutions change values of existing entries; without them every reduced
    # entry is an original one
    with lpg.Presolve(lp, doubletons=0) as P:
        r = P.reduced
        rm, cm = P.maps()
        assert np.all(np.diff(rm) > 0) and np.all(np.diff(cm) > 0)
        assert r.row_ptr[0] == 0 and np.all(np.diff(r.row_ptr) >= 0) and r.row_ptr[-1] == P.info.nnz
        for i in range(r.m):
            cols = r.col_idx[r.row_ptr[i]:r.row_ptr[i + 1]]
            assert np.all(np.diff(cols) > 0)
        # each reduced entry is an original entry of (row_map[i], col_map[j]) with the same value
        A = lp.dense()
        rows = np.repeat(np.arange(r.m), np.diff(r.row_ptr))
        np.testing.assert_array_equal(A[rm[rows], cm[r.col_idx]], r.vals)
        # variable bounds only tighten
        assert np.all(r.x_lo >= lp.x_lo[cm]) and np.all(r.x_hi <= lp.x_hi[cm])
        # the reduced LP is accepted by the solver's validation
        s = lpg.Solver(r, deferred=1)
        s.close()


def _lp(A, c, bl, bh, xl, xh):
    return synth.tiny_lp(dict(A=A, c=c, b_lo=bl, b_hi=bh, x_lo=xl, x_hi=xh))


@pytest.mark.parametrize("case", ["activity", "empty_row", "crossing_bounds"])
def test_infeasible_detected(case):
    if case == "activity":  # x in [0,1]^2 cannot reach x1 + x2 >= 3
        lp = _lp([[1, 1], [1, -1]], [1, 1], [3, -5], ["inf", 5], [0, 0], [1, 1])
    elif case == "empty_row":  # 0 x1 >= 1 (an explicit-zero row)
        lp = _lp([[0.0, 0.0], [1, 1]], [1, 1], [1, 0], ["inf", 4], [0, 0], [3, 3])
        lp.row_ptr = np.array([0, 0, 2], np.int32)
        lp.col_idx = np.array([0, 1], np.int32)
        lp.vals = np.array([1.0, 1.0])
    else:  # x <= 1 by bounds and x >= 2 by a singleton row
        lp = _lp([[1.0]], [1], [2], ["inf"], [0], [1])
    assert highs(lp)["status"] == "infeasible"
    with lpg.Presolve(lp) as P:
        assert P.status == "infeasible"
        with pytest.raises(lpg.LpError):
            P.postsolve()


def test_unbounded_detected():
    # min -x1 with x1 >= 0 unbounded above; the only row x1 - x2 >= 0 does not stop x1 growing
    lp = _lp([[1, -1]], [-1, 1], [0], ["inf"], [0, 0], ["inf", 5])
    assert highs(lp)["status"] == "unbounded"
    with lpg.Presolve(lp) as P:
        assert P.status == "unbounded"


def test_validation_errors():
    lp = synth.presolve_lp(0, m=50, n=100, density=0.05)
    bad = synth.LP(lp.m, lp.n, lp.row_ptr.copy(), lp.col_idx.copy(), lp.vals.copy(), lp.c, lp.b_lo, lp.b_hi,
                   lp.x_lo, lp.x_hi)
    bad.col_idx[0] = lp.n  # out of range
    with pytest.raises(lpg.LpError) as e:
        lpg.Presolve(bad)
    assert lpg.ERRORS[e.value.code] == "LP_ERR_INVALID_MATRIX"
    nan = synth.LP(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals, lp.c.copy(), lp.b_lo, lp.b_hi, lp.x_lo, lp.x_hi)
    nan.c[3] = np.nan
    with pytest.raises(lpg.LpError) as e:
        lpg.Presolve(nan)
    assert lpg.ERRORS[e.value.code] == "LP_ERR_NAN_INPUT"
    with pytest.raises(TypeError):
        lpg.Presolve(lp, no_such_option=1)


def test_doubleton_bound_transfer_hand_lp():
    """Doubleton equality x1 + 2 x2 = 4 (Table 1): x2 has fewer entries and every other row
    with x2 also holds x1, so x2 = (4 - x1) / 2 is substituted without fill-in and its bounds
    [0, 1.5] become x1 in [1, 4]. At the optimum (x1 = 1, x2 = 1.5, x3 = 0.5, objective 3.5,
    checked by HiGHS on the original) x1 rests on the bound it took from x2, so postsolve must
    move that multiplier to x2 for the point to pass the KKT check."""
    lp = _lp([[1, 2, 0], [1, 1, 1], [1, 0, -1]], [3, 0, 1], [4, 3, "-inf"], [4, "inf", 8],
             [0, 0, 0], [10, 1.5, 5])
    ref = highs(lp)
    assert ref["obj"] == pytest.approx(3.5, abs=1e-12)
    with lpg.Presolve(lp, dual_reductions=0) as P:
        assert P.stats()["doubleton_cols"] == 1
        x, y, z, k, red_obj = exact_roundtrip(lp, P)
        assert red_obj == pytest.approx(3.5, abs=1e-12)
        np.testing.assert_allclose(x, [1.0, 1.5, 0.5], atol=1e-12)
        assert z[1] < 0 and z[0] == 0.0  # x2 at its upper bound carries the multiplier


def _with_doubletons(seed, m=60, n=80, pairs=25):
    """A random boxed LP with a known feasible point, plus `pairs` planted doubleton pairs:
    a new column k whose rows are a subset of an existing column j's rows, tied to x_j by a new
    equality row a_j x_j + a_k x_k = b that the feasible point satisfies."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, n))
    mask = rng.random((m, n)) < 0.08
    A[mask] = rng.choice([-1, 1], mask.sum()) * rng.uniform(0.5, 2.0, mask.sum())
    xl = rng.choice([0.0, -5.0], n)
    xh = xl + rng.uniform(2.0, 10.0, n)
    x0 = rng.uniform(xl, xh)
    rows, cols = [A], []
    for _ in range(pairs):
        j = int(rng.integers(n))
        sup = np.nonzero(rows[0][:, j])[0]
        colk = np.zeros(rows[0].shape[0])
        take = sup[rng.random(sup.size) < 0.6]
        colk[take] = rng.uniform(-2, 2, take.size)
        cols.append((j, colk))
    mk = A.shape[0]
    nk = n + pairs
    B = np.zeros((mk + pairs, nk))
    B[:mk, :n] = A
    lo = np.concatenate([xl, np.zeros(pairs)])
    hi = np.concatenate([xh, np.zeros(pairs)])
    xx = np.concatenate([x0, np.zeros(pairs)])
    for t, (j, colk) in enumerate(cols):
        k = n + t
        B[:mk, k] = colk
        lo[k] = -rng.uniform(1, 6)
        hi[k] = rng.uniform(1, 6)
        xx[k] = rng.uniform(lo[k], hi[k])
        aj, ak = rng.choice([-1, 1]) * rng.uniform(0.5, 2), rng.choice([-1, 1]) * rng.uniform(0.5, 2)
        B[mk + t, j] = aj
        B[mk + t, k] = ak
    act = B @ xx
    bl = act - rng.uniform(0.0, 3.0, act.size)
    bh = act + rng.uniform(0.0, 3.0, act.size)
    eq = rng.random(mk) < 0.3
    bh[:mk][eq] = bl[:mk][eq] = act[:mk][eq]
    bl[mk:] = bh[mk:] = act[mk:]
    bl[:mk][~eq & (rng.random(mk) < 0.3)] = -np.inf
    c = rng.normal(size=nk)
    return _lp(B.tolist(), c.tolist(), bl.tolist(), bh.tolist(), lo.tolist(), hi.tolist())


@pytest.mark.parametrize("seed", range(8))
def test_planted_doubletons(seed):
    """Random boxed LPs with planted doubleton pairs: the doubletons are eliminated, the
    reduced LP's optimum plus its offset equals the original's (HiGHS), and postsolve of the
    reduced optimum passes the oracle's KKT check on the original."""
    lp = _with_doubletons(seed)
    ref = highs(lp)
    assert ref["status"] == "optimal"
    for opts in (dict(), dict(dual_reductions=0, substitute=0)):
        with lpg.Presolve(lp, **opts) as P:
            assert P.status in ("reduced", "solved")
            assert P.stats()["doubleton_cols"] > 0
            assert P.info.nnz <= lp.nnz
            _, _, _, k, red_obj = exact_roundtrip(lp, P, tol=1e-8)
            assert red_obj == pytest.approx(ref["obj"], rel=1e-9, abs=1e-9)
            assert k["pobj"] == pytest.approx(ref["obj"], rel=1e-8, abs=1e-8)



def test_doubleton_cancellation_drops_the_entry():
    """A +-1 doubleton that cancels an entry: row 0 is x1 + x2 = 1, row 1 is x1 + x2 + x3 >= 0.5.
    Substituting x1 = 1 - x2 (or x2 = 1 - x1) through row 0 turns row 1's other entry into
    1 - 1 = 0, so row 1 is x3 >= -0.5: the cancelled entry leaves the counts and the reduced
    LP, and row 1 is then found as a singleton row (a bound on x3). The postsolved point
    solves the original (HiGHS's optimum, the oracle's KKT check)."""
    lp = _lp([[1, 1, 0], [1, 1, 1], [0, 1, -1]], [1, 2, 1], [1, 0.5, -3], [1, "inf", 3],
             [0, 0, -1], [4, 4, 4])
    ref = highs(lp)
    assert ref["status"] == "optimal"
    with lpg.Presolve(lp, dual_reductions=0) as P:
        st = P.stats()
        assert st["doubleton_cols"] == 1 and st["cancelled_entries"] == 1
        assert st["singleton_rows"] >= 1
        red = P.reduced
        assert np.all(red.vals != 0.0)
        assert red.row_ptr[-1] <= 2  # row 0 gone, row 1 gone as a singleton, row 2 keeps 2 entries at most
        x, y, z, k, red_obj = exact_roundtrip(lp, P)
        assert red_obj == pytest.approx(ref["obj"], abs=1e-12)
        chk = oracle.kkt(lp, x, y)
        assert chk["erel"] <= 1e-12


def test_explicit_zeros_are_not_exported():
    """Explicit zeros of the input count nowhere: a row whose only other entry is an explicit
    zero is a singleton row, and the reduced LP holds no zero value."""
    lp = _lp([[1, 0, 1], [2, 1, 0], [0, 1, 1]], [1, 1, 1], [1, 1, 1], ["inf", "inf", "inf"],
             [0, 0, 0], [5, 5, 5])
    # store the zero of row 1, column 2 explicitly
    rows = [[0, 2], [0, 1, 2], [1, 2]]
    vals = [[1.0, 1.0], [2.0, 1.0, 0.0], [1.0, 1.0]]
    lp.row_ptr = np.array([0, 2, 5, 7], np.int32)
    lp.col_idx = np.array([c for r in rows for c in r], np.int32)
    lp.vals = np.array([v for r in vals for v in r])
    ref = highs(lp)
    with lpg.Presolve(lp, dual_reductions=0, substitute=0, doubletons=0) as P:
        if P.reduced is not None and P.reduced.row_ptr[-1] > 0:
            assert np.all(P.reduced.vals != 0.0)
        x, y, z, k, red_obj = exact_roundtrip(lp, P)
        assert red_obj == pytest.approx(ref["obj"], abs=1e-12)
