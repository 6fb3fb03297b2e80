"""Infeasibility certificates of the oracle (the remark after Section 2, eq. (2): an LP without
a solution of eq. (2) is infeasible or unbounded). The certificates are checked against their
definitions with plain numpy (Farkas: A^T y + z = 0 with y, z sign-feasible and a positive ray
objective; or a recession direction with negative cost), and the verdicts against scipy's
HiGHS."""
import math

import numpy as np
import pytest

import synth
from conftest import load_golden
from exact_lp import highs

EPS = 1e-8


def infeasible_lps():
    return {s["name"]: (synth.tiny_lp(s), s) for s in load_golden("infeasible_lps.json")["lps"]}


def check_dual_ray(lp, y, z, tol):
    """Farkas certificate of primal infeasibility, normalised so that its objective is 1."""
    A = lp.dense()
    assert np.linalg.norm(A.T @ y + z) <= tol
    lo, hi, xl, xu = lp.b_lo, lp.b_hi, lp.x_lo, lp.x_hi
    assert np.all(y[~np.isfinite(lo)] <= tol) and np.all(y[~np.isfinite(hi)] >= -tol)
    assert np.all(z[~np.isfinite(xl)] <= tol) and np.all(z[~np.isfinite(xu)] >= -tol)
    def fin(b):
        return np.where(np.isfinite(b), b, 0.0)

    D = (np.sum(np.where((y > 0) & np.isfinite(lo), fin(lo) * y, 0.0)) + np.sum(np.where((y < 0) & np.isfinite(hi), fin(hi) * y, 0.0))
         + np.sum(np.where((z > 0) & np.isfinite(xl), fin(xl) * z, 0.0)) + np.sum(np.where((z < 0) & np.isfinite(xu), fin(xu) * z, 0.0)))
    assert D == pytest.approx(1.0, rel=1e-9)


def check_primal_ray(lp, x, tol):
    """Recession direction with cost -1: A x in the recession cone of the row bounds, x in the
    recession cone of the variable bounds."""
    A = lp.dense()
    assert float(lp.c @ x) == pytest.approx(-1.0, rel=1e-9)
    v = A @ x

    def viol(w, lo, hi):
        fl, fh = np.isfinite(lo), np.isfinite(hi)
        out = np.where(fl & fh, w, 0.0)
        out = np.where(fl & ~fh, np.minimum(w, 0.0), out)
        out = np.where(~fl & fh, np.maximum(w, 0.0), out)
        return out

    assert np.linalg.norm(viol(v, lp.b_lo, lp.b_hi)) ** 2 + np.linalg.norm(viol(x, lp.x_lo, lp.x_hi)) ** 2 <= tol ** 2


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["I1", "I2", "U1", "U2"])
def test_hand_built_infeasible_lps(oracle_lib, name, method):
    lp, spec = infeasible_lps()[name]
    assert highs(lp)["status"] == ("infeasible" if spec["status"] == "primal_infeasible" else "unbounded")
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=20000, eps_infeas=EPS, method=method)
    assert r.status == spec["status"], (r.status, r.iters)
    if r.status == "primal_infeasible":
        check_dual_ray(lp, r.y, r.z, 2 * EPS)
    else:
        check_primal_ray(lp, r.x, 2 * EPS)


def test_detection_off_runs_to_the_limit(oracle_lib):
    """Without the certificates the unbounded example can only stop at the iteration limit."""
    lp, _ = infeasible_lps()["U1"]
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=5000, eps_infeas=0.0)
    assert r.status == "iteration_limit"
    assert r.x[0] > 100.0  # x1 keeps growing


def _contradicting_rows(base, rng, k):
    """Add k pairs of rows a^T x >= t and a^T x <= t - 1 over bounded columns (infeasible)."""
    A = base.dense()
    m, n = base.m, base.n
    bounded = np.flatnonzero(np.isfinite(base.x_lo) & np.isfinite(base.x_hi))
    rows, lo, hi = [], [], []
    for _ in range(k):
        a = np.zeros(n)
        cols = rng.choice(bounded, size=4, replace=False)
        a[cols] = rng.standard_normal(4)
        t = float(a @ base.x_star)
        rows += [a, a]
        lo += [t, -math.inf]
        hi += [math.inf, t - 1.0]
    A2 = np.vstack([A, np.array(rows)])
    spec = dict(A=A2.tolist(), c=base.c.tolist(), b_lo=list(base.b_lo) + lo, b_hi=list(base.b_hi) + hi,
                x_lo=base.x_lo.tolist(), x_hi=base.x_hi.tolist())
    return synth.tiny_lp(spec)


def _free_descent_column(base, rng):
    """Add a free column with cost -1 entering one '>=' row with a positive coefficient
    (unbounded: increasing it keeps every row satisfied)."""
    A = base.dense()
    ge = np.flatnonzero(np.isinf(base.b_hi) & np.isfinite(base.b_lo))
    col = np.zeros((base.m, 1))
    col[ge[0], 0] = 1.0 + rng.random()
    spec = dict(A=np.hstack([A, col]).tolist(), c=list(base.c) + [-1.0], b_lo=base.b_lo.tolist(),
                b_hi=base.b_hi.tolist(), x_lo=list(base.x_lo) + [-math.inf], x_hi=list(base.x_hi) + [math.inf])
    return synth.tiny_lp(spec)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("j", range(3))
def test_random_primal_infeasible(oracle_lib, j, method):
    rng = np.random.default_rng([synth.SEED_ROOT, 6, j])
    base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.5)
    lp = _contradicting_rows(base, rng, 1 + j)
    assert highs(lp)["status"] == "infeasible"
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method)
    assert r.status == "primal_infeasible", (r.status, r.iters)
    check_dual_ray(lp, r.y, r.z, 2 * EPS)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("j", range(3))
def test_random_unbounded(oracle_lib, j, method):
    rng = np.random.default_rng([synth.SEED_ROOT, 7, j])
    base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.3)
    lp = _free_descent_column(base, rng)
    assert highs(lp)["status"] == "unbounded"
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method)
    assert r.status == "dual_infeasible", (r.status, r.iters)
    check_primal_ray(lp, r.x, 2 * EPS)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("j", range(4))
def test_no_false_certificate_on_feasible_lps(oracle_lib, j, method):
    """Feasible, bounded LPs solved to a tight tolerance never report a certificate."""
    lp = synth.cfg0(j) if j < 2 else synth.transportation(40 + 20 * j, np.random.default_rng(j))
    r = oracle_lib.solve(lp, eps_rel=1e-7, max_iters=200000, eps_infeas=EPS, method=method)
    assert r.status == "optimal"


# ---- the second candidate ray: the averaged point's displacement from the restart anchor
def _infeasible_cases():
    cases = {name: lp for name, (lp, _) in infeasible_lps().items()}
    for j in range(3):
        rng = np.random.default_rng([synth.SEED_ROOT, 6, j])
        base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.5)
        cases[f"pinf{j}"] = _contradicting_rows(base, rng, 1 + j)
    for j in range(3):
        rng = np.random.default_rng([synth.SEED_ROOT, 7, j])
        base = synth.kkt_constructed(40, 80, synth.random_sparse_pattern(40, 80, 0.08, rng), rng, eq_frac=0.3)
        cases[f"unb{j}"] = _free_descent_column(base, rng)
    return cases


CASES = _infeasible_cases()


def _check_certificate(lp, r):
    if r.status == "primal_infeasible":
        check_dual_ray(lp, r.y, r.z, 2 * EPS)
    else:
        assert r.status == "dual_infeasible", r.status
        check_primal_ray(lp, r.x, 2 * EPS)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_anchored_average_ray_alone_certifies(oracle_lib, name, method):
    """With only the anchored-average candidate tested, every LP without a solution still gets
    a certificate that meets its definition."""
    lp = CASES[name]
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method, ray_candidates=2)
    assert r.ray_source == 2
    _check_certificate(lp, r)


@pytest.mark.parametrize("method", [0, 1])
def test_both_candidates_stop_at_the_first_of_either(oracle_lib, method):
    """The candidates do not change the iterates, so with both tested the solve stops at the
    first evaluation where either certifies, with that candidate's certificate (the
    displacement first when both do), bit for bit."""
    earlier = 0
    for name, lp in CASES.items():
        kw = dict(eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method)
        r1 = oracle_lib.solve(lp, ray_candidates=1, **kw)
        r2 = oracle_lib.solve(lp, ray_candidates=2, **kw)
        rb = oracle_lib.solve(lp, **kw)
        assert rb.iters == min(r1.iters, r2.iters), name
        src = r1 if r1.iters <= r2.iters else r2
        assert rb.ray_source == src.ray_source and rb.status == src.status, name
        for a, b in ((rb.x, src.x), (rb.y, src.y), (rb.z, src.z)):
            np.testing.assert_array_equal(a, b)
        earlier += r2.iters < r1.iters
    if method == 0:
        assert earlier >= 1  # on these LPs the averaged candidate certifies first at least once


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["pinf1", "pinf2", "unb0", "unb1"])
def test_anchored_ray_is_average_minus_anchor(oracle_lib, name, method):
    """Recompute the anchored-average ray from snapshots: the anchor is the candidate chosen at
    the last restart before the detecting evaluation (trace columns 6 and 7), or the start
    point; the ray is C (x~avg - x~anchor) or R (y~avg - y~anchor), normalised."""
    lp = CASES[name]
    kw = dict(eps_rel=1e-8, max_iters=100000, eps_infeas=EPS, method=method, ray_candidates=2)
    r = oracle_lib.solve(lp, **kw)
    tr = r.trace
    rst = [int(row[0]) for row in tr[:-1] if row[7] != 0]
    k_r = rst[-1] if rst else 0
    use_avg = {int(row[0]): int(row[6]) for row in tr}
    snaps = [k_r, r.iters] if k_r else [r.iters]
    rs = oracle_lib.solve(lp, snap_k=snaps, **kw)
    assert rs.iters == r.iters and rs.status == r.status
    n, m = lp.n, lp.m
    _, R, Cc, _, _, _ = oracle_lib.scaled_problem(lp)
    _, _, xa, ya = oracle_lib.split_snap(rs.snaps[-1], n, m)
    if k_r:
        x, y, xav, yav = oracle_lib.split_snap(rs.snaps[0], n, m)
        xan, yan = (xav, yav) if use_avg[k_r] else (x, y)
    else:  # the start point: x~ = clamp(0, x~lo, x~hi), y~ = 0
        xan, yan = np.clip(0.0, lp.x_lo / Cc, lp.x_hi / Cc), np.zeros(m)
    if r.status == "dual_infeasible":
        d = Cc * (xa - xan)
        expect = d / (-(lp.c @ d))
        np.testing.assert_allclose(r.x, expect, rtol=1e-9, atol=1e-12 * np.max(np.abs(expect)))
    else:
        d = R * (ya - yan)
        scale = r.y[np.argmax(np.abs(d))] / d[np.argmax(np.abs(d))]
        assert scale > 0
        np.testing.assert_allclose(r.y, scale * d, rtol=1e-9, atol=1e-12 * np.max(np.abs(r.y)))
