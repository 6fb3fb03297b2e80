"""Oracle pins against exact results: brute-force vertex enumeration, closed forms of the
iteration, the PDHG contraction property, and a third-party LP solver as a cross-check."""
import math

import numpy as np
import pytest

import synth
from brute import enumerate_min

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _random_bounded_lp(rng, m, n):
    """Dense random LP with finite variable bounds and a feasible interior point."""
    a = rng.standard_normal((m, n))
    a[rng.random((m, n)) < 0.25] = 0.0
    x_lo = rng.uniform(-1, 0, n)
    x_hi = x_lo + rng.uniform(0.5, 3, n)
    xin = x_lo + rng.random(n) * (x_hi - x_lo)
    ax = a @ xin
    b_lo = np.empty(m)
    b_hi = np.empty(m)
    for i in range(m):
        kind = rng.integers(4)
        if kind == 0:
            b_lo[i] = b_hi[i] = ax[i]
        elif kind == 1:
            b_lo[i], b_hi[i] = ax[i] - rng.random(), math.inf
        elif kind == 2:
            b_lo[i], b_hi[i] = -math.inf, ax[i] + rng.random()
        else:
            b_lo[i], b_hi[i] = ax[i] - rng.random(), ax[i] + rng.random()
    c = rng.standard_normal(n)
    rows, cols = np.nonzero(a)
    keys = rows.astype(np.int64) * n + cols
    rp, ci, v = synth.csr_from_keys(keys, m, n, a[rows, cols])
    return synth.LP(m, n, rp, ci, v, c, b_lo, b_hi, x_lo, x_hi), a


@pytest.mark.parametrize("case", range(12))
def test_vertex_enumeration(oracle_lib, case):
    rng = np.random.default_rng([7, case])
    n = int(rng.integers(2, 9))
    m = int(rng.integers(1, 7)) if n <= 6 else int(rng.integers(1, 4))
    lp, a = _random_bounded_lp(rng, m, n)
    best, _ = enumerate_min(a, lp.c, lp.b_lo, lp.b_hi, lp.x_lo, lp.x_hi)
    r = oracle_lib.solve(lp, eps_rel=1e-10, max_iters=1_000_000)
    assert r.status == "optimal", (r.status, r.erel, r.iters)
    assert abs(r.pobj - best) <= 1e-7 * (1 + abs(best)), (r.pobj, best)


def test_box_lp_without_rows(oracle_lib):
    """m = 0: the minimiser sits at x_lo where c > 0 and at x_hi where c < 0."""
    c = np.array([1.0, -2.0, 0.5, -1.0, 3.0])
    x_lo = np.array([-1.0, 0.0, 2.0, -3.0, 0.25])
    x_hi = np.array([1.0, 5.0, 4.0, 7.0, 0.5])
    lp = synth.LP(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c, np.zeros(0), np.zeros(0),
                  x_lo, x_hi)
    r = oracle_lib.solve(lp, eps_rel=1e-12, max_iters=10000)
    assert r.status == "optimal"
    expect = np.where(c > 0, x_lo, x_hi)
    assert np.array_equal(r.x, expect)
    assert r.pobj == pytest.approx(float(c @ expect), abs=1e-14)


def test_fractional_knapsack(oracle_lib):
    """max v^T x s.t. w^T x <= W, 0 <= x <= 1: greedy by v/w is optimal (closed form)."""
    rng = np.random.default_rng(11)
    n = 30
    v = rng.uniform(1, 10, n)
    w = rng.uniform(1, 5, n)
    W = 0.4 * w.sum()
    order = np.argsort(-v / w)
    cap, best = W, 0.0
    for k in order:
        take = min(1.0, cap / w[k])
        best += take * v[k]
        cap -= take * w[k]
        if cap <= 0:
            break
    rp, ci, vals = synth.csr_from_keys(np.arange(n, dtype=np.int64), 1, n, w)
    lp = synth.LP(1, n, rp, ci, vals, -v, np.array([-math.inf]), np.array([W]), np.zeros(n), np.ones(n))
    r = oracle_lib.solve(lp, eps_rel=1e-11, max_iters=1_000_000)
    assert r.status == "optimal"
    assert abs(r.pobj + best) <= 1e-8 * best


def _free_equality_lp(seed, m=12, n=20):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    c = rng.standard_normal(n)
    rows, cols = np.nonzero(a)
    rp, ci, v = synth.csr_from_keys(rows.astype(np.int64) * n + cols, m, n, a[rows, cols])
    lp = synth.LP(m, n, rp, ci, v, c, b.copy(), b.copy(), np.full(n, -math.inf), np.full(n, math.inf))
    return lp, a, b, c


def test_linear_recurrence_all_free_equalities(oracle_lib):
    """All-free, equality-only LP: without restarts the iteration is linear,
    x+ = x - tau (c - A^T y), y+ = y - sigma (A (2x+ - x) - b), and the averages are the
    plain means of the iterates since the start."""
    lp, a, b, c = _free_equality_lp(3)
    eta, omega = 0.9 / np.linalg.norm(a, 2), 1.7
    tau, sigma = eta / omega, eta * omega
    ks = list(range(1, 201))
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=200, scaling=False, restarts=False, eta=eta, omega0=omega,
                         snap_k=ks)
    x = np.zeros(lp.n)
    y = np.zeros(lp.m)
    sx = np.zeros(lp.n)
    sy = np.zeros(lp.m)
    for k in ks:
        xn = x - tau * (c - a.T @ y)
        y = y - sigma * (a @ (2 * xn - x) - b)
        x = xn
        sx += x
        sy += y
        xs, ys, xa, ya = oracle_lib.split_snap(r.snaps[k - 1], lp.n, lp.m)
        scale = max(1.0, np.abs(x).max(), np.abs(y).max())
        assert np.abs(xs - x).max() <= 1e-12 * scale
        assert np.abs(ys - y).max() <= 1e-12 * scale
        assert np.abs(xa - sx / k).max() <= 1e-12 * scale
        assert np.abs(ya - sy / k).max() <= 1e-12 * scale


def test_kkt_point_is_fixed_point(oracle_lib):
    lp = synth.cfg0(1)
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=3, scaling=False, x0=lp.x_star, y0=lp.y_star, snap_k=[1, 2, 3])
    for s in r.snaps:
        xs, ys, _, _ = oracle_lib.split_snap(s, lp.n, lp.m)
        np.testing.assert_allclose(xs, lp.x_star, atol=1e-12)
        np.testing.assert_allclose(ys, lp.y_star, atol=1e-12)


def test_nonexpansive_in_pdhg_metric(oracle_lib):
    """Without restarts, ||z_k - z*||_M is non-increasing for M = [[I/tau, A^T], [A, I/sigma]]
    (PDHG as a proximal point method with K = -A)."""
    lp = synth.cfg0(2)
    a = lp.dense()
    eta = 0.95 / np.linalg.norm(a, 2)
    omega = 1.3
    tau, sigma = eta / omega, eta * omega
    ks = list(range(1, 301))
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=300, scaling=False, restarts=False, eta=eta, omega0=omega,
                         snap_k=ks)

    def mnorm(x, y):
        dx, dy = x - lp.x_star, y - lp.y_star
        return dx @ dx / tau + 2 * dy @ (a @ dx) + dy @ dy / sigma

    prev = mnorm(np.clip(np.zeros(lp.n), lp.x_lo, lp.x_hi), np.zeros(lp.m))
    for s in r.snaps:
        xs, ys, _, _ = oracle_lib.split_snap(s, lp.n, lp.m)
        cur = mnorm(xs, ys)
        assert cur <= prev * (1 + 1e-12) + 1e-12
        prev = cur


@pytest.mark.parametrize("j", range(4))
def test_crosscheck_highs(oracle_lib, j):
    """Cross-check only (a third-party solver): objective of random KKT-constructed and
    transportation LPs against scipy's HiGHS."""
    from scipy.optimize import linprog
    import scipy.sparse as sp

    rng = np.random.default_rng([5, j])
    if j % 2 == 0:
        m = 60 + 40 * j
        lp = synth.kkt_constructed(m, 2 * m, synth.random_sparse_pattern(m, 2 * m, 0.03, rng), rng)
    else:
        lp = synth.transportation(40 + 20 * j, rng)
    A = sp.csr_matrix((lp.vals, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    fin_hi = np.isfinite(lp.b_hi)
    fin_lo = np.isfinite(lp.b_lo)
    A_ub = sp.vstack([A[fin_hi], -A[fin_lo]])
    b_ub = np.concatenate([lp.b_hi[fin_hi], -lp.b_lo[fin_lo]])
    bounds = [(None if math.isinf(l) else l, None if math.isinf(u) else u) for l, u in zip(lp.x_lo, lp.x_hi)]
    ref = linprog(lp.c, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
    assert ref.status == 0
    r = oracle_lib.solve(lp, eps_rel=1e-9, max_iters=2_000_000)
    assert r.status == "optimal", (r.erel, r.iters)
    assert abs(r.pobj - ref.fun) <= 1e-6 * (1 + abs(ref.fun)), (r.pobj, ref.fun)
    if lp.p_star is not None:
        assert abs(ref.fun - lp.p_star) <= 1e-8 * (1 + abs(lp.p_star))
