"""Pins of the oracle's restart cycle: the candidate choice, the three restart tests, the
primal-weight update and the reset of iterate, anchor, averages and A~x at a restart.

The paper names the restarted PDHG family of its GPU solver (Sections 1 and 4) without its
restart rules, so the constants (0.2, 0.8, 0.36) and the evaluation period are readings and
stay unpinned. What is pinned here is that the oracle does what the rules say:

* A restart is a fresh start. Right after a restart the solve must continue exactly as a new
  solve started at the restart candidate with the new primal weight would: iterate, anchor,
  running averages and the stored A~x are all reset. Compared bit for bit over the 64
  iterations that follow, in both iteration forms, with and without scaling.
* Every decision, recomputed in dense numpy from the iterates at each evaluation: the
  KKT error in the omega-weighted norm of the current point and of the average, the
  candidate (the average only if strictly smaller), the anchor's and the previous
  candidate's error, the restart reason (first of: deep decay, no progress after some decay,
  long cycle), and the invariant that the candidate is never worse than the current point.
* The primal-weight update balances the weighted distances moved in the cycle: with s
  square-root steps the log of the imbalance omega * dx / dy shrinks by exactly 2^-s.
* Restarts on the fixed-point residual (Halpern form, restart_metric 1): the norm is the one
  in which the PDHG map is firmly nonexpansive (checked on the map itself, which fixes the
  sign of its coupling term), and every residual, anchor residual and decision of a solve is
  recomputed from snapshots.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.usefixtures("oracle_lib")

EVAL = 64


def _lp(j):
    rng = np.random.default_rng([11, j])
    m = 40 + 10 * j
    return synth.kkt_constructed(m, 2 * m, synth.random_sparse_pattern(m, 2 * m, 0.06, rng), rng)


def _kkt_w(lp, a, x, y, omega):
    """KKT error of (x, y) in the omega-weighted norm, from the definitions of eq. 2 on the
    unscaled data: row-bound violation of Ax, the reduced cost minus its projection on the
    sign cone of the bounds (plus sign violations of y), and the gap of the primal and dual
    objectives (0 * inf taken as 0)."""
    ax = a @ x
    rp = ax - np.clip(ax, lp.b_lo, lp.b_hi)
    lam = lp.c - a.T @ y
    flo, fhi = np.isfinite(lp.x_lo), np.isfinite(lp.x_hi)
    z = np.where(flo & fhi, lam, np.where(flo, np.maximum(lam, 0.0), np.where(fhi, np.minimum(lam, 0.0), 0.0)))
    rd2 = float(np.sum((lam - z) ** 2))
    viol = np.where(np.isneginf(lp.b_lo) & (y > 0), y, 0.0) + np.where(np.isposinf(lp.b_hi) & (y < 0), -y, 0.0)
    rd2 += float(np.sum(viol**2))
    yp, ym = np.maximum(y, 0.0), np.minimum(y, 0.0)
    zp, zm = np.maximum(z, 0.0), np.minimum(z, 0.0)
    dual = (np.sum(np.where(yp > 0, lp.b_lo, 0.0) * yp) + np.sum(np.where(ym < 0, lp.b_hi, 0.0) * ym)
            + np.sum(np.where(zp > 0, lp.x_lo, 0.0) * zp) + np.sum(np.where(zm < 0, lp.x_hi, 0.0) * zm))
    gap = float(lp.c @ x) - float(dual)
    return math.sqrt(omega**2 * float(rp @ rp) + rd2 / omega**2 + gap**2)


def _close(a, b, rel=1e-9, noise=1e-11):
    """Agreement of two evaluations of a KKT error: the gap term cancels the objectives
    (O(10) here), so the recomputation carries an absolute rounding noise besides the
    relative one."""
    if math.isinf(a) or math.isinf(b):
        return a == b
    return abs(a - b) <= rel * max(abs(a), abs(b)) + noise


def _tie(a, b):
    return _close(a, b, 1e-8, 1e-10)


def _solve(oracle_lib, lp, eta, method, scaling, **kw):
    return oracle_lib.solve(lp, eps_rel=1e-9, max_iters=6000, scaling=scaling, eta=eta, method=method,
                            omega0=1.0, trace_cap=4096, **kw)


@pytest.mark.parametrize("scaling", [False, True])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("j", [0, 2])
def test_restart_equals_fresh_start(oracle_lib, j, method, scaling):
    lp = _lp(j)
    eta = 0.95 / np.linalg.norm(lp.dense(), 2)
    base = _solve(oracle_lib, lp, eta, method, scaling)
    tr = base.trace
    # one restart of each reason that has 64 iterations after it (the last record is the stop)
    picks = {}
    for rec in tr[:-1]:
        why, k = int(rec[7]), int(rec[0])
        if why and why not in picks and k + EVAL <= base.iters:
            picks[why] = rec
    assert picks, "no restart to check"
    R = C = None
    if scaling:
        _, R, C, _, _, _ = oracle_lib.scaled_problem(lp)
    for why, rec in picks.items():
        k, use_avg, omega = int(rec[0]), bool(rec[6]) or method == 1, float(rec[8])
        ks = [k] + list(range(k + 1, k + EVAL + 1))
        run = _solve(oracle_lib, lp, eta, method, scaling, snap_k=ks)
        x, y, xa, ya = oracle_lib.split_snap(run.snaps[0], lp.n, lp.m)
        xc, yc = (xa, ya) if use_avg else (x, y)
        x0, y0 = (xc * C, yc * R) if scaling else (xc.copy(), yc.copy())
        fresh = oracle_lib.solve(lp, eps_rel=0.0, max_iters=EVAL, scaling=scaling, eta=eta, omega0=omega,
                                 method=method, x0=x0, y0=y0, snap_k=list(range(1, EVAL + 1)))
        for i in range(EVAL):
            after = oracle_lib.split_snap(run.snaps[i + 1], lp.n, lp.m)
            new = oracle_lib.split_snap(fresh.snaps[i], lp.n, lp.m)
            for name, u, v in zip(("x", "y", "x_avg", "y_avg"), after, new):
                assert np.array_equal(u, v), f"reason {why} at k={k}: {name} differs {i + 1} iterations later"


def _check_decisions(oracle_lib, lp, method, omega_steps=0, seen=None, pid=None):
    """pid = (kp, ki, kd) selects the PID rule of the primal weight, checked against the
    closed form of its cumulative change: with the errors e_i = log(omega_i dx_i / dy_i) of
    the restarts so far and I_i = e_1 + ... + e_i, the derivative terms telescope and
    log omega_n - log omega_0 = -(kp sum e_i + ki sum I_i + kd e_n)."""
    a = lp.dense()
    eta = 0.95 / np.linalg.norm(a, 2)
    kw = dict(omega_steps=omega_steps)
    if pid is not None:
        kw.update(pw_rule=2, pid_kp=pid[0], pid_ki=pid[1], pid_kd=pid[2])
    base = _solve(oracle_lib, lp, eta, method, False, **kw)
    tr = base.trace
    ks = [int(r[0]) for r in tr]
    run = _solve(oracle_lib, lp, eta, method, False, snap_k=ks, **kw)
    assert np.array_equal(run.trace, tr)
    steps = omega_steps if omega_steps else (2 if method == 1 else 1)
    errors = []
    x_an = np.clip(np.zeros(lp.n), lp.x_lo, lp.x_hi)
    y_an = np.zeros(lp.m)
    omega = 1.0
    prev = math.inf
    k_last = 0
    anc = _kkt_w(lp, a, x_an, y_an, omega)
    for idx, rec in enumerate(tr[:-1]):
        k = int(rec[0])
        x, y, xa, ya = oracle_lib.split_snap(run.snaps[idx], lp.n, lp.m)
        cur = (xa, ya) if method == 1 else (x, y)
        kc = _kkt_w(lp, a, *cur, omega)
        ka = _kkt_w(lp, a, xa, ya, omega)
        assert _close(rec[2], kc) and _close(rec[3], ka), (k, rec[2], kc, rec[3], ka)
        assert _close(rec[9], anc), (k, rec[9], anc)
        assert _close(rec[10], prev), (k, rec[10], prev)
        t = k - k_last
        assert int(rec[1]) == t
        # candidate: the average only when its error is strictly smaller (the Halpern form has one)
        if method == 0 and not _tie(ka, kc):
            assert bool(rec[6]) == (ka < kc), (k, ka, kc)
        use_avg = method == 1 or bool(rec[6])
        kcand = ka if use_avg else kc
        assert kcand <= kc * (1 + 1e-12)
        # restart reason: the first test that holds
        ties = [_tie(kcand, 0.2 * anc), _tie(kcand, 0.8 * anc), t == 0.36 * k, _tie(kcand, prev)]
        if not any(ties):
            if kcand <= 0.2 * anc:
                why = 1
            elif kcand <= 0.8 * anc and kcand > prev:
                why = 2
            elif t >= 0.36 * k:
                why = 3
            else:
                why = 0
            assert int(rec[7]) == why, (k, int(rec[7]), why, kcand / anc, kcand, prev, t / k)
        why = int(rec[7])
        if seen is not None:
            seen.add(why)
        if why:
            xc, yc = (xa, ya) if use_avg else (x, y)
            dx, dy = np.linalg.norm(xc - x_an), np.linalg.norm(yc - y_an)
            new = float(rec[8])
            if dx > 1e-10 and dy > 1e-10:
                before = math.log(omega * dx / dy)
                after = math.log(new * dx / dy)
                if pid is None:
                    assert abs(after - before * 2.0**-steps) <= 1e-12 * (1 + abs(before)), (k, before, after, steps)
                else:
                    errors.append(before)
                    e = np.array(errors)
                    total = -(pid[0] * e.sum() + pid[1] * np.cumsum(e).sum() + pid[2] * e[-1])
                    assert abs(math.log(new) - total) <= 1e-11 * (1 + abs(total)), (k, math.log(new), total)
            else:
                assert new == omega
            omega = new
            x_an, y_an = xc.copy(), yc.copy()
            anc = _kkt_w(lp, a, x_an, y_an, omega)
            prev = math.inf
            k_last = k
        else:
            assert float(rec[8]) == omega
            prev = kcand


@pytest.mark.parametrize("method", [0, 1])
def test_restart_decisions_recomputed(oracle_lib, method):
    seen = set()
    for j in range(4):
        _check_decisions(oracle_lib, _lp(j), method, seen=seen)
    # the cases exercise every restart reason (the Halpern form rarely meets "no progress")
    assert {1, 3} <= seen and (method == 1 or 2 in seen), seen


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_primal_weight_balances_distances(oracle_lib, steps):
    _check_decisions(oracle_lib, _lp(1), 0, omega_steps=steps)


@pytest.mark.parametrize("gains", [(0.99, 0.01, 0.0), (0.6, 0.15, 0.3)])
@pytest.mark.parametrize("method", [0, 1])
def test_pid_primal_weight_closed_form(oracle_lib, method, gains):
    """PID rule of the primal weight (omega starts at 1, so log omega_0 = 0): every decision
    recomputed as above and the weight after each restart equal to the closed form of the
    controller's cumulative output."""
    seen = set()
    for j in range(2):
        _check_decisions(oracle_lib, _lp(j), method, seen=seen, pid=gains)
    assert 1 in seen and 3 in seen


def test_pid_proportional_is_smoothing(oracle_lib):
    """With ki = kd = 0 the PID rule moves log omega by the fraction kp toward log(dy/dx): at
    kp = 1/2 it is the one-step smoothing, so the weights and decisions of both runs agree
    (to the rounding of exp/log against the square root, which the iteration then carries:
    the first weights agree to 1e-14, later ones drift by up to ~1e-7)."""
    lp = _lp(1)
    eta = 0.95 / np.linalg.norm(lp.dense(), 2)
    a = _solve(oracle_lib, lp, eta, 0, False, pw_rule=1, omega_steps=1)
    b = _solve(oracle_lib, lp, eta, 0, False, pw_rule=2, pid_kp=0.5, pid_ki=0.0, pid_kd=0.0)
    assert a.iters == b.iters and a.restarts == b.restarts
    assert np.array_equal(a.trace[:, [0, 1, 6, 7]], b.trace[:, [0, 1, 6, 7]])
    np.testing.assert_allclose(b.trace[:6, 8], a.trace[:6, 8], rtol=1e-14)
    np.testing.assert_allclose(b.trace[:, 8], a.trace[:, 8], rtol=1e-6)


# ---- restarts on the fixed-point residual (Halpern form, restart_metric = 1) -------------

def _pdhg_map(oracle_lib, lp, x, y, eta, omega):
    """T(z): one step of the oracle's PDHG from the warm start z (no scaling, no restarts)."""
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=1, scaling=False, restarts=False, eta=eta, omega0=omega,
                         method=0, x0=x, y0=y, snap_k=[1])
    xs, ys, _, _ = oracle_lib.split_snap(r.snaps[0], lp.n, lp.m)
    return xs.copy(), ys.copy()


def _m_inner(a, u, v, eta, omega, sign=1.0):
    """eta <u, M v> with the PDHG preconditioner M = [[I/tau, A^T], [A, I/sigma]]."""
    tau, sigma = eta / omega, eta * omega
    return eta * (u[0] @ v[0] / tau + sign * (u[1] @ (a @ v[0]) + v[1] @ (a @ u[0])) + u[1] @ v[1] / sigma)


def _fpr(a, x, xt, y, yt, omega, eta):
    """||z - T(z)|| in that norm, from its definition."""
    d = (x - xt, y - yt)
    return math.sqrt(max(_m_inner(a, d, d, eta, omega), 0.0))


def test_residual_norm_makes_the_map_firmly_nonexpansive(oracle_lib):
    """The norm of the residual restarts is the one in which the PDHG map is firmly
    nonexpansive, ||Tz - Tz'||^2 <= <Tz - Tz', z - z'> (the property the Halpern iteration's
    convergence rests on): it holds for every pair of random points with the metric above and
    fails for most with the sign of the coupling term flipped, so the sign is fixed by the
    map itself."""
    held = broken = 0
    for j in range(3):
        lp = _lp(j)
        a = lp.dense()
        eta = 0.95 / np.linalg.norm(a, 2)
        rng = np.random.default_rng([23, j])
        lo, hi = lp.x_lo, lp.x_hi

        def point():
            x = np.where(np.isfinite(lo) & np.isfinite(hi), lo + rng.random(lp.n) * (hi - lo), 3 * rng.normal(size=lp.n))
            return np.clip(x, lo, hi), 3 * rng.normal(size=lp.m)

        for omega in (0.3, 1.0, 4.0):
            for _ in range(6):
                z1, z2 = point(), point()
                t1, t2 = _pdhg_map(oracle_lib, lp, *z1, eta, omega), _pdhg_map(oracle_lib, lp, *z2, eta, omega)
                dt, dz = (t1[0] - t2[0], t1[1] - t2[1]), (z1[0] - z2[0], z1[1] - z2[1])
                lhs, rhs = _m_inner(a, dt, dt, eta, omega), _m_inner(a, dt, dz, eta, omega)
                assert lhs <= rhs + 1e-12 * abs(lhs), (j, omega, lhs, rhs)
                held += 1
                flhs, frhs = _m_inner(a, dt, dt, eta, omega, -1.0), _m_inner(a, dt, dz, eta, omega, -1.0)
                broken += flhs > frhs
    assert held == 54 and broken >= 27


def _check_fpr_decisions(oracle_lib, lp, pid=None, seen=None):
    """Every decision of a Halpern solve with residual restarts, recomputed from snapshots:
    the residual of the iterate before each evaluation (z_{k-1} against T(z_{k-1}), the
    snapshot pair k-1, k) and of the cycle's anchor (the anchor against its image, the first
    iteration of the cycle), the restart reason from them, and the primal-weight update."""
    a = lp.dense()
    eta = 0.95 / np.linalg.norm(a, 2)
    kw = dict(restart_metric=1)
    if pid is not None:
        kw.update(pw_rule=2, pid_kp=pid[0], pid_ki=pid[1], pid_kd=pid[2])
    base = _solve(oracle_lib, lp, eta, 1, False, **kw)
    tr = base.trace
    ks = [int(r[0]) for r in tr]
    snaps = sorted({1} | {k + d for k in ks for d in (-1, 0, 1)})
    run = _solve(oracle_lib, lp, eta, 1, False, snap_k=snaps, **kw)
    assert np.array_equal(run.trace, tr)
    S = {k: oracle_lib.split_snap(run.snaps[i], lp.n, lp.m) for i, k in enumerate(snaps)}
    omega = 1.0
    x_an, y_an = np.clip(np.zeros(lp.n), lp.x_lo, lp.x_hi), np.zeros(lp.m)
    anc = _fpr(a, x_an, S[1][2], y_an, S[1][3], omega, eta)
    prev, k_last, errors = math.inf, 0, []
    for rec in tr[:-1]:
        k = int(rec[0])
        xa, ya = S[k][2], S[k][3]
        r = _fpr(a, S[k - 1][0], xa, S[k - 1][1], ya, omega, eta)
        # the oracle's A~x of the Halpern iterate is carried by linearity, numpy's is A @ x: the
        # coupling term differs by ~1e-16 |Ax| sqrt(m), an absolute noise far below 1e-13
        assert _close(rec[2], r, noise=1e-13) and rec[3] == rec[2], (k, rec[2], r)
        assert _close(rec[9], anc, noise=1e-13), (k, rec[9], anc)
        assert _close(rec[10], prev, noise=1e-13), (k, rec[10], prev)
        t = k - k_last
        assert int(rec[1]) == t
        ties = [_tie(r, 0.2 * anc), _tie(r, 0.8 * anc), t == 0.36 * k, _tie(r, prev)]
        if not any(ties):
            why = 1 if r <= 0.2 * anc else 2 if (r <= 0.8 * anc and r > prev) else 3 if t >= 0.36 * k else 0
            assert int(rec[7]) == why, (k, int(rec[7]), why, r / anc, r, prev, t / k)
        why = int(rec[7])
        if seen is not None:
            seen.add(why)
        if why:
            dx, dy = np.linalg.norm(xa - x_an), np.linalg.norm(ya - y_an)
            new = float(rec[8])
            before = math.log(omega * dx / dy)
            if pid is None:
                assert abs(math.log(new * dx / dy) - before / 4.0) <= 1e-12 * (1 + abs(before)), (k, before)
            else:
                errors.append(before)
                e = np.array(errors)
                total = -(pid[0] * e.sum() + pid[1] * np.cumsum(e).sum() + pid[2] * e[-1])
                assert abs(math.log(new) - total) <= 1e-11 * (1 + abs(total)), (k, math.log(new), total)
            omega = new
            x_an, y_an = xa.copy(), ya.copy()
            anc = _fpr(a, x_an, S[k + 1][2], y_an, S[k + 1][3], omega, eta)
            prev, k_last = math.inf, k
        else:
            assert float(rec[8]) == omega
            prev = r


@pytest.mark.parametrize("pid", [None, (0.7, 0.05, 0.2)], ids=["smoothing", "pid"])
def test_residual_restart_decisions_recomputed(oracle_lib, pid):
    seen = set()
    for j in range(4):
        _check_fpr_decisions(oracle_lib, _lp(j), pid=pid, seen=seen)
    assert {1, 3} <= seen, seen


def test_residual_restarts_solve_and_change_the_run(oracle_lib):
    """The residual restarts solve these LPs to 1e-8 (E_rel rechecked by the oracle's KKT on
    the original data) and restart at other evaluations than the KKT restarts; the averaged
    form ignores the option."""
    for j in range(3):
        lp = _lp(j)
        kkt = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=200000, method=1)
        res = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=200000, method=1, restart_metric=1)
        assert res.status == "optimal" and res.erel <= 1e-8
        assert not np.array_equal(kkt.trace[:, [0, 7]], res.trace[:, [0, 7]]) or kkt.iters != res.iters
        avg = oracle_lib.solve(lp, eps_rel=1e-6, max_iters=200000, method=0)
        avg1 = oracle_lib.solve(lp, eps_rel=1e-6, max_iters=200000, method=0, restart_metric=1)
        assert np.array_equal(avg.trace, avg1.trace) and np.array_equal(avg.x, avg1.x)
