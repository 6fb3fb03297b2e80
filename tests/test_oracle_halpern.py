"""Pins of the oracle's Halpern form (method 1): z <- w ((1 + rho) T(z) - rho z) + (1 - w) z0,
w = (t + 1) / (t + 2), with T the PDHG map; evaluations, restarts and the output act on T(z)."""
import math

import numpy as np
import pytest

import synth
from conftest import golden_lps
from test_oracle_exact import _free_equality_lp


def pdhg_map(a, c, bl, bu, xl, xu, tau, sigma, x, y):
    xn = np.clip(x - tau * (c - a.T @ y), xl, xu)
    v = y - sigma * (a @ (2 * xn - x))
    yn = np.maximum(v + sigma * bl, 0) + np.minimum(v + sigma * bu, 0)
    return xn, yn


@pytest.mark.parametrize("name", ["T1", "T2", "T3", "T4", "T5"])
@pytest.mark.parametrize("rho", [1.0, 0.5])
def test_worked_examples(oracle_lib, name, rho):
    lp, spec = golden_lps()[name]
    r = oracle_lib.solve(lp, eps_rel=1e-9, max_iters=200000, method=1, reflection=rho)
    assert r.status == "optimal"
    assert r.pobj == pytest.approx(spec["p_star"], abs=1e-7)
    k = oracle_lib.kkt(lp, r.x, r.y)
    assert k["erel"] == pytest.approx(r.erel, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("rho", [1.0, 0.3])
def test_linear_recurrence_all_free_equalities(oracle_lib, rho):
    """All-free equality LP: T is affine, so without restarts the Halpern iterates follow a
    linear recurrence that dense numpy reproduces."""
    lp, a, b, c = _free_equality_lp(5)
    eta, omega = 0.9 / np.linalg.norm(a, 2), 1.3
    tau, sigma = eta / omega, eta * omega
    ks = list(range(1, 201))
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=200, scaling=False, restarts=False, eta=eta, omega0=omega,
                         snap_k=ks, method=1, reflection=rho)
    x0, y0 = np.zeros(lp.n), np.zeros(lp.m)
    x, y = x0.copy(), y0.copy()
    for k in ks:
        xt = x - tau * (c - a.T @ y)
        yt = y - sigma * (a @ (2 * xt - x) - b)
        w = k / (k + 1)  # (t + 1) / (t + 2) with t = k - 1 iterations before this one
        x, y = w * ((1 + rho) * xt - rho * x) + (1 - w) * x0, w * ((1 + rho) * yt - rho * y) + (1 - w) * y0
        xs, ys, xa, ya = oracle_lib.split_snap(r.snaps[k - 1], lp.n, lp.m)
        scale = max(1.0, np.abs(x).max(), np.abs(y).max())
        assert np.abs(xs - x).max() <= 1e-12 * scale
        assert np.abs(ys - y).max() <= 1e-12 * scale
        assert np.abs(xa - xt).max() <= 1e-12 * scale
        assert np.abs(ya - yt).max() <= 1e-12 * scale


def test_kkt_point_is_fixed_point(oracle_lib):
    lp = synth.cfg0(1)
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=3, scaling=False, x0=lp.x_star, y0=lp.y_star, snap_k=[1, 2, 3],
                         method=1)
    for s in r.snaps:
        xs, ys, xa, ya = oracle_lib.split_snap(s, lp.n, lp.m)
        for u, v in ((xs, lp.x_star), (ys, lp.y_star), (xa, lp.x_star), (ya, lp.y_star)):
            np.testing.assert_allclose(u, v, atol=1e-12)


@pytest.mark.parametrize("rho", [1.0, 0.5, 0.0])
def test_halpern_rate_bound(oracle_lib, rho):
    """Halpern's bound for the nonexpansive map R = (1 + rho) T - rho I (T is firmly
    nonexpansive in the PDHG metric M): ||z_k - T(z_k)||_M <= 2 ||z_0 - z*||_M / ((1 + rho)(k + 1))
    without restarts, for every k."""
    lp = synth.cfg0(2)
    a = lp.dense()
    eta = 0.95 / np.linalg.norm(a, 2)
    omega = 1.3
    tau, sigma = eta / omega, eta * omega
    ks = list(range(1, 401))
    r = oracle_lib.solve(lp, eps_rel=0.0, max_iters=400, scaling=False, restarts=False, eta=eta, omega0=omega,
                         snap_k=ks, method=1, reflection=rho)

    def mnorm(dx, dy):
        return math.sqrt(max(0.0, dx @ dx / tau + 2 * dy @ (a @ dx) + dy @ dy / sigma))

    x0 = np.clip(np.zeros(lp.n), lp.x_lo, lp.x_hi)
    bound0 = 2 * mnorm(x0 - lp.x_star, -lp.y_star) / (1 + rho)
    worst = 0.0
    for k, s in zip(ks, r.snaps):
        xs, ys, _, _ = oracle_lib.split_snap(s, lp.n, lp.m)
        xt, yt = pdhg_map(a, lp.c, lp.b_lo, lp.b_hi, lp.x_lo, lp.x_hi, tau, sigma, xs, ys)
        res = mnorm(xs - xt, ys - yt)
        assert res <= bound0 / (k + 1) * (1 + 1e-9) + 1e-12, (k, res, bound0 / (k + 1))
        worst = max(worst, res * (k + 1) / bound0)
    assert worst > 0.01  # the bound is not vacuous for this LP


def test_restarted_halpern_reaches_known_optimum(oracle_lib):
    for j in range(3):
        lp = synth.cfg0(j)
        r = oracle_lib.solve(lp, eps_rel=1e-7, max_iters=300000, method=1)
        assert r.status == "optimal"
        assert abs(r.pobj - lp.p_star) <= 1e-5 * (1 + abs(lp.p_star))
