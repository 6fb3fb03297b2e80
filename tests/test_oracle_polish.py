"""Pins of the oracle's feasibility polishing and of its residual-only stopping rules.

* Stopping rule: with term_mode 1 (2) a solve stops at the first evaluation where the
  relative primal (dual) residual of the current point or of the average is at most eps_rel;
  recomputed in dense numpy from the returned points, it is at most eps at the stop and above
  eps at the evaluation before.
* Polishing: the primal solve's point satisfies the constraints to eps and the dual solve's y
  has a dual residual of at most eps, both recomputed in numpy from the definitions of eq. 2;
  bounds and sign conditions hold exactly; a point that is already feasible is returned
  unchanged after 0 iterations."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _rel_p(lp, x):
    ax = lp.dense() @ x
    rp = ax - np.clip(ax, lp.b_lo, lp.b_hi)
    q = np.maximum(np.where(np.isfinite(lp.b_lo), np.abs(lp.b_lo), 0), np.where(np.isfinite(lp.b_hi), np.abs(lp.b_hi), 0))
    return float(np.linalg.norm(rp)) / (1 + float(np.linalg.norm(q)))


def _rel_d(lp, y):
    lam = lp.c - lp.dense().T @ y
    flo, fhi = np.isfinite(lp.x_lo), np.isfinite(lp.x_hi)
    z = np.where(flo & fhi, lam, np.where(flo, np.maximum(lam, 0), np.where(fhi, np.minimum(lam, 0), 0.0)))
    viol = np.where(np.isneginf(lp.b_lo) & (y > 0), y, 0.0) + np.where(np.isposinf(lp.b_hi) & (y < 0), -y, 0.0)
    r = math.sqrt(float(np.sum((lam - z) ** 2) + np.sum(viol**2)))
    return r / (1 + float(np.linalg.norm(lp.c)))


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_residual_stopping_rule(oracle_lib, mode, method):
    # the dual residual needs unbounded variables (a boxed variable takes any reduced cost)
    lp = synth.cfg0(1) if mode == 1 else synth.cfg1(0, m=400, n=800, nnz=4000)
    eps = 1e-6
    r = oracle_lib.solve(lp, eps_rel=eps, max_iters=200000, method=method, term_mode=mode)
    assert r.status == "optimal" and r.iters > 64
    measure = _rel_p if mode == 1 else _rel_d
    val = measure(lp, r.x if mode == 1 else r.y)
    assert val <= eps * (1 + 1e-6), val
    before = oracle_lib.solve(lp, eps_rel=0.0, max_iters=r.iters - 64, method=method, term_mode=mode)
    assert measure(lp, before.x if mode == 1 else before.y) > eps


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("name", ["cfg0", "large_recipe", "transport"])
def test_polish_feasibility(oracle_lib, name, method):
    lp = {"cfg0": lambda: synth.cfg0(0), "large_recipe": lambda: synth.cfg1(0, m=400, n=800, nnz=4000),
          "transport": lambda: synth.transportation(60, np.random.default_rng(2))}[name]()
    r = oracle_lib.solve(lp, eps_rel=1e-4, max_iters=200000, method=method)
    eps = 1e-9
    p = oracle_lib.polish(lp, r.x, r.y, eps=eps, method=method)
    assert p.primal_status == "optimal" and p.dual_status == "optimal"
    assert _rel_p(lp, p.x) <= eps * (1 + 1e-6)
    assert _rel_d(lp, p.y) <= eps * (1 + 1e-6)
    assert np.all(p.x >= lp.x_lo) and np.all(p.x <= lp.x_hi)
    assert np.all(p.y[np.isposinf(lp.b_hi)] >= 0) and np.all(p.y[np.isneginf(lp.b_lo)] <= 0)
    # the oracle's own KKT record of the polished pair agrees with the recomputation
    assert p.kkt["rel_p"] == pytest.approx(_rel_p(lp, p.x), rel=1e-6, abs=1e-15)
    # polishing stays near the point it started from
    assert np.linalg.norm(p.x - r.x) <= 0.1 * (1 + np.linalg.norm(r.x))


def test_polish_of_a_feasible_point_is_the_point(oracle_lib):
    lp = synth.cfg0(0)
    p = oracle_lib.polish(lp, lp.x_star, lp.y_star, eps=1e-6)
    assert p.primal_iters == 0 and p.dual_iters == 0
    assert np.array_equal(p.x, lp.x_star) and np.array_equal(p.y, lp.y_star)
