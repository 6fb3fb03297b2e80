"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

- Worked examples of the paper (golden/tiny_lps.json, hand-solved from Section 2, eq. 2).
- Hand-computed KKT residuals at chosen points (golden/kkt_points.json).
- KKT-constructed LPs whose optimum is known by construction.
"""
import math

import numpy as np
import pytest

import synth
from conftest import golden_lps, load_golden

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _kkt_sign_ok(lp, x, y, z, tol):
    """Sign/complementarity rules of eq. (2): z>0 => x=x_lo, z<0 => x=x_hi, y>0 => Ax=b_lo,
    y<0 => Ax=b_hi, free x => z=0; b_lo=-inf => y<=0, b_hi=+inf => y>=0."""
    ax = lp.dense() @ x
    for k in range(lp.n):
        if z[k] > tol:
            assert abs(x[k] - lp.x_lo[k]) <= tol * 10
        if z[k] < -tol:
            assert abs(x[k] - lp.x_hi[k]) <= tol * 10
        if math.isinf(lp.x_lo[k]) and math.isinf(lp.x_hi[k]):
            assert abs(z[k]) <= tol
    for i in range(lp.m):
        if y[i] > tol:
            assert abs(ax[i] - lp.b_lo[i]) <= tol * 10
        if y[i] < -tol:
            assert abs(ax[i] - lp.b_hi[i]) <= tol * 10
        if lp.b_lo[i] == -math.inf:
            assert y[i] <= tol
        if lp.b_hi[i] == math.inf:
            assert y[i] >= -tol


@pytest.mark.parametrize("name", ["T1", "T2", "T3", "T4", "T5"])
@pytest.mark.parametrize("scaling", [False, True])
def test_worked_examples(oracle_lib, name, scaling):
    lp, spec = golden_lps()[name]
    r = oracle_lib.solve(lp, eps_rel=1e-10, max_iters=200000, scaling=scaling)
    assert r.status == "optimal", (r.status, r.erel)
    assert abs(r.pobj - spec["p_star"]) <= 1e-8 * (1 + abs(spec["p_star"]))
    if spec.get("x_unique"):
        np.testing.assert_allclose(r.x, spec["x_star"], atol=1e-7)
    if "x1_star" in spec:
        assert abs(r.x[0] - spec["x1_star"]) <= 1e-7
    if "x_sum" in spec:
        assert abs(r.x.sum() - spec["x_sum"]) <= 1e-7
    if spec.get("y_unique"):
        np.testing.assert_allclose(r.y, spec["y_star"], atol=1e-7)
        np.testing.assert_allclose(r.z, spec["z_star"], atol=1e-7)
    if name == "T1":
        # y is not unique: any y in [0, 1/2] is optimal, z = (1 - y, 1 - 2y)
        assert -1e-7 <= r.y[0] <= 0.5 + 1e-7
        np.testing.assert_allclose(r.z, [1 - r.y[0], 1 - 2 * r.y[0]], atol=1e-7)
    _kkt_sign_ok(lp, r.x, r.y, r.z, 1e-6)


@pytest.mark.parametrize("pt", range(5))
def test_kkt_hand_computed_points(oracle_lib, pt):
    spec = load_golden("kkt_points.json")["points"][pt]
    lp, _ = golden_lps()[spec["lp"]]
    k = oracle_lib.kkt(lp, np.array(spec["x"], float), np.array(spec["y"], float))
    for key in ("rel_p", "rel_d", "rel_gap", "erel", "pobj", "dobj"):
        assert abs(k[key] - spec[key]) <= 1e-15 * (1 + abs(spec[key])), (key, k[key], spec[key])


@pytest.mark.parametrize("j", range(3))
def test_constructed_optimum_passes_kkt(oracle_lib, j):
    lp = synth.cfg0(j)
    k = oracle_lib.kkt(lp, lp.x_star, lp.y_star)
    assert k["erel"] < 1e-14
    np.testing.assert_allclose(k["z"], lp.z_star, atol=1e-13)
    assert abs(k["pobj"] - lp.p_star) < 1e-12 * (1 + abs(lp.p_star))
    # strong duality at the constructed point
    assert abs(k["pobj"] - k["dobj"]) < 1e-12 * (1 + abs(lp.p_star))


def test_kkt_detects_perturbation(oracle_lib):
    """Moving x* off a bound, or flipping the sign of y* on an active row, must show up."""
    lp = synth.cfg0(0)
    x = lp.x_star.copy()
    k_at = np.flatnonzero(lp.z_star > 0)[0]
    x[k_at] += 0.5
    k = oracle_lib.kkt(lp, x, lp.y_star)
    assert k["rel_gap"] > 1e-3 or k["rel_p"] > 1e-3
    y = lp.y_star.copy()
    i_act = np.flatnonzero((lp.b_hi == math.inf) & (lp.y_star > 0))[0]
    y[i_act] = -y[i_act]
    k = oracle_lib.kkt(lp, lp.x_star, y)
    assert k["rel_d"] > 1e-3


@pytest.mark.parametrize("j", range(3))
def test_constructed_lp_solved_to_known_optimum(oracle_lib, j):
    lp = synth.cfg0(j)
    r = oracle_lib.solve(lp, eps_rel=1e-9, max_iters=400000)
    assert r.status == "optimal"
    assert r.erel <= 1e-9
    assert abs(r.pobj - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))
    k = oracle_lib.kkt(lp, r.x, r.y)
    assert k["erel"] <= 2e-9
    _kkt_sign_ok(lp, r.x, r.y, r.z, 1e-5)


def test_two_sided_and_free_rows_constructed(oracle_lib):
    """Small instance of the large-LP recipe (free columns, two-sided rows, power-law columns)."""
    lp = synth.cfg1(0, m=300, n=600, nnz=3000)
    k = oracle_lib.kkt(lp, lp.x_star, lp.y_star)
    assert k["erel"] < 1e-14
    r = oracle_lib.solve(lp, eps_rel=1e-8, max_iters=400000)
    assert r.status == "optimal"
    assert abs(r.pobj - lp.p_star) <= 1e-6 * (1 + abs(lp.p_star))


@pytest.mark.parametrize("j", range(2))
def test_reported_error_matches_external_check(oracle_lib, j):
    """The E_rel terms the solver reports (computed on the scaled problem and unscaled by
    exact powers of two) equal a direct check on the original data at the returned point."""
    lp = synth.cfg1(j, m=200, n=400, nnz=1500)
    r = oracle_lib.solve(lp, eps_rel=1e-6, max_iters=100000)
    k = oracle_lib.kkt(lp, r.x, r.y)
    for key in ("rel_p", "rel_d", "rel_gap"):
        assert abs(getattr(r, key) - k[key]) <= 1e-12 * abs(k[key]) + 1e-300, (key, getattr(r, key), k[key])
    np.testing.assert_array_equal(r.z, k["z"])
