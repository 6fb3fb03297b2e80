"""Oracle pins for the one-time steps: CSR transpose (bit-exact against brute force and
scipy), power-of-two scaling (exactness, equilibration band) and the spectral-norm estimate
(against LAPACK's SVD)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _lps():
    return [synth.cfg0(0), synth.cfg1(0, m=500, n=1000, nnz=6000), synth.transportation(80, np.random.default_rng(1)),
            synth.cfg4_lp(0, m_hi=400)]


@pytest.mark.parametrize("idx", range(4))
def test_transpose_bitexact(oracle_lib, idx):
    lp = _lps()[idx]
    rpT, ciT, vT = oracle_lib.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals)
    # brute force: walk the dense transpose column by column
    d = lp.dense().T
    rows, cols = np.nonzero(d)
    exp_rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=lp.n))]).astype(np.int32)
    assert np.array_equal(rpT, exp_rp)
    assert np.array_equal(ciT, cols.astype(np.int32))
    assert np.array_equal(vT.view(np.uint64), d[rows, cols].view(np.uint64))
    # scipy
    t = sp.csr_matrix((lp.vals, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).T.tocsr()
    t.sort_indices()
    assert np.array_equal(rpT, t.indptr.astype(np.int32))
    assert np.array_equal(ciT, t.indices.astype(np.int32))
    assert np.array_equal(vT.view(np.uint64), t.data.view(np.uint64))


def test_transpose_empty_rows_and_columns(oracle_lib):
    rp = np.array([0, 0, 2, 2, 3], np.int32)
    ci = np.array([1, 4, 4], np.int32)
    v = np.array([1.5, -2.0, 3.0])
    rpT, ciT, vT = oracle_lib.transpose(4, 6, rp, ci, v)
    assert rpT.tolist() == [0, 0, 1, 1, 1, 3, 3]
    assert ciT.tolist() == [1, 1, 3]
    assert vT.tolist() == [1.5, -2.0, 3.0]


@pytest.mark.parametrize("idx", range(4))
def test_scaling_exact_and_power_of_two(oracle_lib, idx):
    lp = _lps()[idx]
    av, R, Cc = oracle_lib.scale(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals)
    rows = np.repeat(np.arange(lp.m), np.diff(lp.row_ptr))
    # factors are exact powers of two
    for f in (R, Cc):
        mant, _ = np.frexp(f)
        assert np.all(mant == 0.5)
    # A~ = R A C exactly, and unscaling recovers A bit for bit
    assert np.array_equal(av, lp.vals * R[rows] * Cc[lp.col_idx])
    back = av / R[rows] / Cc[lp.col_idx]
    assert np.array_equal(back.view(np.uint64), lp.vals.view(np.uint64))


@pytest.mark.parametrize("idx", range(4))
def test_ruiz_equilibration_band(oracle_lib, idx):
    """After the infinity-norm Ruiz passes alone, every non-empty row and column has its
    largest |entry| in [1/4, 4] (power-of-two Ruiz settles within a factor of two of 1 per
    side, the coupling widens that by at most another factor of two)."""
    lp = _lps()[idx]
    av, R, Cc = oracle_lib.scale(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals, ruiz=10, pock_chambolle=False)
    a = sp.csr_matrix((np.abs(av), lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    rmax = a.max(axis=1).toarray().ravel()
    cmax = a.max(axis=0).toarray().ravel()
    rmax = rmax[np.diff(lp.row_ptr) > 0]
    cmax = cmax[np.bincount(lp.col_idx, minlength=lp.n) > 0]
    assert rmax.min() >= 0.25 and rmax.max() <= 4.0, (rmax.min(), rmax.max())
    assert cmax.min() >= 0.25 and cmax.max() <= 4.0, (cmax.min(), cmax.max())


@pytest.mark.parametrize("idx", range(4))
def test_power_norm_against_svd(oracle_lib, idx):
    lp = _lps()[idx]
    true = np.linalg.norm(lp.dense(), 2)
    est = oracle_lib.power_norm(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.vals, iters=200)
    # a Rayleigh quotient of A^T A never exceeds ||A||^2
    assert est <= true * (1 + 1e-13)
    assert est >= true * (1 - 1e-3)


def test_validation_codes(oracle_lib):
    lp = synth.cfg0(0)
    assert oracle_lib.validate(lp) == 0
    bad = synth.cfg0(0)
    bad.col_idx = bad.col_idx.copy()
    r0, r1 = bad.row_ptr[3], bad.row_ptr[4]
    bad.col_idx[r0:r1] = bad.col_idx[r0:r1][::-1]
    if r1 - r0 >= 2:
        assert oracle_lib.validate(bad) == 2
    bad = synth.cfg0(0)
    bad.vals = bad.vals.copy()
    bad.vals[5] = math.nan
    assert oracle_lib.validate(bad) == 4
    bad = synth.cfg0(0)
    bad.x_lo = bad.x_lo.copy()
    bad.x_lo[3] = 11.0
    assert oracle_lib.validate(bad) == 3


def _csr_of_dense(D):
    import scipy.sparse as sp
    S = sp.csr_matrix(D)
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def test_power_norm_close_top_singular_values(oracle_lib):
    """Two leading singular values 0.1% apart: 200 fixed steps leave sigma_hat about 3e-4
    low, which would break the PDHG step condition eta ||A~|| < 1 at eta = 0.998 / sigma_hat
    once combined with a slightly larger gap; the chunked iteration runs until the estimate
    stops rising and lands within 2e-5 (the singular values are set, so the norm is known)."""
    rng = np.random.default_rng(11)
    m, n = 40, 60
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.concatenate([[2.0, 2.0 * 0.999], np.linspace(1.5, 0.1, m - 2)])
    D = (U * s) @ V[:, :m].T
    rp, ci, v = _csr_of_dense(D)
    est = oracle_lib.power_norm(m, n, rp, ci, v, iters=200)
    assert est <= 2.0 * (1 + 1e-13)
    assert est >= 2.0 * (1 - 2e-5), est


def test_power_norm_small_lp_with_close_gap(oracle_lib):
    """A small LP of the batched recipe whose scaled matrix has its two largest singular
    values 0.4% apart: the estimate is within 1e-4 of LAPACK's norm, so eta = 0.998 /
    sigma_hat keeps eta ||A~|| below 1."""
    lp = synth.cfg3_lp(2564)
    av, R, Cc, *_ = oracle_lib.scaled_problem(lp)
    import scipy.sparse as sp
    true = np.linalg.norm(sp.csr_matrix((av, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray(), 2)
    est = oracle_lib.power_norm(lp.m, lp.n, lp.row_ptr, lp.col_idx, av, iters=200)
    assert true * (1 - 1e-4) <= est <= true * (1 + 1e-13)
    assert 0.998 / est * true < 1.0
