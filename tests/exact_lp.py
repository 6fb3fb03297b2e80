"""Exact LP solutions by scipy's HiGHS, in the sign convention of the paper's eq. 2.

Used as a third-party cross-check only (the presolve tests compare optimal values and check
postsolved points with the oracle's KKT routine). y_i > 0 means the row is held at b_lo,
y_i < 0 at b_hi; z = c - A^T y.
"""
import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def highs(lp):
    m, n = lp.m, lp.n
    A = sp.csr_matrix((lp.vals, lp.col_idx, lp.row_ptr), shape=(m, n))
    lo, hi = np.asarray(lp.b_lo, float), np.asarray(lp.b_hi, float)
    eq = np.flatnonzero(lo == hi)
    up = np.flatnonzero((lo != hi) & np.isfinite(hi))
    dn = np.flatnonzero((lo != hi) & np.isfinite(lo))
    A_ub = sp.vstack([A[up], -A[dn]]) if len(up) + len(dn) else None
    b_ub = np.concatenate([hi[up], -lo[dn]]) if len(up) + len(dn) else None
    A_eq = A[eq] if len(eq) else None
    b_eq = lo[eq] if len(eq) else None
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b) for a, b in zip(lp.x_lo, lp.x_hi)]
    r = linprog(lp.c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq, bounds=bounds, method="highs")
    out = {"status": {0: "optimal", 2: "infeasible", 3: "unbounded"}.get(r.status, str(r.status)),
           "message": r.message}
    if r.status != 0:
        return out
    y = np.zeros(m)
    if len(eq):
        y[eq] = r.eqlin.marginals
    if len(up):
        y[up] += r.ineqlin.marginals[: len(up)]
    if len(dn):
        y[dn] -= r.ineqlin.marginals[len(up):]
    x = np.asarray(r.x, float)
    z = np.asarray(lp.c, float) - A.T @ y
    out.update(x=x, y=y, z=z, obj=float(r.fun) + float(getattr(lp, "c0", 0.0)))
    return out
