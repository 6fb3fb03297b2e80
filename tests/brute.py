"""Brute-force vertex enumeration for tiny bounded LPs (independent of the oracle).

Every vertex of {x : b_lo <= Ax <= b_hi, x_lo <= x <= x_hi} is the solution of n linearly
independent active constraints; the minimum of c^T x over a non-empty polytope is attained
at a vertex. All choices of n constraints are solved (batched, partial pivoting via LAPACK)
and the feasible solutions kept.
"""
import itertools
import math

import numpy as np


def enumerate_min(a: np.ndarray, c, b_lo, b_hi, x_lo, x_hi, feas_tol: float = 1e-9):
    m, n = a.shape
    rows, rhs = [], []
    for i in range(m):
        if math.isfinite(b_lo[i]):
            rows.append(a[i]); rhs.append(b_lo[i])
        if math.isfinite(b_hi[i]) and b_hi[i] != b_lo[i]:
            rows.append(a[i]); rhs.append(b_hi[i])
    eye = np.eye(n)
    for k in range(n):
        if math.isfinite(x_lo[k]):
            rows.append(eye[k]); rhs.append(x_lo[k])
        if math.isfinite(x_hi[k]) and x_hi[k] != x_lo[k]:
            rows.append(eye[k]); rhs.append(x_hi[k])
    G = np.array(rows)
    h = np.array(rhs)
    combos = np.array(list(itertools.combinations(range(len(G)), n)), dtype=np.int64)
    best = math.inf
    best_x = None
    for start in range(0, len(combos), 20000):
        cb = combos[start : start + 20000]
        M = G[cb]
        rhs_b = h[cb]
        det = np.linalg.det(M)
        ok = np.abs(det) > 1e-10
        if not ok.any():
            continue
        X = np.linalg.solve(M[ok], rhs_b[ok][..., None])[..., 0]
        AX = X @ a.T
        feas = np.all(X >= np.asarray(x_lo) - feas_tol, axis=1) & np.all(X <= np.asarray(x_hi) + feas_tol, axis=1)
        if m:
            feas &= np.all(AX >= np.asarray(b_lo) - feas_tol, axis=1) & np.all(AX <= np.asarray(b_hi) + feas_tol, axis=1)
        if feas.any():
            obj = X[feas] @ np.asarray(c)
            j = int(np.argmin(obj))
            if obj[j] < best:
                best = float(obj[j])
                best_x = X[feas][j]
    return best, best_x
