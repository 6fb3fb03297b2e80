"""Seeded LP instance generators.

Every instance is an LP of the paper's form (Section 2, eq. 1):

    minimize c^T x + c0   subject to   b_lo <= A x <= b_hi,   x_lo <= x <= x_hi,

with A in CSR form (int32 row pointers, int32 column indices strictly increasing
within a row, float64 values) and IEEE +-inf for absent bounds.

"KKT-constructed" instances pick a point (x*, y*, z*) first and then choose the
bounds and the cost so that (x*, y*, z*) satisfies the optimality conditions of
Section 2, eq. 2 exactly: the sign and complementarity rules there (z* > 0 only
where x* sits at its lower bound, y* > 0 only on rows active at b_lo, y* < 0 only
on rows active at b_hi, y* >= 0 where b_hi = +inf, y* <= 0 where b_lo = -inf).
Hence c^T x* + c0 is the optimal value.

Seeds: numpy.random.default_rng([SEED_ROOT, cfg, j]) for instance j of workload cfg.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_ROOT = 260423951
INF = math.inf


@dataclasses.dataclass
class LP:
    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray  # float64 [nnz]
    c: np.ndarray  # float64 [n]
    b_lo: np.ndarray  # float64 [m]
    b_hi: np.ndarray  # float64 [m]
    x_lo: np.ndarray  # float64 [n]
    x_hi: np.ndarray  # float64 [n]
    c0: float = 0.0
    name: str = ""
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None
    z_star: Optional[np.ndarray] = None
    p_star: Optional[float] = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        a[rows, self.col_idx] = self.vals
        return a

    def astype32(self) -> "LP":
        """Return the same LP with the values rounded to float32 and back (for FP32 studies)."""
        out = dataclasses.replace(self)
        out.vals = self.vals.astype(np.float32).astype(np.float64)
        return out


def csr_from_keys(keys: np.ndarray, m: int, n: int, vals: np.ndarray) -> tuple:
    """Build CSR arrays from sorted, unique int64 keys row*n+col."""
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    return row_ptr.astype(np.int32), cols, np.ascontiguousarray(vals, dtype=np.float64)


def _matvec(row_ptr, col_idx, vals, x):
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    return np.bincount(rows, weights=vals * x[col_idx], minlength=m)


def _rmatvec(row_ptr, col_idx, vals, y, n):
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    return np.bincount(col_idx, weights=vals * y[rows], minlength=n)


def random_sparse_pattern(m: int, n: int, density: float, rng: np.random.Generator) -> np.ndarray:
    """Bernoulli(density) pattern as sorted unique keys; every empty row gets one random entry."""
    total = m * n
    k = rng.binomial(total, density)
    if total <= 4_000_000:
        keys = np.flatnonzero(rng.random(total) < density).astype(np.int64)
    else:
        # sample with replacement and drop duplicates; the count is binomial up to the few duplicates
        keys = np.unique(rng.integers(0, total, size=k, dtype=np.int64))
    counts = np.bincount(keys // n, minlength=m)
    empty = np.flatnonzero(counts == 0)
    if len(empty):
        extra = empty.astype(np.int64) * n + rng.integers(0, n, size=len(empty))
        keys = np.union1d(keys, extra)
    return keys


def kkt_constructed(
    m: int,
    n: int,
    keys: np.ndarray,
    rng: np.random.Generator,
    *,
    free_frac: float = 0.0,
    eq_frac: float = 0.5,
    two_sided_frac: float = 0.0,
    literal: bool = False,
    vals: Optional[np.ndarray] = None,
    name: str = "",
) -> LP:
    """Turn a sparsity pattern into an LP whose optimum (x*, y*, z*) is known.

    Columns: a `free_frac` share are free (x* ~ N(0,1), z* = 0); the rest have bounds
    [0, 10], half of them at the lower bound (x* = 0, z* ~ U(0,1]) and half strictly
    inside (x* ~ U(0,1], z* = 0).
    Rows: `eq_frac` equalities (b_lo = b_hi = (Ax*)_i, y* ~ N(0,1)); `two_sided_frac`
    two-sided rows split in thirds (active at b_lo with y* = |N|, active at b_hi with
    y* = -|N|, or slack with y* = 0); the rest one-sided ">=" rows (b_hi = +inf), half
    active (y* = |N|) and half slack (b_lo = (Ax*)_i - U(0,1], y* = 0).
    Cost c = A^T y* + z*.

    literal=True keeps the plain recipe (x* ~ U[0,1] everywhere, y* ~ N(0,1) on every
    row, slack inequality rows): the data has the same shape, but x* is not optimal.
    """
    if vals is None:
        vals = rng.standard_normal(len(keys))
    row_ptr, col_idx, vals = csr_from_keys(keys, m, n, vals)

    x_lo = np.zeros(n)
    x_hi = np.full(n, 10.0)
    x_star = np.empty(n)
    z_star = np.zeros(n)
    perm = rng.permutation(n)
    n_free = int(round(free_frac * n))
    free = perm[:n_free]
    bounded = perm[n_free:]
    at_lb = bounded[: len(bounded) // 2]
    inside = bounded[len(bounded) // 2 :]
    if literal:
        x_star[:] = rng.random(n)
        x_lo[free] = -INF
        x_hi[free] = INF
    else:
        x_lo[free] = -INF
        x_hi[free] = INF
        x_star[free] = rng.standard_normal(n_free)
        x_star[at_lb] = 0.0
        z_star[at_lb] = 1.0 - rng.random(len(at_lb))  # U(0,1]
        x_star[inside] = 1.0 - rng.random(len(inside))  # U(0,1]

    ax = _matvec(row_ptr, col_idx, vals, x_star)
    b_lo = np.empty(m)
    b_hi = np.empty(m)
    y_star = np.zeros(m)
    rperm = rng.permutation(m)
    n_eq = int(round(eq_frac * m))
    n_two = int(round(two_sided_frac * m))
    eq = rperm[:n_eq]
    two = rperm[n_eq : n_eq + n_two]
    one = rperm[n_eq + n_two :]
    b_lo[eq] = ax[eq]
    b_hi[eq] = ax[eq]
    y_star[eq] = rng.standard_normal(len(eq))
    if literal:
        b_lo[one] = ax[one] - rng.random(len(one))
        b_hi[one] = INF
        y_star[one] = rng.standard_normal(len(one))
        b_lo[two] = ax[two] - rng.random(len(two))
        b_hi[two] = ax[two] + rng.random(len(two))
        y_star[two] = rng.standard_normal(len(two))
    else:
        act = one[: len(one) // 2]
        slk = one[len(one) // 2 :]
        b_hi[one] = INF
        b_lo[act] = ax[act]
        y_star[act] = np.abs(rng.standard_normal(len(act)))
        b_lo[slk] = ax[slk] - (1.0 - rng.random(len(slk)))
        k3 = len(two) // 3
        t_lo, t_hi, t_sl = two[:k3], two[k3 : 2 * k3], two[2 * k3 :]
        b_lo[t_lo] = ax[t_lo]
        b_hi[t_lo] = ax[t_lo] + (1.0 - rng.random(len(t_lo)))
        y_star[t_lo] = np.abs(rng.standard_normal(len(t_lo)))
        b_hi[t_hi] = ax[t_hi]
        b_lo[t_hi] = ax[t_hi] - (1.0 - rng.random(len(t_hi)))
        y_star[t_hi] = -np.abs(rng.standard_normal(len(t_hi)))
        b_lo[t_sl] = ax[t_sl] - (1.0 - rng.random(len(t_sl)))
        b_hi[t_sl] = ax[t_sl] + (1.0 - rng.random(len(t_sl)))
    c = _rmatvec(row_ptr, col_idx, vals, y_star, n) + z_star
    lp = LP(m, n, row_ptr, col_idx, vals, c, b_lo, b_hi, x_lo, x_hi, name=name)
    if not literal:
        lp.x_star, lp.y_star, lp.z_star = x_star, y_star, z_star
        lp.p_star = float(np.dot(c, x_star))
    return lp


def cfg0(j: int = 0, *, literal: bool = False) -> LP:
    """Small LP: m=200, n=400, 2% Bernoulli pattern, values N(0,1), bounds [0,10],
    rows 50% equality / 50% one-sided inequality."""
    rng = np.random.default_rng([SEED_ROOT, 0, j])
    m, n = 200, 400
    keys = random_sparse_pattern(m, n, 0.02, rng)
    return kkt_constructed(m, n, keys, rng, eq_frac=0.5, literal=literal, name=f"cfg0[{j}]")


def _powerlaw_degrees(n: int, exponent: float, dmax: int, rng) -> np.ndarray:
    d = np.arange(1, dmax + 1, dtype=np.float64)
    p = d ** (-exponent)
    p /= p.sum()
    return rng.choice(dmax, size=n, p=p).astype(np.int64) + 1


def powerlaw_pattern(m: int, n: int, nnz: int, rng, exponent: float = 2.2, dmax: int = 5000,
                     min_row: int = 2) -> np.ndarray:
    """Keys of an m x n pattern: column degrees from a discrete power law on [1, dmax],
    distinct uniform rows per column, every row topped up to >= min_row entries, then
    uniform random extra entries until exactly `nnz` entries."""
    deg = _powerlaw_degrees(n, exponent, dmax, rng)
    cols = np.repeat(np.arange(n, dtype=np.int64), deg)
    rows = rng.integers(0, m, size=len(cols), dtype=np.int64)
    keys = np.unique(rows * n + cols)
    for _ in range(64):
        cnt = np.bincount(keys // n, minlength=m)
        short = np.flatnonzero(cnt < min_row)
        if len(short) == 0:
            break
        need = np.repeat(short.astype(np.int64), min_row - cnt[short])
        extra = need * n + rng.integers(0, n, size=len(need))
        keys = np.union1d(keys, extra)
    if len(keys) > nnz:
        raise ValueError("power-law part already exceeds the requested nnz")
    for _ in range(64):
        need = nnz - len(keys)
        if need == 0:
            break
        cand = rng.integers(0, m, size=need + need // 16 + 1024, dtype=np.int64) * n + rng.integers(
            0, n, size=need + need // 16 + 1024, dtype=np.int64
        )
        cand = np.unique(cand)
        cand = cand[~np.isin(cand, keys, assume_unique=True)]
        rng.shuffle(cand)
        keys = np.union1d(keys, cand[:need])
    if len(keys) != nnz:
        raise RuntimeError("could not reach the requested nnz")
    return keys


def cfg1(j: int = 0, *, m: int = 1_000_000, n: int = 2_000_000, nnz: int = 12_000_000,
         literal: bool = False) -> LP:
    """Large LP: m=1e6, n=2e6, nnz=1.2e7; power-law column degrees (exponent 2.2, max 5000),
    rows with >= 2 entries, values N(0,1); 20% free columns; rows 35% equality,
    35% one-sided, 30% two-sided. Smaller m, n, nnz give the same recipe at reduced size."""
    rng = np.random.default_rng([SEED_ROOT, 1, j])
    keys = powerlaw_pattern(m, n, nnz, rng, dmax=min(5000, m))
    return kkt_constructed(m, n, keys, rng, free_frac=0.2, eq_frac=0.35, two_sided_frac=0.30,
                           literal=literal, name=f"cfg1[{j}] m={m} n={n} nnz={nnz}")


def transportation(m: int, rng: np.random.Generator, name: str = "") -> LP:
    """Transportation-structured LP with m rows and n = 2m edge columns.

    floor(m/2) supply rows (sum of outgoing flow <= supply, b_lo = -inf) and the rest
    demand rows (sum of incoming flow >= demand, b_hi = +inf); each edge column has
    two +1 entries. A spanning pairing gives every row an edge, the other edges are
    random distinct pairs. A flow x ~ U[0,1] makes the instance feasible; costs are
    U[1,100] and x >= 0, so it is bounded. The optimum is not known in closed form.
    """
    S = m // 2
    D = m - S
    n = 2 * m
    base = max(S, D)
    s_idx = np.arange(base) % S
    d_idx = np.arange(base) % D
    pairs = s_idx.astype(np.int64) * D + d_idx
    pairs = np.unique(pairs)
    while len(pairs) < n:
        extra = rng.integers(0, S, size=n) .astype(np.int64) * D + rng.integers(0, D, size=n)
        extra = np.setdiff1d(np.unique(extra), pairs)
        rng.shuffle(extra)
        pairs = np.union1d(pairs, extra[: n - len(pairs)])
    pairs = rng.permutation(pairs)  # column order is random
    sup = pairs // D
    dem = pairs - sup * D
    col = np.arange(n, dtype=np.int64)
    keys = np.concatenate([sup * n + col, (S + dem) * n + col])
    keys.sort()
    row_ptr, col_idx, vals = csr_from_keys(keys, m, n, np.ones(len(keys)))
    flow = rng.random(n)
    ax = _matvec(row_ptr, col_idx, vals, flow)
    b_lo = np.empty(m)
    b_hi = np.empty(m)
    b_lo[:S] = -INF
    b_hi[:S] = ax[:S] + (1.0 - rng.random(S))
    b_lo[S:] = ax[S:]
    b_hi[S:] = INF
    c = rng.uniform(1.0, 100.0, size=n)
    return LP(m, n, row_ptr, col_idx, vals, c, b_lo, b_hi, np.zeros(n), np.full(n, INF), name=name)


def cfg3_sizes(count: int = 4096) -> np.ndarray:
    """Row counts m_j = round(exp(U[ln 50, ln 5000])) of the batched workload."""
    out = np.empty(count, dtype=np.int64)
    for j in range(count):
        rng = np.random.default_rng([SEED_ROOT, 3, j])
        out[j] = int(round(math.exp(rng.uniform(math.log(50), math.log(5000)))))
    return out


def cfg3_lp(j: int, *, m_max: Optional[int] = None) -> LP:
    """LP j of the batched workload: n = 2m; even j random-sparse (density U[0.5%, 5%],
    KKT-constructed as in the small LP), odd j transportation-structured."""
    rng = np.random.default_rng([SEED_ROOT, 3, j])
    m = int(round(math.exp(rng.uniform(math.log(50), math.log(5000)))))
    if m_max is not None:
        m = min(m, m_max)
    n = 2 * m
    if j % 2 == 0:
        rho = rng.uniform(0.005, 0.05)
        keys = random_sparse_pattern(m, n, rho, rng)
        return kkt_constructed(m, n, keys, rng, eq_frac=0.5, name=f"cfg3[{j}] random m={m}")
    return transportation(m, rng, name=f"cfg3[{j}] transport m={m}")


def cfg4_lp(j: int, *, m_lo: int = 100, m_hi: int = 200_000) -> LP:
    """LP j of the serving pool: m log-uniform on [m_lo, m_hi], n = 1.5m, row lengths
    U{3..20} with distinct random columns, KKT-constructed as in the small LP."""
    rng = np.random.default_rng([SEED_ROOT, 4, j])
    m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
    n = int(round(1.5 * m))
    k = rng.integers(3, 21, size=m)
    rows = np.repeat(np.arange(m, dtype=np.int64), k)
    cols = rng.integers(0, n, size=len(rows), dtype=np.int64)
    keys = np.unique(rows * n + cols)
    return kkt_constructed(m, n, keys, rng, eq_frac=0.5, name=f"cfg4[{j}] m={m}")


def tiny_lp(spec: dict) -> LP:
    """Build an LP from a small dense JSON-style spec (used by the golden fixtures).

    spec keys: A (list of rows), c, b_lo, b_hi, x_lo, x_hi; "inf"/"-inf" strings allowed.
    """
    def vec(v):
        return np.array([float(t) for t in v], dtype=np.float64)

    a = np.array([[float(t) for t in row] for row in spec["A"]], dtype=np.float64).reshape(
        len(spec["A"]), len(spec["c"])
    )
    m, n = a.shape
    rows, cols = np.nonzero(a)
    keys = rows.astype(np.int64) * n + cols
    row_ptr, col_idx, vals = csr_from_keys(keys, m, n, a[rows, cols])
    return LP(m, n, row_ptr, col_idx, vals, vec(spec["c"]), vec(spec["b_lo"]), vec(spec["b_hi"]),
              vec(spec["x_lo"]), vec(spec["x_hi"]), c0=float(spec.get("c0", 0.0)),
              name=spec.get("name", ""))


def with_planted_reductions(
    base: LP,
    rng: np.random.Generator,
    *,
    fixed_cols: int = 0,
    empty_cols: int = 0,
    lock_cols: int = 0,
    singleton_rows: int = 0,
    redundant_rows: int = 0,
    free_singletons: int = 0,
    empty_rows: int = 0,
    name: str = "",
) -> LP:
    """Append structure that a presolver can remove to a KKT-constructed LP, keeping a known
    optimum (the paper's Section 3 explorers: Table 1). All new rows and columns are shuffled
    in with the old ones.

    - fixed columns: x_lo = x_hi = v ~ U[0,10], 1-4 entries in existing rows whose bounds are
      shifted by a*v (so Ax* moves with them); z* = c - a^T y* with c ~ N(0,1);
    - empty columns: no entries, bounds [0,10], c ~ U(0,1], x* = 0, z* = c;
    - lock columns: bounds [0,10], x* = 0, c ~ U(0,1], a single entry a > 0 in a new slack
      "<=" row (y* = 0) that also holds 2-4 bounded old columns, so no row stops the column
      from decreasing;
    - singleton rows: a x_j >= a x*_j - U(0,1] on a bounded column (slack, y* = 0);
    - redundant rows: 2-5 bounded columns, b_lo below the minimum activity over the bounds
      by U(0,1], b_hi = +inf (y* = 0);
    - free column singletons: a free column (x* ~ N(0,1)) in a new equality row with 2-4 old
      columns; y* ~ N(0,1) on the row, the column's cost is a y* (z* = 0) and the old
      columns' costs move by a_j y* so their z* is unchanged;
    - empty rows: b_lo = -U(0,1], b_hi = U(0,1] (y* = 0).
    """
    if base.x_star is None:
        raise ValueError("base LP must be KKT-constructed")
    m0, n0 = base.m, base.n
    rows0 = np.repeat(np.arange(m0), np.diff(base.row_ptr)).tolist()
    R, Cc, V = list(rows0), base.col_idx.astype(np.int64).tolist(), base.vals.tolist()
    c = base.c.tolist()
    b_lo, b_hi = base.b_lo.tolist(), base.b_hi.tolist()
    x_lo, x_hi = base.x_lo.tolist(), base.x_hi.tolist()
    xs, ys, zs = base.x_star.tolist(), base.y_star.tolist(), base.z_star.tolist()
    bounded = np.flatnonzero(np.isfinite(base.x_lo) & np.isfinite(base.x_hi))
    m, n = m0, n0

    def new_col(lo, hi, cost, x, z):
        nonlocal n
        x_lo.append(lo), x_hi.append(hi), c.append(cost), xs.append(x), zs.append(z)
        n += 1
        return n - 1

    def new_row(lo, hi, y):
        nonlocal m
        b_lo.append(lo), b_hi.append(hi), ys.append(y)
        m += 1
        return m - 1

    for _ in range(fixed_cols):
        v = 10.0 * rng.random()
        cost = rng.standard_normal()
        k = new_col(v, v, cost, v, 0.0)
        rr = rng.choice(m0, size=min(m0, int(rng.integers(1, 5))), replace=False)
        zk = cost
        for i in rr:
            a = rng.standard_normal()
            R.append(int(i)), Cc.append(k), V.append(a)
            if math.isfinite(b_lo[i]):
                b_lo[i] += a * v
            if math.isfinite(b_hi[i]):
                b_hi[i] += a * v
            zk -= a * ys[i]
        zs[k] = zk
    for _ in range(empty_cols):
        cost = 1.0 - rng.random()
        new_col(0.0, 10.0, cost, 0.0, cost)
    for _ in range(lock_cols):
        cost = 1.0 - rng.random()
        k = new_col(0.0, 10.0, cost, 0.0, cost)
        js = rng.choice(bounded, size=min(len(bounded), int(rng.integers(2, 5))), replace=False)
        a_k = 0.5 + rng.random()
        act = 0.0
        entries = [(k, a_k)]
        for j in js:
            a = rng.standard_normal()
            entries.append((int(j), a))
            act += a * xs[j]
        i = new_row(-INF, act + (1.0 - rng.random()), 0.0)
        for j, a in entries:
            R.append(i), Cc.append(j), V.append(a)
    for _ in range(singleton_rows):
        j = int(rng.choice(bounded))
        a = rng.standard_normal()
        lo = a * xs[j] - (1.0 - rng.random())
        i = new_row(lo, INF, 0.0)
        R.append(i), Cc.append(j), V.append(a)
    for _ in range(redundant_rows):
        js = rng.choice(bounded, size=min(len(bounded), int(rng.integers(2, 6))), replace=False)
        amin = 0.0
        entries = []
        for j in js:
            a = rng.standard_normal()
            entries.append((int(j), a))
            amin += min(a * x_lo[j], a * x_hi[j])
        i = new_row(amin - (1.0 - rng.random()), INF, 0.0)
        for j, a in entries:
            R.append(i), Cc.append(j), V.append(a)
    for _ in range(free_singletons):
        xk = rng.standard_normal()
        a_k = np.sign(rng.standard_normal()) * (0.5 + rng.random())
        yi = rng.standard_normal()
        k = new_col(-INF, INF, a_k * yi, xk, 0.0)
        js = rng.choice(n0, size=min(n0, int(rng.integers(2, 5))), replace=False)
        b = a_k * xk
        entries = [(k, a_k)]
        for j in js:
            a = rng.standard_normal()
            entries.append((int(j), a))
            b += a * xs[j]
            c[j] += a * yi
        i = new_row(b, b, yi)
        for j, a in entries:
            R.append(i), Cc.append(j), V.append(a)
    for _ in range(empty_rows):
        new_row(-(1.0 - rng.random()), 1.0 - rng.random(), 0.0)

    # shuffle rows and columns
    rp = rng.permutation(m)
    cp = rng.permutation(n)
    R = rp[np.asarray(R, dtype=np.int64)]
    Cn = cp[np.asarray(Cc, dtype=np.int64)]
    V = np.asarray(V)
    keys = R * n + Cn
    order = np.argsort(keys, kind="stable")
    keys, V = keys[order], V[order]
    if len(keys) and np.any(np.diff(keys) == 0):
        raise AssertionError("duplicate entry in planted LP")
    row_ptr, col_idx, vals = csr_from_keys(keys, m, n, V)

    def perm(vec, p, size):
        out = np.empty(size)
        out[p] = np.asarray(vec, dtype=np.float64)
        return out

    lp = LP(m, n, row_ptr, col_idx, vals, perm(c, cp, n), perm(b_lo, rp, m), perm(b_hi, rp, m),
            perm(x_lo, cp, n), perm(x_hi, cp, n), c0=base.c0, name=name or base.name + "+planted")
    lp.x_star, lp.z_star, lp.y_star = perm(xs, cp, n), perm(zs, cp, n), perm(ys, rp, m)
    lp.p_star = float(np.dot(lp.c, lp.x_star) + lp.c0)
    return lp


def presolve_lp(j: int = 0, *, m: int = 2000, n: int = 4000, density: float = 0.002, share: float = 0.1) -> LP:
    """A KKT-constructed LP (small-LP recipe: 50% equality rows, bounds [0,10], 10% free
    columns) with every planted reduction type at `share` of m (rows) or n (columns)."""
    rng = np.random.default_rng([SEED_ROOT, 5, j])
    base = kkt_constructed(m, n, random_sparse_pattern(m, n, density, rng), rng, free_frac=0.1, eq_frac=0.5,
                           name=f"presolve[{j}]")
    kr, kc = max(1, int(share * m)), max(1, int(share * n))
    return with_planted_reductions(base, rng, fixed_cols=kc, empty_cols=kc // 4, lock_cols=kc // 2,
                                   singleton_rows=kr, redundant_rows=kr, free_singletons=kr // 2,
                                   empty_rows=kr // 4)
