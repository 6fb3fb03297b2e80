"""Seeded synthetic LP generators shared by the tests, the oracle checks and the bench.

This package only builds problem data (a CSR matrix, costs and bounds) and, for the
KKT-constructed instances, the primal-dual point that is optimal by construction.
It contains none of the solver's arithmetic.
"""
from .lpgen import (  # noqa: F401
    LP,
    SEED_ROOT,
    csr_from_keys,
    kkt_constructed,
    random_sparse_pattern,
    cfg0,
    cfg1,
    cfg3_lp,
    cfg3_sizes,
    cfg4_lp,
    transportation,
    tiny_lp,
    with_planted_reductions,
    presolve_lp,
)
