"""Row-tile shapes (tile_nnz 1024 / 2048 / 4096) against the oracle and each other: iterates
of the first 200 iterations within 1e-12 for every shape on the row-tile layout and in the
batched paths, rows longer than a tile (reduced by a tree) included; the shape the tuned table
picks gives the same result, bit for bit, as that shape set explicitly."""
import numpy as np
import pytest

import oracle
import paper_2604_23951_amd as lpg
import synth
from test_gpu_parity import ITER_TOL, _close

pytestmark = pytest.mark.gpu
SHAPES = (1024, 2048, 4096)


def _long_row_lp():
    """The large-LP recipe at reduced size with a few dense rows (1500 and 3000 entries): long
    for the 1024 tile, one row is long for 2048, none for 4096."""
    rng = np.random.default_rng(17)
    base = synth.cfg1(0, m=1500, n=4000, nnz=16000)
    rows = [list(base.col_idx[base.row_ptr[i]:base.row_ptr[i + 1]]) for i in range(base.m)]
    for i, length in ((3, 1500), (700, 3000)):
        rows[i] = sorted(rng.choice(base.n, size=length, replace=False).tolist())
    keys = np.concatenate([np.asarray(r, np.int64) + i * base.n for i, r in enumerate(rows)])
    return synth.kkt_constructed(base.m, base.n, np.unique(keys), rng, eq_frac=0.5, name="long rows")


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("name", ["cfg0", "long_rows"])
def test_iterates_every_shape(oracle_lib, name, shape):
    lp = synth.cfg0(0) if name == "cfg0" else _long_row_lp()
    ks = [1, 2, 64, 65, 128, 200]
    ref = oracle.solve(lp, eps_rel=0.0, max_iters=200, snap_k=ks)
    print(f"{name} tile {shape}", flush=True)
    with lpg.Solver(lp, eps_rel=0.0, max_iters=1, spmv_layout=lpg.LP_LAYOUT_TILES, tile_nnz=shape) as s:
        assert s.layout()["tile_nnz"] == shape
        for i, k in enumerate(ks):
            s.update(eps_rel=0.0, max_iters=k)
            s.solve()
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[i], lp.n, lp.m)):
                assert _close(a, b) <= ITER_TOL, (name, shape, k)
    # the batched paths (persistent, and block-diagonal for this LP's size) with the same shape
    for split in (10**9, 0):
        with lpg.Solver(lp, spmv_layout=lpg.LP_LAYOUT_TILES, tile_nnz=shape) as s:
            lpg.solve_batch([s], eps_rel=0.0, max_iters=200, batch_split_nnz=split)
            for a, b in zip(s.iterates(), oracle.split_snap(ref.snaps[-1], lp.n, lp.m)):
                assert _close(a, b) <= ITER_TOL, (name, shape, "batch", split)


def test_tuned_shape_equals_fixed_shape():
    """tile_nnz = 0 takes the table's shape for the LP's class; the same shape given
    explicitly solves every LP bit for bit alike, in a batch and alone."""
    lps = [synth.cfg3_lp(j, m_max=600) for j in range(6)] + [synth.cfg4_lp(2, m_hi=3000)]
    for prec in (lpg.LP_PREC_FP64, lpg.LP_PREC_FP32_REFINED):
        tuned = [lpg.Solver(lp, spmv_layout=1, precision=prec) for lp in lps]
        shapes = [s.layout()["tile_nnz"] for s in tuned]
        fixed = [lpg.Solver(lp, spmv_layout=1, precision=prec, tile_nnz=sh) for lp, sh in zip(lps, shapes)]
        try:
            a = lpg.solve_batch(tuned, eps_rel=1e-5, max_iters=100000)
            b = lpg.solve_batch(fixed, eps_rel=1e-5, max_iters=100000)
            single = [s.solve() for s in fixed[:2]]
        finally:
            for s in tuned + fixed:
                s.close()
        for u, v in zip(a, b):
            assert u.info.iterations == v.info.iterations
            assert np.array_equal(u.x, v.x) and np.array_equal(u.y, v.y)
        for u, v in zip(single, b[:2]):
            assert u.status == v.status
