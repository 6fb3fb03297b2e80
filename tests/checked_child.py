"""Solves run by tests/test_gpu_checked_build.py in a process of their own: the library that
process loads is chosen by LPGPU_CHECKED when the package is imported. Writes the returned
points and the check word to the .npz file named on the command line."""
import sys

import numpy as np

import paper_2604_23951_amd as lpg
import synth


def solves():
    """(name, x) of every solve: lp_solve in both layouts and forms, a certificate, polishing,
    a paused and resumed run, both batched launches and a server."""
    rng = np.random.default_rng(7)
    small, mid = synth.cfg0(0), synth.cfg1(0, m=3000, n=6000, nnz=36000)
    out = []
    for name, lp in (("cfg0", small), ("mid", mid)):
        for layout in (0, 1):
            for method, prec in ((0, 0), (1, 1)):
                with lpg.Solver(lp, eps_rel=1e-6, max_iters=200000, spmv_layout=layout, method=method,
                                precision=prec) as s:
                    out.append((f"{name}_l{layout}_m{method}_p{prec}", s.solve().x))
    with lpg.Solver(mid, eps_rel=1e-4, max_iters=200000, method=1) as s:
        s.solve()
        out.append(("polish", s.polish(1e-8).x))
    with lpg.Solver(small, eps_rel=1e-7, max_iters=200000, small_lp_lds=0) as s:
        s.solve_until(640)
        out.append(("resumed", s.resume().x))
    lps = [synth.cfg0(1), synth.transportation(80, rng), synth.cfg4_lp(4, m_hi=600), synth.cfg3_lp(9, m_max=300)]
    for split in (10**9, 0):
        solvers = [lpg.Solver(lp, spmv_layout=1, precision=1, method=1) for lp in lps]
        try:
            sols = lpg.solve_batch(solvers, eps_rel=1e-5, max_iters=200000, method=1, precision=1,
                                   batch_split_nnz=split)
        finally:
            for s in solvers:
                s.close()
        out += [(f"batch{split}_{i}", r.x) for i, r in enumerate(sols)]
    tmpls = [lpg.Solver(lp, deferred=1, spmv_layout=1, method=1) for lp in lps[:2]]
    try:
        with lpg.Server(1 << 33, 4, eps_rel=1e-5, max_iters=200000, method=1) as srv:
            tickets = [srv.submit(t) for t in tmpls]
            srv.wait(120.0)
            out += [(f"served{i}", srv.result(t).x) for i, t in enumerate(tickets)]
    finally:
        for t in tmpls:
            t.close()
    return out


if __name__ == "__main__":
    res = solves()
    word, checked = lpg.lp_check_word(0)
    np.savez(sys.argv[1], word=word, checked=int(checked), **dict(res))
    print(f"{len(res)} solves, checked build {checked}, check word {word}", flush=True)
