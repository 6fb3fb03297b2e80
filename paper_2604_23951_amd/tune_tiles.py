"""Row-tile shape tuner of the batched and row-tile products (run on the GPU).

For each LP class (precision x mean row length of A x size), a set of synthetic LPs of that
class (KKT-constructed, random sparse pattern with the class's row length, n = 2m) is solved
with lp_solve_batch for a fixed number of iterations with every row-tile shape (1024, 2048
and 4096 nonzeros per tile), LPs at or below 20000 nonzeros in the persistent launch and the
larger ones in the block-diagonal launches, as in a production batch. The two smallest size
classes hold fewer LPs than the device has compute units, so their time is the iteration
latency of one workgroup, which sets a batch's time when one small LP needs many iterations. The fastest shape of
each class becomes a rule of csrc/lp_tile_table.h, which the library reads at lp_create
when tile_nnz is 0:

    python -m paper_2604_23951_amd.tune_tiles --write      (then rebuild the library)

Shapes only change which rows are long (summed by a tree) and how rows are grouped into
tiles, so every result stays deterministic for a given shape; the tuner measures speed only.
"""
from __future__ import annotations

import argparse
import datetime
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "lp_tile_table.h")
SHAPES = (1024, 2048, 4096)
ROW_LEN_EDGES = (6.0, 12.0, 24.0, math.inf)   # mean nonzeros per row of A
SIZE_CLASSES = (                              # (max nnz, LPs, nnz range, iterations)
    (1024, 24, (200, 1024), 2000),            # fewer LPs than CUs: the time is one LP's latency
    (2048, 24, (1025, 2048), 2000),
    (20000, 48, (2049, 20000), 640),
    (500000, 6, (50000, 500000), 256),
    (2**62, 1, (1000000, 1500000), 128),
)


def class_lps(row_len_lo, row_len_hi, nnz_lo, nnz_hi, count, seed):
    import numpy as np

    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth

    rng = np.random.default_rng([260423951, 99, seed])
    out = []
    for _ in range(count):
        r = rng.uniform(row_len_lo, min(row_len_hi, 2 * row_len_lo + 8))
        nnz = math.exp(rng.uniform(math.log(nnz_lo), math.log(nnz_hi)))
        m = max(20, int(nnz / r))
        n = 2 * m
        keys = synth.random_sparse_pattern(m, n, min(0.5, r / n), rng)
        out.append(synth.kkt_constructed(m, n, keys, rng, eq_frac=0.5, name=f"tune m={m} r={r:.1f}"))
    return out


def time_shape(lps, shape, fp32, iters):
    import paper_2604_23951_amd as lpg

    prec = lpg.LP_PREC_FP32_REFINED if fp32 else lpg.LP_PREC_FP64
    solvers = [lpg.Solver(lp, spmv_layout=lpg.LP_LAYOUT_TILES, precision=prec, tile_nnz=shape) for lp in lps]
    try:
        lpg.solve_batch(solvers, eps_rel=0.0, max_iters=64)  # warm-up: code, caches
        best = math.inf
        for _ in range(2):
            t = time.perf_counter()
            lpg.solve_batch(solvers, eps_rel=0.0, max_iters=iters)
            best = min(best, time.perf_counter() - t)
        return best
    finally:
        for s in solvers:
            s.close()


def sweep(quick=False):
    rules = []
    seed = 0
    for fp32 in (0, 1):
        lo = 2.0
        for hi in ROW_LEN_EDGES:
            for max_nnz, count, (nlo, nhi), iters in SIZE_CLASSES:
                seed += 1
                if quick:
                    count = max(1, count // 8)
                lps = class_lps(lo, hi if math.isfinite(hi) else 64.0, nlo, nhi, count, seed)
                times = {s: time_shape(lps, s, fp32, iters) for s in SHAPES}
                best = min(times, key=times.get)
                print(f"[tune] fp32={fp32} row_len<= {hi} nnz<= {max_nnz}: " +
                      ", ".join(f"{s}: {times[s] * 1e3:.1f} ms" for s in SHAPES) + f" -> {best}", flush=True)
                rules.append((fp32, hi, max_nnz, SHAPES.index(best), times))
            lo = hi
    return rules


def write_table(rules, source, out=TABLE):
    text = open(TABLE).read()
    head, rest = text.split("// TUNED-TABLE-BEGIN", 1)
    _, tail = rest.split("// TUNED-TABLE-END", 1)
    lines = ["// TUNED-TABLE-BEGIN (generated; a class the sweep did not measure takes shape 1)",
             "constexpr TileRule kTileRules[] = {"]
    for fp32, hi, max_nnz, shape, times in rules:
        rl = "1e300" if not math.isfinite(hi) else repr(float(hi))
        mn = "INT64_MAX" if max_nnz >= 2**62 else str(max_nnz)
        ms = ", ".join(f"{s}: {times[s] * 1e3:.1f} ms" for s in SHAPES)
        lines.append(f"    {{{fp32}, {rl}, {mn}, {shape}}},  // {ms}")
    lines.append("};")
    lines.append(f'constexpr const char* kTileTableSource = "{source}";')
    lines.append("// TUNED-TABLE-END")
    with open(out, "w") as f:
        f.write(head + "\n".join(lines) + tail)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="rewrite csrc/lp_tile_table.h with the measured rules")
    ap.add_argument("--quick", action="store_true", help="an eighth of the LPs per class")
    ap.add_argument("--out", default=TABLE, help="where --write puts the table (default: the library's header)")
    args = ap.parse_args(argv)
    import torch

    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "unknown device"
    rules = sweep(args.quick)
    if args.write:
        src = f"tune_tiles.py on {dev}, {datetime.date.today().isoformat()}"
        write_table(rules, src, args.out)
        print(f"[tune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
