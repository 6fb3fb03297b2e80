"""Benchmark of the restarted-PDHG hot path on one MI355X.

Workload: the single large LP (m = 1e6 rows, n = 2e6 columns, nnz = 1.2e7, power-law
column degrees with exponent 2.2 and maximum 5000, every row with >= 2 entries, values
N(0,1), 20% free columns, 35% equality / 35% one-sided / 30% two-sided rows,
KKT-constructed so the optimum is known), solved in FP64 with the power-of-two
Ruiz + Pock-Chambolle scaling.

A step is one evaluation period of the solver: eval_every = 64 PDHG iterations (each a
fused A^T y + primal update and a fused A x + dual update), the FP64 KKT evaluation of
the current and the average iterate, and the restart / primal-weight / termination
decision. `value` is PDHG iterations per second with the problem resident in HBM.

The per-kernel durations of the primal and the dual kernel are measured with HIP events
on the solver stream during the timed region (one sampled iteration per step).

The default run adds the rest of the metric as extra keys of the same JSON line, each leg
bounded in time: `small_lp` (the latency-bound 200 x 400 LP, microseconds per iteration),
`batch` (a 256-LP sample of the 4096-LP batch to E_rel 1e-4: LPs/s against the per-LP FP64
loop on the same GPU) and `serving` (Poisson arrivals at 2000/s for 20 s: LPs/s, and p50/p99
latency at half that throughput), each with its own CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Random 8-byte gathers in the panel-sweep pattern of the product kernels (12-byte entries,
# 8-32 column panels, 4 waves per CU) peaked at 1.66e11 gathers/s in a micro-benchmark on
# MI355X: one L1-to-L2 request per gathered entry, bounded by the requests a CU keeps in
# flight. A product of nnz entries therefore needs at least nnz / 1.66e11 s.
GATHER_CEILING_PER_S = 1.66e11
# The same micro-benchmark with the gathered vector resident in L2 (1 MiB footprint): 2.2e11
# gathers/s, the bound of products whose vectors fit the cache (the served LPs' rounds).
L2_GATHER_RATE_PER_S = 2.2e11
METRIC = "PDHG iters/s & HBM GB/s vs roofline; batched LPs/s to 1e-4 KKT, p50/p99"


def algorithmic_bytes(m: int, n: int, nnz: int, sv: int = 8, halpern: bool = False):
    """Bytes the method must move per launch (int32 indices, sv-byte values).

    primal kernel: A^T values + indices, A^T row pointers, one gather of y, read x, c,
                   x_lo, x_hi, x_avg (Halpern form: the anchor x0) and write x, x_avg (T(z)).
    dual kernel:   A values + indices, A row pointers, one gather of x, read y, b_lo, b_hi,
                   y_avg, A x and write y, y_avg, A x; the Halpern form reads the anchor y0
                   and its A x0 instead of y_avg and also writes A T(z).
    """
    primal = (sv + 4) * nnz + 4 * (n + 1) + sv * (7 * n + m)
    dual = (sv + 4) * nnz + 4 * (m + 1) + sv * (n + (10 if halpern else 8) * m)
    return primal, dual


METHODS = {"averaged": 0, "halpern": 1}


def method_of(args, default: str) -> int:
    """The PDHG form a workload runs: --method, else the workload's default."""
    return METHODS[args.method or default]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def environment() -> dict:
    """Where a line was measured: GPU, ROCm (HIP) version, host CPU and thread count, the
    generators' seed root."""
    env = {"cpu": cpu_model(), "nproc": os.cpu_count()}
    try:
        import torch

        env["gpu"] = torch.cuda.get_device_name(0) if torch.cuda.is_available() else None
        env["hip"] = getattr(torch.version, "hip", None)
    except Exception:  # the line is still written without the device description
        env["gpu"] = env["hip"] = None
    try:
        import synth

        env["seed_root"] = synth.SEED_ROOT
    except Exception:
        env["seed_root"] = None
    return env


def run_cpu_baseline(lp, iters: int) -> dict:
    """The oracle as it stands, single-threaded on the host, on a bounded sample."""
    import oracle

    r = oracle.solve(lp, eps_rel=0.0, max_iters=iters, pow_iters=10)
    rate = iters / r.iter_s
    return {"value": rate, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"same LP, first {iters} PDHG iterations incl. {iters // 64} KKT evaluations; "
                      f"setup (transpose, scaling, 10-step power iteration) not timed; "
                      f"{r.iter_s:.1f} s of CPU time on '{cpu_model()}' (nproc={os.cpu_count()})"}


def run_cpu_baseline_batch(lps, method: int, budget_s: float = 20.0, eval_every: int = 64) -> dict:
    """The oracle as it stands, single-threaded, solving LPs of the batch one after another
    to E_rel 1e-4 (same method) in index order (sizes are random in that order) until
    about `budget_s` seconds of solve time have been spent."""
    import oracle

    spent = 0.0
    done = 0
    for lp in lps:
        r = oracle.solve(lp, eps_rel=1e-4, max_iters=400000, method=method, eval_every=eval_every)
        spent += r.setup_s + r.iter_s
        done += 1
        if spent >= budget_s:
            break
    return {"value": done / spent, "unit": "LPs/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {done} LPs of the batch in index order, each to E_rel 1e-4 with the same "
                      f"method, setup included, {spent:.1f} s of CPU time on '{cpu_model()}' (nproc={os.cpu_count()})"}


def leg_batch(count: int, loop_count: int, max_iters: int, method: int, cpu_budget_s: float = 0.0,
              eval_every: int = 64) -> dict:
    """Batched workload: `count` LPs of the 4096-LP batch (every (4096 / count)-th; m
    log-uniform in [50, 5000], n = 2m, random-sparse with density U[0.5%, 5%] for even j,
    transportation for odd j), solved to E_rel 1e-4 together (one persistent launch for the
    small LPs beside block-diagonal launches for the large ones) in the FP32 storage form,
    against the plain per-LP FP64 lp_solve loop on the same GPU (a sub-sample) and, with a
    budget, the oracle on the host."""
    import numpy as np

    import paper_2604_23951_amd as lpg
    import synth

    total = 4096
    stride = max(1, total // count)
    ids = list(range(0, total, stride))[:count]
    t0 = time.time()
    lps = [synth.cfg3_lp(j) for j in ids]
    gen_s = time.time() - t0
    nnz = np.array([lp.nnz for lp in lps])
    print(f"[bench] generated {len(lps)} LPs (nnz total {nnz.sum():.3e}, max {nnz.max()}) in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    t1 = time.time()
    solvers = [lpg.Solver(lp, spmv_layout=1, precision=lpg.LP_PREC_FP32_REFINED, method=method) for lp in lps]
    create_s = time.time() - t1
    print(f"[bench] created {len(solvers)} handles in {create_s:.1f}s", file=sys.stderr, flush=True)
    lpg.solve_batch(solvers[-8:], eps_rel=1e-4, max_iters=64, method=method, eval_every=eval_every)  # warm-up launch
    t2 = time.perf_counter()
    sols = lpg.solve_batch(solvers, eps_rel=1e-4, max_iters=max_iters, method=method, eval_every=eval_every)
    dt = time.perf_counter() - t2
    ok = sum(s.status == "optimal" for s in sols)
    iters = np.array([s.info.iterations for s in sols])
    # per-LP completion instants on the device clock, relative to the first LP to finish
    done = np.array([s.info.done_clock for s in sols], dtype=np.float64)
    hz = sols[0].info.clock_hz or 1e8
    rel = (done - done.min()) / hz
    hist, _ = np.histogram(rel / max(rel.max(), 1e-12), bins=10, range=(0.0, 1.0))
    print(f"[bench] batch: {len(sols)} LPs in {dt:.2f}s ({len(sols) / dt:.1f} LPs/s), {ok} optimal, "
          f"iterations median {int(np.median(iters))} max {iters.max()}; completions (s after the first) "
          f"p50 {np.percentile(rel, 50):.3f} p90 {np.percentile(rel, 90):.3f} p99 {np.percentile(rel, 99):.3f} "
          f"max {rel.max():.3f}", file=sys.stderr, flush=True)
    for s in solvers:
        s.close()
    # plain per-LP FP64 loop on a sub-sample
    sub = lps[:: max(1, len(lps) // max(loop_count, 1))][:loop_count]
    loop_t = 0.0
    loop_ok = 0
    for lp in sub:
        with lpg.Solver(lp, eps_rel=1e-4, max_iters=max_iters, method=method, spmv_layout=lpg.LP_LAYOUT_TUNED,
                        eval_every=eval_every) as s1:
            t3 = time.perf_counter()
            r = s1.solve()
            loop_t += time.perf_counter() - t3
            loop_ok += r.status == "optimal"
    loop_rate = loop_ok / loop_t if loop_t > 0 else float("nan")  # LPs that reached 1e-4
    print(f"[bench] per-LP FP64 loop: {len(sub)} LPs in {loop_t:.2f}s ({loop_rate:.2f} LPs/s)",
          file=sys.stderr, flush=True)
    out = {
        # LPs that reached E_rel 1e-4 per second of the batched solve
        "lps_per_s": ok / dt, "seconds": dt,
        "workload": ("batched LPs to E_rel 1e-4: the 4096-LP batch " if len(lps) == total else
                     f"batched LPs to E_rel 1e-4: every {stride}th LP of the 4096-LP batch ") +
                    "(m log-uniform [50,5000], n=2m, random-sparse density U[0.5%,5%] / transportation "
                    "50/50), FP32 storage form with FP64 evaluation and refinement",
        "method": {v: k for k, v in METHODS.items()}[method],
        "lps": len(sols), "nnz_total": int(nnz.sum()), "optimal": ok,
        "iterations_median": int(np.median(iters)), "iterations_p99": float(np.percentile(iters, 99)),
        "iterations_max": int(iters.max()),
        "completion_s_after_first": {"p50": float(np.percentile(rel, 50)), "p90": float(np.percentile(rel, 90)),
                                     "p99": float(np.percentile(rel, 99)), "max": float(rel.max()),
                                     "histogram_tenths_of_span": hist.tolist()},
        "per_lp_fp64_loop": {"lps": len(sub), "seconds": loop_t, "lps_per_s": loop_rate, "optimal": loop_ok,
                             "method": "same as the batch", "layout": "tuned per LP"},
        "speedup_vs_per_lp_loop": (ok / dt) / loop_rate,
        "create_s": create_s,
        "cpu_baseline": None,
    }
    if cpu_budget_s > 0:
        print("[bench] cpu baseline: oracle on the first LPs of the batch", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline_batch(lps, method, cpu_budget_s, eval_every)
    out["eval_every"] = eval_every
    return out


def run_batch(args) -> int:
    """The batched workload alone (--workload batch): one JSON line with LPs/s as `value`."""
    meth = method_of(args, "halpern")
    leg = leg_batch(args.batch_count, args.loop_count, args.batch_max_iters, meth,
                    0.0 if args.no_cpu_baseline else 20.0, args.batch_eval_every)
    result = {
        "metric": METRIC, "value": leg["lps_per_s"], "unit": "LPs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": leg["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": leg["workload"], "method": leg["method"], "lps": leg["lps"],
                   "nnz_total": leg["nnz_total"], "optimal": leg["optimal"],
                   "iterations_median": leg["iterations_median"], "iterations_max": leg["iterations_max"]},
        "completion_s_after_first": leg["completion_s_after_first"],
        "per_lp_fp64_loop": leg["per_lp_fp64_loop"], "speedup_vs_per_lp_loop": leg["speedup_vs_per_lp_loop"],
        "create_s": leg["create_s"], "cpu_baseline": leg["cpu_baseline"],
    }
    result["environment"] = environment()
    print(json.dumps(result), flush=True)
    return 0


def run_blockdiag(args) -> int:
    """Block-diagonal launches of the batch form over a fixed set: the batch's LPs above
    20000 nonzeros among the even indices (random-sparse recipe), FP32 storage, Halpern form,
    128 iterations with every LP in the block-diagonal group, so every primal / dual launch
    covers the same tiles (the set for per-launch counters of those kernels)."""
    import paper_2604_23951_amd as lpg
    import synth

    lps = [lp for lp in (synth.cfg3_lp(j) for j in range(0, 4096, 2)) if lp.nnz > 20000]
    nnz = sum(lp.nnz for lp in lps)
    m = sum(lp.m for lp in lps)
    n = sum(lp.n for lp in lps)
    # per launch: FP32 values + int32 indices, row pointers, one gather of the FP32 vector,
    # 4 bytes per epilogue float (7 per column for the primal, 8 per row for the dual)
    prim = 8 * nnz + 4 * (n + len(lps)) + 4 * m + 4 * 7 * n
    dual = 8 * nnz + 4 * (m + len(lps)) + 4 * n + 4 * 8 * m
    solvers = [lpg.Solver(lp, spmv_layout=1, precision=lpg.LP_PREC_FP32_REFINED, method=lpg.LP_METHOD_HALPERN)
               for lp in lps]
    iters = 128
    times = []
    for _ in range(2):
        t = time.perf_counter()
        lpg.solve_batch(solvers, eps_rel=0.0, max_iters=iters, method=lpg.LP_METHOD_HALPERN, batch_split_nnz=0)
        times.append(time.perf_counter() - t)
    for s in solvers:
        s.close()
    dt = min(times)
    print(f"[bench] block-diagonal set: {len(lps)} LPs, {nnz:.3e} nonzeros; {iters} iterations in {dt:.3f}s",
          file=sys.stderr, flush=True)
    result = {
        "metric": METRIC, "value": iters / dt, "unit": "iters/s", "n_gpus": 1, "steps": 2, "warmup": 0,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"block-diagonal launches of {len(lps)} LPs of the batch (nnz > 20000, even "
                               f"indices), FP32 storage, Halpern form, {iters} iterations",
                   "lps": len(lps), "nnz": nnz, "m": m, "n": n},
        "alg_bytes_primal_launch": prim, "alg_bytes_dual_launch": dual,
        "iteration_alg_gbs": (prim + dual) * iters / dt / 1e9,
    }
    result["environment"] = environment()
    print(json.dumps(result), flush=True)
    return 0


def simulate_mgc(service, rate: float, seconds: float, servers: int, seed: int) -> dict:
    """First-come first-served queue with `servers` servers: Poisson arrivals at `rate` for
    `seconds`, service times drawn at random from `service`. Returns the completions inside
    the window per second and the latency percentiles of every arrival of the window (run to
    completion)."""
    import heapq
    import random

    import numpy as np

    rng = random.Random(seed)
    free = [0.0] * servers
    t, lat, in_window = 0.0, [], 0
    while t < seconds:
        s = service[rng.randrange(len(service))]
        start = max(t, heapq.heappop(free))
        heapq.heappush(free, start + s)
        lat.append(start + s - t)
        in_window += start + s <= seconds
        t += rng.expovariate(rate)
    lat = np.array(lat) if lat else np.array([np.nan])
    return {"lps_per_s": in_window / seconds, "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)), "arrivals": len(lat)}


def cpu_serving_baseline(pool, requests, rate: float, seconds: float, method: int, budget_s: float,
                         eval_every: int = 64) -> dict:
    """The oracle as the host's server, simulated: its rate in nonzero-iterations per second is
    measured on 8 LPs spread over the pool's size range (same method, single-threaded, each
    for about budget_s / 8 seconds of iterations); each completed GPU request of the drained
    phase (its LP's nnz and the iterations it needed) then gets the service time
    iterations * nnz / that rate, and an M/G/c queue with c = the host's cores serves Poisson
    arrivals at `rate` (saturated) and at half the simulated capacity (latency)."""
    import numpy as np

    import oracle

    order = sorted(range(len(pool)), key=lambda j: pool[j].nnz)
    picks = [order[round(q * (len(order) - 1) / 7)] for q in range(8)]
    work = spent = 0.0
    for j in picks:
        # about budget_s / 8 seconds each at ~2.5e8 nonzero-iterations per second
        its = int(max(64, min(20000, budget_s / 8 * 2.5e8 / max(pool[j].nnz, 1))))
        r = oracle.solve(pool[j], eps_rel=0.0, max_iters=its, method=method, eval_every=eval_every)
        work += float(r.iters) * pool[j].nnz
        spent += r.iter_s
    solved = len(picks)
    per_s = work / spent
    service = [it * pool[j].nnz / per_s for j, it in requests]
    cores = os.cpu_count() or 1
    sat = simulate_mgc(service, rate, seconds, cores, 11)
    cap = cores / float(np.mean(service))
    sub = simulate_mgc(service, 0.5 * cap, seconds, cores, 12)
    return {"value": sat["lps_per_s"], "unit": "LPs/s", "cores": cores, "kind": "oracle",
            "simulated": True, "latency_p50_s": sub["latency_p50_s"], "latency_p99_s": sub["latency_p99_s"],
            "latency_offered_lps_per_s": 0.5 * cap,
            "sample": f"simulated: the oracle ran {solved} pool LPs spread over its size range for {spent:.1f} s "
                      f"({per_s:.3g} nnz-iterations/s on one core of '{cpu_model()}'); service time of each of "
                      f"the {len(service)} requests of the GPU's drained phase = its iterations x nnz / that rate; "
                      f"M/G/{cores} first-come first-served queue, Poisson arrivals at {rate}/s for {seconds}s "
                      f"(LPs/s) and at half the simulated capacity (p50/p99)"}


def leg_serve(pool_size: int, rate: float, seconds: float, sub_seconds: float, drain_seconds: float,
              hbm_budget_gb: int, slots: int, max_iters: int, method: int, loop_count: int,
              cpu_budget_s: float = 0.0, eval_every: int = 64) -> dict:
    """Serving workload: Poisson arrivals drawn from a pre-generated pool of LPs
    (m log-uniform on [100, 2e5], n = 1.5m, 3-20 nonzeros per row, KKT-constructed),
    FP32 storage form with FP64 evaluation and refinement, to E_rel 1e-4; continuous
    batching with admission by device footprint. A saturated phase at `rate` gives LPs/s;
    a second phase at half that throughput, drained, gives the latency percentiles."""
    import random

    import numpy as np

    import paper_2604_23951_amd as lpg
    import synth

    t0 = time.time()
    pool = [synth.cfg4_lp(j) for j in range(pool_size)]
    nnz = np.array([lp.nnz for lp in pool])
    tmpl = [lpg.Solver(lp, spmv_layout=1, deferred=1, precision=lpg.LP_PREC_FP32_REFINED, method=method)
            for lp in pool]
    print(f"[bench] pool of {len(pool)} LPs (mean nnz {nnz.mean():.3g}, max {nnz.max()}) ready in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def phase(rate, seconds, seed, drain):
        """Poisson arrivals at `rate` for `seconds`; with `drain`, keep serving (no new
        arrivals) until every request submitted in the window has completed, at most
        drain_seconds more, so that latency covers the whole window."""
        rng = random.Random(seed)
        srv = lpg.Server(hbm_budget_gb * 2**30, slots, eps_rel=1e-4, max_iters=max_iters, method=method,
                         eval_every=eval_every)
        tickets = {}
        start = time.perf_counter()
        t_next = 0.0
        done = []
        while True:
            now = time.perf_counter() - start
            if now >= seconds:
                break
            if now >= t_next:
                j = rng.randrange(len(tmpl))
                tickets[srv.submit(tmpl[j])] = j
                t_next += rng.expovariate(rate)
                continue
            done += srv.poll()
            time.sleep(min(0.0005, max(0.0, t_next - now)))
        done += srv.poll()
        in_window = len(done)
        st_window = srv.stats()
        if drain:
            while len(done) < len(tickets) and time.perf_counter() - start < seconds + drain_seconds:
                time.sleep(0.002)
                done += srv.poll()
        span = time.perf_counter() - start
        st = srv.stats()
        lat, wait, status, reqs = [], [], [], []
        for t in done:
            ts, ta, td = srv.times(t)
            lat.append(td - ts)
            wait.append(ta - ts)
            try:
                r = srv.result(t)
                status.append(r.status)
                reqs.append((tickets[t], int(r.info.iterations)))
            except lpg.LpError:  # the request could not be set up on the device
                status.append("failed")
        srv.close()
        opt_in_window = sum(st_ == "optimal" for st_ in status[:in_window])
        lat = np.array(lat) if lat else np.array([np.nan])
        wait = np.array(wait) if wait else np.array([np.nan])
        # work: PDHG iterations x nnz(A) run by the server; with FP32 storage both products
        # stream 8 bytes (value + index) per nonzero, a lower bound on the traffic
        wsec = st_window["nnz_iterations"] / seconds
        # LPs/s counts the requests that reached E_rel 1e-4 inside the window; the others that
        # completed stopped at the iteration cap
        return {"offered_lps_per_s": rate, "seconds": seconds, "submitted": len(tickets),
                "completed_in_window": in_window, "optimal_in_window": opt_in_window,
                "lps_per_s": opt_in_window / seconds,
                "optimal": sum(st_ == "optimal" for st_ in status),
                "completed": len(done), "drained": bool(drain and len(done) == len(tickets)),
                "span_s": span,
                "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
                "admission_wait_p50_s": float(np.percentile(wait, 50)),
                "backlog_at_window_end": st_window["queued"] + st_window["running"], "rounds": st["rounds"],
                "peak_device_bytes": st["peak_bytes"],
                "nnz_iterations_per_s": wsec, "matrix_stream_GBps": 16 * wsec / 1e9,
                # each iteration gathers once per nonzero in each of its two products
                "gathered_entries_per_s": 2 * wsec,
                "fraction_of_l2_gather_rate": 2 * wsec / L2_GATHER_RATE_PER_S,
                "lp_iterations_per_s": st_window["lp_iterations"] / seconds}, reqs

    full, _ = phase(rate, seconds, 1, False)
    print(f"[bench] offered {rate}/s: {full['lps_per_s']:.1f} LPs/s to 1e-4 ({full['completed_in_window']} "
          f"completed), p50 {full['latency_p50_s']:.3f}s, "
          f"p99 {full['latency_p99_s']:.3f}s, backlog {full['backlog_at_window_end']}, "
          f"{full['nnz_iterations_per_s']:.3g} nnz-it/s ({full['matrix_stream_GBps']:.0f} GB/s of A)",
          file=sys.stderr, flush=True)
    sub_rate = max(0.5, 0.5 * full["lps_per_s"])
    sub, sub_reqs = phase(sub_rate, sub_seconds, 2, True)
    print(f"[bench] offered {sub_rate:.2f}/s: {sub['completed']}/{sub['submitted']} completed (drained "
          f"{sub['drained']}), p50 {sub['latency_p50_s']:.3f}s, p99 {sub['latency_p99_s']:.3f}s, "
          f"{sub['nnz_iterations_per_s']:.3g} nnz-it/s", file=sys.stderr, flush=True)
    for t in tmpl:
        t.close()
    # plain per-LP FP64 loop: every 12th LP of the pool (the pool is drawn at random), same
    # method and tolerance, lp_solve one after another on the same GPU
    sub_lps = pool[::12][:loop_count]
    loop_t = 0.0
    loop_ok = 0
    for lp in sub_lps:
        with lpg.Solver(lp, eps_rel=1e-4, max_iters=max_iters, method=method, spmv_layout=lpg.LP_LAYOUT_TUNED,
                        eval_every=eval_every) as s1:
            t3 = time.perf_counter()
            r = s1.solve()
            loop_t += time.perf_counter() - t3
            loop_ok += r.status == "optimal"
    loop_rate = loop_ok / loop_t if loop_t > 0 else float("nan")  # LPs that reached 1e-4
    print(f"[bench] per-LP FP64 loop: {len(sub_lps)} LPs in {loop_t:.2f}s ({loop_rate:.2f} LPs/s)",
          file=sys.stderr, flush=True)
    out = {
        "lps_per_s": full["lps_per_s"],
        "workload": f"serving: Poisson arrivals at {rate}/s for {seconds}s from a pool of {len(pool)} LPs "
                    f"(m log-uniform [100, 2e5], n=1.5m, 3-20 nnz/row), FP32 storage form + FP64 refinement to "
                    f"E_rel 1e-4, continuous batching, HBM budget {hbm_budget_gb} GiB, {slots} slots",
        "pool_mean_nnz": float(nnz.mean()), "method": {v: k for k, v in METHODS.items()}[method],
        # latency of every request of the half-load window (drained); under saturation the
        # queue grows without bound and only early, small requests complete in the window
        "latency_p50_s": sub["latency_p50_s"], "latency_p99_s": sub["latency_p99_s"],
        "latency_phase": f"offered {sub_rate:.2f}/s (half the saturated rate), all requests of a "
                         f"{sub_seconds}s window",
        "saturated": full, "sub_saturation": sub,
        "per_lp_fp64_loop": {"lps": len(sub_lps), "seconds": loop_t, "lps_per_s": loop_rate, "optimal": loop_ok,
                             "method": "same as the server", "layout": "tuned per LP"},
        "speedup_vs_per_lp_loop": full["lps_per_s"] / loop_rate,
        "cpu_baseline": None,
    }
    if cpu_budget_s > 0 and sub_reqs:
        print("[bench] cpu baseline: oracle service rate on the pool, M/G/c simulation", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_serving_baseline(pool, sub_reqs, rate, seconds, method, cpu_budget_s, eval_every)
    out["eval_every"] = eval_every
    return out


def run_serve(args) -> int:
    """The serving workload alone (--workload serve): one JSON line with LPs/s as `value`."""
    leg = leg_serve(args.pool, args.rate, args.serve_seconds, args.sub_seconds, args.drain_seconds,
                    args.hbm_budget_gb, args.slots, args.batch_max_iters, method_of(args, "halpern"),
                    args.loop_count, 0.0 if args.no_cpu_baseline else 20.0, args.serve_eval_every)
    result = {
        "metric": METRIC, "value": leg["lps_per_s"], "unit": "LPs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": args.serve_seconds * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": leg["workload"], "pool_mean_nnz": leg["pool_mean_nnz"], "method": leg["method"]},
    }
    result.update({k: v for k, v in leg.items() if k not in ("workload", "pool_mean_nnz", "method", "lps_per_s")})
    result["environment"] = environment()
    print(json.dumps(result), flush=True)
    return 0


def leg_small_lp(cpu: bool) -> dict:
    """The small LP (m = 200, n = 400, 2% density, KKT-constructed), 5000 FP64 iterations with
    eps 0 and restarts active: its working set (~80 KB) sits in the caches, so it is bound by
    latency, not HBM; reported as microseconds per iteration for lp_solve as it runs by default
    (one workgroup from LDS: the LP fits the small-LP budget), for the kernel-per-phase loop
    (hipGraph bundles of 64 iterations) with panels and with row tiles, and the oracle's
    iterations per second on one host core."""
    import numpy as np

    import paper_2604_23951_amd as lpg
    import synth

    lp = synth.cfg0(0)
    iters = 5000
    out = {"workload": "small LP m=200 n=400 (2% density, KKT-constructed), FP64, 5000 iterations, eps 0",
           "iterations": iters, "bound": "latency (working set in cache)"}
    for name, opts in (("lp_solve_us_per_iter", {}),
                       ("kernel_loop_panels_us_per_iter", dict(spmv_layout=0, small_lp_lds=0)),
                       ("kernel_loop_tiles_us_per_iter", dict(spmv_layout=1, small_lp_lds=0))):
        with lpg.Solver(lp, eps_rel=0.0, max_iters=iters, **opts) as s:
            s.solve()
            ts = []
            for _ in range(3):
                t = time.perf_counter()
                sol = s.solve()
                ts.append(time.perf_counter() - t)
        out[name] = float(np.median(ts)) / iters * 1e6
        if not opts:
            out["lp_solve_path"] = "one workgroup" if sol.info.solve_path == 1 else "kernel per phase"
    print(f"[bench] small LP: lp_solve {out['lp_solve_us_per_iter']:.1f} us/it ({out['lp_solve_path']}), "
          f"kernel loop {out['kernel_loop_panels_us_per_iter']:.1f} (panels) / "
          f"{out['kernel_loop_tiles_us_per_iter']:.1f} (row tiles) us/it", file=sys.stderr, flush=True)
    out["cpu_baseline"] = None
    if cpu:
        import oracle

        r = oracle.solve(lp, eps_rel=0.0, max_iters=iters, scaling=True)
        out["cpu_baseline"] = {"value": iters / r.iter_s, "unit": "iters/s", "cores": 1, "kind": "oracle",
                               "us_per_iter": r.iter_s / iters * 1e6,
                               "sample": f"the same 5000 iterations on one core of '{cpu_model()}'"}
    return out


def run_presolve(args) -> int:
    """Presolve workload: a KKT-constructed LP (small-LP recipe, m x 2m, 10% free columns) with
    planted reducible structure (fixed, empty and lock-fixable columns, singleton, redundant and
    empty rows, free column singletons in equality rows, each at 10% of m or n), solved to
    E_rel 1e-4 directly on the GPU and through host presolve + GPU solve + host postsolve."""
    import paper_2604_23951_amd as lpg
    import synth

    m = args.presolve_m
    t0 = time.time()
    lp = synth.presolve_lp(0, m=m, n=2 * m, density=args.presolve_density)
    print(f"[bench] presolve workload m={lp.m} n={lp.n} nnz={lp.nnz} generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    # both legs with the layout tuner (row tiles beat panels at this size)
    opts = dict(eps_rel=1e-4, max_iters=args.batch_max_iters, method=method_of(args, "halpern"),
                spmv_layout=lpg.LP_LAYOUT_TUNED)
    lpg.solve_presolved(synth.presolve_lp(1, m=200, n=400, density=0.02), **opts)  # warm-up
    t1 = time.perf_counter()
    with lpg.Solver(lp, **opts) as s:
        direct = s.solve()
    direct_s = time.perf_counter() - t1
    t2 = time.perf_counter()
    r = lpg.solve_presolved(lp, **opts)
    pre_s = time.perf_counter() - t2
    ev = lpg.evaluate(lp, r.x, r.y)
    print(f"[bench] direct: {direct.status} {direct.info.iterations} it in {direct_s:.2f}s; presolved: "
          f"{r.presolve['m']}x{r.presolve['n']} nnz {r.presolve['nnz']}, {r.reduced.info.iterations} it, "
          f"{pre_s:.2f}s end to end (presolve {r.times['presolve_s'] * 1e3:.1f} ms); postsolved E_rel {ev.rel_kkt:.2e}",
          file=sys.stderr, flush=True)
    result = {
        "metric": METRIC, "value": pre_s, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": pre_s * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"presolve + solve to E_rel 1e-4 vs solve alone: KKT-constructed LP m={lp.m} "
                               f"n={lp.n} nnz={lp.nnz} with planted reducible structure (10% of rows / columns "
                               f"per type)", "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                   "method": {v: k for k, v in METHODS.items()}[opts["method"]], "layout": "tuned"},
        "presolve": r.presolve, "times": r.times,
        "reduced": {"status": r.reduced.status, "iterations": int(r.reduced.info.iterations),
                    "rel_kkt": r.reduced.info.rel_kkt},
        "postsolved": {"rel_kkt_original": ev.rel_kkt, "primal_obj": ev.primal_obj, "p_star": lp.p_star},
        "direct": {"status": direct.status, "iterations": int(direct.info.iterations), "seconds": direct_s,
                   "rel_kkt": direct.info.rel_kkt},
        "speedup_end_to_end": direct_s / pre_s,
    }
    result["environment"] = environment()
    print(json.dumps(result), flush=True)
    return 0


COUNTERS_FILE = os.path.join(ROOT, "profiles", "pdhg_large_lp_fp64_hbm_counters.md")


def recorded_traffic(layout_info, kernel):
    """HBM bytes per launch of `kernel` ("primal" or "dual") from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE figures, scaled by the copy calibration. None unless the kernel
    sources still hash to the recorded value and the layout is the one the counters saw."""
    try:
        text = open(COUNTERS_FILE).read()
        blk = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        h = hashlib.sha256()
        for f in blk["source_files"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != blk["source_sha256"]:
            return None
        if any(layout_info.get(k) != v for k, v in blk["layout"].items()):
            return None
        c = blk[kernel]
        return (c["fetch_kib"] * blk["fetch_scale"] + c["write_kib"] * blk["write_scale"]) * 1024.0
    except (OSError, IndexError, KeyError, ValueError):
        return None


def run_copy_calibration(args) -> int:
    """A plain device-to-device copy of known size (512 MiB read, 512 MiB written), the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = 64 * 2**20  # doubles
    a = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 10
    print(json.dumps({"copy_bytes_each_way": n * 8, "us_per_copy": dt * 1e6,
                      "read_plus_write_gbs": 2 * n * 8 / dt / 1e9}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eval-every", type=int, default=64)
    # evaluation periods of the batched and the served LPs (also of their per-LP loops and
    # oracle baselines); the library's default of 64 unless asked otherwise
    ap.add_argument("--batch-eval-every", type=int, default=64)
    ap.add_argument("--serve-eval-every", type=int, default=64)
    ap.add_argument("--cpu-iters", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solve", action="store_true", help="also solve the LP to E_rel 1e-4 and toward 1e-8 (long)")
    ap.add_argument("--solve-time-limit", type=float, default=90.0)
    ap.add_argument("--size", default="full", help="full, or m,n,nnz for a reduced instance")
    ap.add_argument("--layout", type=int, default=0, help="0 panel-packed wave units, 1 row tiles")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 storage form measurement")
    ap.add_argument("--method", choices=sorted(METHODS), default=None,
                    help="PDHG form (default: averaged for the large-LP iteration rate, halpern for the "
                         "workloads measured to a tolerance)")
    ap.add_argument("--no-halpern-leg", action="store_true")
    ap.add_argument("--workload", default="large", choices=["large", "batch", "serve", "copy", "presolve", "blockdiag"])
    ap.add_argument("--presolve-m", type=int, default=20000)
    ap.add_argument("--presolve-density", type=float, default=0.0003)
    ap.add_argument("--pool", type=int, default=96)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--sub-seconds", type=float, default=20.0)
    ap.add_argument("--drain-seconds", type=float, default=60.0)
    ap.add_argument("--hbm-budget-gb", type=int, default=128)
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--loop-count", type=int, default=8)
    ap.add_argument("--batch-max-iters", type=int, default=400000)
    ap.add_argument("--no-legs", action="store_true",
                    help="large LP only (skip the small-LP, batch-sample and serving legs of the default run)")
    ap.add_argument("--leg-batch-count", type=int, default=256)
    ap.add_argument("--leg-serve-seconds", type=float, default=20.0)
    ap.add_argument("--leg-sub-seconds", type=float, default=15.0)
    ap.add_argument("--slice-bytes", type=int, default=0)
    ap.add_argument("--units-per-cu", type=int, default=0)
    ap.add_argument("--long-row-len", type=int, default=0)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is a design note, not built", file=sys.stderr)
        return 2
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "presolve":
        return run_presolve(args)
    if args.workload == "blockdiag":
        return run_blockdiag(args)
    if args.workload == "copy":
        return run_copy_calibration(args)

    import numpy as np

    import paper_2604_23951_amd as lpg
    import synth

    if args.size == "full":
        m, n, nnz = 1_000_000, 2_000_000, 12_000_000
    else:
        m, n, nnz = (int(v) for v in args.size.split(","))
    t0 = time.time()
    lp = synth.cfg1(0, m=m, n=n, nnz=nnz)
    gen_s = time.time() - t0
    print(f"[bench] generated {lp.name} in {gen_s:.1f}s", file=sys.stderr, flush=True)

    E = args.eval_every
    tun = dict(spmv_layout=args.layout)
    if args.slice_bytes:
        tun["panel_slice_bytes"] = args.slice_bytes
    if args.units_per_cu:
        tun["units_per_cu"] = args.units_per_cu
    if args.long_row_len:
        tun["long_row_len"] = args.long_row_len
    solver = lpg.Solver(lp, eps_rel=0.0, max_iters=E * max(args.warmup, 1), eval_every=E, **tun)
    layout_info = solver.layout()
    sol = solver.solve()  # warmup (also captures the iteration graph)
    setup_s = sol.info.setup_seconds
    print(f"[bench] setup {setup_s:.2f}s, warmup {sol.info.iterations} iterations in {sol.info.solve_seconds:.3f}s",
          file=sys.stderr, flush=True)

    # timed region: exactly `steps` evaluation periods, kernel events on the solver stream
    K = args.steps
    solver.update(eps_rel=0.0, max_iters=E * K, eval_every=E)
    lpg.lp_set_kernel_timing(solver.h, True)
    t1 = time.perf_counter()
    sol = solver.solve()
    dt = time.perf_counter() - t1
    p_ms, d_ms, samples = lpg.lp_get_kernel_times(solver.h)
    lpg.lp_set_kernel_timing(solver.h, False)
    assert sol.info.iterations == E * K
    iters_per_s = E * K / dt
    print(f"[bench] timed {K} steps ({E * K} iterations) in {dt:.3f}s: {iters_per_s:.1f} it/s; "
          f"primal {p_ms * 1e3:.1f} us, dual {d_ms * 1e3:.1f} us ({samples} samples)", file=sys.stderr, flush=True)

    # same region replayed as hipGraph bundles without events
    t2 = time.perf_counter()
    sol_g = solver.solve()
    dt_g = time.perf_counter() - t2

    fp32_res = None
    if not args.no_fp32:
        # the FP32 storage form on the same LP (matrix and iterates FP32, FP64 evaluation,
        # restart decisions and refinement), same step definition
        s32 = lpg.Solver(lp, eps_rel=0.0, max_iters=E * max(args.warmup, 1), eval_every=E,
                         precision=lpg.LP_PREC_FP32_REFINED, **tun)
        s32.solve()
        s32.update(eps_rel=0.0, max_iters=E * K, eval_every=E)
        lpg.lp_set_kernel_timing(s32.h, True)
        t5 = time.perf_counter()
        s32.solve()
        dt5 = time.perf_counter() - t5
        p32, d32, n32 = lpg.lp_get_kernel_times(s32.h)
        s32.close()
        bp32, bd32 = algorithmic_bytes(m, n, nnz, sv=4)
        fp32_res = {"workload": "same LP, FP32 storage form (FP64 evaluation / restarts / refinement)",
                    "iters_per_s": E * K / dt5, "ms_per_step": dt5 / K * 1e3,
                    "primal_ms": p32, "dual_ms": d32, "primal_alg_bytes": bp32, "dual_alg_bytes": bd32,
                    "primal_gbs": bp32 / (p32 * 1e-3) / 1e9, "dual_gbs": bd32 / (d32 * 1e-3) / 1e9, "samples": n32}
        print(f"[bench] fp32 form: {E * K / dt5:.1f} it/s; primal {p32 * 1e3:.1f} us, dual {d32 * 1e3:.1f} us",
              file=sys.stderr, flush=True)

    halpern_res = None
    if not args.no_halpern_leg:
        # the reflected Halpern form on the same LP (FP64), same step definition
        sh = lpg.Solver(lp, eps_rel=0.0, max_iters=E * max(args.warmup, 1), eval_every=E,
                        method=lpg.LP_METHOD_HALPERN, **tun)
        sh.solve()
        sh.update(eps_rel=0.0, max_iters=E * K, eval_every=E, method=lpg.LP_METHOD_HALPERN)
        lpg.lp_set_kernel_timing(sh.h, True)
        t6 = time.perf_counter()
        sh.solve()
        dt6 = time.perf_counter() - t6
        ph, dh, nh = lpg.lp_get_kernel_times(sh.h)
        sh.close()
        bph, bdh = algorithmic_bytes(m, n, nnz, halpern=True)
        halpern_res = {"workload": "same LP, reflected Halpern form (FP64)",
                       "iters_per_s": E * K / dt6, "ms_per_step": dt6 / K * 1e3,
                       "primal_ms": ph, "dual_ms": dh, "primal_alg_bytes": bph, "dual_alg_bytes": bdh,
                       "primal_gbs": bph / (ph * 1e-3) / 1e9, "dual_gbs": bdh / (dh * 1e-3) / 1e9, "samples": nh}
        print(f"[bench] halpern form: {E * K / dt6:.1f} it/s; primal {ph * 1e3:.1f} us, dual {dh * 1e3:.1f} us",
              file=sys.stderr, flush=True)

    bp, bd = algorithmic_bytes(m, n, nnz)
    gbs_p = bp / (p_ms * 1e-3) / 1e9
    gbs_d = bd / (d_ms * 1e-3) / 1e9
    if p_ms >= d_ms:
        dom = dict(kernel="primal: A^T y + primal update", bytes=bp, ms=p_ms, gbs=gbs_p, key="primal")
    else:
        dom = dict(kernel="dual: A x + dual update", bytes=bd, ms=d_ms, gbs=gbs_d, key="dual")
    traffic = recorded_traffic(layout_info, dom["key"])
    iter_bytes = bp + bd
    result = {
        "metric": METRIC,
        "value": iters_per_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single large LP, FP64: m=%d n=%d nnz=%d, power-law columns (exp 2.2, max 5000), "
                               "20%% free columns, 30%% two-sided rows, KKT-constructed" % (m, n, nnz),
                   "m": m, "n": n, "nnz": nnz, "iters_per_step": E, "precision": "fp64", "scaling": "ruiz10+pc",
                   "layout": layout_info},
        "roofline": {"bound": "hbm", "achieved": dom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["gbs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom["kernel"],
                     "alg_bytes_per_launch": dom["bytes"], "avg_launch_ms": dom["ms"],
                     # the counted HBM traffic (FETCH_SIZE / WRITE_SIZE, scaled) over the same launch time
                     "traffic_gbs": traffic / (dom["ms"] * 1e-3) / 1e9 if traffic else None,
                     "traffic_frac": traffic / (dom["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "gather_ceiling": {"gathers_per_launch": nnz, "rate_per_s": GATHER_CEILING_PER_S,
                                        "min_launch_ms": nnz / GATHER_CEILING_PER_S * 1e3,
                                        "frac": (nnz / GATHER_CEILING_PER_S * 1e3) / dom["ms"]}},
        "kernels": {"primal_ms": p_ms, "primal_alg_bytes": bp, "primal_gbs": gbs_p,
                    "dual_ms": d_ms, "dual_alg_bytes": bd, "dual_gbs": gbs_d, "samples": samples},
        "iteration_alg_bytes": iter_bytes,
        "effective_gbs_per_iteration": iter_bytes * iters_per_s / 1e9,
        "graph_mode_iters_per_s": E * K / dt_g,
        "setup_s": setup_s,
        "generate_s": gen_s,
        "fp32_form": fp32_res,
        "halpern_form": halpern_res,
    }
    if args.solve:
        # to E_rel 1e-4 in the FP64 and FP32 storage forms of the reflected Halpern iteration
        # (the averaged form needs several times the iterations on this LP), then the FP32
        # form toward 1e-8 within the time limit
        legs = []
        for prec, eps in ((lpg.LP_PREC_FP64, 1e-4), (lpg.LP_PREC_FP32_REFINED, 1e-4), (lpg.LP_PREC_FP32_REFINED, 1e-8)):
            with lpg.Solver(lp, precision=prec, method=lpg.LP_METHOD_HALPERN, eps_rel=eps, max_iters=10**7,
                            time_limit_s=args.solve_time_limit, eval_every=E) as s4:
                t3 = time.perf_counter()
                r4 = s4.solve()
                dt4 = time.perf_counter() - t3
                polished = None
                if eps == 1e-4 and r4.status == "optimal":
                    # feasibility polishing of the 1e-4 point to primal and dual residuals of 1e-8
                    t7 = time.perf_counter()
                    p4 = s4.polish(eps=1e-8, max_iters=400000)
                    polished = {"eps": 1e-8, "seconds": time.perf_counter() - t7,
                                "primal_iterations": int(p4.info.polish_primal_iterations),
                                "dual_iterations": int(p4.info.polish_dual_iterations),
                                "rel_primal_res": p4.info.rel_primal_res, "rel_dual_res": p4.info.rel_dual_res,
                                "rel_gap": p4.info.rel_gap,
                                "rel_obj_err": abs(p4.info.primal_obj - lp.p_star) / (1 + abs(lp.p_star))}
            legs.append({"precision": "fp64" if prec == lpg.LP_PREC_FP64 else "fp32+fp64", "eps_rel": eps,
                         "status": r4.status, "iterations": int(r4.info.iterations),
                         "restarts": int(r4.info.restarts), "seconds": dt4, "rel_kkt": r4.info.rel_kkt,
                         "primal_obj": r4.info.primal_obj, "p_star": lp.p_star,
                         "rel_obj_err": abs(r4.info.primal_obj - lp.p_star) / (1 + abs(lp.p_star)),
                         "polished": polished})
            print(f"[bench] solve ({legs[-1]['precision']}, Halpern) to {eps:g}: {r4.status} after "
                  f"{r4.info.iterations} iterations in {dt4:.1f}s, E_rel {r4.info.rel_kkt:.3e}",
                  file=sys.stderr, flush=True)
            if polished:
                print(f"[bench]   polished to 1e-8 in {polished['seconds']:.2f}s ({polished['primal_iterations']} + "
                      f"{polished['dual_iterations']} iterations): rel primal {polished['rel_primal_res']:.2e}, "
                      f"rel dual {polished['rel_dual_res']:.2e}, gap {polished['rel_gap']:.2e}",
                      file=sys.stderr, flush=True)
        result["solves"] = legs
    solver.close()
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle, {args.cpu_iters} iterations", file=sys.stderr, flush=True)
        result["cpu_baseline"] = run_cpu_baseline(lp, args.cpu_iters)
    else:
        result["cpu_baseline"] = None
    del lp
    if not args.no_legs:
        # the rest of the metric, each bounded so that the whole run stays within minutes:
        # the latency-bound small LP, a sample of the batch and a shorter serving window
        cpu = not args.no_cpu_baseline
        meth = method_of(args, "halpern")
        result["small_lp"] = leg_small_lp(cpu)
        result["batch"] = leg_batch(args.leg_batch_count, 8, args.batch_max_iters, meth, 10.0 if cpu else 0.0,
                                    args.batch_eval_every)
        result["serving"] = leg_serve(args.pool, args.rate, args.leg_serve_seconds, args.leg_sub_seconds, 30.0,
                                      args.hbm_budget_gb, args.slots, args.batch_max_iters, meth, 4,
                                      10.0 if cpu else 0.0, args.serve_eval_every)
    result["environment"] = environment()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
