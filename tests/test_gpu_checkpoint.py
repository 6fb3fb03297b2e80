"""Checkpoint and resume: a run split by lp_solve_until / lp_resume, or carried to another
handle through lp_export_state / lp_import_state, against one uninterrupted lp_solve of the
same handle options: same iterations, restarts, decision trace, certificate and returned
point, bit for bit, in both iteration forms, both precisions, both product layouts and with
the PID primal-weight rule; a tolerance loosened at a pause stops where a run with that
tolerance from the start stops; every misuse is an error code."""
import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth
from test_oracle_infeasible import CASES as INFEASIBLE
from test_oracle_infeasible import EPS

pytestmark = pytest.mark.gpu
ERR_INVALID_ARG, ERR_NOT_SOLVED = 1, 7


def _lp(name):
    return {"cfg0": lambda: synth.cfg0(0),
            "transport": lambda: synth.transportation(120, np.random.default_rng(3)),
            "mixed": lambda: synth.cfg4_lp(1, m_lo=400, m_hi=900),
            "pinf2": lambda: INFEASIBLE["pinf2"]}[name]()


def _same(a, b):
    assert (a.status, a.info.iterations, a.info.restarts) == (b.status, b.info.iterations, b.info.restarts)
    assert a.info.ray_source == b.info.ray_source and a.info.output_is_avg == b.info.output_is_avg
    np.testing.assert_array_equal(a.trace, b.trace)
    for u, v in zip((a.x, a.y, a.z), (b.x, b.y, b.z)):
        np.testing.assert_array_equal(u, v)
    assert a.info.rel_kkt == b.info.rel_kkt and a.info.primal_obj == b.info.primal_obj
    assert a.info.omega == b.info.omega


def _opts(name, method, precision, layout, pid=False):
    """cfg0 ends on max_iters (6000: a short last period), the others on the tolerance or a
    certificate."""
    o = dict(eps_rel=1e-7, max_iters=200000, method=method, precision=precision, spmv_layout=layout, small_lp_lds=0)
    if name == "cfg0":
        o.update(max_iters=6000)
    if name == "mixed":
        o.update(eps_rel=1e-4, max_iters=20000)
    if name == "pinf2":
        o.update(eps_rel=1e-8, max_iters=100000, eps_infeas=EPS)
    if pid:
        o["pw_rule"] = lpg.LP_PW_PID
    return o


def _straight(lp, opts):
    with lpg.Solver(lp, **opts) as s:
        return s.solve(with_trace=True)


def _pauses(total):
    """Two pause requests inside a run of `total` iterations (evaluations every 64)."""
    assert total >= 4 * 64, total
    return max(1, total // 3 - 17), max(2, (2 * total) // 3 - 5)


FORMS = [(0, lpg.LP_PREC_FP64, 0, False), (1, lpg.LP_PREC_FP64, 1, False), (0, lpg.LP_PREC_FP32_REFINED, 1, False),
         (1, lpg.LP_PREC_FP32_REFINED, 0, False), (0, lpg.LP_PREC_FP64, 1, True)]
FORM_IDS = ["avg_fp64_panels", "halpern_fp64_tiles", "avg_fp32_tiles", "halpern_fp32_panels", "avg_fp64_pid"]


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("name", ["cfg0", "transport", "mixed", "pinf2"])
def test_split_run_equals_straight_run(name, form):
    method, precision, layout, pid = form
    lp = _lp(name)
    opts = _opts(name, method, precision, layout, pid)
    ref = _straight(lp, opts)
    k1, k2 = _pauses(ref.info.iterations)
    print(f"{name} {form}: straight {ref.status} at {ref.info.iterations}, pauses at {k1}, {k2}", flush=True)
    with lpg.Solver(lp, **opts) as s:
        p1 = s.solve_until(k1)
        assert p1.status == "iteration_limit" and k1 <= p1.info.iterations < k1 + 64
        assert p1.info.iterations % 64 == 0
        p2 = s.resume(k2)
        assert p2.status == "iteration_limit" and k2 <= p2.info.iterations < k2 + 64
        out = s.resume(with_trace=True)
    _same(out, ref)


@pytest.mark.parametrize("form", [FORMS[0], FORMS[1], FORMS[2], FORMS[3]], ids=FORM_IDS[:4])
def test_state_carried_to_a_new_handle(form):
    method, precision, layout, _ = form
    lp = _lp("transport")
    opts = _opts("transport", method, precision, layout)
    ref = _straight(lp, opts)
    k1, _ = _pauses(ref.info.iterations)
    print(f"export/import {form}: straight at {ref.info.iterations}, pause at {k1}", flush=True)
    with lpg.Solver(lp, **opts) as a:
        paused = a.solve_until(k1)
        state = a.export_state()
        assert len(state) == len(a.export_state())
        with lpg.Solver(lp, **opts) as b:
            loaded = b.import_state(state)
            assert (loaded.status, loaded.info.iterations) == (paused.status, paused.info.iterations)
            for u, v in zip((loaded.x, loaded.y, loaded.z), (paused.x, paused.y, paused.z)):
                np.testing.assert_array_equal(u, v)
            assert loaded.info.rel_kkt == paused.info.rel_kkt
            assert b.export_state() == state  # the loaded handle holds the same state, bytes and all
            out_b = b.resume(with_trace=True)
        out_a = a.resume(with_trace=True)
    _same(out_b, ref)
    _same(out_a, ref)


def test_state_survives_a_file(tmp_path):
    lp = _lp("cfg0")
    opts = _opts("cfg0", 0, lpg.LP_PREC_FP64, 1)
    ref = _straight(lp, opts)
    k1, k2 = _pauses(ref.info.iterations)
    f = tmp_path / "run.state"
    with lpg.Solver(lp, **opts) as a:
        a.solve_until(k1)
        f.write_bytes(a.export_state())
    with lpg.Solver(lp, **opts) as b:  # another handle reads the file and pauses again
        b.import_state(f.read_bytes())
        b.resume(k2)
        f.write_bytes(b.export_state())
    with lpg.Solver(lp, **opts) as c:
        c.import_state(f.read_bytes())
        out = c.resume(with_trace=True)
    _same(out, ref)


def test_loosened_tolerance_stops_where_a_loose_run_stops():
    """The restart decisions do not depend on eps_rel, so a 1e-7 run paused before a 1e-4 run
    would stop and resumed with 1e-4 stops at that run's evaluation with its point."""
    lp = _lp("transport")
    loose = _opts("transport", 0, lpg.LP_PREC_FP64, 1)
    loose["eps_rel"] = 1e-4
    ref = _straight(lp, loose)
    assert ref.status == "optimal" and ref.info.iterations >= 4 * 64
    tight = dict(loose, eps_rel=1e-7)
    with lpg.Solver(lp, **tight) as s:
        s.solve_until(ref.info.iterations // 2)
        s.update(**loose)
        out = s.resume(with_trace=True)
    _same(out, ref)


def _code(fn, *a):
    with pytest.raises(lpg.LpError) as e:
        fn(*a)
    return e.value.code


def test_misuse_is_an_error():
    lp = _lp("cfg0")
    opts = _opts("cfg0", 0, lpg.LP_PREC_FP64, 1)
    with lpg.Solver(lp, **opts) as s:
        assert _code(s.resume) == ERR_NOT_SOLVED       # nothing paused
        assert _code(s.solve_until, 0) == ERR_INVALID_ARG
        assert _code(s.export_state) == ERR_NOT_SOLVED
        done = s.solve()
        assert _code(s.resume) == ERR_NOT_SOLVED       # a finished lp_solve is not resumable
        late = s.solve_until(10 * done.info.iterations)  # ends on max_iters before the pause
        assert (late.status, late.info.iterations) == (done.status, done.info.iterations) == ("iteration_limit", 6000)
        assert _code(s.resume) == ERR_NOT_SOLVED
        paused = s.solve_until(128)
        state = s.export_state()
        # max_iters at or below the paused count: nothing runs and the handle stays paused
        s.update(**dict(opts, max_iters=64))
        again = s.resume()
        assert (again.status, again.info.iterations) == ("iteration_limit", paused.info.iterations)
        np.testing.assert_array_equal(again.x, paused.x)
        # the iteration form must not change across a pause
        s.update(**dict(opts, eval_every=32))
        assert _code(s.resume) == ERR_INVALID_ARG
        s.update(**dict(opts, method=1))
        assert _code(s.resume) == ERR_INVALID_ARG
        s.update(**opts)
        assert s.export_state() == state
        # bad buffers
        assert _code(s.import_state, state[:-8]) == ERR_INVALID_ARG
        assert _code(s.import_state, b"x" + state[1:]) == ERR_INVALID_ARG
        assert _code(s.import_state, b"") == ERR_INVALID_ARG
        s.resume()
    with lpg.Solver(lp, **dict(opts, eval_every=32)) as t:   # another iteration form
        assert _code(t.import_state, state) == ERR_INVALID_ARG
    other = synth.cfg0(0)
    other.c = other.c + 1.0                                   # same sizes, another LP
    with lpg.Solver(other, **opts) as t:
        assert _code(t.import_state, state) == ERR_INVALID_ARG
    with lpg.Solver(lp, **dict(opts, precision=lpg.LP_PREC_FP32_REFINED)) as t:
        assert _code(t.import_state, state) == ERR_INVALID_ARG
    with lpg.Solver(lp, deferred=1, **opts) as t:             # no device memory yet
        assert _code(t.import_state, state) == ERR_INVALID_ARG


def test_batch_ends_the_pause():
    lp = _lp("cfg0")
    opts = _opts("cfg0", 0, lpg.LP_PREC_FP64, 1)
    with lpg.Solver(lp, **opts) as s:
        s.solve_until(128)
        lpg.solve_batch([s], eps_rel=1e-7, max_iters=200000, spmv_layout=1)
        assert _code(s.resume) == ERR_NOT_SOLVED
