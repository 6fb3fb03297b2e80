"""lp_server_cancel: a queued request completes at once with no point, a running one stops
after its round with the point of its current iterate, which (Halpern form: the PDHG output
T(z)) is the point a single solve stopped by max_iters at the same iteration returns, bit for
bit; the server keeps serving; misuse is an error code."""
import time

import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu
ERR_INVALID_ARG = 1


def _single(lp, k, precision):
    with lpg.Solver(lp, eps_rel=1e-14, max_iters=k, method=lpg.LP_METHOD_HALPERN, spmv_layout=1,
                    precision=precision) as s:
        return s.solve()


def _wait_running(srv, count, limit=30.0):
    t = time.perf_counter()
    while srv.stats()["running"] < count:
        assert time.perf_counter() - t < limit, srv.stats()
        time.sleep(0.01)


def _wait_completed(srv, count, limit=30.0):
    t = time.perf_counter()
    while srv.stats()["completed"] < count:
        assert time.perf_counter() - t < limit, srv.stats()
        time.sleep(0.01)


@pytest.mark.parametrize("precision", [lpg.LP_PREC_FP64, lpg.LP_PREC_FP32_REFINED])
def test_cancel_queued_and_running(precision):
    rng = np.random.default_rng(41)
    lps = [synth.cfg4_lp(3, m_lo=400, m_hi=900), synth.transportation(60, rng), synth.cfg0(0)]
    opts = dict(method=lpg.LP_METHOD_HALPERN, spmv_layout=1, precision=precision)
    tmpls = [lpg.Solver(lp, deferred=1, **opts) for lp in lps]
    print(f"cancel, precision {precision}", flush=True)
    try:
        # one slot: the first request runs, the others wait in the queue; nothing reaches 1e-14
        with lpg.Server(1 << 34, 1, eps_rel=1e-14, max_iters=10**7, **opts) as srv:
            ta, tb, tc = (srv.submit(t) for t in tmpls)
            srv.cancel(tb)                        # queued: completed at once
            _wait_running(srv, 1)
            time.sleep(0.2)
            srv.cancel(ta)                        # running: stopped after its round
            _wait_completed(srv, 2)
            _wait_running(srv, 1)                 # the slot went to the third request
            time.sleep(0.1)
            srv.cancel(tc)
            srv.wait(60.0)
            st = srv.stats()
            assert (st["submitted"], st["completed"], st["running"], st["queued"]) == (3, 3, 0, 0)
            assert st["bytes_in_use"] == 0
            for bad in (tb, ta, 10**6):             # completed, completed, unknown
                with pytest.raises(lpg.LpError) as e:
                    srv.cancel(bad)
                assert e.value.code == ERR_INVALID_ARG
            ra, rb, rc = srv.result(ta), srv.result(tb), srv.result(tc)
    finally:
        for t in tmpls:
            t.close()
    assert rb.status == "cancelled" and rb.info.iterations == 0
    assert np.all(np.isnan(rb.x)) and np.all(np.isnan(rb.y)) and np.all(np.isnan(rb.z))
    for lp, r in ((lps[0], ra), (lps[2], rc)):
        k = r.info.iterations
        print(f"  cancelled at iteration {k}", flush=True)
        assert r.status == "cancelled" and k >= 64 and k % 64 == 0
        ref = _single(lp, k, precision)
        assert ref.status == "iteration_limit" and ref.info.iterations == k
        np.testing.assert_array_equal(r.x, ref.x)
        np.testing.assert_array_equal(r.y, ref.y)
        np.testing.assert_array_equal(r.z, ref.z)
        assert r.info.rel_kkt == ref.info.rel_kkt


def test_cancel_leaves_other_requests_untouched():
    """Cancelling one request of a running set: the others finish with their solo results."""
    rng = np.random.default_rng(43)
    lps = [synth.cfg4_lp(j, m_lo=300, m_hi=700) for j in range(3)] + [synth.transportation(50, rng)]
    opts = dict(method=lpg.LP_METHOD_HALPERN, spmv_layout=1)
    solo = []
    for lp in lps:
        with lpg.Solver(lp, eps_rel=1e-6, max_iters=200000, **opts) as s:
            solo.append(s.solve())
    long_lp = synth.cfg4_lp(7, m_lo=400, m_hi=900)
    tmpls = [lpg.Solver(lp, deferred=1, **opts) for lp in lps]
    blocker = lpg.Solver(long_lp, deferred=1, **opts)
    try:
        with lpg.Server(1 << 34, 8, eps_rel=1e-6, max_iters=10**7, **opts) as srv:
            tb = srv.submit(blocker)
            tickets = [srv.submit(t) for t in tmpls]
            _wait_running(srv, 1)
            srv.cancel(tb)
            srv.wait(120.0)
            rb = srv.result(tb)
            outs = [srv.result(t) for t in tickets]
    finally:
        for t in tmpls:
            t.close()
        blocker.close()
    assert rb.status in ("cancelled", "optimal")  # it may finish before the worker acts
    for a, b in zip(solo, outs):
        assert a.status == b.status == "optimal" and a.info.iterations == b.info.iterations
        np.testing.assert_array_equal(a.x, b.x)
        np.testing.assert_array_equal(a.y, b.y)
