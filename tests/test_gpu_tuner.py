"""Layout tuner (spmv_layout 2): both product layouts are built, timed on the device at
set-up, and the faster one runs the whole solve. Bars: the choice is the layout with the
smaller recorded trial time, and the tuned solve is bit-identical to a solve with that
layout fixed (the tuner only selects among existing kernels)."""
import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth

pytestmark = pytest.mark.gpu

FP32 = lpg.LP_PREC_FP32_REFINED


def _lps():
    return [synth.cfg0(1), synth.cfg4_lp(3, m_hi=3000), synth.cfg1(0, m=3000, n=6000, nnz=40000)]


@pytest.mark.parametrize("precision", [lpg.LP_PREC_FP64, FP32])
@pytest.mark.parametrize("deferred", [0, 1])
def test_tuned_equals_fixed_choice(precision, deferred):
    for lp in _lps():
        kw = dict(precision=precision, eps_rel=1e-6, max_iters=20000)
        with lpg.Solver(lp, spmv_layout=lpg.LP_LAYOUT_TUNED, deferred=deferred, **kw) as s:
            a = s.solve()
            L = s.layout()
        assert L["layout"] in (0, 1), lp.name
        assert L["trial_ns_panels"] > 0 and L["trial_ns_tiles"] > 0
        faster = 1 if L["trial_ns_tiles"] < L["trial_ns_panels"] else 0
        assert L["layout"] == faster
        with lpg.Solver(lp, spmv_layout=L["layout"], **kw) as s:
            b = s.solve()
        assert a.status == b.status and a.info.iterations == b.info.iterations, lp.name
        assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y) and np.array_equal(a.z, b.z), lp.name


def test_tuned_handle_resolves_with_same_choice():
    """A second solve of the handle (and a solve after update) keeps the layout."""
    lp = synth.cfg4_lp(5, m_hi=2000)
    with lpg.Solver(lp, spmv_layout=lpg.LP_LAYOUT_TUNED, eps_rel=1e-5) as s:
        a = s.solve()
        first = s.layout()["layout"]
        b = s.solve()
        assert s.layout()["layout"] == first
    assert np.array_equal(a.x, b.x)
