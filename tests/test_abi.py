"""The C-ABI library loads on a machine without a GPU, exports every function the header
declares, and rejects invalid input with the documented error codes before touching a
device (validation runs on the host, ahead of any HIP call)."""
import math
import os
import re

import numpy as np
import pytest

import paper_2604_23951_amd as lpg
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lp_\w+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = lpg.lib()
    declared = _declared()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lpg.EXPORTS) == declared


def test_error_strings():
    for code in range(9):
        assert lpg.lp_error_string(code)
    assert lpg.lp_error_string(99) == "unknown error code"


def _args(lp):
    return dict(m=lp.m, n=lp.n, nnz=lp.nnz, row_ptr=np.ascontiguousarray(lp.row_ptr, np.int32),
                col_idx=np.ascontiguousarray(lp.col_idx, np.int32), vals=np.ascontiguousarray(lp.vals),
                c=np.ascontiguousarray(lp.c), c0=0.0, b_lo=np.ascontiguousarray(lp.b_lo),
                b_hi=np.ascontiguousarray(lp.b_hi), x_lo=np.ascontiguousarray(lp.x_lo),
                x_hi=np.ascontiguousarray(lp.x_hi))


def _create_code(**a):
    try:
        h = lpg.lp_create(**a)
    except lpg.LpError as e:
        return e.code
    lpg.lp_destroy(h)
    return 0


@pytest.mark.parametrize("case,code", [
    ("nan_value", 4), ("inf_value", 4), ("nan_cost", 4), ("inf_cost", 4), ("nan_bound", 4),
    ("lo_gt_hi_row", 3), ("lo_gt_hi_col", 3), ("lo_plus_inf", 3), ("hi_minus_inf", 3),
    ("unsorted_row", 2), ("duplicate_col", 2), ("col_out_of_range", 2), ("row_ptr_decreasing", 2),
    ("row_ptr_bad_end", 2), ("negative_m", 1), ("zero_n", 1), ("null_cost", 1), ("bad_eval_every", 1),
    ("nan_c0", 4), ("bad_layout", 1), ("omega_steps_negative", 1), ("omega_steps_nine", 1),
    ("pw_rule_three", 1), ("pid_gain_negative", 1), ("pid_gain_nan", 1),
])
def test_invalid_input_codes(case, code):
    lp = synth.cfg0(0)
    a = _args(lp)
    r = int(np.flatnonzero(np.diff(lp.row_ptr) >= 2)[0])
    e0 = int(lp.row_ptr[r])
    if case == "nan_value":
        a["vals"] = a["vals"].copy(); a["vals"][3] = math.nan
    elif case == "inf_value":
        a["vals"] = a["vals"].copy(); a["vals"][3] = math.inf
    elif case == "nan_cost":
        a["c"] = a["c"].copy(); a["c"][1] = math.nan
    elif case == "inf_cost":
        a["c"] = a["c"].copy(); a["c"][1] = -math.inf
    elif case == "nan_bound":
        a["b_lo"] = a["b_lo"].copy(); a["b_lo"][2] = math.nan
    elif case == "lo_gt_hi_row":
        a["b_lo"] = a["b_lo"].copy(); a["b_hi"] = a["b_hi"].copy(); a["b_lo"][0] = 2.0; a["b_hi"][0] = 1.0
    elif case == "lo_gt_hi_col":
        a["x_lo"] = a["x_lo"].copy(); a["x_lo"][0] = 11.0
    elif case == "lo_plus_inf":
        a["x_lo"] = a["x_lo"].copy(); a["x_hi"] = a["x_hi"].copy(); a["x_lo"][0] = math.inf; a["x_hi"][0] = math.inf
    elif case == "hi_minus_inf":
        a["b_lo"] = a["b_lo"].copy(); a["b_hi"] = a["b_hi"].copy(); a["b_lo"][0] = -math.inf
        a["b_hi"][0] = -math.inf
    elif case == "unsorted_row":
        a["col_idx"] = a["col_idx"].copy(); a["col_idx"][e0], a["col_idx"][e0 + 1] = a["col_idx"][e0 + 1], a["col_idx"][e0]
    elif case == "duplicate_col":
        a["col_idx"] = a["col_idx"].copy(); a["col_idx"][e0 + 1] = a["col_idx"][e0]
    elif case == "col_out_of_range":
        a["col_idx"] = a["col_idx"].copy(); a["col_idx"][-1] = lp.n
    elif case == "row_ptr_decreasing":
        a["row_ptr"] = a["row_ptr"].copy(); a["row_ptr"][r + 1] = a["row_ptr"][r] - 1
    elif case == "row_ptr_bad_end":
        a["nnz"] = lp.nnz + 1
    elif case == "negative_m":
        a["m"] = -1
    elif case == "zero_n":
        a["n"] = 0
    elif case == "null_cost":
        a["c"] = None
    elif case == "bad_eval_every":
        a["opt"] = lpg.make_options(eval_every=0)
    elif case == "nan_c0":
        a["c0"] = math.nan
    elif case == "bad_layout":
        a["opt"] = lpg.make_options(spmv_layout=3)
    elif case == "omega_steps_negative":
        a["opt"] = lpg.make_options(omega_steps=-1)
    elif case == "omega_steps_nine":
        a["opt"] = lpg.make_options(omega_steps=9)
    elif case == "pw_rule_three":
        a["opt"] = lpg.make_options(pw_rule=3)
    elif case == "pid_gain_negative":
        a["opt"] = lpg.make_options(pw_rule=lpg.LP_PW_PID, pid_ki=-0.1)
    elif case == "pid_gain_nan":
        a["opt"] = lpg.make_options(pw_rule=lpg.LP_PW_PID, pid_kd=math.nan)
    assert _create_code(**a) == code
    assert lpg.lp_last_error()  # a message is recorded


def test_null_out_pointer():
    import ctypes
    lp = synth.cfg0(0)
    a = _args(lp)
    rc = lpg.lib().lp_create(None, a["m"], a["n"], a["nnz"], a["row_ptr"].ctypes.data, a["col_idx"].ctypes.data,
                             a["vals"].ctypes.data, a["c"].ctypes.data, 0.0, a["b_lo"].ctypes.data,
                             a["b_hi"].ctypes.data, a["x_lo"].ctypes.data, a["x_hi"].ctypes.data, None)
    assert rc == 1


def test_null_handle_calls():
    assert lpg.lib().lp_solve(None) == 1
    assert lpg.lib().lp_get_solution(None, None, None, None, None) == 1
    lpg.lib().lp_destroy(None)  # ignored


def test_deferred_handle_needs_no_device():
    """A deferred handle is validated and laid out on the host; its device footprint is
    known before any device memory is touched."""
    lp = synth.cfg0(0)
    with lpg.Solver(lp, deferred=1, spmv_layout=1) as s:
        fp = s.layout()["device_bytes"]
    assert fp > 24 * lp.nnz


def test_tuned_layout_builds_both_on_the_host():
    """spmv_layout 2 lays out both product forms (panels and row tiles) at create; the
    choice between them is made on the device, so a deferred handle reports none yet."""
    lp = synth.cfg0(0)
    with lpg.Solver(lp, deferred=1, spmv_layout=lpg.LP_LAYOUT_TUNED) as s:
        L = s.layout()
    with lpg.Solver(lp, deferred=1, spmv_layout=lpg.LP_LAYOUT_TILES) as s:
        T = s.layout()
    assert L["units_a"] > 0 and L["units_at"] > 0 and L["tiles_a"] == T["tiles_a"]
    assert T["units_a"] == 0 and L["device_bytes"] > T["device_bytes"]
    assert L["layout"] == -1 and L["trial_ns_panels"] == 0 and L["trial_ns_tiles"] == 0


def test_library_has_no_unresolved_internal_symbols():
    """Every function of the library's own namespace that one source file calls and another
    defines is resolved inside the shared object (a lazily bound miss would only fail at
    its first call, on the device path)."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    path = lpg.lib()._name
    out = subprocess.run(["nm", "-D", "--undefined-only", "-C", path], capture_output=True, text=True, check=True)
    assert "lpgpu::" not in out.stdout, out.stdout


def test_default_options_match_the_header():
    """lp_default_options fills in the defaults that include/lp.h documents for each field."""
    o = lpg.lp_default_options()
    expected = dict(eps_rel=1e-4, max_iters=100000, time_limit_s=0.0, eval_every=64,
                    precision=lpg.LP_PREC_FP64, scaling=1, ruiz_passes=10, pow_iters=200, restarts=1,
                    step_size=0.0, omega0=0.0, device=0, trace_cap=4096, spmv_layout=0, long_row_len=256,
                    units_per_cu=4, batch_wg_per_cu=3, panel_slice_bytes=512 * 1024, batch_split_nnz=20000,
                    deferred=0, eps_infeas=1e-8, method=lpg.LP_METHOD_AVERAGED, reflection=1.0,
                    omega_steps=0, pw_rule=lpg.LP_PW_DEFAULT, pid_kp=0.7, pid_ki=0.05, pid_kd=0.2, tile_nnz=0,
                    small_lp_lds=112 * 1024)
    for k, v in expected.items():
        assert getattr(o, k) == v, (k, getattr(o, k), v)


PRESET_FIELDS = {
    "default": {},
    "small": dict(spmv_layout=lpg.LP_LAYOUT_TILES, method=lpg.LP_METHOD_HALPERN),
    "large": dict(spmv_layout=lpg.LP_LAYOUT_PANELS, method=lpg.LP_METHOD_HALPERN),
    "large_fp32": dict(spmv_layout=lpg.LP_LAYOUT_PANELS, method=lpg.LP_METHOD_HALPERN,
                       precision=lpg.LP_PREC_FP32_REFINED),
    "batch": dict(spmv_layout=lpg.LP_LAYOUT_TILES, method=lpg.LP_METHOD_HALPERN, precision=lpg.LP_PREC_FP32_REFINED),
    "serving": dict(spmv_layout=lpg.LP_LAYOUT_TILES, method=lpg.LP_METHOD_HALPERN,
                    precision=lpg.LP_PREC_FP32_REFINED, deferred=1),
}


@pytest.mark.parametrize("name", sorted(PRESET_FIELDS))
def test_presets_are_the_defaults_plus_their_fields(name):
    """Every preset is lp_default_options with the fields include/lp.h lists for it."""
    o = lpg.lp_preset_options(name)
    d = lpg.lp_default_options()
    for k, _ in lpg.lp_options._fields_:
        want = PRESET_FIELDS[name].get(k, getattr(d, k))
        assert getattr(o, k) == want, (name, k, getattr(o, k), want)
    s = lpg.make_options(preset=name, eps_rel=1e-6)  # the binding's helper starts from the preset
    assert s.eps_rel == 1e-6 and s.spmv_layout == o.spmv_layout and s.precision == o.precision


def test_unknown_preset_is_rejected():
    import ctypes as C

    o = lpg.lp_default_options()
    o.eps_rel = 0.5
    for bad in (-1, 6, 99):
        assert lpg.lib().lp_preset_options(C.byref(o), bad) == 1  # LP_ERR_INVALID_ARG
        assert o.eps_rel == 0.5  # left unchanged
    assert lpg.lib().lp_preset_options(None, 1) == 1  # LP_ERR_INVALID_ARG


def test_presolve_default_options_match_the_header():
    o = lpg.lp_presolve_options()
    lpg.lib().lp_presolve_default_options(__import__("ctypes").byref(o))
    expected = dict(max_rounds=32, dual_reductions=1, substitute=1, doubletons=1, feas_tol=1e-9, pivot_tol=1e-3)
    for k, v in expected.items():
        assert getattr(o, k) == v, (k, getattr(o, k), v)


@pytest.mark.parametrize("struct", ["lp_options", "lp_info", "lp_server_stats", "lp_presolve_options",
                                    "lp_presolve_info"])
def test_binding_structs_match_the_header(tmp_path, struct):
    """The binding's ctypes structures have the size and field offsets of the C structs of
    include/lp.h (compiled with the host C compiler)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    cls = getattr(lpg, struct)
    fields = [f[0] for f in cls._fields_ if not f[0].startswith("pad")]
    lines = [f'printf("%zu\\n", sizeof({struct}));']
    lines += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = tmp_path / "probe.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lp.h"\nint main(void) {\n'
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    import ctypes
    assert out[0] == ctypes.sizeof(cls), (struct, out[0], ctypes.sizeof(cls))
    for f, off in zip(fields, out[1:]):
        assert getattr(cls, f).offset == off, (struct, f, getattr(cls, f).offset, off)


def test_entry_count_bound():
    """nnz above 2^31 - 2^16 - 1 is rejected before any array is read (the kernels form entry
    offsets in 32 bits and prefetch a few thousand entries past a unit's end); at the bound
    the size check passes and validation goes on to the arrays."""
    import ctypes
    L = lpg.lib()
    bound = 2**31 - 2**16 - 1
    rp = np.array([0, 1], np.int32)
    ci = np.zeros(1, np.int32)
    v = np.ones(1)
    c = np.zeros(2)
    bl, bu = np.zeros(1), np.ones(1)
    xl, xu = np.zeros(2), np.ones(2)
    h = ctypes.c_void_p()
    args = lambda nnz: (ctypes.byref(h), 1, 2, nnz, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, c.ctypes.data,
                        0.0, bl.ctypes.data, bu.ctypes.data, xl.ctypes.data, xu.ctypes.data, None)
    assert L.lp_create(*args(bound + 1)) == 1
    assert "2^31" in lpg.lp_last_error()
    assert L.lp_create(*args(bound)) == 2  # size accepted; row_ptr[m] != nnz
    p = ctypes.c_void_p()
    assert L.lp_presolve(ctypes.byref(p), 1, 2, bound + 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                         c.ctypes.data, 0.0, bl.ctypes.data, bu.ctypes.data, xl.ctypes.data, xu.ctypes.data,
                         None, None) == 1
