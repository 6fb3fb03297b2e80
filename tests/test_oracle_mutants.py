"""The oracle's pins must catch plausible mistakes. Each mutant below plants one mistake in
a temporary copy of the oracle source (CPU only), and the quick pin subset must fail on it.

The restart cycle is covered by mutants of its implementation (candidate choice, primal-weight
update direction, the no-progress test, the anchor reset), and so are the fixed-point
residual restarts (the norm's coupling sign and weights, which iterate it is taken at, the
anchor's residual). Its constants (0.2, 0.8, 0.36) are
readings the paper does not fix, so no mutant changes them (parity unpinned for them)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pdhg_oracle.c")

MUTANTS = {
    "primal_step_sign": ("double xn = x - tau * g;", "double xn = x + tau * g;"),
    "no_extrapolation": ("double w = 2.0 * axn - ax;", "double w = axn;"),
    "dual_prox_sign": ("double lo = v + sigma * blo;", "double lo = v - sigma * blo;"),
    "swapped_sign_cone": ("else if (flo && !fhi) zs = ls > 0.0 ? ls : 0.0;",
                          "else if (flo && !fhi) zs = ls < 0.0 ? ls : 0.0;"),
    "dropped_dual_bound_term": ("if (zo > 0.0) dobj += P->oxlo[k] * zo;", "if (zo > 0.0) dobj += 0.0;"),
    "transpose_wrong_index": ("ciT[dst] = i;", "ciT[dst] = ci[e];"),
    "average_sign": ("xa[j] = xa[j] + wt * (x[j] - xa[j]);", "xa[j] = xa[j] + wt * (xa[j] - x[j]);"),
    "residual_swapped_bounds": ("double rs = ax[i] - clampd(ax[i], P->blo[i], P->bhi[i]);",
                                "double rs = ax[i] - clampd(ax[i], P->bhi[i], P->blo[i]);"),
    "scaling_exponent_sign": ("return ldexp(1.0, -h);", "return ldexp(1.0, h);"),
    "power_iteration_transposed_operand": ("csr_mv(n, rpT, ciT, vT, u, w);", "csr_mv(n, rp, ci, v, u, w);"),
    "power_iteration_fixed_count": ("if ((it + 1) % iters == 0 && sigma - prev <= 1e-8 * sigma) break;",
                                    "if ((it + 1) % iters == 0) break;"),
    "gap_denominator": ("K->rel_gap = fabs(p - d) / (1.0 + fabs(p) + fabs(d));",
                        "K->rel_gap = fabs(p - d) / (1.0 + fabs(p));"),
    "dual_residual_unscaled": ("double rdo = rds * P->Ci[k];", "double rdo = rds;"),
    "ray_objective_sign": ("if (zs > 0.0) D += P->oxlo[k] * zs;", "if (zs > 0.0) D -= P->oxlo[k] * zs;"),
    "ray_row_cone_side": ("else if (flo) w = v < 0.0 ? v : 0.0;", "else if (flo) w = v > 0.0 ? v : 0.0;"),
    "halpern_anchor_weight": ("double wk = (double)(t + 1) / (double)(t + 2);",
                              "double wk = (double)(t + 1) / (double)(t + 3);"),
    "halpern_reflection_sign": ("x[j] = wk * (r1 * xa[j] - rho * x[j]) + wa * xan[j];",
                                "x[j] = wk * (r1 * xa[j] + rho * x[j]) + wa * xan[j];"),
    "restart_candidate_inverted": ("int use_avg = halpern ? 1 : ka < kc;", "int use_avg = halpern ? 1 : ka > kc;"),
    "primal_weight_inverted": ("omega = sqrt((omega * dy) / dx);", "omega = sqrt((omega * dx) / dy);"),
    "restart_no_progress_flipped": ("kcand > kkt_prev) why = 2;", "kcand < kkt_prev) why = 2;"),
    "restart_anchor_not_reset": ("memcpy(xan, x, nb);", "(void)0;"),
    "pid_integral_not_accumulated": ("pid_int += e;", "pid_int = e;"),
    "pid_derivative_sign": ("o->pid_kd * (e - pid_prev);", "o->pid_kd * (pid_prev - e);"),
    "polish_stops_on_wrong_residual": ("if (mode == 1) return isnan(K->erel) ? NAN : K->rel_p;",
                                       "if (mode == 1) return isnan(K->erel) ? NAN : K->rel_d;"),
    "anchored_ray_from_previous_point": (
        "eval_rays(&P, xa, ya, axa, atya, xan, yan, axan, atyan, &Rray, NULL, NULL, NULL);",
        "eval_rays(&P, xa, ya, axa, atya, xp, yp, axp, atyp, &Rray, NULL, NULL, NULL);"),
    "anchor_products_not_moved": ("memcpy(atyan, atya, nb);", "(void)0;"),
    "residual_coupling_sign": ("double r2 = omega * s1 + 2.0 * eta * s2 + s3 / omega;",
                               "double r2 = omega * s1 - 2.0 * eta * s2 + s3 / omega;"),
    "residual_weights_swapped": ("double r2 = omega * s1 + 2.0 * eta * s2 + s3 / omega;",
                                 "double r2 = s1 / omega + 2.0 * eta * s2 + omega * s3;"),
    "residual_anchor_not_refreshed": ("if (t == 0) r_anchor = r;", "if (k == 0) r_anchor = r;"),
    "residual_from_first_iterate_of_period": ("(t == 0 || (k + 1) % o->eval_every == 0 || k + 1 >= o->max_iters)",
                                              "(t == 0 || k % o->eval_every == 0 || k + 1 >= o->max_iters)"),
    "residual_restarts_on_kkt": ("kc = ka = r_cur;", "(void)0;"),
}

QUICK = [
    "tests/test_oracle_pins.py",
    "tests/test_oracle_exact.py::test_linear_recurrence_all_free_equalities",
    "tests/test_oracle_exact.py::test_vertex_enumeration",
    "tests/test_oracle_exact.py::test_kkt_point_is_fixed_point",
    "tests/test_oracle_structure.py",
    "tests/test_oracle_infeasible.py",
    "tests/test_oracle_halpern.py",
    "tests/test_oracle_restarts.py",
    "tests/test_oracle_polish.py",
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    import oracle

    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut_src = tmp_path / "mutant.c"
    mut_src.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(mut_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *QUICK],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
