// Lightweight host presolve and postsolve (the paper's Section 3), built from the atomic
// reductions of Section 2.1:
//   - fix a variable (and substitute its value into the rows and the objective),
//   - remove a constraint,
//   - change bounds (of a variable, or drop the redundant side of a row),
//   - substitute a variable out through an equality row,
// driven by the fast explorers of Section 3.1 (Table 1): empty and singleton rows, redundant
// rows and row sides by minimum / maximum activity (the redundant-constraint explorer of
// Section 2.2), empty and fixed columns, column singletons of equality rows, doubleton
// equality rows (Table 1; here only those whose substitution adds no nonzero), and variable
// locks (Section 2.3); the activities, counts and locks are the internal statistics of
// Section 3.2. Every reduction pushes a postsolve record;
// lp_postsolve replays the records in reverse and maps a solution of the reduced LP to
// (x, y, z) of the original one (eq. 2). Sequential CPU code: no device is touched.
//
// Data: the original CSR and its CSC copy keep their structure; rows and columns are switched
// off as they leave the problem (no reduction here adds nonzeros; a doubleton substitution
// changes values of existing entries in both copies), and the active row and column
// counts are kept up to date. Explorers run in rounds over all active rows and columns until
// a round changes nothing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "lp.h"
#include "lp_check.h"

namespace {

constexpr double kInf = HUGE_VAL;

enum RecKind : int { kDelRow = 0, kSingletonRow = 1, kFixCol = 2, kSubstCol = 3, kDoubleton = 4 };

// One postsolve record. Entry lists (rows of a fixed column, columns of a substituted row)
// live in the presolver's shared idx / val arrays at [off, off + len).
struct Rec {
    int kind;
    int i;          // row
    int k;          // column
    int j;          // doubleton: the column that stays
    double a;       // a_ik (singleton row, substitution, doubleton)
    double aj;      // doubleton: a_ij
    double v;       // fixed value (fix), equality right-hand side (substitution)
    double ck;      // cost of column k when the reduction was applied
    int from_row;   // singleton row: bit 0 = new lower bound of x_k came from the row, bit 1 = upper;
                    // doubleton: the same for x_j's bounds taken from x_k's
    int64_t off;
    int64_t len;
};

}  // namespace

struct lp_presolver {
    int m0 = 0, n0 = 0;
    std::vector<int32_t> rp, ci, cp, ri;
    std::vector<double> av, cv;
    std::vector<double> c, lo, hi, lb, ub;
    double c0 = 0.0;
    std::vector<char> row_on, col_on;
    std::vector<int32_t> row_cnt, col_cnt;
    std::vector<Rec> recs;
    std::vector<int32_t> rec_idx;
    std::vector<double> rec_val;
    lp_presolve_options opt{};
    lp_presolve_info info{};
    int status = LP_PRESOLVE_REDUCED;
    // reduced problem
    std::vector<int32_t> row_map, col_map;  // reduced index -> original index
    std::vector<int32_t> row_new, col_new;  // original index -> reduced index or -1
    int64_t red_nnz = 0;
};

namespace {

bool finite(double v) { return std::isfinite(v); }

// a * bound with the convention 0 * inf = 0.
double mul_bound(double a, double b) {
    if (a == 0.0) return 0.0;
    return a * b;
}

struct Activity {
    double min_fin = 0.0, max_fin = 0.0;  // sums of the finite contributions
    int min_inf = 0, max_inf = 0;         // number of infinite contributions
    double min() const { return min_inf ? -kInf : min_fin; }
    double max() const { return max_inf ? kInf : max_fin; }
};

class Presolve {
public:
    explicit Presolve(lp_presolver& P) : P(P) {}

    void run() {
        const int max_rounds = P.opt.max_rounds > 0 ? P.opt.max_rounds : 32;
        for (int round = 0; round < max_rounds && P.status == LP_PRESOLVE_REDUCED; ++round) {
            changed = false;
            rows_pass();
            if (P.status != LP_PRESOLVE_REDUCED) break;
            cols_pass();
            if (P.status != LP_PRESOLVE_REDUCED) break;
            if (P.opt.substitute) substitution_pass();
            if (P.status != LP_PRESOLVE_REDUCED) break;
            if (P.opt.doubletons) doubleton_pass();
            if (P.status != LP_PRESOLVE_REDUCED) break;
            activity_pass();
            if (P.status != LP_PRESOLVE_REDUCED) break;
            if (P.opt.dual_reductions) lock_pass();
            P.info.rounds = round + 1;
            if (!changed) break;
        }
    }

private:
    lp_presolver& P;
    bool changed = false;

    double tol() const { return P.opt.feas_tol > 0 ? P.opt.feas_tol : 1e-9; }

    // The counts are of active nonzero entries: an explicit zero, or an entry that a
    // substitution cancels to zero, counts nowhere.
    void remove_row(int i) {
        P.row_on[i] = 0;
        for (int e = P.rp[i]; e < P.rp[i + 1]; ++e)
            if (P.col_on[P.ci[e]] && P.av[e] != 0.0) --P.col_cnt[P.ci[e]];
        changed = true;
    }

    void remove_col(int k) {
        P.col_on[k] = 0;
        for (int e = P.cp[k]; e < P.cp[k + 1]; ++e)
            if (P.row_on[P.ri[e]] && P.cv[e] != 0.0) --P.row_cnt[P.ri[e]];
        changed = true;
    }

    // Fix x_k = v: substitute into the active rows and the objective, record the active
    // column entries so that postsolve can form z_k = c_k - a_k^T y.
    void fix_col(int k, double v) {
        Rec r{};
        r.kind = kFixCol;
        r.k = k;
        r.v = v;
        r.ck = P.c[k];
        r.off = static_cast<int64_t>(P.rec_idx.size());
        for (int e = P.cp[k]; e < P.cp[k + 1]; ++e) {
            const int i = P.ri[e];
            if (!P.row_on[i]) continue;
            const double a = P.cv[e];
            P.rec_idx.push_back(i);
            P.rec_val.push_back(a);
            const double s = a * v;
            if (finite(P.lo[i])) P.lo[i] -= s;
            if (finite(P.hi[i])) P.hi[i] -= s;
        }
        r.len = static_cast<int64_t>(P.rec_idx.size()) - r.off;
        P.c0 += P.c[k] * v;
        P.recs.push_back(r);
        remove_col(k);
    }

    void del_row(int i) {
        Rec r{};
        r.kind = kDelRow;
        r.i = i;
        P.recs.push_back(r);
        remove_row(i);
    }

    void infeasible() { P.status = LP_PRESOLVE_INFEASIBLE; }

    // Empty rows (feasibility check, removal) and singleton rows (bounds on the variable).
    void rows_pass() {
        for (int i = 0; i < P.m0; ++i) {
            if (!P.row_on[i]) continue;
            if (P.row_cnt[i] == 0) {
                if (P.lo[i] > tol() || P.hi[i] < -tol()) return infeasible();
                ++P.info.empty_rows;
                del_row(i);
            } else if (P.row_cnt[i] == 1) {
                int e = P.rp[i];
                while (!P.col_on[P.ci[e]] || P.av[e] == 0.0) ++e;
                const int k = P.ci[e];
                const double a = P.av[e];
                double ilb = a > 0 ? P.lo[i] / a : P.hi[i] / a;
                double iub = a > 0 ? P.hi[i] / a : P.lo[i] / a;
                if (std::isnan(ilb)) ilb = -kInf;
                if (std::isnan(iub)) iub = kInf;
                Rec r{};
                r.kind = kSingletonRow;
                r.i = i;
                r.k = k;
                r.a = a;
                if (ilb > P.lb[k]) {
                    P.lb[k] = ilb;
                    r.from_row |= 1;
                }
                if (iub < P.ub[k]) {
                    P.ub[k] = iub;
                    r.from_row |= 2;
                }
                if (P.lb[k] > P.ub[k]) {
                    if (P.lb[k] - P.ub[k] > tol() * (1.0 + std::fabs(P.ub[k]))) return infeasible();
                    // equal up to rounding: meet in the middle of the two bounds
                    const double mid = 0.5 * (P.lb[k] + P.ub[k]);
                    P.lb[k] = P.ub[k] = mid;
                }
                ++P.info.singleton_rows;
                P.recs.push_back(r);
                remove_row(i);
            }
        }
    }

    // Empty columns (fixed at the bound their cost prefers) and fixed columns (lb = ub).
    void cols_pass() {
        for (int k = 0; k < P.n0; ++k) {
            if (!P.col_on[k]) continue;
            if (P.col_cnt[k] == 0) {
                double v;
                if (P.c[k] > 0) {
                    if (!finite(P.lb[k])) {
                        P.status = LP_PRESOLVE_UNBOUNDED;
                        return;
                    }
                    v = P.lb[k];
                } else if (P.c[k] < 0) {
                    if (!finite(P.ub[k])) {
                        P.status = LP_PRESOLVE_UNBOUNDED;
                        return;
                    }
                    v = P.ub[k];
                } else {
                    v = std::min(std::max(0.0, P.lb[k]), P.ub[k]);
                }
                ++P.info.empty_cols;
                fix_col(k, v);
            } else if (P.lb[k] == P.ub[k]) {
                ++P.info.fixed_cols;
                fix_col(k, P.lb[k]);
            }
        }
    }

    // A column k whose only active entry is in an equality row i: x_k = (b - sum_j a_ij x_j) / a_ik.
    // Its cost is moved onto the other columns of the row and the offset, the column leaves,
    // and the row keeps the other columns with the bounds that x_k's bounds imply.
    void substitution_pass() {
        const double ptol = P.opt.pivot_tol > 0 ? P.opt.pivot_tol : 1e-3;
        for (int k = 0; k < P.n0; ++k) {
            if (!P.col_on[k] || P.col_cnt[k] != 1) continue;
            int e = P.cp[k];
            while (!P.row_on[P.ri[e]] || P.cv[e] == 0.0) ++e;
            const int i = P.ri[e];
            const double a = P.cv[e];
            if (!(P.lo[i] == P.hi[i]) || P.row_cnt[i] < 2) continue;
            double amax = 0.0;
            for (int f = P.rp[i]; f < P.rp[i + 1]; ++f)
                if (P.col_on[P.ci[f]]) amax = std::max(amax, std::fabs(P.av[f]));
            if (std::fabs(a) < ptol * amax) continue;
            const double b = P.lo[i];
            Rec r{};
            r.kind = kSubstCol;
            r.i = i;
            r.k = k;
            r.a = a;
            r.v = b;
            r.ck = P.c[k];
            r.off = static_cast<int64_t>(P.rec_idx.size());
            const double ratio = P.c[k] / a;
            for (int f = P.rp[i]; f < P.rp[i + 1]; ++f) {
                const int j = P.ci[f];
                if (j == k || !P.col_on[j]) continue;
                P.rec_idx.push_back(j);
                P.rec_val.push_back(P.av[f]);
                P.c[j] -= ratio * P.av[f];
            }
            r.len = static_cast<int64_t>(P.rec_idx.size()) - r.off;
            P.c0 += ratio * b;
            // sum_{j != k} a_ij x_j = b - a x_k with x_k in [lb_k, ub_k]
            const double t1 = b - mul_bound(a, P.lb[k]);
            const double t2 = b - mul_bound(a, P.ub[k]);
            P.lo[i] = std::min(t1, t2);
            P.hi[i] = std::max(t1, t2);
            if (std::isnan(P.lo[i])) P.lo[i] = -kInf;
            if (std::isnan(P.hi[i])) P.hi[i] = kInf;
            ++P.info.substituted_cols;
            P.recs.push_back(r);
            remove_col(k);
        }
    }

    // Adds d to the entry (q, j), which exists, in the CSR and the CSC copy (both hold the
    // same value). An entry that becomes exactly zero leaves the counts of its row and
    // column (and the reduced LP); one that becomes nonzero joins them.
    void add_to_entry(int q, int j, double d) {
        double before = 0.0, after = 0.0;
        for (int e = P.rp[q]; e < P.rp[q + 1]; ++e)
            if (P.ci[e] == j) {
                before = P.av[e];
                P.av[e] += d;
                after = P.av[e];
                break;
            }
        for (int e = P.cp[j]; e < P.cp[j + 1]; ++e)
            if (P.ri[e] == q) {
                P.cv[e] = after;
                break;
            }
        if ((before != 0.0) != (after != 0.0)) {
            const int step = after != 0.0 ? 1 : -1;
            P.row_cnt[q] += step;
            P.col_cnt[j] += step;
            ++P.info.cancelled_entries;
        }
    }

    // True when every active row other than i that holds a nonzero of column k also holds
    // column j, so that substituting x_k through row i adds no nonzero.
    bool no_fill(int i, int k, int j) const {
        for (int e = P.cp[k]; e < P.cp[k + 1]; ++e) {
            const int q = P.ri[e];
            if (q == i || !P.row_on[q] || P.cv[e] == 0.0) continue;
            bool has = false;
            for (int f = P.rp[q]; f < P.rp[q + 1] && !has; ++f) has = P.ci[f] == j;
            if (!has) return false;
        }
        return true;
    }

    // Doubleton equality row i: a_ij x_j + a_ik x_k = b, so x_k = beta - alpha x_j with
    // alpha = a_ij / a_ik, beta = b / a_ik. Every other row q with x_k gets a_qj -= a_qk alpha
    // and its sides shifted by a_qk beta; c_j -= c_k alpha and the offset gains c_k beta; the
    // bounds of x_k become bounds of x_j; row i and column k leave.
    void eliminate_doubleton(int i, int k, int j, double ak, double aj) {
        const double b = P.lo[i];
        const double alpha = aj / ak, beta = b / ak;
        Rec r{};
        r.kind = kDoubleton;
        r.i = i;
        r.k = k;
        r.j = j;
        r.a = ak;
        r.aj = aj;
        r.v = b;
        r.ck = P.c[k];
        r.off = static_cast<int64_t>(P.rec_idx.size());
        for (int e = P.cp[k]; e < P.cp[k + 1]; ++e) {
            const int q = P.ri[e];
            if (q == i || !P.row_on[q]) continue;
            const double aqk = P.cv[e];
            P.rec_idx.push_back(q);
            P.rec_val.push_back(aqk);
            if (aqk == 0.0) continue;
            add_to_entry(q, j, -aqk * alpha);
            const double s = aqk * beta;
            if (finite(P.lo[q])) P.lo[q] -= s;
            if (finite(P.hi[q])) P.hi[q] -= s;
        }
        r.len = static_cast<int64_t>(P.rec_idx.size()) - r.off;
        P.c[j] -= P.c[k] * alpha;
        P.c0 += P.c[k] * beta;
        // x_k = beta - alpha x_j in [lb_k, ub_k]
        const double l = alpha > 0 ? (beta - P.ub[k]) / alpha : (beta - P.lb[k]) / alpha;
        const double u = alpha > 0 ? (beta - P.lb[k]) / alpha : (beta - P.ub[k]) / alpha;
        if (l > P.lb[j]) {
            P.lb[j] = l;
            r.from_row |= 1;
        }
        if (u < P.ub[j]) {
            P.ub[j] = u;
            r.from_row |= 2;
        }
        if (P.lb[j] > P.ub[j]) {
            if (P.lb[j] - P.ub[j] > tol() * (1.0 + std::fabs(P.ub[j]))) return infeasible();
            const double mid = 0.5 * (P.lb[j] + P.ub[j]);
            P.lb[j] = P.ub[j] = mid;
        }
        ++P.info.doubleton_cols;
        P.recs.push_back(r);
        remove_row(i);
        remove_col(k);
    }

    // Doubleton equality rows (Table 1) whose substitution adds no nonzero: the column with
    // fewer entries is eliminated if its pivot passes the pivot tolerance and no fill-in
    // arises, else the other one under the same conditions.
    void doubleton_pass() {
        const double ptol = P.opt.pivot_tol > 0 ? P.opt.pivot_tol : 1e-3;
        for (int i = 0; i < P.m0 && P.status == LP_PRESOLVE_REDUCED; ++i) {
            if (!P.row_on[i] || P.row_cnt[i] != 2 || !(P.lo[i] == P.hi[i]) || !finite(P.lo[i])) continue;
            int e1 = -1, e2 = -1;
            for (int e = P.rp[i]; e < P.rp[i + 1]; ++e)
                if (P.col_on[P.ci[e]] && P.av[e] != 0.0) (e1 < 0 ? e1 : e2) = e;
            if (e2 < 0) continue;
            int cand[2] = {e1, e2};
            if (P.col_cnt[P.ci[e2]] < P.col_cnt[P.ci[e1]]) std::swap(cand[0], cand[1]);
            for (int t = 0; t < 2; ++t) {
                const int ek = cand[t], ej = cand[1 - t];
                const int k = P.ci[ek], j = P.ci[ej];
                const double ak = P.av[ek], aj = P.av[ej];
                if (std::fabs(ak) < ptol * std::max(std::fabs(ak), std::fabs(aj))) continue;
                if (!no_fill(i, k, j)) continue;
                eliminate_doubleton(i, k, j, ak, aj);
                break;
            }
        }
    }

    Activity activity(int i) const {
        Activity A;
        for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
            const int j = P.ci[e];
            if (!P.col_on[j]) continue;
            const double a = P.av[e];
            if (a == 0.0) continue;
            const double lo_c = a > 0 ? P.lb[j] : P.ub[j];  // the bound giving the minimum
            const double hi_c = a > 0 ? P.ub[j] : P.lb[j];
            if (finite(lo_c)) A.min_fin += a * lo_c; else ++A.min_inf;
            if (finite(hi_c)) A.max_fin += a * hi_c; else ++A.max_inf;
        }
        return A;
    }

    // Redundant rows and row sides from the minimum / maximum activity (the
    // redundant-constraint explorer of Section 2.2); rows that no point satisfies make the LP
    // infeasible.
    void activity_pass() {
        for (int i = 0; i < P.m0; ++i) {
            if (!P.row_on[i] || P.row_cnt[i] < 2) continue;
            const Activity A = activity(i);
            const double amin = A.min(), amax = A.max();
            const double scale = 1.0 + std::max(std::fabs(finite(P.lo[i]) ? P.lo[i] : 0.0),
                                                std::fabs(finite(P.hi[i]) ? P.hi[i] : 0.0));
            if (amin > P.hi[i] + tol() * scale || amax < P.lo[i] - tol() * scale) return infeasible();
            const bool lo_red = !finite(P.lo[i]) || amin >= P.lo[i];
            const bool hi_red = !finite(P.hi[i]) || amax <= P.hi[i];
            if (lo_red && hi_red) {
                ++P.info.redundant_rows;
                del_row(i);
            } else if (lo_red && finite(P.lo[i])) {
                P.lo[i] = -kInf;
                ++P.info.dropped_sides;
                changed = true;
            } else if (hi_red && finite(P.hi[i])) {
                P.hi[i] = kInf;
                ++P.info.dropped_sides;
                changed = true;
            }
        }
    }

    // Variable locks: a row locks x_k upward if it stops x_k from growing (a_ik > 0 with a
    // finite upper side, or a_ik < 0 with a finite lower side) and downward symmetrically.
    // A variable whose cost pushes it toward an unlocked direction sits at that bound in every
    // optimal solution (weak dual reduction); with zero cost it may be put there (strong).
    void lock_pass() {
        std::vector<int32_t> up(P.n0, 0), down(P.n0, 0);
        for (int i = 0; i < P.m0; ++i) {
            if (!P.row_on[i]) continue;
            const bool fl = finite(P.lo[i]), fh = finite(P.hi[i]);
            for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
                const int j = P.ci[e];
                if (!P.col_on[j] || P.av[e] == 0.0) continue;
                if (P.av[e] > 0) {
                    up[j] += fh;
                    down[j] += fl;
                } else {
                    up[j] += fl;
                    down[j] += fh;
                }
            }
        }
        for (int k = 0; k < P.n0; ++k) {
            if (!P.col_on[k]) continue;
            const double ck = P.c[k];
            if (ck > 0 && down[k] == 0) {
                if (!finite(P.lb[k])) {
                    P.status = LP_PRESOLVE_UNBOUNDED;
                    return;
                }
                ++P.info.lock_fixed_cols;
                fix_col(k, P.lb[k]);
            } else if (ck < 0 && up[k] == 0) {
                if (!finite(P.ub[k])) {
                    P.status = LP_PRESOLVE_UNBOUNDED;
                    return;
                }
                ++P.info.lock_fixed_cols;
                fix_col(k, P.ub[k]);
            } else if (ck == 0) {
                if (down[k] == 0 && up[k] == 0) {
                    ++P.info.lock_fixed_cols;
                    fix_col(k, std::min(std::max(0.0, P.lb[k]), P.ub[k]));
                } else if (down[k] == 0 && finite(P.lb[k])) {
                    ++P.info.lock_fixed_cols;
                    fix_col(k, P.lb[k]);
                } else if (up[k] == 0 && finite(P.ub[k])) {
                    ++P.info.lock_fixed_cols;
                    fix_col(k, P.ub[k]);
                }
            }
        }
    }
};

void build_reduced(lp_presolver& P) {
    P.row_new.assign(P.m0, -1);
    P.col_new.assign(P.n0, -1);
    P.row_map.clear();
    P.col_map.clear();
    for (int i = 0; i < P.m0; ++i)
        if (P.row_on[i]) {
            P.row_new[i] = static_cast<int32_t>(P.row_map.size());
            P.row_map.push_back(i);
        }
    for (int k = 0; k < P.n0; ++k)
        if (P.col_on[k]) {
            P.col_new[k] = static_cast<int32_t>(P.col_map.size());
            P.col_map.push_back(k);
        }
    int64_t nnz = 0;
    for (int i : P.row_map)
        for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) nnz += P.col_on[P.ci[e]] && P.av[e] != 0.0 ? 1 : 0;
    P.red_nnz = nnz;
    P.info.m = static_cast<int32_t>(P.row_map.size());
    P.info.n = static_cast<int32_t>(P.col_map.size());
    P.info.nnz = nnz;
    if (P.status == LP_PRESOLVE_REDUCED && P.info.n == 0) P.status = LP_PRESOLVE_SOLVED;
    P.info.status = P.status;
}

int32_t fail(int32_t code, const std::string& msg) {
    lpgpu::set_last_error(msg);
    return code;
}

}  // namespace

extern "C" {

void lp_presolve_default_options(lp_presolve_options* opt) {
    if (!opt) return;
    opt->max_rounds = 32;
    opt->dual_reductions = 1;
    opt->substitute = 1;
    opt->doubletons = 1;
    opt->feas_tol = 1e-9;
    opt->pivot_tol = 1e-3;
}

int32_t lp_presolve(lp_presolver** out, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                    const int32_t* col_idx, const double* vals, const double* c, double c0, const double* b_lo,
                    const double* b_hi, const double* x_lo, const double* x_hi, const lp_presolve_options* opt,
                    lp_presolve_info* info) {
    if (!out) return fail(LP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::string msg;
    if (int32_t rc = lpgpu::validate_lp(m, n, nnz, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi, &msg))
        return fail(rc, msg);
    try {
        const auto t0 = std::chrono::steady_clock::now();
        auto* P = new lp_presolver();
        std::unique_ptr<lp_presolver> guard(P);
        lp_presolve_default_options(&P->opt);
        if (opt) P->opt = *opt;
        if (P->opt.max_rounds < 0 || !(P->opt.feas_tol >= 0) || !(P->opt.pivot_tol >= 0))
            return fail(LP_ERR_INVALID_ARG, "presolve options out of range");
        P->m0 = m;
        P->n0 = n;
        P->rp.assign(row_ptr, row_ptr + m + 1);
        P->ci.assign(col_idx, col_idx + nnz);
        P->av.assign(vals, vals + nnz);
        P->c.assign(c, c + n);
        P->c0 = c0;
        P->lo.assign(b_lo, b_lo + m);
        P->hi.assign(b_hi, b_hi + m);
        P->lb.assign(x_lo, x_lo + n);
        P->ub.assign(x_hi, x_hi + n);
        // CSC copy (stable counting sort: rows ascend inside a column)
        P->cp.assign(n + 1, 0);
        for (int64_t e = 0; e < nnz; ++e) ++P->cp[col_idx[e] + 1];
        for (int k = 0; k < n; ++k) P->cp[k + 1] += P->cp[k];
        P->ri.resize(nnz);
        P->cv.resize(nnz);
        {
            std::vector<int32_t> next(P->cp.begin(), P->cp.end() - 1);
            for (int i = 0; i < m; ++i)
                for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    const int32_t p = next[col_idx[e]]++;
                    P->ri[p] = i;
                    P->cv[p] = vals[e];
                }
        }
        P->row_on.assign(m, 1);
        P->col_on.assign(n, 1);
        P->row_cnt.resize(m);
        P->col_cnt.resize(n);
        for (int i = 0; i < m; ++i) {
            P->row_cnt[i] = 0;
            for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) P->row_cnt[i] += vals[e] != 0.0;
        }
        for (int k = 0; k < n; ++k) {
            P->col_cnt[k] = 0;
            for (int e = P->cp[k]; e < P->cp[k + 1]; ++e) P->col_cnt[k] += P->cv[e] != 0.0;
        }
        Presolve(*P).run();
        build_reduced(*P);
        P->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = P->info;
        *out = guard.release();
        return LP_OK;
    } catch (const std::bad_alloc&) {
        return fail(LP_ERR_OUT_OF_MEMORY, "host allocation failed in presolve");
    } catch (const std::exception& ex) {
        return fail(LP_ERR_INTERNAL, ex.what());
    }
}

int32_t lp_presolve_get_info(const lp_presolver* p, lp_presolve_info* info) {
    if (!p || !info) return fail(LP_ERR_INVALID_ARG, "NULL argument");
    *info = p->info;
    return LP_OK;
}

int32_t lp_presolve_get_reduced(const lp_presolver* p, int32_t* row_ptr, int32_t* col_idx, double* vals, double* c,
                                double* c0, double* b_lo, double* b_hi, double* x_lo, double* x_hi) {
    if (!p) return fail(LP_ERR_INVALID_ARG, "presolver is NULL");
    const lp_presolver& P = *p;
    const int mr = P.info.m, nr = P.info.n;
    if (!row_ptr || (P.red_nnz > 0 && (!col_idx || !vals)) || (nr > 0 && (!c || !x_lo || !x_hi)) ||
        (mr > 0 && (!b_lo || !b_hi)) || !c0)
        return fail(LP_ERR_INVALID_ARG, "a required output array is NULL");
    int64_t e_out = 0;
    row_ptr[0] = 0;
    for (int r = 0; r < mr; ++r) {
        const int i = P.row_map[r];
        for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
            const int k = P.ci[e];
            if (!P.col_on[k] || P.av[e] == 0.0) continue;
            col_idx[e_out] = P.col_new[k];
            vals[e_out] = P.av[e];
            ++e_out;
        }
        row_ptr[r + 1] = static_cast<int32_t>(e_out);
        b_lo[r] = P.lo[i];
        b_hi[r] = P.hi[i];
    }
    for (int j = 0; j < nr; ++j) {
        const int k = P.col_map[j];
        c[j] = P.c[k];
        x_lo[j] = P.lb[k];
        x_hi[j] = P.ub[k];
    }
    *c0 = P.c0;
    return LP_OK;
}

int32_t lp_presolve_get_maps(const lp_presolver* p, int32_t* row_map, int32_t* col_map) {
    if (!p) return fail(LP_ERR_INVALID_ARG, "presolver is NULL");
    if ((p->info.m > 0 && !row_map) || (p->info.n > 0 && !col_map)) return fail(LP_ERR_INVALID_ARG, "NULL map");
    std::copy(p->row_map.begin(), p->row_map.end(), row_map);
    std::copy(p->col_map.begin(), p->col_map.end(), col_map);
    return LP_OK;
}

int32_t lp_postsolve(const lp_presolver* p, const double* x, const double* y, const double* z, double* x_out,
                     double* y_out, double* z_out) {
    if (!p) return fail(LP_ERR_INVALID_ARG, "presolver is NULL");
    const lp_presolver& P = *p;
    if (P.status == LP_PRESOLVE_INFEASIBLE || P.status == LP_PRESOLVE_UNBOUNDED)
        return fail(LP_ERR_INVALID_ARG, "presolve found no reduced LP to postsolve");
    if ((P.info.n > 0 && (!x || !z)) || (P.info.m > 0 && !y) || !x_out || !z_out || (P.m0 > 0 && !y_out))
        return fail(LP_ERR_INVALID_ARG, "a required array is NULL");
    try {
        std::vector<double> X(P.n0, 0.0), Y(P.m0, 0.0), Z(P.n0, 0.0);
        for (int j = 0; j < P.info.n; ++j) {
            X[P.col_map[j]] = x[j];
            Z[P.col_map[j]] = z[j];
        }
        for (int r = 0; r < P.info.m; ++r) Y[P.row_map[r]] = y[r];
        for (auto it = P.recs.rbegin(); it != P.recs.rend(); ++it) {
            const Rec& R = *it;
            switch (R.kind) {
                case kDelRow:
                    Y[R.i] = 0.0;
                    break;
                case kSingletonRow: {
                    // The row gave x_k the bound its multiplier belongs to: move z_k onto y_i.
                    const double zk = Z[R.k];
                    Y[R.i] = 0.0;
                    if ((zk > 0 && (R.from_row & 1)) || (zk < 0 && (R.from_row & 2))) {
                        Y[R.i] = zk / R.a;
                        Z[R.k] = 0.0;
                    }
                    break;
                }
                case kFixCol: {
                    X[R.k] = R.v;
                    double s = R.ck;
                    for (int64_t q = R.off; q < R.off + R.len; ++q) s -= P.rec_val[q] * Y[P.rec_idx[q]];
                    Z[R.k] = s;
                    break;
                }
                case kDoubleton: {
                    // x_k from row i; then the multipliers: S_k = c_k - sum_q a_qk y_q over the
                    // other rows. If x_j rests on a bound it took from x_k, that multiplier is
                    // x_k's: z_j = 0, z_k = -(a_ik / a_ij) z_j', y_i = z_j' / a_ij + S_k / a_ik;
                    // otherwise z_k = 0 and y_i = S_k / a_ik (z_j is unchanged).
                    X[R.k] = (R.v - R.aj * X[R.j]) / R.a;
                    double sk = R.ck;
                    for (int64_t q = R.off; q < R.off + R.len; ++q) sk -= P.rec_val[q] * Y[P.rec_idx[q]];
                    const double zj = Z[R.j];
                    if ((zj > 0 && (R.from_row & 1)) || (zj < 0 && (R.from_row & 2))) {
                        Y[R.i] = zj / R.aj + sk / R.a;
                        Z[R.k] = -(R.a / R.aj) * zj;
                        Z[R.j] = 0.0;
                    } else {
                        Y[R.i] = sk / R.a;
                        Z[R.k] = 0.0;
                    }
                    break;
                }
                case kSubstCol: {
                    double s = R.v;
                    for (int64_t q = R.off; q < R.off + R.len; ++q) s -= P.rec_val[q] * X[P.rec_idx[q]];
                    X[R.k] = s / R.a;
                    const double yr = Y[R.i];
                    Y[R.i] = yr + R.ck / R.a;
                    Z[R.k] = -R.a * yr;
                    break;
                }
                default:
                    return fail(LP_ERR_INTERNAL, "unknown postsolve record");
            }
        }
        std::copy(X.begin(), X.end(), x_out);
        if (P.m0 > 0) std::copy(Y.begin(), Y.end(), y_out);
        std::copy(Z.begin(), Z.end(), z_out);
        return LP_OK;
    } catch (const std::bad_alloc&) {
        return fail(LP_ERR_OUT_OF_MEMORY, "host allocation failed in postsolve");
    }
}

void lp_presolve_destroy(lp_presolver* p) { delete p; }

}  // extern "C"
