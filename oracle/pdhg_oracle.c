/*
 * Plain FP64 CPU oracle for restarted, averaged PDHG on the LP of the paper's
 * Section 2, eq. (1):  minimize c^T x + c0  s.t.  b_lo <= A x <= b_hi,  x_lo <= x <= x_hi.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct reference that the
 * GPU solver is checked against. Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load it. The solver library never includes, links or
 * calls it, and it shares no source with the solver.
 *
 * Single-threaded, every loop in index order, compiled with -ffp-contract=off so each
 * multiply and add is rounded on its own.
 *
 * What it follows:
 *  - The problem form and the sign conventions of the duals (y, z) are the paper's
 *    Section 2, eq. (1) and eq. (2), including its remarks that a free variable has z = 0,
 *    that b_lo = -inf forces y <= 0 and that b_hi = +inf forces y >= 0.
 *  - The reduced cost of a column is c_k - a_k^T y (Section 2.1, the dual postsolve of a
 *    fixed variable, which follows from the second line of eq. (2)).
 *  - Termination uses one relative tolerance (Section 4.2, the cuPDLPx setup).
 *  - The paper names PDHG (Zhu-Chan, Chambolle-Pock) and the PDLP family but does not spell
 *    the iteration out. The iteration, restarts, step size and primal weight below are the
 *    published averaged, restarted PDHG of that family, in the reading stated beside each
 *    function. The restart constants (0.2 / 0.8 / 0.36) and the evaluation period are
 *    heuristics the paper does not fix: parity unpinned for them. The implementation of the
 *    restart cycle is pinned by the tests (a restart equals a fresh start at the candidate,
 *    every decision recomputed from the iterates, the primal-weight update balancing the
 *    weighted distances), and the power-of-two scaling by its exactness.
 *  - Method 1 is the reflected Halpern form of the same family (see ora_solve); the
 *    infeasibility certificates follow the remark after eq. (2) that an LP with no solution
 *    of eq. (2) is infeasible or unbounded (see eval_rays).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORA_OK 0
#define ORA_ERR_INVALID_ARG 1
#define ORA_ERR_INVALID_MATRIX 2
#define ORA_ERR_INCONSISTENT_BOUNDS 3
#define ORA_ERR_NAN_INPUT 4
#define ORA_ERR_OUT_OF_MEMORY 5

#define ORA_OPTIMAL 0
#define ORA_ITERATION_LIMIT 1
#define ORA_NUMERICAL_ERROR 2
#define ORA_PRIMAL_INFEASIBLE 3 /* a dual ray certifies that no x satisfies the constraints */
#define ORA_DUAL_INFEASIBLE 4   /* a primal ray certifies that the dual has no solution */

#define ORA_TRACE_W 12

typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr, *col_idx;
    const double *vals, *c;
    double c0;
    const double *b_lo, *b_hi, *x_lo, *x_hi;
} ora_lp;

typedef struct {
    double eps_rel;
    int64_t max_iters;
    int32_t eval_every;
    int32_t scaling;     /* 0: identity, 1: Ruiz passes then one Pock-Chambolle pass */
    int32_t ruiz_passes;
    int32_t pow_iters;
    int32_t restarts;    /* 1: restarts and primal-weight updates on; 0: plain averaged PDHG */
    int32_t pad0;
    double eta;          /* <= 0: 0.998 / sigma_hat */
    double omega0;       /* <= 0: ||c~|| / ||q~|| */
    uint64_t seed;       /* start vector of the power iteration */
    const double *x0, *y0; /* optional warm start, original space */
    int32_t n_snap, pad1;
    const int64_t *snap_k;
    double *snap_out;    /* per snapshot: x~[n], y~[m], x~avg[n], y~avg[m] */
    int32_t trace_cap, pad2;
    double *trace;       /* trace_cap * ORA_TRACE_W */
    double eps_infeas;   /* relative tolerance of the infeasibility certificates; 0: off */
    int32_t method;      /* 0: averaged PDHG; 1: reflected Halpern PDHG */
    int32_t restart_metric; /* what the restart tests compare in the Halpern form: 0 KKT_omega
                               of T(z), 1 the fixed-point residual ||z - T(z)|| in the PDHG
                               norm (ignored by the averaged form) */
    double reflection;   /* rho of the Halpern form, in [0, 1] */
    int32_t omega_steps; /* square-root steps of the primal-weight update (O11); 0: the form's */
    int32_t pad4;
    int32_t pw_rule;     /* primal-weight update at a restart: 1 smoothing (omega_steps), 2 PID
                            controller; 0: the default (smoothing) */
    int32_t pad5;
    double pid_kp, pid_ki, pid_kd; /* gains of the PID rule */
    int32_t term_mode;   /* what must fall to eps_rel to stop: 0 E_rel, 1 the relative primal
                            residual alone, 2 the relative dual residual alone (the two
                            feasibility polishing solves) */
    int32_t ray_candidates; /* which candidate rays are tested: 0 both (default), 1 the
                               displacement since the previous evaluation only, 2 the averaged
                               point's displacement from the restart anchor only */
} ora_opts;

typedef struct {
    int32_t status;
    int32_t output_is_avg;
    int64_t iters, restarts, n_trace;
    double pobj, dobj, rel_p, rel_d, rel_gap, erel;
    double sigma_max, eta, omega;
    double setup_s, iter_s;
    int32_t ray_source; /* candidate that gave the certificate: 1 displacement, 2 anchored average */
    int32_t pad;
} ora_info;

/* ---------------------------------------------------------------- helpers */

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static double clampd(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* SplitMix64 (Steele, Lea, Flood 2014) used as a counter-based generator: output k is the
 * finaliser applied to seed + (k+1) * golden-gamma. Mapped to [-1/2, 1/2) with 53 bits. */
static double splitmix_centered(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

/* Power-of-two stand-in for 1/sqrt(v): with v = f * 2^E, f in [1/2, 1), return 2^(-floor(E/2)).
 * Scaling by it is exact in floating point. v = 0 (an empty row or column) gives 1. */
static double pow2_rsqrt(double v) {
    if (!(v > 0.0) || !isfinite(v)) return 1.0;
    int e;
    frexp(v, &e);
    int h = (e >= 0) ? e / 2 : -((1 - e) / 2);
    return ldexp(1.0, -h);
}

/* --------------------------------------------------------------- O1 validate */

int ora_validate(const ora_lp *lp) {
    if (!lp || lp->m < 0 || lp->n < 1 || lp->nnz < 0) return ORA_ERR_INVALID_ARG;
    if (!lp->row_ptr || !lp->c || (lp->m > 0 && (!lp->b_lo || !lp->b_hi)) || !lp->x_lo || !lp->x_hi)
        return ORA_ERR_INVALID_ARG;
    if (lp->nnz > 0 && (!lp->col_idx || !lp->vals)) return ORA_ERR_INVALID_ARG;
    if (lp->row_ptr[0] != 0 || (int64_t)lp->row_ptr[lp->m] != lp->nnz) return ORA_ERR_INVALID_MATRIX;
    for (int32_t i = 0; i < lp->m; i++) {
        if (lp->row_ptr[i + 1] < lp->row_ptr[i]) return ORA_ERR_INVALID_MATRIX;
        for (int32_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; e++) {
            int32_t j = lp->col_idx[e];
            if (j < 0 || j >= lp->n) return ORA_ERR_INVALID_MATRIX;
            if (e > lp->row_ptr[i] && lp->col_idx[e - 1] >= j) return ORA_ERR_INVALID_MATRIX;
        }
    }
    for (int64_t e = 0; e < lp->nnz; e++)
        if (!isfinite(lp->vals[e])) return ORA_ERR_NAN_INPUT;
    for (int32_t j = 0; j < lp->n; j++) {
        if (!isfinite(lp->c[j]) || isnan(lp->x_lo[j]) || isnan(lp->x_hi[j])) return ORA_ERR_NAN_INPUT;
        if (lp->x_lo[j] > lp->x_hi[j] || lp->x_lo[j] == INFINITY || lp->x_hi[j] == -INFINITY)
            return ORA_ERR_INCONSISTENT_BOUNDS;
    }
    for (int32_t i = 0; i < lp->m; i++) {
        if (isnan(lp->b_lo[i]) || isnan(lp->b_hi[i])) return ORA_ERR_NAN_INPUT;
        if (lp->b_lo[i] > lp->b_hi[i] || lp->b_lo[i] == INFINITY || lp->b_hi[i] == -INFINITY)
            return ORA_ERR_INCONSISTENT_BOUNDS;
    }
    if (!isfinite(lp->c0)) return ORA_ERR_NAN_INPUT;
    return ORA_OK;
}

/* --------------------------------------------------------------- O2 transpose */

/* CSR of A^T (= CSC of A) by a stable counting sort on the column index: inside each row of
 * A^T the original row indices ascend and every value is moved, never recomputed. This is
 * the CSR + CSC pairing the paper's Section 3.2 keeps for fast row and column access. */
void ora_transpose(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   int32_t *rpT, int32_t *ciT, double *vT) {
    memset(rpT, 0, sizeof(int32_t) * ((size_t)n + 1));
    int64_t nnz = rp[m];
    for (int64_t e = 0; e < nnz; e++) rpT[ci[e] + 1]++;
    for (int32_t j = 0; j < n; j++) rpT[j + 1] += rpT[j];
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    memcpy(next, rpT, sizeof(int32_t) * ((size_t)n + 1));
    for (int32_t i = 0; i < m; i++)
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
            int32_t dst = next[ci[e]]++;
            ciT[dst] = i;
            vT[dst] = v[e];
        }
    free(next);
}

/* --------------------------------------------------------------- O3 scaling */

/* Diagonal scaling A~ = R A C with power-of-two entries: `ruiz` passes of infinity-norm Ruiz
 * equilibration (row and column factors from the same current matrix, applied together),
 * then one Pock-Chambolle pass with alpha = 1 (factors from the row and column sums of
 * |a~|). `av` holds A's values on entry and A~'s on exit; R and C are the products of the
 * factors. Column sums are accumulated row by row, i.e. in ascending row order. */
void ora_scale(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, double *av, int32_t ruiz,
               int32_t pock_chambolle, double *R, double *C) {
    double *rs = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    double *cs = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    for (int32_t i = 0; i < m; i++) R[i] = 1.0;
    for (int32_t j = 0; j < n; j++) C[j] = 1.0;
    for (int32_t pass = 0; pass < ruiz + (pock_chambolle ? 1 : 0); pass++) {
        int use_sum = pass >= ruiz;
        for (int32_t i = 0; i < m; i++) rs[i] = 0.0;
        for (int32_t j = 0; j < n; j++) cs[j] = 0.0;
        for (int32_t i = 0; i < m; i++)
            for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
                double a = fabs(av[e]);
                int32_t j = ci[e];
                if (use_sum) {
                    rs[i] += a;
                    cs[j] += a;
                } else {
                    if (a > rs[i]) rs[i] = a;
                    if (a > cs[j]) cs[j] = a;
                }
            }
        for (int32_t i = 0; i < m; i++) rs[i] = pow2_rsqrt(rs[i]);
        for (int32_t j = 0; j < n; j++) cs[j] = pow2_rsqrt(cs[j]);
        for (int32_t i = 0; i < m; i++)
            for (int32_t e = rp[i]; e < rp[i + 1]; e++) av[e] = av[e] * rs[i] * cs[ci[e]];
        for (int32_t i = 0; i < m; i++) R[i] *= rs[i];
        for (int32_t j = 0; j < n; j++) C[j] *= cs[j];
    }
    free(rs);
    free(cs);
}

/* ------------------------------------------------------------ sparse products */

static void csr_mv(int32_t rows, const int32_t *rp, const int32_t *ci, const double *v, const double *x,
                   double *out) {
    for (int32_t i = 0; i < rows; i++) {
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) s += v[e] * x[ci[e]];
        out[i] = s;
    }
}

/* ---------------------------------------------------------- a3 power iteration */

/* sigma_hat ~ ||A~||_2 by power iteration on A~^T A~ from the SplitMix64 start vector
 * v_k = U[-1/2, 1/2)(seed, k): u = A~ v, w = A~^T u, sigma_hat = ||u||, v = w / ||w||.
 * Reading: PDHG needs eta ||A~||_2 < 1 and eta = 0.998 / sigma_hat, while sigma_hat only
 * approaches ||A~||_2 from below, slowly when the two largest singular values are close.
 * So the steps run in chunks of `iters`; after each chunk the iteration stops when its last
 * step raised sigma_hat by at most 1e-8 sigma_hat, else it goes on, for at most 25 chunks.
 * (With mass a^2 on the top direction and b^2 on the next, the remaining error of
 * sigma_hat^2 is at most sqrt(step gain * ||A~||^2) * b / a, so the rule leaves well under the
 * 0.2% margin of eta.) */
double ora_power_norm(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                      const int32_t *rpT, const int32_t *ciT, const double *vT, int32_t iters,
                      uint64_t seed) {
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double s = 0.0;
    for (int32_t k = 0; k < n; k++) {
        x[k] = splitmix_centered(seed, (uint64_t)k);
        s += x[k] * x[k];
    }
    s = sqrt(s);
    for (int32_t k = 0; k < n; k++) x[k] = x[k] / s;
    double sigma = 0.0, prev = 0.0;
    const int64_t cap = 25 * (int64_t)iters;
    for (int64_t it = 0; it < cap; it++) {
        csr_mv(m, rp, ci, v, x, u);
        csr_mv(n, rpT, ciT, vT, u, w);
        double nu = 0.0, nw = 0.0;
        for (int32_t i = 0; i < m; i++) nu += u[i] * u[i];
        for (int32_t k = 0; k < n; k++) nw += w[k] * w[k];
        prev = sigma;
        sigma = sqrt(nu);
        nw = sqrt(nw);
        if (!(nw > 0.0)) break;
        for (int32_t k = 0; k < n; k++) x[k] = w[k] / nw;
        if ((it + 1) % iters == 0 && sigma - prev <= 1e-8 * sigma) break;
    }
    free(x);
    free(u);
    free(w);
    return sigma;
}

/* ------------------------------------------------------------ problem in scaled space */

typedef struct {
    int32_t m, n;
    int32_t *rp, *ci, *rpT, *ciT;
    double *av, *avT;
    double *c, *blo, *bhi, *xlo, *xhi; /* scaled data */
    double *R, *C, *Ri, *Ci;           /* scale factors and their (exact) inverses */
    const double *oc, *oblo, *obhi, *oxlo, *oxhi; /* original data */
    double c0, qnorm, cnorm;
} prob;

typedef struct {
    double rp2, rd2;   /* ||r_p||^2, ||r_d||^2 on the original data */
    double rps2, rds2; /* the same on the scaled problem */
    double pobj, dobj; /* without c0 */
    double rel_p, rel_d, rel_gap, erel;
} kkt_t;

/* O8: residuals, objectives and E_rel of a candidate (x~, y~) given A~x~ and A~^T y~.
 * Original-scale quantities follow from exact power-of-two unscaling:
 * A x = R^-1 A~x~, c - A^T y = C^-1 (c~ - A~^T y~), x = C x~, y = R y~.
 *   r_p,i = (Ax)_i - clamp((Ax)_i, b_lo,i, b_hi,i)
 *   z = projection of lambda = c - A^T y onto the sign cone of eq. (2) (free: 0; only x_lo
 *       finite: >= 0; only x_hi finite: <= 0; both finite: any)
 *   r_d = lambda - z, plus any sign violation of y (y > 0 where b_lo = -inf, y < 0 where
 *       b_hi = +inf), which the iteration never produces
 *   p = c^T x + c0,  d = sum_i (b_lo,i y_i^+ - b_hi,i y_i^-) + sum_k (x_lo,k z_k^+ - x_hi,k z_k^-) + c0
 *       with 0 * inf := 0
 *   E_rel = max(||r_p|| / (1 + ||q||), ||r_d|| / (1 + ||c||), |p - d| / (1 + |p| + |d|)). */
static void eval_kkt(const prob *P, const double *x, const double *y, const double *ax, const double *aty,
                     kkt_t *K, double *z_out) {
    double rp2 = 0, rps2 = 0, rd2 = 0, rds2 = 0, pobj = 0, dobj = 0;
    for (int32_t i = 0; i < P->m; i++) {
        double rs = ax[i] - clampd(ax[i], P->blo[i], P->bhi[i]);
        double ro = rs * P->Ri[i];
        rps2 += rs * rs;
        rp2 += ro * ro;
        double yo = y[i] * P->R[i];
        if (yo > 0.0 && isfinite(P->oblo[i])) dobj += P->oblo[i] * yo;
        if (yo < 0.0 && isfinite(P->obhi[i])) dobj += P->obhi[i] * yo;
        double vs = 0.0;
        if (P->oblo[i] == -INFINITY && y[i] > 0.0) vs += y[i];
        if (P->obhi[i] == INFINITY && y[i] < 0.0) vs -= y[i];
        double vo = vs * P->R[i];
        rds2 += vs * vs;
        rd2 += vo * vo;
    }
    for (int32_t k = 0; k < P->n; k++) {
        double ls = P->c[k] - aty[k];
        int flo = isfinite(P->oxlo[k]), fhi = isfinite(P->oxhi[k]);
        double zs = ls;
        if (!flo && !fhi) zs = 0.0;
        else if (flo && !fhi) zs = ls > 0.0 ? ls : 0.0;
        else if (!flo && fhi) zs = ls < 0.0 ? ls : 0.0;
        double rds = ls - zs;
        double zo = zs * P->Ci[k];
        double rdo = rds * P->Ci[k];
        rds2 += rds * rds;
        rd2 += rdo * rdo;
        double xo = x[k] * P->C[k];
        pobj += P->oc[k] * xo;
        if (zo > 0.0) dobj += P->oxlo[k] * zo;
        if (zo < 0.0) dobj += P->oxhi[k] * zo;
        if (z_out) z_out[k] = zo;
    }
    K->rp2 = rp2;
    K->rd2 = rd2;
    K->rps2 = rps2;
    K->rds2 = rds2;
    K->pobj = pobj;
    K->dobj = dobj;
    double p = pobj + P->c0, d = dobj + P->c0;
    K->rel_p = sqrt(rp2) / (1.0 + P->qnorm);
    K->rel_d = sqrt(rd2) / (1.0 + P->cnorm);
    K->rel_gap = fabs(p - d) / (1.0 + fabs(p) + fabs(d));
    double e = K->rel_p;
    if (K->rel_d > e) e = K->rel_d;
    if (K->rel_gap > e) e = K->rel_gap;
    if (isnan(K->rel_p) || isnan(K->rel_d) || isnan(K->rel_gap)) e = NAN;
    K->erel = e;
}

/* The quantity termination compares with eps_rel (term_mode of ora_opts). */
static double term_value(const kkt_t *K, int32_t mode) {
    if (mode == 1) return isnan(K->erel) ? NAN : K->rel_p;
    if (mode == 2) return isnan(K->erel) ? NAN : K->rel_d;
    return K->erel;
}

/* KKT error in the primal-weighted norm on the scaled problem (restart metric). */
static double kkt_omega(const kkt_t *K, double omega) {
    double w2 = omega * omega;
    double g = K->pobj - K->dobj;
    return sqrt(w2 * K->rps2 + K->rds2 / w2 + g * g);
}

/* Infeasibility certificates (the sign remarks after eq. (2): an LP with no solution of
 * eq. (2) is infeasible or unbounded). Reading: a candidate ray is the difference of two
 * points, taken on the original scale. Two candidates are tested at every evaluation, in
 * this order: (1) the evaluated point minus the one of the previous evaluation (after its
 * restart decision); (2) the averaged point (the running average; the PDHG output in the
 * Halpern form) minus the anchor of the current restart cycle: for an LP without a
 * solution the iterates drift along the infimal displacement, and the average's distance
 * from the anchor grows along it about linearly in the iterations since the restart, with
 * the oscillations of the iterates averaged out (the normalised average). For a pair
 * (x~, y~) minus (x~p, y~p), with their products:
 *   dual ray   y^ = R (y~ - y~p), with lambda = -A^T y^ = -C^-1 (A~^T y~ - A~^T y~p) and
 *              z^ = lambda projected onto the sign cone of eq. (2);
 *              rd2 = ||lambda - z^||^2 + ||sign violations of y^||^2 (y^ > 0 where b_lo = -inf,
 *              y^ < 0 where b_hi = +inf);
 *              D = sum_i (b_lo,i y^_i^+ - b_hi,i y^_i^-) + sum_k (x_lo,k z^_k^+ - x_hi,k z^_k^-)
 *              (finite bounds only). A ray with D > 0 and sqrt(rd2) <= eps * D certifies that
 *              the constraints have no solution (Farkas).
 *   primal ray x^ = C (x~ - x~p), A x^ = R^-1 (A~x~ - A~x~p);
 *              rp2 = ||part of A x^ outside the recession cone of [b_lo, b_hi]||^2
 *                  + ||part of x^ outside the recession cone of [x_lo, x_hi]||^2
 *              (both bounds finite: the whole component; only the lower: its negative part;
 *              only the upper: its positive part; none: nothing);
 *              G = -c^T x^. A ray with G > 0 and sqrt(rp2) <= eps * G certifies that the
 *              objective decreases without bound along a feasible direction, so the dual is
 *              infeasible. */
typedef struct {
    double rd2, D, rp2, G;
} ray_t;

static void eval_rays(const prob *P, const double *x, const double *y, const double *ax, const double *aty,
                      const double *xp, const double *yp, const double *axp, const double *atyp, ray_t *Rr,
                      double *xray, double *yray, double *zray) {
    double rd2 = 0, D = 0, rp2 = 0, G = 0;
    for (int32_t i = 0; i < P->m; i++) {
        double dy = (y[i] - yp[i]) * P->R[i];
        double v = (ax[i] - axp[i]) * P->Ri[i];
        int flo = isfinite(P->oblo[i]), fhi = isfinite(P->obhi[i]);
        if (dy > 0.0 && flo) D += P->oblo[i] * dy;
        if (dy < 0.0 && fhi) D += P->obhi[i] * dy;
        double vs = 0.0;
        if (!flo && dy > 0.0) vs += dy;
        if (!fhi && dy < 0.0) vs -= dy;
        rd2 += vs * vs;
        double w = 0.0;
        if (flo && fhi) w = v;
        else if (flo) w = v < 0.0 ? v : 0.0;
        else if (fhi) w = v > 0.0 ? v : 0.0;
        rp2 += w * w;
        if (yray) yray[i] = dy;
    }
    for (int32_t k = 0; k < P->n; k++) {
        double lam = -(aty[k] - atyp[k]) * P->Ci[k];
        int flo = isfinite(P->oxlo[k]), fhi = isfinite(P->oxhi[k]);
        double zs = lam;
        if (!flo && !fhi) zs = 0.0;
        else if (flo && !fhi) zs = lam > 0.0 ? lam : 0.0;
        else if (!flo && fhi) zs = lam < 0.0 ? lam : 0.0;
        double r = lam - zs;
        rd2 += r * r;
        if (zs > 0.0) D += P->oxlo[k] * zs;
        if (zs < 0.0) D += P->oxhi[k] * zs;
        double xh = (x[k] - xp[k]) * P->C[k];
        G -= P->oc[k] * xh;
        double w = 0.0;
        if (flo && fhi) w = xh;
        else if (flo) w = xh < 0.0 ? xh : 0.0;
        else if (fhi) w = xh > 0.0 ? xh : 0.0;
        rp2 += w * w;
        if (zray) zray[k] = zs;
        if (xray) xray[k] = xh;
    }
    Rr->rd2 = rd2;
    Rr->D = D;
    Rr->rp2 = rp2;
    Rr->G = G;
}

static double combined_bound_norm(int32_t m, const double *lo, const double *hi) {
    double s = 0.0;
    for (int32_t i = 0; i < m; i++) {
        double q = 0.0;
        if (isfinite(lo[i]) && fabs(lo[i]) > q) q = fabs(lo[i]);
        if (isfinite(hi[i]) && fabs(hi[i]) > q) q = fabs(hi[i]);
        s += q * q;
    }
    return sqrt(s);
}

static double vec_norm(int32_t n, const double *v) {
    double s = 0.0;
    for (int32_t k = 0; k < n; k++) s += v[k] * v[k];
    return sqrt(s);
}

static double diff_norm(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t k = 0; k < n; k++) {
        double d = a[k] - b[k];
        s += d * d;
    }
    return sqrt(s);
}

static void prob_free(prob *P) {
    free(P->rp); free(P->ci); free(P->rpT); free(P->ciT); free(P->av); free(P->avT);
    free(P->c); free(P->blo); free(P->bhi); free(P->xlo); free(P->xhi);
    free(P->R); free(P->C); free(P->Ri); free(P->Ci);
}

/* O2 + O3: copies, transpose and (optionally) scaling; original norms for E_rel. */
static int prob_build(const ora_lp *lp, int scaling, int ruiz, prob *P) {
    int32_t m = lp->m, n = lp->n;
    int64_t nnz = lp->nnz;
    memset(P, 0, sizeof(*P));
    P->m = m;
    P->n = n;
    P->rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
    P->ci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    P->rpT = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    P->ciT = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    P->av = (double *)malloc(sizeof(double) * ((size_t)nnz + 1));
    P->avT = (double *)malloc(sizeof(double) * ((size_t)nnz + 1));
    P->c = (double *)malloc(sizeof(double) * (size_t)n);
    P->xlo = (double *)malloc(sizeof(double) * (size_t)n);
    P->xhi = (double *)malloc(sizeof(double) * (size_t)n);
    P->C = (double *)malloc(sizeof(double) * (size_t)n);
    P->Ci = (double *)malloc(sizeof(double) * (size_t)n);
    P->blo = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    P->bhi = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    P->R = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    P->Ri = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    if (!P->rp || !P->ci || !P->rpT || !P->ciT || !P->av || !P->avT || !P->c || !P->xlo || !P->xhi ||
        !P->C || !P->Ci || !P->blo || !P->bhi || !P->R || !P->Ri) {
        prob_free(P);
        return ORA_ERR_OUT_OF_MEMORY;
    }
    memcpy(P->rp, lp->row_ptr, sizeof(int32_t) * ((size_t)m + 1));
    if (nnz) {
        memcpy(P->ci, lp->col_idx, sizeof(int32_t) * (size_t)nnz);
        memcpy(P->av, lp->vals, sizeof(double) * (size_t)nnz);
    }
    if (scaling) {
        ora_scale(m, n, P->rp, P->ci, P->av, ruiz, 1, P->R, P->C);
    } else {
        for (int32_t i = 0; i < m; i++) P->R[i] = 1.0;
        for (int32_t k = 0; k < n; k++) P->C[k] = 1.0;
    }
    ora_transpose(m, n, P->rp, P->ci, P->av, P->rpT, P->ciT, P->avT);
    for (int32_t i = 0; i < m; i++) {
        P->Ri[i] = 1.0 / P->R[i];
        P->blo[i] = lp->b_lo[i] * P->R[i];
        P->bhi[i] = lp->b_hi[i] * P->R[i];
    }
    for (int32_t k = 0; k < n; k++) {
        P->Ci[k] = 1.0 / P->C[k];
        P->c[k] = lp->c[k] * P->C[k];
        P->xlo[k] = lp->x_lo[k] * P->Ci[k];
        P->xhi[k] = lp->x_hi[k] * P->Ci[k];
    }
    P->oc = lp->c;
    P->oblo = lp->b_lo;
    P->obhi = lp->b_hi;
    P->oxlo = lp->x_lo;
    P->oxhi = lp->x_hi;
    P->c0 = lp->c0;
    P->qnorm = combined_bound_norm(m, lp->b_lo, lp->b_hi);
    P->cnorm = vec_norm(n, lp->c);
    return ORA_OK;
}

void ora_default_opts(ora_opts *o) {
    memset(o, 0, sizeof(*o));
    o->eps_rel = 1e-4;
    o->max_iters = 100000;
    o->eval_every = 64;
    o->scaling = 1;
    o->ruiz_passes = 10;
    o->pow_iters = 200;
    o->restarts = 1;
    o->eta = 0.0;
    o->omega0 = 0.0;
    o->seed = 0x5EED0C0FFEEull;
    o->eps_infeas = 1e-8;
    o->method = 0;
    o->reflection = 1.0;
    o->omega_steps = 0;
    o->pw_rule = 0;
    o->pid_kp = 0.7;
    o->pid_ki = 0.05;
    o->pid_kd = 0.2;
}

/* Export the scaled problem: A~ values (in the caller's CSR order), R, C, and A~^T. */
int ora_scaled_problem(const ora_lp *lp, int32_t scaling, int32_t ruiz, double *av, double *R, double *C,
                       int32_t *rpT, int32_t *ciT, double *avT) {
    int rc = ora_validate(lp);
    if (rc) return rc;
    prob P;
    rc = prob_build(lp, scaling, ruiz, &P);
    if (rc) return rc;
    if (av) memcpy(av, P.av, sizeof(double) * (size_t)lp->nnz);
    if (R) memcpy(R, P.R, sizeof(double) * (size_t)lp->m);
    if (C) memcpy(C, P.C, sizeof(double) * (size_t)lp->n);
    if (rpT) memcpy(rpT, P.rpT, sizeof(int32_t) * ((size_t)lp->n + 1));
    if (ciT) memcpy(ciT, P.ciT, sizeof(int32_t) * (size_t)lp->nnz);
    if (avT) memcpy(avT, P.avT, sizeof(double) * (size_t)lp->nnz);
    prob_free(&P);
    return ORA_OK;
}

/* KKT check of an original-space point (x, y) against the original data (no scaling):
 * out = [rel_p, rel_d, rel_gap, E_rel, p, d] with p, d including c0; z (optional) is the
 * projected reduced cost. */
int ora_kkt(const ora_lp *lp, const double *x, const double *y, double *out, double *z) {
    int rc = ora_validate(lp);
    if (rc) return rc;
    prob P;
    rc = prob_build(lp, 0, 0, &P);
    if (rc) return rc;
    double *ax = (double *)malloc(sizeof(double) * ((size_t)lp->m + 1));
    double *aty = (double *)malloc(sizeof(double) * (size_t)lp->n);
    csr_mv(lp->m, P.rp, P.ci, P.av, x, ax);
    csr_mv(lp->n, P.rpT, P.ciT, P.avT, y, aty);
    kkt_t K;
    eval_kkt(&P, x, y, ax, aty, &K, z);
    out[0] = K.rel_p;
    out[1] = K.rel_d;
    out[2] = K.rel_gap;
    out[3] = K.erel;
    out[4] = K.pobj + lp->c0;
    out[5] = K.dobj + lp->c0;
    free(ax);
    free(aty);
    prob_free(&P);
    return ORA_OK;
}

/* ------------------------------------------------------------------ O4 - O12 */

/* O7, primal half of the PDHG map: x+ = clamp(x - tau (c~ - A~^T y)) for one column. */
static double primal_step(double x, double c, double aty, double tau, double lo, double hi) {
    double g = c - aty;
    double xn = x - tau * g;
    return clampd(xn, lo, hi);
}

/* O7, dual half: v = y - sigma (2 A~x+ - A~x), y+ = max(v + sigma b~lo, 0) + min(v + sigma b~hi, 0)
 * (the closed-form prox of the row bounds) for one row. */
static double dual_step(double y, double axn, double ax, double sigma, double blo, double bhi) {
    double w = 2.0 * axn - ax;
    double v = y - sigma * w;
    double lo = v + sigma * blo;
    double hi = v + sigma * bhi;
    return (lo > 0.0 ? lo : 0.0) + (hi < 0.0 ? hi : 0.0);
}

/* Fixed-point residual of the Halpern iterate z = (x, y) in the norm of the PDHG map: with
 * d = z - T(z) = (dx, dy) and A~dx = ax - axa,
 *   r^2 = omega ||dx||^2 + 2 eta <dy, A~dx> + ||dy||^2 / omega,
 * which is eta times the quadratic form of [[I / tau, A~^T], [A~, I / sigma]] (tau = eta /
 * omega, sigma = eta omega): the metric in which the map of O7 is firmly nonexpansive, a norm
 * while eta ||A~||_2 < 1. */
static double fixed_point_residual(int32_t m, int32_t n, const double *x, const double *xa, const double *y,
                                   const double *ya, const double *ax, const double *axa, double omega,
                                   double eta) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int32_t j = 0; j < n; j++) {
        double d = x[j] - xa[j];
        s1 += d * d;
    }
    for (int32_t i = 0; i < m; i++) {
        double d = y[i] - ya[i];
        s2 += d * (ax[i] - axa[i]);
        s3 += d * d;
    }
    double r2 = omega * s1 + 2.0 * eta * s2 + s3 / omega;
    return sqrt(r2 > 0.0 ? r2 : 0.0);
}

/* Restarted, averaged PDHG (primal step first) on the scaled problem.
 *
 * O4  omega0 = ||c~|| / ||q~|| when both exceed 1e-10, else 1 (q: combined bounds).
 * O5  eta = 0.998 / sigma_hat; tau = eta / omega, sigma = eta * omega.
 * O6  x0 = clamp(0) (or the warm start), y0 = 0; averages and anchor equal the start.
 * O7  x+ = clamp(x - tau (c~ - A~^T y)), y+ = max(v + sigma b~_lo, 0) + min(v + sigma b~_hi, 0)
 *     with v = y - sigma (2 A~x+ - A~x); running means of x and y since the last restart
 *     (constant step, so the weights are uniform: x_avg += (x+ - x_avg) / t).
 * O8  every `eval_every` iterations (and at max_iters) both the current and the average
 *     iterate are evaluated as in eval_kkt.
 * O9  stop when E_rel(current) <= eps (then the average); at max_iters return the better.
 *     (term_mode 1 / 2 compare the relative primal / dual residual instead of E_rel: the
 *     feasibility polishing solves, see ora_polish in the Python module.)
 * O10 candidate = average if its KKT_omega is strictly smaller; restart if
 *     (i) KKT_c <= 0.2 KKT_anchor, (ii) KKT_c <= 0.8 KKT_anchor and KKT_c > KKT_prev, or
 *     (iii) t >= 0.36 k.
 * O11 on restart, when dx, dy > 1e-10 (the distances the candidate moved from the anchor),
 *     the primal weight is updated so that the weighted distances omega * dx and dy / omega
 *     move toward balance, i.e. log omega toward log(dy/dx):
 *     - smoothing (pw_rule 1): omega <- sqrt(omega * dy / dx) applied `omega_steps` times,
 *       log omega moving by the fraction theta = 1 - 2^-omega_steps, from correctly rounded
 *       operations only (0 selects one step, theta = 1/2, for the averaged form and two,
 *       theta = 3/4, for the Halpern form);
 *     - PID controller (pw_rule 2) on the error e = log(omega * dx / dy) of this restart:
 *       I += e, log omega -= kp e + ki I + kd (e - e_prev), e_prev = e (I and e_prev start
 *       at 0). With ki = kd = 0 it is the smoothing with theta = kp.
 *     The candidate becomes iterate, anchor and average.
 * O12 x = C x~, y = R y~, z = projected reduced cost.
 *
 * Halpern form (method 1, a reading of the newer cuPDLPx-family iteration the paper names):
 * the iterate is z <- w ((1 + rho) T(z) - rho z) + (1 - w) z_anchor with T the map of O7,
 * w = (t + 1) / (t + 2); no averages; O8-O11 act on T(z) (the only candidate), a restart
 * moves the iterate and the anchor to T(z). With restart_metric 1 (the restart rule of that
 * solver family) the three tests of O10 compare fixed-point residuals instead of KKT_omega
 * values: the current one is that of the last iterate before the evaluation (whose T(z) is
 * the candidate), the anchor's that of the first iterate of the cycle (the anchor itself),
 * both in the cycle's weight. */
int ora_solve(const ora_lp *lp, const ora_opts *o, double *x_out, double *y_out, double *z_out,
              ora_info *info) {
    double t0 = now_s();
    memset(info, 0, sizeof(*info));
    int rc = ora_validate(lp);
    if (rc) {
        info->status = -rc;
        return rc;
    }
    if (o->eval_every < 1) return ORA_ERR_INVALID_ARG;
    prob P;
    rc = prob_build(lp, o->scaling, o->ruiz_passes, &P);
    if (rc) return rc;
    int32_t m = lp->m, n = lp->n;
    size_t mb = sizeof(double) * ((size_t)m + 1), nb = sizeof(double) * (size_t)n;
    double *x = (double *)malloc(nb), *xa = (double *)malloc(nb), *xan = (double *)malloc(nb);
    double *aty = (double *)malloc(nb), *atya = (double *)malloc(nb);
    double *y = (double *)malloc(mb), *ya = (double *)malloc(mb), *yan = (double *)malloc(mb);
    double *ax = (double *)malloc(mb), *axn = (double *)malloc(mb), *axa = (double *)malloc(mb);
    /* point at the previous evaluation (after its restart decision), for the candidate rays */
    double *xp = (double *)malloc(nb), *atyp = (double *)malloc(nb);
    double *yp = (double *)malloc(mb), *axp = (double *)malloc(mb);
    double *axan = (double *)malloc(mb); /* A~ x~ of the anchor */
    double *atyan = (double *)malloc(nb); /* A~^T y~ of the anchor (anchored-average rays) */
    const int halpern = o->method == 1;
    const double rho = o->reflection;

    /* a3 / O5: step size */
    double sig = 0.0;
    double eta = o->eta;
    if (!(eta > 0.0)) {
        sig = ora_power_norm(m, n, P.rp, P.ci, P.av, P.rpT, P.ciT, P.avT, o->pow_iters, o->seed);
        eta = sig > 0.0 ? 0.998 / sig : 1.0;
    }
    /* O4: primal weight */
    double omega = o->omega0;
    if (!(omega > 0.0)) {
        double cn = vec_norm(n, P.c), qn = combined_bound_norm(m, P.blo, P.bhi);
        omega = (cn > 1e-10 && qn > 1e-10) ? cn / qn : 1.0;
    }
    double tau = eta / omega, sigma = eta * omega;

    /* O6 */
    for (int32_t k = 0; k < n; k++) {
        double s = o->x0 ? o->x0[k] * P.Ci[k] : 0.0;
        x[k] = clampd(s, P.xlo[k], P.xhi[k]);
        xa[k] = x[k];
        xan[k] = x[k];
    }
    for (int32_t i = 0; i < m; i++) {
        y[i] = o->y0 ? o->y0[i] * P.Ri[i] : 0.0;
        ya[i] = y[i];
        yan[i] = y[i];
    }
    csr_mv(m, P.rp, P.ci, P.av, x, ax);
    csr_mv(n, P.rpT, P.ciT, P.avT, y, aty);
    memcpy(axan, ax, sizeof(double) * (size_t)m);
    memcpy(atyan, aty, nb);
    memcpy(axa, ax, sizeof(double) * (size_t)m);
    memcpy(atya, aty, nb);
    kkt_t Kc, Ka, Kanc;
    eval_kkt(&P, x, y, ax, aty, &Kc, NULL);
    memcpy(xp, x, nb);
    memcpy(atyp, aty, nb);
    memcpy(yp, y, sizeof(double) * (size_t)m);
    memcpy(axp, ax, sizeof(double) * (size_t)m);
    ray_t Rray;
    memset(&Rray, 0, sizeof(Rray));
    int ray_src = 0;
    const int try_disp = o->ray_candidates != 2, try_anch = o->ray_candidates != 1;
    Kanc = Kc;
    double kkt_anchor = kkt_omega(&Kanc, omega);
    double kkt_prev = INFINITY;
    /* primal-weight rule and the PID controller's state (integral, previous error) */
    const int pid = o->pw_rule == 2;
    double pid_int = 0.0, pid_prev = 0.0;
    /* fixed-point residual restarts: residual of the latest iterate and of the cycle's anchor */
    const int fpr = halpern && o->restart_metric == 1;
    double r_cur = 0.0, r_anchor = 0.0;
    int64_t k = 0, t = 0, restarts = 0, ntr = 0;
    int status = -1, out_avg = 0;
    int64_t snap_i = 0;
    info->setup_s = now_s() - t0;
    double t1 = now_s();

    if (isnan(Kc.erel)) status = ORA_NUMERICAL_ERROR;
    else if (term_value(&Kc, o->term_mode) <= o->eps_rel) status = ORA_OPTIMAL;
    else if (o->max_iters <= 0) status = ORA_ITERATION_LIMIT;

    while (status < 0) {
        if (halpern) {
            /* Reflected Halpern PDHG (a reading; the paper names cuPDLPx's family but does not
             * print its iteration): with T the PDHG map of O7 and the anchor z0 of the current
             * restart cycle, z <- w ((1 + rho) T(z) - rho z) + (1 - w) z0, w = (t + 1) / (t + 2),
             * t the iterations since the restart. xa, ya hold T(z) (bounded and sign-feasible),
             * axa = A~ xa; A~x of the Halpern iterate follows by linearity. */
            csr_mv(n, P.rpT, P.ciT, P.avT, y, aty);
            for (int32_t j = 0; j < n; j++) xa[j] = primal_step(x[j], P.c[j], aty[j], tau, P.xlo[j], P.xhi[j]);
            csr_mv(m, P.rp, P.ci, P.av, xa, axa);
            for (int32_t i = 0; i < m; i++) ya[i] = dual_step(y[i], axa[i], ax[i], sigma, P.blo[i], P.bhi[i]);
            if (fpr && (t == 0 || (k + 1) % o->eval_every == 0 || k + 1 >= o->max_iters)) {
                double r = fixed_point_residual(m, n, x, xa, y, ya, ax, axa, omega, eta);
                if (t == 0) r_anchor = r;
                r_cur = r;
            }
            double wk = (double)(t + 1) / (double)(t + 2);
            double wa = 1.0 - wk;
            double r1 = 1.0 + rho;
            for (int32_t j = 0; j < n; j++) x[j] = wk * (r1 * xa[j] - rho * x[j]) + wa * xan[j];
            for (int32_t i = 0; i < m; i++) {
                y[i] = wk * (r1 * ya[i] - rho * y[i]) + wa * yan[i];
                ax[i] = wk * (r1 * axa[i] - rho * ax[i]) + wa * axan[i];
            }
            k++;
            t++;
        } else {
        /* O7: primal step (A~^T y computed for the current y) */
        csr_mv(n, P.rpT, P.ciT, P.avT, y, aty);
        for (int32_t j = 0; j < n; j++) x[j] = primal_step(x[j], P.c[j], aty[j], tau, P.xlo[j], P.xhi[j]);
        /* O7: dual step with the extrapolation 2 A~x+ - A~x */
        csr_mv(m, P.rp, P.ci, P.av, x, axn);
        for (int32_t i = 0; i < m; i++) {
            y[i] = dual_step(y[i], axn[i], ax[i], sigma, P.blo[i], P.bhi[i]);
            ax[i] = axn[i];
        }
        k++;
        t++;
        if (t == 1) {
            memcpy(xa, x, nb);
            memcpy(ya, y, sizeof(double) * (size_t)m);
        } else {
            double wt = 1.0 / (double)t;
            for (int32_t j = 0; j < n; j++) xa[j] = xa[j] + wt * (x[j] - xa[j]);
            for (int32_t i = 0; i < m; i++) ya[i] = ya[i] + wt * (y[i] - ya[i]);
        }
        }
        while (snap_i < o->n_snap && o->snap_k[snap_i] < k) snap_i++;
        if (snap_i < o->n_snap && o->snap_k[snap_i] == k) {
            double *s = o->snap_out + (size_t)snap_i * (2 * (size_t)n + 2 * (size_t)m);
            memcpy(s, x, nb);
            memcpy(s + n, y, sizeof(double) * (size_t)m);
            memcpy(s + n + m, xa, nb);
            memcpy(s + 2 * (size_t)n + m, ya, sizeof(double) * (size_t)m);
            snap_i++;
        }
        if (!(k % o->eval_every == 0 || k >= o->max_iters)) continue;

        /* O8 (Halpern form: the only candidate is T(z) = (xa, ya), whose A~x is axa) */
        if (halpern) {
            csr_mv(n, P.rpT, P.ciT, P.avT, ya, atya);
            eval_kkt(&P, xa, ya, axa, atya, &Kc, NULL);
            Ka = Kc;
        } else {
        csr_mv(n, P.rpT, P.ciT, P.avT, y, aty);
        csr_mv(m, P.rp, P.ci, P.av, xa, axa);
        csr_mv(n, P.rpT, P.ciT, P.avT, ya, atya);
        eval_kkt(&P, x, y, ax, aty, &Kc, NULL);
        eval_kkt(&P, xa, ya, axa, atya, &Ka, NULL);
        }
        /* the point each evaluation looks at: (x, y) or, in the Halpern form, T(z) */
        const double *ex = halpern ? xa : x, *ey = halpern ? ya : y;
        const double *eax = halpern ? axa : ax, *eaty = halpern ? atya : aty;
        double kc = kkt_omega(&Kc, omega), ka = kkt_omega(&Ka, omega);
        if (fpr) {
            kc = ka = r_cur;
            kkt_anchor = r_anchor;
        }
        double rec[ORA_TRACE_W];
        memset(rec, 0, sizeof(rec));
        rec[0] = (double)k;
        rec[1] = (double)t;
        rec[2] = kc;
        rec[3] = ka;
        rec[4] = Kc.erel;
        rec[5] = Ka.erel;
        rec[9] = kkt_anchor;
        rec[10] = kkt_prev;
        /* O9 */
        if (isnan(Kc.erel) || isnan(Ka.erel)) {
            status = ORA_NUMERICAL_ERROR;
        } else if (term_value(&Kc, o->term_mode) <= o->eps_rel) {
            status = ORA_OPTIMAL;
            out_avg = halpern;
        } else if (term_value(&Ka, o->term_mode) <= o->eps_rel) {
            status = ORA_OPTIMAL;
            out_avg = 1;
        } else {
            if (o->eps_infeas > 0.0 && try_disp) {
                eval_rays(&P, ex, ey, eax, eaty, xp, yp, axp, atyp, &Rray, NULL, NULL, NULL);
                if (Rray.D > 0.0 && sqrt(Rray.rd2) <= o->eps_infeas * Rray.D) status = ORA_PRIMAL_INFEASIBLE;
                else if (Rray.G > 0.0 && sqrt(Rray.rp2) <= o->eps_infeas * Rray.G) status = ORA_DUAL_INFEASIBLE;
                if (status >= 0) ray_src = 1;
            }
            if (status < 0 && o->eps_infeas > 0.0 && try_anch) {
                eval_rays(&P, xa, ya, axa, atya, xan, yan, axan, atyan, &Rray, NULL, NULL, NULL);
                if (Rray.D > 0.0 && sqrt(Rray.rd2) <= o->eps_infeas * Rray.D) status = ORA_PRIMAL_INFEASIBLE;
                else if (Rray.G > 0.0 && sqrt(Rray.rp2) <= o->eps_infeas * Rray.G) status = ORA_DUAL_INFEASIBLE;
                if (status >= 0) ray_src = 2;
            }
            if (status < 0 && k >= o->max_iters) {
                status = ORA_ITERATION_LIMIT;
                out_avg = halpern ? 1 : term_value(&Ka, o->term_mode) < term_value(&Kc, o->term_mode);
            }
        }
        if (status >= 0) {
            if (status == ORA_PRIMAL_INFEASIBLE || status == ORA_DUAL_INFEASIBLE) out_avg = halpern;
            rec[6] = out_avg;
            rec[8] = omega;
            rec[11] = INFINITY;
            if (o->trace && ntr < o->trace_cap) memcpy(o->trace + ntr * ORA_TRACE_W, rec, sizeof(rec));
            ntr++;
            break;
        }
        /* O10 */
        int use_avg = halpern ? 1 : ka < kc;
        double kcand = use_avg ? ka : kc;
        double margin = fabs(ka - kc) / fmax(fmax(ka, kc), 1e-300);
        int why = 0;
        if (o->restarts) {
            double mi = fabs(kcand - 0.2 * kkt_anchor) / fmax(kkt_anchor, 1e-300);
            double mii = fabs(kcand - 0.8 * kkt_anchor) / fmax(kkt_anchor, 1e-300);
            double mprev = isfinite(kkt_prev) ? fabs(kcand - kkt_prev) / fmax(kkt_prev, 1e-300) : INFINITY;
            double miii = fabs((double)t - 0.36 * (double)k) / (double)k;
            margin = fmin(margin, fmin(fmin(mi, mii), fmin(mprev, miii)));
            if (kcand <= 0.2 * kkt_anchor) why = 1;
            else if (kcand <= 0.8 * kkt_anchor && kcand > kkt_prev) why = 2;
            else if ((double)t >= 0.36 * (double)k) why = 3;
        }
        rec[6] = use_avg;
        rec[7] = why;
        rec[11] = margin;
        if (why) {
            /* O11 */
            const double *xc = use_avg ? xa : x, *yc = use_avg ? ya : y;
            double dx = diff_norm(n, xc, xan), dy = diff_norm(m, yc, yan);
            const int32_t steps = o->omega_steps > 0 ? o->omega_steps : (halpern ? 2 : 1);
            if (dx > 1e-10 && dy > 1e-10) {
                if (pid) {
                    const double e = log((omega * dx) / dy);
                    pid_int += e;
                    const double u = o->pid_kp * e + o->pid_ki * pid_int + o->pid_kd * (e - pid_prev);
                    pid_prev = e;
                    omega = omega * exp(-u);
                } else {
                    for (int32_t q = 0; q < steps; q++) omega = sqrt((omega * dy) / dx);
                }
            }
            tau = eta / omega;
            sigma = eta * omega;
            if (use_avg) {
                memcpy(x, xa, nb);
                memcpy(y, ya, sizeof(double) * (size_t)m);
                memcpy(ax, axa, sizeof(double) * (size_t)m);
                memcpy(axan, axa, sizeof(double) * (size_t)m);
                memcpy(atyan, atya, nb);
                Kanc = Ka;
            } else {
                memcpy(xa, x, nb);
                memcpy(ya, y, sizeof(double) * (size_t)m);
                memcpy(axan, ax, sizeof(double) * (size_t)m);
                memcpy(atyan, aty, nb);
                Kanc = Kc;
            }
            memcpy(xan, x, nb);
            memcpy(yan, y, sizeof(double) * (size_t)m);
            kkt_anchor = kkt_omega(&Kanc, omega);
            kkt_prev = INFINITY;
            t = 0;
            restarts++;
        } else {
            kkt_prev = kcand;
        }
        /* the point the next evaluation's rays start from */
        if (halpern) {
            memcpy(xp, xa, nb);
            memcpy(yp, ya, sizeof(double) * (size_t)m);
            memcpy(axp, axa, sizeof(double) * (size_t)m);
            memcpy(atyp, atya, nb);
        } else {
            memcpy(xp, x, nb);
            memcpy(yp, y, sizeof(double) * (size_t)m);
            memcpy(axp, ax, sizeof(double) * (size_t)m);
            memcpy(atyp, (why && use_avg) ? atya : aty, nb);
        }
        rec[8] = omega;
        if (o->trace && ntr < o->trace_cap) memcpy(o->trace + ntr * ORA_TRACE_W, rec, sizeof(rec));
        ntr++;
    }
    info->iter_s = now_s() - t1;

    /* O12 */
    const double *xo = out_avg ? xa : x, *yo = out_avg ? ya : y;
    kkt_t Ko;
    if (k == 0) {
        Ko = Kc;
        if (z_out) eval_kkt(&P, x, y, ax, aty, &Ko, z_out);
    } else {
        const double *ato = out_avg ? atya : aty;
        const double *axo = out_avg ? axa : ax;
        eval_kkt(&P, xo, yo, axo, ato, &Ko, z_out);
    }
    if (x_out)
        for (int32_t j = 0; j < n; j++) x_out[j] = xo[j] * P.C[j];
    if (y_out)
        for (int32_t i = 0; i < m; i++) y_out[i] = yo[i] * P.R[i];
    if (status == ORA_PRIMAL_INFEASIBLE || status == ORA_DUAL_INFEASIBLE) {
        /* the certificate, normalised so that D = 1 (dual ray in y, z) or G = 1 (primal ray in x) */
        double *xr = (double *)malloc(nb), *yr = (double *)malloc(mb), *zr = (double *)malloc(nb);
        if (ray_src == 2) eval_rays(&P, xa, ya, axa, atya, xan, yan, axan, atyan, &Rray, xr, yr, zr);
        else if (halpern) eval_rays(&P, xa, ya, axa, atya, xp, yp, axp, atyp, &Rray, xr, yr, zr);
        else eval_rays(&P, x, y, ax, aty, xp, yp, axp, atyp, &Rray, xr, yr, zr);
        if (status == ORA_PRIMAL_INFEASIBLE) {
            double s = 1.0 / Rray.D;
            if (y_out)
                for (int32_t i = 0; i < m; i++) y_out[i] = yr[i] * s;
            if (z_out)
                for (int32_t j = 0; j < n; j++) z_out[j] = zr[j] * s;
        } else {
            double s = 1.0 / Rray.G;
            if (x_out)
                for (int32_t j = 0; j < n; j++) x_out[j] = xr[j] * s;
        }
        free(xr);
        free(yr);
        free(zr);
    }
    info->status = status;
    info->ray_source = ray_src;
    info->output_is_avg = out_avg;
    info->iters = k;
    info->restarts = restarts;
    info->n_trace = ntr;
    info->pobj = Ko.pobj + lp->c0;
    info->dobj = Ko.dobj + lp->c0;
    info->rel_p = Ko.rel_p;
    info->rel_d = Ko.rel_d;
    info->rel_gap = Ko.rel_gap;
    info->erel = Ko.erel;
    info->sigma_max = sig;
    info->eta = eta;
    info->omega = omega;
    free(xp); free(yp); free(axp); free(atyp); free(axan); free(atyan);
    free(x); free(xa); free(xan); free(aty); free(atya);
    free(y); free(ya); free(yan); free(ax); free(axn); free(axa);
    prob_free(&P);
    return ORA_OK;
}
