/*
 * lp.h - C ABI of the MI355X restarted-PDHG linear-programming solver.
 *
 * Problem (the paper's Section 2, eq. 1):
 *
 *     minimize    c^T x + c0
 *     subject to  b_lo <= A x <= b_hi
 *                 x_lo <= x <= x_hi
 *
 * with A an m x n matrix in CSR form. Infinite entries of b_lo, b_hi, x_lo, x_hi are
 * IEEE +-inf and mean "no bound"; an equality row has b_lo = b_hi.
 *
 * Solution (eq. 2): a primal x and duals (y, z) with c - A^T y - z = 0 up to the dual
 * residual, y_i > 0 only where (Ax)_i = b_lo_i, y_i < 0 only where (Ax)_i = b_hi_i,
 * z_k > 0 only where x_k = x_lo_k, z_k < 0 only where x_k = x_hi_k, z_k = 0 for a free
 * x_k, y_i <= 0 where b_lo_i = -inf and y_i >= 0 where b_hi_i = +inf. z is returned as
 * the reduced cost c - A^T y projected onto that sign pattern (Section 2.1, the dual
 * postsolve identity z_k = c_k - a_k^T y).
 *
 * Termination: one relative tolerance eps_rel (Section 4.2) on
 *   E_rel = max(||r_p|| / (1 + ||q||), ||r_d|| / (1 + ||c||), |p - d| / (1 + |p| + |d|)),
 * with r_p the bound violation of Ax, r_d = c - A^T y - z (plus any sign violation of y),
 * p, d the primal and dual objectives and q_i the largest finite |b_lo_i|, |b_hi_i|.
 *
 * Conventions for every function:
 *  - The return value is an lp_error code (LP_OK = 0). No C++ exception crosses the ABI.
 *  - Array arguments are host pointers unless stated otherwise; the library copies what
 *    it needs before returning, so the caller may free its arrays afterwards.
 *  - A handle owns all host and device memory it allocates until lp_destroy.
 *  - A handle is not re-entrant: one call at a time per handle. Distinct handles may be
 *    used from different threads.
 *  - After a failed call, lp_last_error(h) (or lp_last_error(NULL) when no handle exists)
 *    returns a message describing the failure.
 */
#ifndef LPGPU_LP_H
#define LPGPU_LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_handle lp_handle;

typedef enum {
    LP_OK = 0,
    LP_ERR_INVALID_ARG = 1,         /* null pointer, negative size, bad option value */
    LP_ERR_INVALID_MATRIX = 2,      /* row_ptr not monotone / not 0..nnz, col_idx out of range or not strictly increasing in a row */
    LP_ERR_INCONSISTENT_BOUNDS = 3, /* lower > upper, or a lower bound of +inf / an upper bound of -inf */
    LP_ERR_NAN_INPUT = 4,           /* NaN anywhere, or an infinite matrix value or cost */
    LP_ERR_OUT_OF_MEMORY = 5,       /* host or device allocation failed */
    LP_ERR_DEVICE = 6,              /* a HIP runtime call failed */
    LP_ERR_NOT_SOLVED = 7,          /* solution requested before lp_solve */
    LP_ERR_INTERNAL = 8
} lp_error;

typedef enum {
    LP_OPTIMAL = 0,         /* E_rel <= eps_rel */
    LP_ITERATION_LIMIT = 1, /* max_iters reached */
    LP_TIME_LIMIT = 2,
    LP_NUMERICAL_ERROR = 3, /* a NaN appeared in the residuals */
    LP_PRIMAL_INFEASIBLE = 4, /* no x satisfies the constraints: lp_get_solution returns in y a
                                 dual ray and in z its projected reduced cost, with
                                 A^T y + z = 0 up to eps_infeas and ray objective
                                 sum_i (b_lo y_i^+ - b_hi y_i^-) + sum_k (x_lo z_k^+ - x_hi z_k^-) = 1;
                                 x is the last iterate */
    LP_DUAL_INFEASIBLE = 5,   /* the dual has no solution (the LP is unbounded if it is feasible):
                                 x is a primal ray with c^T x = -1 and A x, x inside the recession
                                 cones of the row and variable bounds up to eps_infeas; y, z are
                                 the last iterate's */
    LP_CANCELLED = 6          /* a server request stopped by lp_server_cancel: the point and
                                 statistics of its current iterate when it was running, no point
                                 (x, y, z NaN, 0 iterations) when it was still queued */
} lp_termination;

typedef enum {
    LP_PREC_FP64 = 0,        /* matrix, iterates and all reductions in FP64 */
    LP_PREC_FP32_REFINED = 1 /* matrix and iterates stored and accumulated in FP32 around an FP64
                                master point; KKT residuals, duality gap, restart, step-size and
                                primal-weight decisions in FP64 on the FP64 matrix; at every
                                restart the master moves to the restart point and the FP32
                                correction data are recomputed in FP64 (iterative refinement) */
} lp_precision;

typedef enum {
    LP_METHOD_AVERAGED = 0, /* restarted PDHG with running averages (PDLP family): the averages
                               and the iterate are the candidates of every evaluation */
    LP_METHOD_HALPERN = 1   /* reflected Halpern PDHG: z <- w ((1 + rho) T(z) - rho z) + (1 - w) z0
                               with T the PDHG map, z0 the anchor of the restart cycle and
                               w = (t + 1) / (t + 2) after t iterations of the cycle; the PDHG
                               output T(z) is the only candidate (termination, restarts,
                               certificates and the returned point), a restart moves the iterate
                               and the anchor to it (the newer cuPDLPx-family form) */
} lp_method;

typedef enum lp_layout {
    LP_LAYOUT_PANELS = 0, /* panel-packed wave units */
    LP_LAYOUT_TILES = 1,  /* row tiles of up to a fixed number of nonzeros per workgroup */
    LP_LAYOUT_TUNED = 2   /* the faster of the two on the device, measured at set-up */
} lp_layout;

typedef struct lp_options {
    double eps_rel;        /* relative tolerance on E_rel (default 1e-4) */
    int64_t max_iters;     /* iteration limit (default 100000) */
    double time_limit_s;   /* wall-clock limit of a solve (default: none, 0), checked at every evaluation
                              (each eval_every iterations): by the host in lp_solve; on the device, against
                              its wall clock, for each LP of lp_solve_batch and lp_solve_batch_static (from
                              the start of the call) and for each request of a server (from its admission).
                              A solve stopped by it returns LP_TIME_LIMIT and the point last evaluated. */
    int32_t eval_every;    /* iterations between KKT evaluations / restart checks (default 64) */
    int32_t precision;     /* lp_precision (default LP_PREC_FP64) */
    int32_t scaling;       /* 1: power-of-two Ruiz + Pock-Chambolle scaling (default), 0: none */
    int32_t ruiz_passes;   /* number of infinity-norm Ruiz passes (default 10) */
    int32_t pow_iters;     /* power-iteration chunk for ||A~||_2 (default 200): after each chunk of
                            * this many steps the iteration stops when its last step raised the
                            * estimate by at most 1e-8 of it; at most 25 chunks */
    int32_t restarts;      /* 1: adaptive restarts and primal-weight updates (default), 0: off */
    double step_size;      /* eta; <= 0 selects 0.998 / ||A~||_2 (default 0) */
    double omega0;         /* initial primal weight; <= 0 selects ||c~|| / ||q~|| (default 0) */
    uint64_t seed;         /* seed of the power-iteration start vector */
    void *hip_stream;      /* hipStream_t to run on; NULL: the library creates its own */
    int32_t device;        /* HIP device ordinal (default 0) */
    int32_t trace_cap;     /* number of evaluation records kept for lp_get_trace (default 4096) */
    int32_t spmv_layout;   /* sparse-product layout: 0 panel-packed wave units (default), 1 row tiles,
                            * 2 tuned: both are built and timed on the device at set-up (a few
                            * products each, on scratch buffers) and the faster one is kept; the
                            * choice depends on the measurement, so two handles of one LP may
                            * differ in rounding (deferred clones share their template's choice) */
    int32_t long_row_len;  /* rows longer than this get a workgroup of their own (default 256) */
    int32_t units_per_cu;  /* wave units per compute unit the panel layout aims for, never exceeds
                              (default 4; a workgroup holds 2 units, each with a producer and a
                              consumer wave, so even values fill every CU evenly) */
    int32_t batch_wg_per_cu; /* lp_solve_batch: workgroups per compute unit (default 3) */
    int64_t panel_slice_bytes; /* bytes of the gathered vector per column panel (default 512 KiB) */
    int64_t batch_split_nnz;   /* lp_solve_batch: LPs with more nonzeros go to the block-diagonal
                                  multi-LP launches, the rest to the persistent kernel (default 20000) */
    int32_t deferred;      /* 1: lp_create validates and prepares on the host only; device memory is
                              allocated (and the setup run) when the LP is first solved or admitted
                              by a server, and released by the server when it completes (default 0) */
    int32_t small_lp_lds;  /* bytes of LDS per workgroup (0 to 114688, default 114688) for LPs
                              held on chip. lp_solve_batch: an LP of the persistent launch whose
                              matrices and iteration vectors (in its precision) fit is solved from
                              LDS by a launch of its own (one workgroup per CU), bit-identical to
                              the solve from global memory. lp_solve: such an LP is solved by one
                              workgroup from LDS (the whole loop in one launch, the row-tile
                              products; not with kernel timing on, and not for lp_polish's
                              solves), bit-identical to the kernel-per-phase loop with row tiles
                              (lp_info.solve_path = 1). 0 turns both off */
    const double *x0;      /* optional warm start (host, length n, original scale) */
    const double *y0;      /* optional warm start (host, length m, original scale) */
    double eps_infeas;     /* relative tolerance of the infeasibility certificates (default 1e-8;
                              0 turns the test off). At each evaluation after the first, two
                              candidate rays are tested as a dual ray (primal infeasibility) and
                              as a primal ray (dual infeasibility), in this order: the
                              displacement of the evaluated point since the previous evaluation,
                              then the averaged point (the PDHG output in the Halpern form)
                              minus the anchor of the restart cycle; see LP_PRIMAL_INFEASIBLE /
                              LP_DUAL_INFEASIBLE and lp_info.ray_source */
    int32_t method;        /* lp_method (default LP_METHOD_AVERAGED) */
    int32_t restart_metric; /* LP_METHOD_HALPERN: what the three restart tests compare. 0 (default):
                              the KKT error of T(z) in the primal-weighted norm; 1: the
                              fixed-point residual ||z - T(z)|| in the norm of the PDHG map,
                              omega ||dx||^2 + 2 eta <dy, A~dx> + ||dy||^2 / omega (the restart
                              rule of the Halpern PDHG family of Section 4's solver), for the
                              last iterate before an evaluation and for the cycle's anchor.
                              Termination still tests E_rel. The averaged form ignores it */
    double reflection;     /* rho of LP_METHOD_HALPERN, in [0, 1] (default 1) */
    int32_t omega_steps;   /* primal-weight update at a restart: omega <- sqrt(omega * dy / dx)
                            * applied this many times, i.e. log omega moves toward log(dy/dx)
                            * by the fraction 1 - 2^-omega_steps; 1 to 8, or 0 (default) for
                            * the form's own: 1 for LP_METHOD_AVERAGED, 2 for LP_METHOD_HALPERN */
    int32_t pad3;
    int32_t pw_rule;       /* lp_primal_weight_rule of the update at a restart (default 0) */
    int32_t pad4;
    double pid_kp, pid_ki, pid_kd; /* gains of LP_PW_PID (defaults 0.7, 0.05, 0.2), each in [0, 2] */
    int32_t tile_nnz;      /* row-tile shape of the row-tile products (lp_solve with spmv_layout 1 or
                              2, lp_solve_batch, servers): 1024, 2048 or 4096 nonzeros per tile (and
                              a quarter as many rows), or 0 (default) for the shape the tuned table
                              gives this LP's precision, mean row length and size (the table is
                              written by paper_2604_23951_amd/tune_tiles.py on the device). A row
                              longer than the tile is reduced by a workgroup of its own, so the
                              shape decides which rows are summed by a tree */
    int32_t pad5;
} lp_options;

/* Primal-weight update at a restart, from the distances dx, dy the restart point moved
 * (scaled space) since the previous restart, when both exceed 1e-10:
 *  LP_PW_SMOOTH: omega <- sqrt(omega * dy / dx), omega_steps times (the default);
 *  LP_PW_PID:    a PID controller on the error e = log(omega * dx / dy) of the imbalance of
 *                the weighted distances: I += e, log omega -= kp e + ki I + kd (e - e_prev),
 *                e_prev = e (I and e_prev are 0 at the start of a solve). With ki = kd = 0
 *                it is the smoothing with fraction kp. */
typedef enum {
    LP_PW_DEFAULT = 0, /* LP_PW_SMOOTH */
    LP_PW_SMOOTH = 1,
    LP_PW_PID = 2
} lp_primal_weight_rule;

typedef struct lp_info {
    int32_t status;        /* lp_termination */
    int32_t output_is_avg; /* 1 if the returned point is the running average */
    int64_t iterations;
    int64_t restarts;
    double primal_obj, dual_obj;          /* p and d of the returned point, c0 included */
    double rel_primal_res, rel_dual_res, rel_gap, rel_kkt; /* the three E_rel terms and E_rel */
    double sigma_max;      /* power-iteration estimate of ||A~||_2 (0 if step_size was given) */
    double step_size;      /* eta used */
    double omega;          /* final primal weight */
    double setup_seconds;  /* lp_create: upload, transpose, scaling, norm estimate */
    double solve_seconds;  /* last lp_solve */
    int64_t done_clock;    /* the device's wall clock when this LP's solve stopped (in a batch:
                              each LP's own instant); ticks of clock_hz, comparable across the
                              LPs of one device */
    double clock_hz;       /* rate of that clock */
    int64_t polish_primal_iterations, polish_dual_iterations; /* of the last lp_polish (0 after lp_solve) */
    double polish_seconds; /* last lp_polish */
    int32_t ray_source;    /* with a certificate (status 4 or 5), the candidate ray it came from:
                              1 the displacement of the evaluated point since the previous
                              evaluation, 2 the averaged point (the PDHG output in the Halpern
                              form) minus the restart anchor; 0 otherwise */
    int32_t solve_path;    /* how lp_solve ran: 0 one kernel per phase (the spmv_layout products,
                              hipGraph periods), 1 one workgroup from LDS (an LP whose iteration
                              arrays fit small_lp_lds, see there); batched and served LPs: 0 */
} lp_info;

/* Fill *opt with the defaults listed above. */
void lp_default_options(lp_options *opt);

/* Option presets for the workloads the library was measured on: *opt is filled with the
 * defaults, then with the preset's fields (the choices that measured best for that
 * workload on MI355X; every field stays adjustable afterwards). LP_ERR_INVALID_ARG for an
 * unknown preset or NULL opt (then *opt is left unchanged).
 *   LP_PRESET_DEFAULT     the defaults.
 *   LP_PRESET_SMALL       one small LP solved for latency by lp_solve (hundreds of rows):
 *                         row-tile layout (its products take one or two tiles), reflected
 *                         Halpern form, FP64.
 *   LP_PRESET_LARGE       one large LP (millions of nonzeros) to eps_rel: panel-packed
 *                         layout, reflected Halpern form, FP64.
 *   LP_PRESET_LARGE_FP32  the same in the FP32 storage form with FP64 refinement (half the
 *                         matrix bytes; E_rel is still evaluated in FP64).
 *   LP_PRESET_BATCH       many LPs through lp_solve_batch / lp_solve_batch_static: FP32
 *                         storage, reflected Halpern form, row tiles (the layout of the batched
 *                         launches).
 *   LP_PRESET_SERVING     template handles for a server: as LP_PRESET_BATCH, with deferred = 1. */
typedef enum lp_preset {
    LP_PRESET_DEFAULT = 0,
    LP_PRESET_SMALL = 1,
    LP_PRESET_LARGE = 2,
    LP_PRESET_LARGE_FP32 = 3,
    LP_PRESET_BATCH = 4,
    LP_PRESET_SERVING = 5
} lp_preset;
int32_t lp_preset_options(lp_options *opt, int32_t preset);

/* Create a solver handle for the LP of eq. (1) and prepare it on the GPU.
 *   m >= 0 rows, n >= 1 columns, nnz = row_ptr[m] entries with nnz <= 2^31 - 2^16 - 1 (the
 *   kernels form entry offsets in 32 bits; LP_ERR_INVALID_ARG above that).
 *   row_ptr[m+1] (int32, row_ptr[0] = 0, non-decreasing), col_idx[nnz] (int32 in [0, n),
 *   strictly increasing inside each row), vals[nnz] (finite float64; explicit zeros kept).
 *   c[n] finite; c0 finite constant; b_lo[m], b_hi[m], x_lo[n], x_hi[n] with lower <= upper,
 *   lower < +inf, upper > -inf. For m = 0, row_ptr must still hold one entry (0) and b_lo,
 *   b_hi may be NULL.
 *   opt may be NULL (defaults). The option struct is copied; x0/y0 are copied if given.
 * The setup (a CSR transpose, the scaling, the ||A~||_2 estimate and the step size) runs
 * on the device selected by opt->device. On success *out receives the handle. */
int32_t lp_create(lp_handle **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                  const int32_t *col_idx, const double *vals, const double *c, double c0,
                  const double *b_lo, const double *b_hi, const double *x_lo, const double *x_hi,
                  const lp_options *opt);

/* Run restarted PDHG (the form of opt->method) from the start point until E_rel <= eps_rel,
 * a certificate or a limit. Every call starts again from x0, y0 (the handle keeps the
 * problem, not the iterates). An LP whose iteration arrays fit small_lp_lds bytes of LDS
 * runs the whole loop on one workgroup in one launch; any other runs one kernel per phase,
 * an evaluation period (eval_every iterations, the evaluation, the decision) per hipGraph
 * replay, the host reading the status once per period. lp_info.solve_path says which. */
int32_t lp_solve(lp_handle *h);

/* Feasibility polishing of the point the last lp_solve returned (the PDLP family's polishing;
 * the paper runs a solver of that family, Section 4), two more solves of the same form on the
 * device, warm-started at that point and stopped on one residual alone:
 *  - primal: the LP's constraints with the objective removed (c = 0), from (x, 0), until the
 *    relative primal residual ||r_p|| / (1 + ||q||) is at most eps: a point that satisfies the
 *    constraints to eps, near x;
 *  - dual: the LP's matrix and costs with every finite row and variable bound set to 0 (the
 *    problem whose dual constraints are those of the LP), from (0, y), until the relative dual
 *    residual ||r_d|| / (1 + ||c||) is at most eps: a dual point feasible to eps, near y.
 * Both start at primal weight 1 (one of ||c||, ||q|| vanishes in each) with the LP's step size
 * and stop at max_iters iterations at most. lp_get_solution then returns x of the first, y of
 * the second and z = the projected reduced cost of that y, and info holds their E_rel terms
 * (the gap is not polished), the status of the lp_solve and the polishing iterations. The
 * handle's data are restored. LP_ERR_NOT_SOLVED before lp_solve; LP_ERR_INVALID_ARG after a
 * solve that returned a certificate, or for eps <= 0. */
int32_t lp_polish(lp_handle *h, double eps, int64_t max_iters);

/* ---- checkpoint and resume ---------------------------------------------------------
 * Not an operation of the paper: a way to split one run of the method of Section 4 (the
 * restarted PDHG loop of lp_solve) into pieces, for callers that must give up the device
 * between pieces or keep a run across processes.
 * lp_solve_until runs lp_solve's loop (one kernel per phase, whatever small_lp_lds says) but
 * pauses after the first evaluation period that ends at or beyond iteration k_pause (> 0,
 * else LP_ERR_INVALID_ARG): the period's decision and restart are applied, the status reads
 * LP_ITERATION_LIMIT, lp_get_solution returns the paused point and its statistics, and the
 * handle is resumable. A solve that stops earlier (tolerance, certificate, max_iters, time
 * limit) returns as lp_solve does and is not resumable.
 * lp_resume continues a resumable handle's run from its device state until the handle's
 * current eps_rel, max_iters, time_limit_s (counted from the lp_resume call) or eps_infeas
 * stop it, or, with k_pause > 0, pauses again as lp_solve_until does; the new tolerances are
 * first tested at the end of the next period, and max_iters at or below the paused
 * iteration count leaves the handle paused. lp_update_options may change those four;
 * eval_every, restarts, the iteration form and the primal-weight rule must stay
 * (LP_ERR_INVALID_ARG). With unchanged options the iterates, restarts, decision trace and
 * result are bit for bit those of one uninterrupted lp_solve, however the run is split.
 * LP_ERR_NOT_SOLVED if the handle is not resumable. lp_solve, lp_polish and the batched
 * solves end a handle's resumable state.
 * lp_export_state copies a resumable handle's state (iterates, averages, anchors, the point
 * of the previous evaluation, the products kept across periods, the FP32 form's corrections,
 * shifted data and master point, the scalar state and the decision trace) into the host
 * buffer buf of cap bytes and sets *size to its length (buf NULL: only *size;
 * LP_ERR_INVALID_ARG if cap is smaller). lp_import_state loads such a buffer into a handle
 * of the same LP with the same precision, trace capacity and iteration options, which must
 * hold its device memory (not deferred, or solved once); the handle is then as the exporting
 * one was at its pause (resumable, same lp_get_solution). LP_ERR_INVALID_ARG for a buffer of
 * another size or version, another iteration form, or another LP (told by its sizes and a
 * hash of the scaled cost and scaling factors). The buffer holds plain bytes of this
 * library build (for a file kept beside it), not a portable format. */
int32_t lp_solve_until(lp_handle *h, int64_t k_pause);
int32_t lp_resume(lp_handle *h, int64_t k_pause);
int32_t lp_export_state(lp_handle *h, void *buf, int64_t cap, int64_t *size);
int32_t lp_import_state(lp_handle *h, const void *buf, int64_t size);

/* Replace the solve-time options of a handle: eps_rel, max_iters, time_limit_s, eval_every,
 * restarts, eps_infeas, method, reflection, omega_steps, pw_rule and the three pid gains are
 * taken from *opt; every other field of *opt is ignored (the problem setup, the step size and the trace capacity are fixed at lp_create). */
int32_t lp_update_options(lp_handle *h, const lp_options *opt);

/* Batched form: solve the LPs of `count` handles (created on the same device) together.
 *  - LPs with at most batch_split_nnz nonzeros run in one persistent launch: each workgroup
 *    takes the next LP from a device work counter (largest first) and runs that LP's whole
 *    restarted PDHG on chip (row-tile sparse products with the fused updates, FP64
 *    evaluations, restart and termination decisions).
 *  - Larger LPs advance together as one block-diagonal problem: every launch covers the row
 *    tiles of all of them, each LP with its own step sizes, restarts and termination;
 *    evaluation periods are replayed as one hipGraph for the group; when a quarter of the
 *    group has stopped the launches are rebuilt over the running LPs. Each such LP follows
 *    exactly the trajectory of its own lp_solve with the row-tile layout. The persistent
 *    launch runs on a stream of its own beside these launches.
 * Each LP's result depends only on that LP (not on the other LPs or on where it ran), so it
 * is the same alone and in any batch. The handles' precisions may differ.
 * Solve-time options: batch_opt's eps_rel, max_iters, time_limit_s, eval_every and restarts for every LP
 * when batch_opt is given, each handle's own otherwise (the LPs of the block-diagonal group
 * must then share eval_every); batch_opt->batch_wg_per_cu and batch_split_nnz set the
 * launches. Afterwards every handle is solved and lp_get_solution returns its result
 * (info.solve_seconds is the batch time). Runs on the first handle's stream (and a
 * temporary second stream for the persistent launch) and waits. */
int32_t lp_solve_batch(lp_handle *const *hs, int32_t count, const lp_options *batch_opt);

/* Allocation-free form of lp_solve_batch, for callers that cannot allocate device memory
 * (work issued inside a stream capture, tight serving loops, harnesses that forbid
 * hipMalloc). On success it calls no hipMalloc, hipFree, stream or event creation and no
 * other allocating routine; it still waits for the GPU before returning.
 *  - Every LP runs in the persistent one-workgroup-per-LP launch of lp_solve_batch, whatever
 *    its size (lp_solve_batch sends LPs above batch_split_nnz to block-diagonal launches,
 *    whose per-call maps would need allocations). An LP's result is bit-identical to the one
 *    lp_solve_batch gives it in the persistent launch.
 *  - The launch's job table, LP order and work counter live in a library-owned static device
 *    array of fixed size (LP_STATIC_BATCH_MAX jobs, 3.2 MB), one copy per device, held
 *    until the process ends; the counter is cleared by a kernel at every call. count above
 *    LP_STATIC_BATCH_MAX returns LP_ERR_INVALID_ARG.
 *  - Every handle must already hold its device memory (created with deferred = 0, or solved
 *    once): LP_ERR_INVALID_ARG otherwise, as for handles on different devices.
 *  - Calls on one device share that array: two calls that overlap in time on one device race
 *    and must be serialised by the caller. Runs on the first handle's stream.
 * Options as for lp_solve_batch (batch_opt's eps_rel, max_iters, time_limit_s, eval_every, restarts,
 * eps_infeas, method, reflection, omega_steps and batch_wg_per_cu, or each handle's own). */
#define LP_STATIC_BATCH_MAX 4096
int32_t lp_solve_batch_static(lp_handle *const *hs, int32_t count, const lp_options *batch_opt);

/* ---- serving form -------------------------------------------------------------------
 * A server solves LPs as they arrive, with continuous batching: a worker thread keeps a
 * running set of LPs on the device and advances all of them together, one evaluation
 * period (eval_every iterations, evaluation, restart decision) per round of shared
 * block-diagonal launches (replayed as a hipGraph while the set is unchanged). Between
 * rounds it retires the LPs that stopped (their result is copied to the host and their
 * device memory released) and takes in the requests that are ready. A second (set-up)
 * thread admits queued requests in arrival order while a slot is free and the request's
 * device footprint fits the HBM budget, and sets each up on the device (upload, scaling,
 * norm estimate) on its own stream while the rounds run. Every LP starts at its own iteration 0 and keeps its own step sizes, restarts and
 * counters, so its result is the same as when it is solved alone.
 * A submitted handle is a template: it must be created with opt->deferred = 1, it is not
 * modified, and it may be submitted any number of times, also while earlier submissions of
 * it are queued or running; every submission is a request of its own, with device memory
 * allocated at admission and released at completion. The result of a request is fetched
 * once with lp_server_result. */
typedef struct lp_server lp_server;

typedef struct lp_server_stats {
    int64_t submitted, admitted, completed, queued, running;
    int64_t rounds;            /* evaluation periods run */
    int64_t bytes_in_use;      /* device bytes of the admitted LPs */
    int64_t peak_bytes;        /* largest bytes_in_use seen */
    int64_t hbm_budget;
    int64_t lp_iterations;     /* PDHG iterations run, summed over the served LPs */
    double nnz_iterations;     /* sum over those iterations of the LP's nnz(A) (work done) */
} lp_server_stats;

/* Start a server on `device` with a device-memory budget for admitted LPs and at most
 * max_slots LPs in the running set. The solve-time fields of *opt (eps_rel, max_iters,
 * time_limit_s counted from each request's admission, eval_every, restarts) apply to every
 * LP; opt may be NULL (defaults). */
int32_t lp_server_create(lp_server **out, int32_t device, int64_t hbm_budget_bytes, int32_t max_slots,
                         const lp_options *opt);

/* Queue a request to solve the LP of a deferred handle; returns at once with its ticket.
 * LP_ERR_INVALID_ARG for a handle that is not deferred or whose footprint exceeds the
 * whole budget. The handle must outlive its requests' admission (its host data is shared). */
int32_t lp_server_submit(lp_server *srv, lp_handle *h, uint64_t *ticket);

/* Result of a completed request (original scale, as lp_get_solution) and its run record;
 * any pointer may be NULL. The request's storage is released: a second call for the same
 * ticket returns LP_ERR_NOT_SOLVED. */
int32_t lp_server_result(lp_server *srv, uint64_t ticket, double *x, double *y, double *z, lp_info *info);

/* Tickets completed since the last poll (each reported once), at most cap of them. For a
 * completed ticket, times[0..2] of lp_server_ticket_times are the submit, admit and
 * completion instants in seconds on the server's clock. Never blocks. */
int32_t lp_server_poll(lp_server *srv, uint64_t *done_tickets, int32_t cap, int32_t *n_done);
int32_t lp_server_ticket_times(lp_server *srv, uint64_t ticket, double *times);

/* Cancel a request. Still queued (not admitted): it completes at once with LP_CANCELLED and
 * no point. Admitted (being set up or running): the worker stops it after the current round
 * (one evaluation period) with LP_CANCELLED and the point and statistics of its current
 * iterate, as a host-side stop of lp_solve gives them, and releases its device memory and
 * slot. A request that completes on its own before the worker acts keeps its own status.
 * LP_ERR_INVALID_ARG for a ticket that is not pending (unknown, completed, or already
 * cancelled). Not an operation of the paper: the serving form's way to drop work. */
int32_t lp_server_cancel(lp_server *srv, uint64_t ticket);

/* Block until every submitted request has completed, or until timeout_s seconds (<= 0: no
 * limit); LP_ERR_INTERNAL on timeout. */
int32_t lp_server_wait(lp_server *srv, double timeout_s);

int32_t lp_server_stats_get(lp_server *srv, lp_server_stats *st);

/* Stop the worker after the current round; queued and running LPs are left unsolved. */
void lp_server_destroy(lp_server *srv);

/* ---- presolve and postsolve (Section 3) -----------------------------------------------
 * A lightweight host presolver built from the atomic reductions of Section 2.1 (fix a
 * variable, remove a constraint, change bounds, substitute a variable out through an
 * equality row), driven by the fast explorers of Section 3.1 (Table 1): empty and singleton rows,
 * redundant rows and row sides by minimum / maximum activity, empty and fixed columns,
 * column singletons of equality rows, doubleton equality rows whose substitution adds no
 * nonzero (it changes values of existing entries of the partner column) and variable locks
 * (Section 2.3). It runs sequentially
 * on the CPU and touches no device. lp_presolve takes an LP of eq. 1 (same arguments and
 * validation as lp_create) and keeps a reduced LP of the same form; lp_postsolve maps an
 * (approximate) solution of the reduced LP to (x, y, z) of the original (eq. 2): y of a
 * removed row and z of a removed column are recovered from the reductions in reverse order,
 * z_k = c_k - a_k^T y for a fixed column (Section 2.1). Reductions never add nonzeros, so
 * nnz(reduced) <= nnz. The presolver owns its memory until lp_presolve_destroy. */
typedef struct lp_presolver lp_presolver;

typedef enum {
    LP_PRESOLVE_REDUCED = 0,    /* a reduced LP with at least one variable is available */
    LP_PRESOLVE_SOLVED = 1,     /* every variable was fixed: the reduced LP is empty (m = n = 0);
                                   lp_postsolve with empty inputs gives the solution */
    LP_PRESOLVE_INFEASIBLE = 2, /* some row or bound is violated by every point */
    LP_PRESOLVE_UNBOUNDED = 3   /* a variable whose cost favours an unlocked direction has no bound
                                   there: the LP is unbounded or infeasible */
} lp_presolve_status;

typedef struct lp_presolve_options {
    int32_t max_rounds;      /* rounds of all explorers at most (default 32) */
    int32_t dual_reductions; /* 1: fixing by variable locks (default); 0: primal reductions only */
    int32_t substitute;      /* 1: eliminate column singletons of equality rows (default) */
    int32_t doubletons;      /* 1: eliminate doubleton equality rows whose substitution adds no
                                nonzero (default) */
    double feas_tol;         /* tolerance of the infeasibility tests (default 1e-9) */
    double pivot_tol;        /* smallest |a_ik| / max_j |a_ij| accepted for a substitution (default 1e-3) */
} lp_presolve_options;

typedef struct lp_presolve_info {
    int32_t status;          /* lp_presolve_status */
    int32_t m, n;            /* reduced sizes */
    int64_t nnz;             /* reduced nonzeros */
    int32_t rounds;
    int64_t empty_rows, singleton_rows, redundant_rows, dropped_sides;
    int64_t empty_cols, fixed_cols, lock_fixed_cols, substituted_cols;
    double seconds;          /* wall time of lp_presolve */
    int64_t doubleton_cols;  /* columns eliminated through doubleton equality rows */
    int64_t cancelled_entries; /* entries a doubleton substitution turned to exactly zero (they
                                  leave the counts and the reduced LP; explicit zeros of the
                                  input are never counted or exported either) */
} lp_presolve_info;

void lp_presolve_default_options(lp_presolve_options *opt);

/* Presolve the LP; opt may be NULL (defaults), info may be NULL. On LP_OK *out holds a
 * presolver whatever the status in info (an infeasible or unbounded status leaves nothing
 * to postsolve). Validation errors as for lp_create. */
int32_t lp_presolve(lp_presolver **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                    const int32_t *col_idx, const double *vals, const double *c, double c0,
                    const double *b_lo, const double *b_hi, const double *x_lo, const double *x_hi,
                    const lp_presolve_options *opt, lp_presolve_info *info);

int32_t lp_presolve_get_info(const lp_presolver *p, lp_presolve_info *info);

/* Copy the reduced LP into caller arrays sized by info (row_ptr[m+1], col_idx[nnz],
 * vals[nnz], c[n], b_lo[m], b_hi[m], x_lo[n], x_hi[n]) and its objective offset to *c0.
 * Rows and columns keep their original relative order. */
int32_t lp_presolve_get_reduced(const lp_presolver *p, int32_t *row_ptr, int32_t *col_idx, double *vals,
                                double *c, double *c0, double *b_lo, double *b_hi, double *x_lo, double *x_hi);

/* Original index of each reduced row (row_map[m]) and column (col_map[n]). */
int32_t lp_presolve_get_maps(const lp_presolver *p, int32_t *row_map, int32_t *col_map);

/* Map a solution (x[n], y[m], z[n]) of the reduced LP to x_out[n0], y_out[m0], z_out[n0] of
 * the original LP. The inputs may be NULL when the reduced size is 0. */
int32_t lp_postsolve(const lp_presolver *p, const double *x, const double *y, const double *z,
                     double *x_out, double *y_out, double *z_out);

void lp_presolve_destroy(lp_presolver *p);

/* Copy the returned point (original scale) to caller buffers x[n], y[m], z[n] and the run
 * record to *info. Any pointer may be NULL to skip it. LP_ERR_NOT_SOLVED before lp_solve. */
int32_t lp_get_solution(lp_handle *h, double *x, double *y, double *z, lp_info *info);

/* Release everything the handle owns. NULL is ignored. */
void lp_destroy(lp_handle *h);

/* The checked build (liblpgpu_checked.so, compiled with LPGPU_CHECKED=1) bounds-checks every
 * gathered column and every accumulator row in the product kernels: an index outside its
 * array sets a bit of a per-device word (1 panel gather, 2 panel accumulator row, 4 row-tile
 * gather, 8 long-row gather) and is replaced by 0, so the kernel goes on without reading
 * outside its arrays. lp_solve, lp_solve_until, lp_resume, lp_polish, lp_solve_batch and
 * lp_solve_batch_static of that build return LP_ERR_INTERNAL when the word is set after them.
 * lp_check_word reads and clears the word of `device` (for servers and for callers of the
 * plain build) and sets *checked to 1 in the checked build, 0 otherwise (*word is then 0).
 * A debugging aid, not an operation of the paper. */
int32_t lp_check_word(int32_t device, uint32_t *word, int32_t *checked);

/* Static description of an error code. */
const char *lp_error_string(int32_t code);

/* Message of the last failed call on h (thread-local last error when h is NULL). */
const char *lp_last_error(const lp_handle *h);

/* ---- inspection (used by the parity tests) ------------------------------------------ */

/* Iterate state in the scaled space right now: x~[n], y~[m], the running averages
 * x~avg[n], y~avg[m]. After lp_solve with max_iters = k this is the state after the update
 * of iteration k, before that iteration's evaluation acts on it. Any pointer may be NULL. */
int32_t lp_get_iterates(lp_handle *h, double *x, double *y, double *x_avg, double *y_avg);

/* The scaled problem: A~ values in the caller's CSR order vals[nnz], the factors R[m] and
 * C[n] (A~ = diag(R) A diag(C)), and A~^T as CSR: t_row_ptr[n+1], t_col_idx[nnz],
 * t_vals[nnz]. Any pointer may be NULL. */
int32_t lp_get_scaled(lp_handle *h, double *vals, double *R, double *C, int32_t *t_row_ptr,
                      int32_t *t_col_idx, double *t_vals);

/* Evaluation records of the last lp_solve, LP_TRACE_WIDTH doubles each:
 *   [k, t, KKT_w(current), KKT_w(average), E_rel(current), E_rel(average), candidate
 *    (1 = average), restart reason (0 none, 1 deep decay, 2 no progress, 3 long cycle),
 *    omega after the decision, KKT_w of the anchor, previous candidate KKT_w, margin]
 * margin = the smallest relative gap between two quantities a decision compared.
 * Writes min(cap, available) records to out and the available count to *n_records. */
#define LP_TRACE_WIDTH 12
int32_t lp_get_trace(lp_handle *h, double *out, int32_t cap, int32_t *n_records);

/* Per-kernel timing of the next lp_solve calls: when enabled, the primal (A^T y + primal
 * update) and dual (A x + dual update) kernels of one iteration per evaluation period are
 * bracketed by HIP events on the solver stream. lp_get_kernel_times returns the mean
 * duration in milliseconds of each and the number of samples since enabling. */
int32_t lp_set_kernel_timing(lp_handle *h, int32_t enable);
int32_t lp_get_kernel_times(lp_handle *h, double *primal_ms, double *dual_ms, int64_t *samples);

/* Sizes the solver chose: sizes[0] = tiles of A, [1] = tiles of A^T, [2] = long rows of
 * A, [3] = long rows of A^T, [4] = device bytes held by the handle, [5] = wave units of A,
 * [6] = wave units of A^T, [7] = column panels of A, [8] = column panels of A^T,
 * [9] = layout of the products (0 panels, 1 row tiles; -1 before the handle is on the
 * device), [10] / [11] = the layout tuner's time in nanoseconds of one A x + A^T y pair in
 * panels / row tiles (0 unless spmv_layout is 2), [12] = nonzeros per row tile (the shape
 * chosen from tile_nnz or the tuned table). */
int32_t lp_get_layout(lp_handle *h, int64_t *sizes, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* LPGPU_LP_H */
