// Internal device-side types and kernel launchers of the restarted-PDHG solver.
// Everything here is private to the library; the public surface is include/lp.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lpgpu {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
// Row-tile shapes of the LDS-staged SpMV: shape h holds at most tile_nnz_of(h) nonzeros
// (1024, 2048, 4096) and a quarter as many rows; the shape of an LP comes from its options or
// the tuned table (lp_tile_table.h).
constexpr int kTileShapes = 3;
__host__ __device__ constexpr int tile_nnz_of(int shape) { return 1024 << shape; }
constexpr int kTileNnzMax = 4096;
constexpr int kMaxRedBlocks = 512;
constexpr int kNQ = 8;            // reduced quantities per candidate
constexpr int kNR = 8;            // reduced quantities of the two candidate rays (infeasibility), 4 each
constexpr int kNF = 6;             // sums of the residual restarts: ||dx||^2, <dy, A~dx>, ||dy||^2 (last iterate, anchor)
constexpr int kNT = 2 * kNQ + kNR + kNF;  // all reduced quantities of one evaluation
constexpr int kTraceW = 12;

constexpr int kRunning = -1;

// Largest nonzero count accepted. The kernels form entry offsets in 32-bit ints and clamp
// indices that run past the end of a row, tile or unit (by at most a few thousand entries:
// the panel producer's prefetch reaches 16 groups of 256 entries ahead); the margin keeps
// every such offset below 2^31.
constexpr long long kMaxEntries = 0x7fffffffLL - (1LL << 16);

// Device-resident scalar state of one solve. The iteration kernels read it; only the
// single-workgroup decision kernels write it.
struct Scalars {
    double tau, sigma, omega, eta, omega0;
    double eps_rel, c0, qnorm, cnorm, sigma_max, sigma_prev;  // sigma_prev: the power step before
    double kkt_anchor, kkt_prev;
    double eps_infeas, ray_scale;  // certificate tolerance (0: off); 1/D or 1/G of a certificate
    double anc_rps2, anc_rds2, anc_gap;
    double pid_int, pid_prev;  // PID rule of the primal weight: integral and previous error
    // statistics of the returned point
    double out_pobj, out_dobj, out_rel_p, out_rel_d, out_rel_gap, out_erel;
    long long k, t, max_iters, restarts, n_trace, trace_cap;
    long long done_clock;  // device wall clock (wall_clock64) when the solve stopped
    long long deadline;    // device wall clock at which an evaluation stops the solve with LP_TIME_LIMIT (0: none)
    int status;        // kRunning or an lp_termination value
    int out_avg;       // returned point: 1 = running average
    int last_restart;  // what the apply kernel must do: 0 nothing, 1 keep current, 2 take average
    int eval_every;
    int restarts_on;
    int term_mode;     // what must fall to eps_rel to stop: 0 E_rel, 1 rel. primal residual, 2 rel. dual residual
    int ray_src;       // candidate ray of a certificate: 1 displacement since the previous evaluation, 2 anchored average
};

// CSR matrix with its LDS tiling: tile b covers rows [tiles[b], tiles[b+1]), or, when
// rowlist is set, the single row rowlist[b].
struct Csr {
    int rows;
    int ntiles;
    int nnz;
    int shape;  // row-tile shape (tile_nnz_of(shape) nonzeros per tile at most)
    const int* rp;
    const int* ci;
    const double* v;
    const int* tiles;
    const int* rowlist;
    const float* v32;  // FP32 copy of v (FP32 storage form only)
    int cols;          // length of the vector the products gather from
};

// Panel-packed layout (see lp_layout.h): unit u (one wave) owns rows
// [unit_row[u], unit_row[u+1]) and the entries [unit_seg[u*(panels+1)], unit_seg[u*(panels+1)+panels]),
// stored panel by panel. packed = (row inside the unit << col_bits) | column.
struct Panels {
    int units;
    int panels;
    int col_bits;
    int nnz;
    int max_rows;  // rows of the largest unit (sizes the LDS accumulators)
    const int* unit_row;
    const int* unit_seg;
    const unsigned* pk;
    const double* v;
    const unsigned char* is_long;  // nullptr when the matrix has no long rows
    const float* v32;              // FP32 copy of v (FP32 storage form only)
    int cols;                      // length of the gathered vector
};

// Index checks of the checked build (compiled with LPGPU_CHECKED=1): a gathered column or
// an accumulator row outside its array sets a bit of a device word and is replaced by 0, so
// the kernel reads nothing outside its arrays; the host reports the word after a call.
// Bits: 1 panel gather, 2 panel accumulator row, 4 row-tile gather, 8 long-row gather.
#ifndef LPGPU_CHECKED
#define LPGPU_CHECKED 0
#endif
constexpr bool kChecked = LPGPU_CHECKED != 0;
// Reads and clears the check word of `device` (0 in a build without checks).
int read_check_word(int device, unsigned* word);

constexpr int kUnitRowCap = 2048;  // rows per wave unit at most
constexpr int kChunks = 4;         // 64-entry chunks a wave loads together (one group)
constexpr int kStreamDepth = 4;    // groups of matrix entries a wave keeps loaded or in flight

// One sparse operand: CSR (scaling, inspection, long rows, row tiles) and its panel layout.
struct Mat {
    Csr csr;
    Panels pan;
    int nlong;
    const int* longrows;
    int layout;  // 0 panels, 1 row tiles
};

struct DevLP {
    int m, n;
    long long nnz;
    int nred;          // blocks of the fixed-grid reductions
    Mat A, AT;
    // scaled problem data
    const double *c, *bl, *bu, *xl, *xu;
    const double *R, *C, *Ri, *Ci;
    // iterate state (scaled space)
    double *x, *y, *xa, *ya;          // current and running averages
    double *ax, *axa, *aty, *atya;    // A~x, A~x_avg, A~^T y, A~^T y_avg
    double *xan, *yan;                // anchor (start of the current restart cycle)
    double *xp, *yp, *axp, *atyp;     // point of the previous evaluation (candidate rays)
    double *axan, *atyan;             // A~x, A~^T y of the anchor
    // Residual restarts of the Halpern form (restart_metric 1): z - T(z) as (x, y, A~x) parts,
    // written by the iteration epilogues for the last iterate before an evaluation (fr_*) and
    // for the first iterate of a restart cycle, the anchor (fa_*).
    int restart_metric;
    double *fr_x, *fr_y, *fr_ax, *fa_x, *fa_y, *fa_ax;
    // iteration form of the current solve: 0 averaged PDHG, 1 reflected Halpern PDHG with
    // reflection rho. In the Halpern form (x, y, ax) is the Halpern iterate and (xa, ya, axa)
    // the PDHG output T(z), the only candidate of the evaluations.
    int method;
    double rho;
    int omega_steps;                  // square-root steps of the primal-weight update (>= 1)
    int pw_rule;                      // 1 smoothing (omega_steps), 2 PID controller
    double kp, ki, kd;                // gains of the PID rule
    double *partials;                 // nred * kNT
    Scalars* sc;
    double* trace;
    double *out_x, *out_y, *out_z;
    // FP32 storage form: the FP32 loop iterates on the correction (dx, dy) around the FP64
    // master point (xh, yh); d32 = c~ - A~^T yh, lo32/hi32 = x~ bounds - xh,
    // rl32/ru32 = b~ bounds - A~ xh and yh32 = yh, all computed in FP64 and rounded.
    int fp32;
    float *dx, *dxa, *dy, *dya, *adx;
    float *d32, *lo32, *hi32, *rl32, *ru32, *yh32;
    double *xh, *yh;
};

// One LP of a batched solve: its device problem and the solve-time options.
struct BatchJob {
    DevLP P;
    double eps_rel;
    double eps_infeas;
    long long max_iters;
    long long trace_cap;
    int eval_every;
    int restarts_on;
    const double* x0;
    const double* y0;
    long long limit_ticks;  // time limit in device wall-clock ticks (0: none)
    const long long* t0;    // device wall clock at the start of the call (null: the LP's reset)
};

// Block maps of a block-diagonal batch: entry b of a map is (LP index, tile or block of it).
struct MultiMaps {
    const BatchJob* jobs;
    int count;
    const int2* map_a;    // row tiles of every A
    int n_a;
    const int2* map_at;   // row tiles of every A^T
    int n_at;
    const int2* map_red;  // reduction blocks (nred per LP)
    int n_red;
    const int2* map_elem; // vector blocks (ceil(max(m, n) / kBlock) per LP)
    int n_elem;
    int* active;          // number of LPs still running (MULTI_ACTIVE) or each LP's status (MULTI_STATUS)
    // The tile maps are grouped by form v = 2 * fp32 + method (FP64 / FP32 storage, averaged /
    // Halpern) and row-tile shape h: the tiles of group g = 3 v + h are entries
    // [off_a[g], off_a[g] + cnt_a[g]) of map_a (and likewise of map_at), so every launch runs
    // one kernel specialised per form and shape present.
    int off_a[12], cnt_a[12], off_at[12], cnt_at[12];
};

constexpr int kMapGroups = 4 * kTileShapes;

enum MultiLaunch {
    MULTI_PRIMAL = 0, MULTI_DUAL, MULTI_AX_ALL, MULTI_AX_FP32, MULTI_ATY, MULTI_AXA, MULTI_ATYA, MULTI_PARTIALS,
    MULTI_DECIDE, MULTI_INIT, MULTI_REBASE_INIT, MULTI_MATERIALIZE, MULTI_APPLY, MULTI_EXTRACT, MULTI_RESET,
    MULTI_ACTIVE, MULTI_STATUS
};

// ---- setup ------------------------------------------------------------------------
void launch_fill(double* p, long long n, double v, hipStream_t s);
void launch_scale_pass(const DevLP& P, int* A_rp, int* A_ci, double* A_v, const int* AT_rp, const int* perm,
                       double* R, double* C, double* rf, double* cf, int use_sum, hipStream_t s);
void launch_gather(const int* perm, const double* src, double* dst, long long nnz, hipStream_t s);
void launch_prepare(const DevLP& P, double* c, double* bl, double* bu, double* xl, double* xu, double* R, double* C,
                    double* Ri, double* Ci, double* x0, double* y0, hipStream_t s);
void launch_norms(const DevLP& P, hipStream_t s);
// Power iteration on A~^T A~: the start vector (normalised into v, sigma_max and sigma_prev
// cleared), then `iters` steps (u = A~ v, w = A~^T u, sigma_max = ||u||, v = w / ||w||).
void launch_power_start(const DevLP& P, unsigned long long seed, double* v, hipStream_t s);
void launch_power_steps(const DevLP& P, int iters, double* v, double* u, double* w, hipStream_t s);
void launch_finalize_setup(const DevLP& P, double eta_override, double omega_override, double c0, hipStream_t s);

// ---- solve ------------------------------------------------------------------------
// omega_override > 0 starts the solve at that primal weight instead of the set-up one.
void launch_reset(const DevLP& P, double eps_rel, double eps_infeas, long long max_iters, int eval_every, int restarts_on,
                  long long trace_cap, hipStream_t s, int term_mode = 0, double omega_override = 0.0);
// Statistics (products, reductions, decision in mode 2) of the point held in x = xa, y = ya.
void launch_evaluate_point(const DevLP& P, hipStream_t s);
// p[i] <- 0 where p[i] is finite (the recession cone of a bound vector).
void launch_zero_finite(double* p, long long n, hipStream_t s);
void launch_init_state(const DevLP& P, const double* x0, const double* y0, hipStream_t s);
void launch_spmv_store(const Mat& M, const double* xin, double* out, const Scalars* gate, hipStream_t s);
// reps pairs of products (A~ x, then A~^T y) in the given layout (0 panels, 1 row tiles) in the
// precision of the solve, stored to the A~x and A~^T y buffers: the trial of the layout tuner.
void launch_layout_trial(const DevLP& P, int layout, int reps, hipStream_t s);
void launch_primal(const DevLP& P, int it, hipStream_t s);
void launch_dual(const DevLP& P, int it, hipStream_t s);
void launch_evaluate(const DevLP& P, int mode, hipStream_t s);  // mode 0 regular, 1 init, 2 final
void launch_apply_restart(const DevLP& P, hipStream_t s);
void launch_stop(const DevLP& P, int status, hipStream_t s);
void launch_extract(const DevLP& P, hipStream_t s);
void launch_to_float(const double* src, float* dst, long long n, hipStream_t s);
void launch_materialize(const DevLP& P, hipStream_t s);
// Batched form: `grid` workgroups take LPs jobs[order[0]], jobs[order[1]], ... from the
// device counter (which must start at 0) and each solves one LP at a time, entirely on chip.
// lds_cap > 0: each workgroup holds lds_cap bytes of LDS (at most kSmallLpLdsMax) and solves an LP
// from LDS when small_lp_lds_bytes(LP) <= lds_cap (bit-identical result, lower latency).
constexpr int kSmallLpLdsMax = 112 * 1024;
void launch_batch(const BatchJob* jobs, const int* order, int count, int* counter, int grid, hipStream_t s,
                  int lds_cap = 0);
size_t small_lp_lds_bytes(const DevLP& P);

// Allocation-free batched form: the job table, LP order and work counter of at most
// kStaticBatchMax LPs live in a file-scope device array of the kernel source (one copy per
// device, kept until the process ends). static_batch_scratch returns its device address on
// `device`, which must be the current device; the address is looked up once per device.
constexpr int kStaticBatchMax = 4096;
struct StaticBatchScratch {
    BatchJob* jobs;  // kStaticBatchMax entries
    int* order;      // kStaticBatchMax entries
    int* counter;    // one work counter
    long long* t0;   // device wall clock at the start of the call
};
hipError_t static_batch_scratch(int device, StaticBatchScratch* out);
size_t static_batch_scratch_bytes();
// Sets *counter = 0 and *t0 = the device wall clock, with a one-thread kernel (no memset
// node if the caller captures the stream).
void launch_batch_start(int* counter, long long* t0, hipStream_t s);
// One launch of a block-diagonal batch; it_or_mode is the iteration inside the bundle for
// MULTI_PRIMAL / MULTI_DUAL and the evaluation mode for MULTI_PARTIALS / MULTI_DECIDE.
void launch_multi(const MultiMaps& M, int kind, int it_or_mode, hipStream_t s);

}  // namespace lpgpu
