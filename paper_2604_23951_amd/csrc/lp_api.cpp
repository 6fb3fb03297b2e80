// C ABI of the restarted-PDHG solver (include/lp.h): input validation, the one-time
// device setup (CSR transpose, scaling, norm estimate, step size) and the solve loop that
// replays hipGraph-captured bundles of iterations and reads one status word per bundle.
#include "lp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <array>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lp_device.h"
#include "lp_layout.h"
#include "lp_check.h"
#include "lp_tile_table.h"

using namespace lpgpu;

namespace {

thread_local std::string g_last_error;

struct Arena {
    size_t off = 0;
    size_t add(size_t bytes) {
        const size_t o = off;
        if (bytes < 8) bytes = 8;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

// Row tiles for the LDS-staged SpMV: consecutive rows while the tile holds at most tn
// nonzeros and tn / 4 rows; a row longer than tn is a tile of its own.
std::vector<int32_t> build_tiles(int32_t rows, const int32_t* rp, int32_t tn, int64_t* n_long) {
    const int32_t tile_rows = tn / 4;
    std::vector<int32_t> t;
    t.reserve(static_cast<size_t>(rows) / 64 + 2);
    t.push_back(0);
    int64_t nl = 0;
    int32_t r = 0;
    while (r < rows) {
        const int32_t start = r;
        const int64_t len = rp[r + 1] - rp[r];
        if (len > tn) {
            ++r;
            ++nl;
        } else {
            int64_t nz = 0;
            while (r < rows && r - start < tile_rows) {
                const int64_t l = rp[r + 1] - rp[r];
                if (l > tn || nz + l > tn) break;
                nz += l;
                ++r;
            }
        }
        t.push_back(r);
    }
    *n_long = nl;
    return t;
}

// Host-side integer structure of an LP, built once at lp_create.
struct Prep {
    std::vector<int32_t> rpT, ciT, perm, tA, tAT;
    PanelLayoutHost LA, LAT;
    int shape = 1;  // row-tile shape
    bool panels = false;
    int nred = 1;
    bool ready = false;
    // layout tuner (spmv_layout 2): the chosen layout (-1 before the first trial) and the
    // mean time in microseconds of one A x + A^T y pair in each layout; shared by the
    // clones of a deferred handle, which take the first trial's choice
    std::atomic<int> tuned{-1};
    double trial_us[2] = {0.0, 0.0};
};

// Device bytes of a one-workgroup lp_solve: the job (256-byte aligned), then the LP order
// (one int), the work counter and the start clock, 256 bytes apart.
constexpr size_t kSoloJobAligned = (sizeof(BatchJob) + 255) / 256 * 256;
constexpr size_t kSoloJobBytes = kSoloJobAligned + 768;

// Offsets of every device array inside a handle's allocation.
struct Offsets {
    size_t arp, aci, av, at, trp, tci, tv, tt, perm, c, xl, xu, C, Ci, bl, bu, R, Ri;
    size_t x, xa, xan, aty, atya, ox, oz, y, ya, yan, ax, axa, oy, x0, y0;
    size_t xp, atyp, yp, axp, axan, atyan;
    size_t fr[6];  // residual restarts: z - T(z) of the last iterate (x, y, A~x parts), then of the anchor
    size_t f32[15] = {0};
    size_t pA[7] = {0}, pAT[7] = {0}, pA32 = 0, pAT32 = 0;
    size_t part, sc, tr, job;
};

// Problem data kept on the host by a deferred handle until it is placed on the device.
struct HostData {
    std::vector<int32_t> rp, ci;
    std::vector<double> v, c, bl, bu, xl, xu, x0, y0;
};

}  // namespace

namespace lpgpu {

int32_t validate_lp(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                 const double* c, double c0, const double* bl, const double* bu, const double* xl, const double* xu,
                 std::string* msg) {
    if (m < 0 || n < 1 || nnz < 0 || nnz > kMaxEntries) {
        *msg = "sizes must satisfy m >= 0, n >= 1, 0 <= nnz <= 2^31 - 2^16 - 1";
        return LP_ERR_INVALID_ARG;
    }
    if (!rp || !c || !xl || !xu || (m > 0 && (!bl || !bu)) || (nnz > 0 && (!ci || !v))) {
        *msg = "a required array pointer is NULL";
        return LP_ERR_INVALID_ARG;
    }
    if (rp[0] != 0 || static_cast<int64_t>(rp[m]) != nnz) {
        *msg = "row_ptr must start at 0 and end at nnz";
        return LP_ERR_INVALID_MATRIX;
    }
    for (int32_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) {
            *msg = "row_ptr decreases at row " + std::to_string(i);
            return LP_ERR_INVALID_MATRIX;
        }
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) {
                *msg = "col_idx out of range at entry " + std::to_string(e);
                return LP_ERR_INVALID_MATRIX;
            }
            if (e > rp[i] && ci[e] <= ci[e - 1]) {
                *msg = "col_idx not strictly increasing in row " + std::to_string(i);
                return LP_ERR_INVALID_MATRIX;
            }
        }
    }
    for (int64_t e = 0; e < nnz; ++e)
        if (!std::isfinite(v[e])) {
            *msg = "matrix value " + std::to_string(e) + " is not finite";
            return LP_ERR_NAN_INPUT;
        }
    if (!std::isfinite(c0)) {
        *msg = "c0 is not finite";
        return LP_ERR_NAN_INPUT;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (!std::isfinite(c[j]) || std::isnan(xl[j]) || std::isnan(xu[j])) {
            *msg = "cost or variable bound " + std::to_string(j) + " is NaN/inf";
            return LP_ERR_NAN_INPUT;
        }
        if (xl[j] > xu[j] || xl[j] == HUGE_VAL || xu[j] == -HUGE_VAL) {
            *msg = "inconsistent bounds on variable " + std::to_string(j);
            return LP_ERR_INCONSISTENT_BOUNDS;
        }
    }
    for (int32_t i = 0; i < m; ++i) {
        if (std::isnan(bl[i]) || std::isnan(bu[i])) {
            *msg = "row bound " + std::to_string(i) + " is NaN";
            return LP_ERR_NAN_INPUT;
        }
        if (bl[i] > bu[i] || bl[i] == HUGE_VAL || bu[i] == -HUGE_VAL) {
            *msg = "inconsistent bounds on row " + std::to_string(i);
            return LP_ERR_INCONSISTENT_BOUNDS;
        }
    }
    return LP_OK;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace lpgpu

struct lp_handle {
    lp_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    double c0 = 0.0;
    int64_t long_a = 0, long_at = 0;
    int64_t units_a = 0, units_at = 0, panels_a = 0, panels_at = 0;
    int tile_shape = 1;  // row-tile shape chosen at lp_create
    double trial_us[2] = {0.0, 0.0};  // layout tuner's times (panels, row tiles)
    char* arena = nullptr;
    size_t arena_bytes = 0;
    DevLP P{};
    int* d_perm = nullptr;
    double* d_x0 = nullptr;
    double* d_y0 = nullptr;
    char* d_job = nullptr;  // job, LP order, work counter and start clock of a one-workgroup lp_solve
    Scalars* h_sc = nullptr;  // pinned host copy of the device scalars
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    bool solved = false;
    bool resumable = false;  // paused by lp_solve_until / lp_resume, or loaded by lp_import_state
    lp_options paused_opt{};  // the options of the paused run (its form must not change on resume)
    lp_info info{};
    std::string err;
    bool timing = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    double sum_p_ms = 0.0, sum_d_ms = 0.0;
    int64_t samples = 0;
    std::shared_ptr<Prep> prep;     // shared with the server's per-request clones
    std::shared_ptr<HostData> raw;
    bool has_x0 = false, has_y0 = false;
    bool deferred = false;
    bool on_device = false;
    std::vector<double> res_x, res_y, res_z;  // result kept on the host after the device copy is released
};

namespace {

int32_t materialize(lp_handle* h);

int32_t fail(lp_handle* h, int32_t code, const std::string& msg) {
    if (h) h->err = msg;
    g_last_error = msg;
    return code;
}

#define HIP_TRY(h, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((h), e_ == hipErrorOutOfMemory ? LP_ERR_OUT_OF_MEMORY : LP_ERR_DEVICE,   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                     \
    } while (0)

int32_t check_launch(lp_handle* h, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, LP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return LP_OK;
}


int32_t validate_options(const lp_options& o, std::string* msg) {
    if (!(o.eps_rel >= 0.0) || o.max_iters < 0 || o.eval_every < 1 || o.ruiz_passes < 0 || o.pow_iters < 0 ||
        o.trace_cap < 0 || o.precision < LP_PREC_FP64 || o.precision > LP_PREC_FP32_REFINED || o.spmv_layout < 0 || o.spmv_layout > 2 ||
        o.long_row_len < 0 || o.units_per_cu < 0 || o.batch_wg_per_cu < 0 || o.batch_split_nnz < 0 || o.panel_slice_bytes < 0 || std::isnan(o.step_size) || std::isnan(o.omega0) ||
        o.small_lp_lds < 0 || o.small_lp_lds > kSmallLpLdsMax ||
        !(o.tile_nnz == 0 || o.tile_nnz == 1024 || o.tile_nnz == 2048 || o.tile_nnz == 4096) ||
        std::isnan(o.time_limit_s) || !(o.eps_infeas >= 0.0) || o.method < LP_METHOD_AVERAGED ||
        o.method > LP_METHOD_HALPERN || !(o.reflection >= 0.0 && o.reflection <= 1.0) || o.omega_steps < 0 ||
        o.omega_steps > 8 || o.pw_rule < LP_PW_DEFAULT || o.pw_rule > LP_PW_PID || !(o.pid_kp >= 0.0 && o.pid_kp <= 2.0) ||
        !(o.pid_ki >= 0.0 && o.pid_ki <= 2.0) || !(o.pid_kd >= 0.0 && o.pid_kd <= 2.0) || o.restart_metric < 0 ||
        o.restart_metric > 1) {
        *msg = "invalid option value";
        return LP_ERR_INVALID_ARG;
    }
    return LP_OK;
}

void destroy_device(lp_handle* h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (auto& e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->arena) (void)hipFree(h->arena);
    if (h->h_sc) (void)hipHostFree(h->h_sc);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->arena = nullptr;
    h->h_sc = nullptr;
    h->stream = nullptr;
    for (auto& e : h->ev) e = nullptr;
    h->on_device = false;
}

// Keep the result on the host and give the device memory back (the handle stays usable:
// a later solve places it on the device again).
int32_t release_device(lp_handle* h) {
    if (!h->on_device) {  // a set-up that failed part way may still hold its allocation
        if (h->arena) (void)hipFree(h->arena);
        h->arena = nullptr;
        if (!h->own_stream) h->stream = nullptr;
        return LP_OK;
    }
    if (h->solved) {
        h->res_x.resize(static_cast<size_t>(h->n));
        h->res_y.resize(static_cast<size_t>(h->m));
        h->res_z.resize(static_cast<size_t>(h->n));
        HIP_TRY(h, hipMemcpyAsync(h->res_x.data(), h->P.out_x, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
        if (h->m > 0)
            HIP_TRY(h, hipMemcpyAsync(h->res_y.data(), h->P.out_y, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipMemcpyAsync(h->res_z.data(), h->P.out_z, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->graph_failed = false;
    if (h->arena) (void)hipFree(h->arena);
    h->arena = nullptr;
    h->on_device = false;
    if (!h->own_stream) h->stream = nullptr;  // a server's stream: not the handle's to keep
    return LP_OK;
}

// One evaluation period: eval_every iterations of (primal, dual), the evaluation and the
// restart. `timed_it` >= 0 brackets that iteration's kernels with the handle's events.
void record_bundle(lp_handle* h, int timed_it) {
    const int E = h->opt.eval_every;
    for (int it = 0; it < E; ++it) {
        if (it == timed_it) (void)hipEventRecord(h->ev[0], h->stream);
        launch_primal(h->P, it, h->stream);
        if (it == timed_it) (void)hipEventRecord(h->ev[1], h->stream);
        launch_dual(h->P, it, h->stream);
        if (it == timed_it) (void)hipEventRecord(h->ev[2], h->stream);
    }
    launch_evaluate(h->P, 0, h->stream);
    launch_apply_restart(h->P, h->stream);
}

void fill_info(lp_handle* h) {
    const Scalars& sc = *h->h_sc;
    lp_info& inf = h->info;
    inf.status = sc.status;
    inf.output_is_avg = sc.out_avg;
    inf.iterations = sc.k;
    inf.restarts = sc.restarts;
    inf.primal_obj = sc.out_pobj;
    inf.dual_obj = sc.out_dobj;
    inf.rel_primal_res = sc.out_rel_p;
    inf.rel_dual_res = sc.out_rel_d;
    inf.rel_gap = sc.out_rel_gap;
    inf.rel_kkt = sc.out_erel;
    inf.sigma_max = sc.sigma_max;
    inf.step_size = sc.eta;
    inf.omega = sc.omega;
    inf.done_clock = sc.done_clock;
    inf.ray_source = (sc.status == LP_PRIMAL_INFEASIBLE || sc.status == LP_DUAL_INFEASIBLE) ? sc.ray_src : 0;
    inf.solve_path = 0;  // the one-workgroup lp_solve sets 1 after this
    int khz = 0;
    inf.clock_hz = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) == hipSuccess ? 1e3 * khz : 0.0;
}


// The iteration form and primal-weight rule of a solve, from its options.
void set_form(DevLP& P, const lp_options& o) {
    P.method = o.method;
    P.rho = o.reflection;
    P.omega_steps = o.omega_steps > 0 ? o.omega_steps : (o.method == LP_METHOD_HALPERN ? 2 : 1);
    P.pw_rule = o.pw_rule == LP_PW_PID ? 2 : 1;
    P.kp = o.pid_kp;
    P.ki = o.pid_ki;
    P.kd = o.pid_kd;
    P.restart_metric = o.method == LP_METHOD_HALPERN ? o.restart_metric : 0;
}

BatchJob make_job(lp_handle* h, const lp_options* bo) {
    const lp_options& o = bo ? *bo : h->opt;
    BatchJob J{};
    J.P = h->P;
    J.eps_rel = o.eps_rel;
    J.eps_infeas = o.eps_infeas;
    set_form(J.P, o);
    J.max_iters = o.max_iters;
    J.trace_cap = h->opt.trace_cap;
    J.eval_every = o.eval_every;
    J.restarts_on = o.restarts;
    J.x0 = h->d_x0;
    J.y0 = h->d_y0;
    // the time limit becomes a device-clock deadline, checked at every evaluation on the device
    J.limit_ticks = 0;
    J.t0 = nullptr;
    int khz = 0;
    if (o.time_limit_s > 0.0 && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) == hipSuccess &&
        khz > 0) {
        const double ticks = o.time_limit_s * 1e3 * khz;
        J.limit_ticks = ticks >= 9.0e18 ? static_cast<long long>(9.0e18) : std::max(1LL, static_cast<long long>(ticks));
    }
    return J;
}

int32_t finish_batch(const std::vector<lp_handle*>& hs, hipStream_t s) {
    for (lp_handle* h : hs) HIP_TRY(h, hipMemcpyAsync(h->h_sc, h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(hs[0], hipStreamSynchronize(s));
    for (lp_handle* h : hs) {
        fill_info(h);
        h->solved = true;
    }
    return LP_OK;
}

// Workgroups of a launch go to the 8 XCDs of the device round-robin by index. The tiles of
// one form (LP after LP) are cut into kXcds contiguous runs of equal length and run k is
// placed at entries k, k + kXcds, k + 2 kXcds, ...: each run executes on one XCD, so an LP's
// gathered vector is cached in the L2 of one or two XCDs rather than all of them. Runs are
// padded with entries of the stand-in job `pad_job`. Short lists keep their order.
constexpr int kXcds = 8;

void append_xcd_order(const std::vector<int2>& tiles, int pad_job, std::vector<int2>& out) {
    const size_t len = tiles.size();
    if (len < static_cast<size_t>(4 * kXcds)) {
        out.insert(out.end(), tiles.begin(), tiles.end());
        return;
    }
    const size_t per = (len + kXcds - 1) / kXcds, base = out.size();
    out.resize(base + per * kXcds, make_int2(pad_job, 0));
    for (size_t t = 0; t < len; ++t) out[base + (t % per) * kXcds + t / per] = tiles[t];
}

// Device jobs table and block maps of a set of LPs (grown as needed, reused across rounds;
// every round ends with a stream synchronisation before the next rebuild).
struct DevMaps {
    char* buf = nullptr;
    size_t cap = 0;
    int* hstatus = nullptr;  // pinned
    int hcap = 0;
    MultiMaps M{};
    int E = 64;
    Scalars stopped{};  // host copy of the stand-in job's scalar block (kept for the async copy)
    // The round's launches as a graph, captured once the same set has run one round
    // uncaptured (a set that changes every round is not worth an instantiation).
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int stable_rounds = 0;
    bool graph_failed = false;

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        stable_rounds = 0;
        graph_failed = false;
    }

    int32_t build(const std::vector<lp_handle*>& hs, const lp_options* o, hipStream_t s, lp_handle* err_to) {
        drop_graph();
        const int count = static_cast<int>(hs.size());
        // jobs[count] is a stand-in whose scalar block says "stopped": map entries that pad
        // the XCD runs below point at it and their workgroups return at once
        std::vector<BatchJob> jobs(static_cast<size_t>(count) + 1);
        std::vector<int2> ma, mat, mred, melem;
        int off_a[kMapGroups], cnt_a[kMapGroups], off_at[kMapGroups], cnt_at[kMapGroups];
        for (int i = 0; i < count; ++i) jobs[i] = make_job(hs[i], o);
        for (int v = 0; v < kMapGroups; ++v) {  // tile maps grouped by form and shape, each in XCD order
            std::vector<int2> ta, tat;
            for (int i = 0; i < count; ++i) {
                const lp_handle* h = hs[i];
                const int form = (jobs[i].P.fp32 ? 2 : 0) + (jobs[i].P.method ? 1 : 0);
                if (form * kTileShapes + jobs[i].P.A.csr.shape != v) continue;
                for (int t = 0; t < h->P.A.csr.ntiles; ++t) ta.push_back(make_int2(i, t));
                for (int t = 0; t < h->P.AT.csr.ntiles; ++t) tat.push_back(make_int2(i, t));
            }
            off_a[v] = static_cast<int>(ma.size());
            off_at[v] = static_cast<int>(mat.size());
            append_xcd_order(ta, count, ma);
            append_xcd_order(tat, count, mat);
            cnt_a[v] = static_cast<int>(ma.size()) - off_a[v];
            cnt_at[v] = static_cast<int>(mat.size()) - off_at[v];
        }
        for (int i = 0; i < count; ++i) {
            const lp_handle* h = hs[i];
            for (int b = 0; b < h->P.nred; ++b) mred.push_back(make_int2(i, b));
            const int mx = h->m > h->n ? h->m : h->n;
            for (int b = 0; b < (mx + kBlock - 1) / kBlock; ++b) melem.push_back(make_int2(i, b));
        }
        E = count > 0 ? jobs[0].eval_every : 64;
        for (int i = 0; i < count; ++i)
            if (jobs[i].eval_every != E) return fail(err_to, LP_ERR_INVALID_ARG, "block-diagonal LPs must share eval_every");
        Arena L;
        const size_t oj = L.add(sizeof(BatchJob) * jobs.size()), oa = L.add(sizeof(int2) * ma.size()),
                     oat = L.add(sizeof(int2) * mat.size()), ored = L.add(sizeof(int2) * mred.size()),
                     oel = L.add(sizeof(int2) * melem.size()), ost = L.add(sizeof(int) * (count + 1)),
                     osc = L.add(sizeof(Scalars));
        if (L.off > cap) {
            if (buf) (void)hipFree(buf);
            buf = nullptr;
            cap = 0;
            const size_t want = L.off * 2;
            HIP_TRY(err_to, hipMalloc(reinterpret_cast<void**>(&buf), want));
            cap = want;
        }
        if (count + 1 > hcap) {
            if (hstatus) (void)hipHostFree(hstatus);
            hstatus = nullptr;
            hcap = 0;
            HIP_TRY(err_to, hipHostMalloc(reinterpret_cast<void**>(&hstatus), sizeof(int) * (count + 1) * 2,
                                          hipHostMallocDefault));
            hcap = (count + 1) * 2;
        }
        M = MultiMaps{};
        M.jobs = reinterpret_cast<const BatchJob*>(buf + oj);
        M.count = count;
        M.map_a = reinterpret_cast<const int2*>(buf + oa);
        M.n_a = static_cast<int>(ma.size());
        M.map_at = reinterpret_cast<const int2*>(buf + oat);
        M.n_at = static_cast<int>(mat.size());
        for (int v = 0; v < kMapGroups; ++v) {
            M.off_a[v] = off_a[v];
            M.cnt_a[v] = cnt_a[v];
            M.off_at[v] = off_at[v];
            M.cnt_at[v] = cnt_at[v];
        }
        M.map_red = reinterpret_cast<const int2*>(buf + ored);
        M.n_red = static_cast<int>(mred.size());
        M.map_elem = reinterpret_cast<const int2*>(buf + oel);
        M.n_elem = static_cast<int>(melem.size());
        M.active = reinterpret_cast<int*>(buf + ost);
        auto H2D = [&](size_t off, const void* src, size_t bytes) {
            return bytes ? hipMemcpyAsync(buf + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
        };
        if (count > 0) {  // the stand-in: any LP's arrays, a stopped scalar block of its own
            jobs[count] = jobs[0];
            jobs[count].P.sc = reinterpret_cast<Scalars*>(buf + osc);
            stopped = Scalars{};
            stopped.status = 0;
            HIP_TRY(err_to, H2D(osc, &stopped, sizeof(Scalars)));
        }
        HIP_TRY(err_to, H2D(oj, jobs.data(), sizeof(BatchJob) * jobs.size()));
        HIP_TRY(err_to, H2D(oa, ma.data(), sizeof(int2) * ma.size()));
        HIP_TRY(err_to, H2D(oat, mat.data(), sizeof(int2) * mat.size()));
        HIP_TRY(err_to, H2D(ored, mred.data(), sizeof(int2) * mred.size()));
        HIP_TRY(err_to, H2D(oel, melem.data(), sizeof(int2) * melem.size()));
        return LP_OK;
    }

    void free_all() {
        drop_graph();
        if (buf) (void)hipFree(buf);
        if (hstatus) (void)hipHostFree(hstatus);
        buf = nullptr;
        hstatus = nullptr;
        cap = 0;
        hcap = 0;
    }
};

// One evaluation period of every LP of D: eval_every (primal, dual) launches, the
// evaluation, the decision, the restart and each LP's status into D.M.active[i]. Replayed
// as a hipGraph once the same set has run `capture_after` rounds uncaptured.
void run_round(DevMaps& D, hipStream_t s, int capture_after) {
    const MultiMaps& M = D.M;
    auto round = [&]() {
        for (int it = 0; it < D.E; ++it) {
            launch_multi(M, MULTI_PRIMAL, it, s);
            launch_multi(M, MULTI_DUAL, it, s);
        }
        launch_multi(M, MULTI_MATERIALIZE, 0, s);
        launch_multi(M, MULTI_AX_FP32, 0, s);
        launch_multi(M, MULTI_ATY, 0, s);
        launch_multi(M, MULTI_AXA, 0, s);
        launch_multi(M, MULTI_ATYA, 0, s);
        launch_multi(M, MULTI_PARTIALS, 0, s);
        launch_multi(M, MULTI_DECIDE, 0, s);
        launch_multi(M, MULTI_APPLY, 0, s);
        launch_multi(M, MULTI_STATUS, 0, s);
    };
    if (!D.gexec && !D.graph_failed && D.stable_rounds >= capture_after) {
        hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
            round();
            ce = hipStreamEndCapture(s, &D.graph);
        }
        if (ce == hipSuccess) ce = hipGraphInstantiate(&D.gexec, D.graph, nullptr, nullptr, 0);
        if (ce != hipSuccess) {  // stay with direct launches for this set
            (void)hipGetLastError();
            if (D.graph) (void)hipGraphDestroy(D.graph);
            D.graph = nullptr;
            D.gexec = nullptr;
            D.graph_failed = true;
        }
    }
    if (D.gexec) (void)hipGraphLaunch(D.gexec, s);
    else round();
    D.stable_rounds++;
}

// LPs solved one per workgroup in a single persistent launch, started on its own stream
// so that it runs beside the block-diagonal launches of the larger LPs. The host arrays
// stay alive until finish_persistent. The runtime spreads streams over a few hardware queues
// in creation order, and two launches whose streams share a queue run one after the other,
// so the block-diagonal launches get the third of three streams created together (s[2])
// rather than an older stream that may share a queue with a persistent launch.
struct PersistentRun {
    std::vector<BatchJob> jobs;
    std::vector<int32_t> order;
    char* buf = nullptr;
    hipStream_t s[3] = {nullptr, nullptr, nullptr};
};

// Two persistent launches at most, each on a stream of its own: the LPs whose iteration
// arrays fit in the small-LP LDS budget (one workgroup per CU, each LP solved from LDS) and
// the others (batch_wg_per_cu workgroups per CU, from global memory). Each launch takes its
// LPs largest first.
int32_t start_persistent(const std::vector<lp_handle*>& hs, const lp_options* bo, PersistentRun& R) {
    const int count = static_cast<int>(hs.size());
    lp_handle* h0 = hs[0];
    for (lp_handle* h : hs)
        if (int32_t rc = materialize(h)) return rc;
    const int budget = bo ? bo->small_lp_lds : h0->opt.small_lp_lds;
    R.jobs.resize(static_cast<size_t>(count));
    R.order.resize(static_cast<size_t>(count));
    std::vector<size_t> need(static_cast<size_t>(count));
    size_t cap = 0;
    int n_lds = 0;
    for (int i = 0; i < count; ++i) {
        R.jobs[i] = make_job(hs[i], bo);
        R.order[i] = i;
        need[i] = small_lp_lds_bytes(R.jobs[i].P);
        if (budget > 0 && need[i] <= static_cast<size_t>(budget)) {
            cap = std::max(cap, need[i]);
            ++n_lds;
        }
    }
    auto in_lds = [&](int32_t i) { return budget > 0 && need[i] <= static_cast<size_t>(budget); };
    // LDS LPs first, then the others; each part largest first
    std::stable_sort(R.order.begin(), R.order.end(), [&](int32_t a, int32_t b) {
        if (in_lds(a) != in_lds(b)) return in_lds(a);
        return hs[a]->nnz > hs[b]->nnz;
    });
    const int lds_cap = n_lds ? static_cast<int>((cap + 16383) / 16384 * 16384) : 0;
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h0->device) != hipSuccess || cus < 1)
        cus = 256;
    const int wpc = (bo && bo->batch_wg_per_cu > 0) ? bo->batch_wg_per_cu : 3;
    const size_t bj = sizeof(BatchJob) * static_cast<size_t>(count), bo_ = sizeof(int32_t) * static_cast<size_t>(count);
    const size_t oc = (bj + bo_ + 255) / 256 * 256;
    HIP_TRY(h0, hipMalloc(reinterpret_cast<void**>(&R.buf), oc + 512));
    BatchJob* djobs = reinterpret_cast<BatchJob*>(R.buf);
    int32_t* dorder = reinterpret_cast<int32_t*>(R.buf + bj);
    int32_t* dcounter = reinterpret_cast<int32_t*>(R.buf + oc);  // one counter per launch, 256 bytes apart
    long long* dt0 = reinterpret_cast<long long*>(R.buf + oc + 128);  // device clock at the start of the call
    for (BatchJob& J : R.jobs) J.t0 = dt0;
    hipError_t e = hipSuccess;
    for (int l = 0; l < 3 && e == hipSuccess; ++l)
        e = hipStreamCreateWithFlags(&R.s[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemcpyAsync(djobs, R.jobs.data(), bj, hipMemcpyHostToDevice, R.s[0]);
    if (e == hipSuccess) e = hipMemcpyAsync(dorder, R.order.data(), bo_, hipMemcpyHostToDevice, R.s[0]);
    if (e == hipSuccess) e = hipMemsetAsync(dcounter, 0, 512, R.s[0]);
    if (e == hipSuccess) {
        launch_batch_start(dcounter, dt0, R.s[0]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(R.s[0]);
    if (e == hipSuccess && n_lds > 0) {
        launch_batch(djobs, dorder, n_lds, dcounter, std::min(cus, n_lds), R.s[1], lds_cap);
        e = hipGetLastError();
    }
    if (e == hipSuccess && count > n_lds) {
        launch_batch(djobs, dorder + n_lds, count - n_lds, dcounter + 64, std::min(cus * wpc, count - n_lds), R.s[0]);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return fail(h0, LP_ERR_DEVICE, std::string("batched solve: ") + hipGetErrorString(e));
    return LP_OK;
}

// Waits for the persistent launches (also after an error elsewhere: their kernels must have
// ended before their memory goes) and collects the results when `collect`.
int32_t finish_persistent(const std::vector<lp_handle*>& hs, PersistentRun& R, bool collect) {
    hipError_t e = hipSuccess;
    for (hipStream_t st : R.s)
        if (st) {
            const hipError_t e1 = hipStreamSynchronize(st);
            if (e == hipSuccess) e = e1;
        }
    if (R.buf) (void)hipFree(R.buf);
    R.buf = nullptr;
    int32_t rc = LP_OK;
    if (e != hipSuccess) rc = fail(hs[0], LP_ERR_DEVICE, std::string("batched solve: ") + hipGetErrorString(e));
    else if (collect) rc = finish_batch(hs, R.s[0]);
    for (hipStream_t& st : R.s) {
        if (st) (void)hipStreamDestroy(st);
        st = nullptr;
    }
    return rc;
}

// LPs advanced together as one block-diagonal problem, one launch per phase for all of
// them, evaluation periods replayed as a hipGraph. When a quarter of the mapped LPs have
// stopped, the maps are rebuilt over the running ones, so finished LPs cost no more
// workgroups (each LP's trajectory does not depend on the others in the map).
int32_t solve_block_diagonal(const std::vector<lp_handle*>& hs, const lp_options* bo, hipStream_t s) {
    lp_handle* h0 = hs[0];
    for (lp_handle* h : hs)
        if (int32_t rc = materialize(h)) return rc;
    DevMaps all, run;
    struct Release {
        DevMaps &a, &b;
        ~Release() {
            a.free_all();
            b.free_all();
        }
    } release{all, run};
    if (int32_t rc = all.build(hs, bo, s, h0)) return rc;
    {
        const MultiMaps& M = all.M;
        launch_multi(M, MULTI_RESET, 0, s);
        launch_multi(M, MULTI_INIT, 0, s);
        launch_multi(M, MULTI_AX_ALL, 0, s);
        launch_multi(M, MULTI_ATY, 1, s);  // 1: products of the initial point
        launch_multi(M, MULTI_PARTIALS, 1, s);
        launch_multi(M, MULTI_DECIDE, 1, s);
        launch_multi(M, MULTI_REBASE_INIT, 0, s);
        HIP_TRY(h0, hipGetLastError());
    }
    long long max_bundles = 0;
    for (lp_handle* h : hs) {
        const long long b = make_job(h, bo).max_iters / all.E + 2;
        if (b > max_bundles) max_bundles = b;
    }
    std::vector<lp_handle*> cur = hs;
    if (int32_t rc = run.build(cur, bo, s, h0)) return rc;
    for (long long b = 0; b < max_bundles; ++b) {
        run_round(run, s, 0);
        HIP_TRY(h0, hipGetLastError());
        HIP_TRY(h0, hipMemcpyAsync(run.hstatus, run.M.active, sizeof(int) * run.M.count, hipMemcpyDeviceToHost, s));
        HIP_TRY(h0, hipStreamSynchronize(s));
        std::vector<lp_handle*> still;
        for (int i = 0; i < run.M.count; ++i)
            if (run.hstatus[i] == kRunning) still.push_back(cur[i]);
        if (still.empty()) break;
        if (4 * still.size() <= 3 * cur.size()) {
            cur.swap(still);
            if (int32_t rc = run.build(cur, bo, s, h0)) return rc;
        }
    }
    launch_multi(all.M, MULTI_EXTRACT, 0, s);
    HIP_TRY(h0, hipGetLastError());
    HIP_TRY(h0, hipStreamSynchronize(s));
    return finish_batch(hs, s);
}

int32_t capture_graph(lp_handle* h) {
    if (h->gexec || h->graph_failed) return LP_OK;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        record_bundle(h, -1);
        e = hipStreamEndCapture(h->stream, &h->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->graph_failed = true;
        if (h->graph) (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
        h->gexec = nullptr;
    }
    return LP_OK;
}

// Host-side integer preparation (a1): transpose structure by a stable counting sort on the
// column index (perm maps each entry of A^T to its entry of A so the values are moved on
// the device), row tiles, panel layouts and the reduction grid.
int32_t host_prep(lp_handle* h, const int32_t* rp, const int32_t* ci) {
    const int32_t m = h->m, n = h->n;
    const int64_t nnz = h->nnz;
    const lp_options& o = h->opt;
    h->prep = std::make_shared<Prep>();
    Prep& Q = *h->prep;
    Q.rpT.assign(static_cast<size_t>(n) + 1, 0);
    Q.ciT.resize(static_cast<size_t>(nnz));
    Q.perm.resize(static_cast<size_t>(nnz));
    for (int64_t e = 0; e < nnz; ++e) Q.rpT[ci[e] + 1]++;
    for (int32_t j = 0; j < n; ++j) Q.rpT[j + 1] += Q.rpT[j];
    {
        std::vector<int32_t> next(Q.rpT.begin(), Q.rpT.end() - 1);
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int32_t p = next[ci[e]]++;
                Q.ciT[p] = i;
                Q.perm[p] = e;
            }
    }
    int64_t dummy_long = 0;
    Q.shape = o.tile_nnz > 0 ? (o.tile_nnz == 1024 ? 0 : o.tile_nnz == 2048 ? 1 : 2)
                             : tuned_tile_shape(o.precision == LP_PREC_FP32_REFINED, m, n, nnz);
    h->tile_shape = Q.shape;
    Q.tA = build_tiles(m, rp, tile_nnz_of(Q.shape), &dummy_long);
    Q.tAT = build_tiles(n, Q.rpT.data(), tile_nnz_of(Q.shape), &dummy_long);
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    const int target_units = cus * (o.units_per_cu > 0 ? o.units_per_cu : 4);
    const int64_t slice = o.panel_slice_bytes > 0 ? o.panel_slice_bytes : (int64_t(1) << 19);
    const int long_len = o.long_row_len > 0 ? o.long_row_len : 256;
    Q.panels = o.spmv_layout == 0 || o.spmv_layout == 2;
    if (Q.panels) {
        Q.LA = build_panel_layout(m, n, rp, ci, nullptr, choose_panels(n, slice), long_len, target_units, kUnitRowCap);
        Q.LAT = build_panel_layout(n, m, Q.rpT.data(), Q.ciT.data(), Q.perm.data(), choose_panels(m, slice), long_len,
                                   target_units, kUnitRowCap);
        h->long_a = static_cast<int64_t>(Q.LA.long_rows.size());
        h->long_at = static_cast<int64_t>(Q.LAT.long_rows.size());
        h->units_a = Q.LA.units;
        h->units_at = Q.LAT.units;
        h->panels_a = Q.LA.panels;
        h->panels_at = Q.LAT.panels;
    }
    const int mx = m > n ? m : n;
    Q.nred = (mx + 1023) / 1024;
    if (Q.nred < 1) Q.nred = 1;
    if (Q.nred > kMaxRedBlocks) Q.nred = kMaxRedBlocks;
    Q.ready = true;
    return LP_OK;
}

// Device layout of one handle: every array at a 256-byte aligned offset of one allocation.
size_t arena_layout(const lp_handle* h, Offsets* O) {
    const int32_t m = h->m, n = h->n;
    const int64_t nnz = h->nnz;
    const lp_options& o = h->opt;
    const Prep& Q = *h->prep;
    const size_t sm = sizeof(double) * static_cast<size_t>(m), sn = sizeof(double) * static_cast<size_t>(n);
    const size_t si_nnz = sizeof(int32_t) * static_cast<size_t>(nnz), sd_nnz = sizeof(double) * static_cast<size_t>(nnz);
    Arena L;
    O->arp = L.add(sizeof(int32_t) * (m + 1));
    O->aci = L.add(si_nnz);
    O->av = L.add(sd_nnz);
    O->at = L.add(sizeof(int32_t) * Q.tA.size());
    O->trp = L.add(sizeof(int32_t) * (n + 1));
    O->tci = L.add(si_nnz);
    O->tv = L.add(sd_nnz);
    O->tt = L.add(sizeof(int32_t) * Q.tAT.size());
    O->perm = L.add(si_nnz);
    O->c = L.add(sn);
    O->xl = L.add(sn);
    O->xu = L.add(sn);
    O->C = L.add(sn);
    O->Ci = L.add(sn);
    O->bl = L.add(sm);
    O->bu = L.add(sm);
    O->R = L.add(sm);
    O->Ri = L.add(sm);
    O->x = L.add(sn);
    O->xa = L.add(sn);
    O->xan = L.add(sn);
    O->aty = L.add(sn);
    O->atya = L.add(sn);
    O->ox = L.add(sn);
    O->oz = L.add(sn);
    O->y = L.add(sm);
    O->ya = L.add(sm);
    O->yan = L.add(sm);
    O->ax = L.add(sm);
    O->axa = L.add(sm);
    O->oy = L.add(sm);
    O->xp = L.add(sn);
    O->atyp = L.add(sn);
    O->yp = L.add(sm);
    O->axp = L.add(sm);
    O->axan = L.add(sm);
    O->atyan = L.add(sn);
    for (int i = 0; i < 6; ++i) O->fr[i] = L.add(i % 3 == 0 ? sn : sm);
    O->x0 = h->has_x0 ? L.add(sn) : 0;
    O->y0 = h->has_y0 ? L.add(sm) : 0;
    const bool fp32 = o.precision == LP_PREC_FP32_REFINED;
    const size_t fn = sizeof(float) * static_cast<size_t>(n), fm = sizeof(float) * static_cast<size_t>(m);
    if (fp32) {
        const size_t sz[15] = {fn, fn, fm, fm, fm, fn, fn, fn, fm, fm, fm, sn, sm,
                               sizeof(float) * static_cast<size_t>(nnz), sizeof(float) * static_cast<size_t>(nnz)};
        for (int i = 0; i < 15; ++i) O->f32[i] = L.add(sz[i]);
    }
    auto add_layout = [&](const PanelLayoutHost& P, size_t* off) {
        off[0] = L.add(sizeof(int32_t) * P.unit_row.size());
        off[1] = L.add(sizeof(int32_t) * P.unit_seg.size());
        off[2] = L.add(sizeof(uint32_t) * P.packed.size());
        off[3] = L.add(sizeof(double) * P.packed.size());
        off[4] = L.add(sizeof(int32_t) * P.src.size());
        off[5] = L.add(sizeof(int32_t) * P.long_rows.size());
        off[6] = L.add(P.is_long.size());
    };
    if (Q.panels) {
        add_layout(Q.LA, O->pA);
        add_layout(Q.LAT, O->pAT);
        if (fp32) {
            O->pA32 = L.add(sizeof(float) * Q.LA.packed.size());
            O->pAT32 = L.add(sizeof(float) * Q.LAT.packed.size());
        }
    }
    O->part = L.add(sizeof(double) * kNT * kMaxRedBlocks);
    O->sc = L.add(sizeof(Scalars));
    O->job = L.add(kSoloJobBytes);
    O->tr = L.add(sizeof(double) * kTraceW * static_cast<size_t>(o.trace_cap > 0 ? o.trace_cap : 1));
    return L.off;
}

// Device part (a2, a3): allocate, bind, upload, scale, permute values, estimate ||A~||_2 and
// the step size. Runs on the handle's stream and waits.
// Times reps pairs of products in each layout, twice in alternation, keeps the smaller
// time of each and records the faster layout in the shared host structure.
int32_t tune_layout(lp_handle* h, hipStream_t s) {
    Prep& Q = *h->prep;
    const DevLP& P = h->P;
    constexpr int kReps = 8;
    if (P.fp32) {
        HIP_TRY(h, hipMemsetAsync(P.dx, 0, sizeof(float) * static_cast<size_t>(P.n), s));
        if (P.m > 0) HIP_TRY(h, hipMemsetAsync(P.dy, 0, sizeof(float) * static_cast<size_t>(P.m), s));
    } else {
        HIP_TRY(h, hipMemsetAsync(P.x, 0, sizeof(double) * static_cast<size_t>(P.n), s));
        if (P.m > 0) HIP_TRY(h, hipMemsetAsync(P.y, 0, sizeof(double) * static_cast<size_t>(P.m), s));
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(h, LP_ERR_DEVICE, "event creation failed");
    }
    float best[2] = {1e30f, 1e30f};
    hipError_t e = hipSuccess;
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
        for (int L = 0; L < 2 && e == hipSuccess; ++L) {
            launch_layout_trial(P, L, 2, s);  // warm-up: caches and code
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) launch_layout_trial(P, L, kReps, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < best[L]) best[L] = ms;
        }
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(h, LP_ERR_DEVICE, std::string("layout trial: ") + hipGetErrorString(e));
    Q.trial_us[0] = 1e3 * best[0] / kReps;
    Q.trial_us[1] = 1e3 * best[1] / kReps;
    int expect = -1;
    (void)Q.tuned.compare_exchange_strong(expect, best[1] < best[0] ? 1 : 0);
    return LP_OK;
}

int32_t device_setup(lp_handle* h, const int32_t* rp, const int32_t* ci, const double* v, const double* c,
                     const double* bl, const double* bu, const double* xl, const double* xu, const double* x0,
                     const double* y0) {
    const int32_t m = h->m, n = h->n;
    const int64_t nnz = h->nnz;
    const lp_options& o = h->opt;
    const Prep& Q = *h->prep;
    HIP_TRY(h, hipSetDevice(h->device));
    if (!h->stream) {
        if (o.hip_stream) {
            h->stream = static_cast<hipStream_t>(o.hip_stream);
        } else {
            HIP_TRY(h, hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            h->own_stream = true;
        }
    }
    Offsets O;
    h->arena_bytes = arena_layout(h, &O);
    HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->arena), h->arena_bytes));
    if (!h->h_sc) {
        HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->h_sc), sizeof(Scalars), hipHostMallocDefault));
        std::memset(h->h_sc, 0, sizeof(Scalars));
    }
    char* b = h->arena;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    auto I = [&](size_t off) { return reinterpret_cast<int32_t*>(b + off); };
    auto F = [&](size_t off) { return reinterpret_cast<float*>(b + off); };
    const int32_t ntA = static_cast<int32_t>(Q.tA.size()) - 1, ntAT = static_cast<int32_t>(Q.tAT.size()) - 1;
    const bool panels = Q.panels;
    const bool fp32 = o.precision == LP_PREC_FP32_REFINED;

    DevLP& P = h->P;
    P = DevLP{};
    P.m = m;
    P.n = n;
    P.nnz = nnz;
    P.nred = Q.nred;
    P.A.csr = Csr{m, ntA, static_cast<int>(nnz), Q.shape, I(O.arp), I(O.aci), D(O.av), I(O.at), nullptr, nullptr, n};
    P.AT.csr = Csr{n, ntAT, static_cast<int>(nnz), Q.shape, I(O.trp), I(O.tci), D(O.tv), I(O.tt), nullptr, nullptr, m};
    P.A.layout = P.AT.layout = panels ? 0 : 1;
    auto bind_layout = [&](const PanelLayoutHost& L, const size_t* off, Mat& M) {
        M.pan = Panels{L.units, L.panels, L.col_bits, static_cast<int>(L.nnz_packed), L.max_unit_rows, I(off[0]), I(off[1]),
                       reinterpret_cast<const unsigned*>(b + off[2]), D(off[3]),
                       L.is_long.empty() ? nullptr : reinterpret_cast<const unsigned char*>(b + off[6]), nullptr,
                       M.csr.cols};
        M.nlong = static_cast<int>(L.long_rows.size());
        M.longrows = M.nlong ? I(off[5]) : nullptr;
    };
    if (panels) {
        bind_layout(Q.LA, O.pA, P.A);
        bind_layout(Q.LAT, O.pAT, P.AT);
    }
    P.fp32 = fp32 ? 1 : 0;
    if (fp32) {
        P.dx = F(O.f32[0]);
        P.dxa = F(O.f32[1]);
        P.dy = F(O.f32[2]);
        P.dya = F(O.f32[3]);
        P.adx = F(O.f32[4]);
        P.d32 = F(O.f32[5]);
        P.lo32 = F(O.f32[6]);
        P.hi32 = F(O.f32[7]);
        P.rl32 = F(O.f32[8]);
        P.ru32 = F(O.f32[9]);
        P.yh32 = F(O.f32[10]);
        P.xh = D(O.f32[11]);
        P.yh = D(O.f32[12]);
        P.A.csr.v32 = F(O.f32[13]);
        P.AT.csr.v32 = F(O.f32[14]);
        if (panels) {
            P.A.pan.v32 = F(O.pA32);
            P.AT.pan.v32 = F(O.pAT32);
        }
    }
    P.c = D(O.c);
    P.xl = D(O.xl);
    P.xu = D(O.xu);
    P.C = D(O.C);
    P.Ci = D(O.Ci);
    P.bl = D(O.bl);
    P.bu = D(O.bu);
    P.R = D(O.R);
    P.Ri = D(O.Ri);
    P.x = D(O.x);
    P.xa = D(O.xa);
    P.xan = D(O.xan);
    P.aty = D(O.aty);
    P.atya = D(O.atya);
    P.out_x = D(O.ox);
    P.out_z = D(O.oz);
    P.y = D(O.y);
    P.ya = D(O.ya);
    P.yan = D(O.yan);
    P.ax = D(O.ax);
    P.axa = D(O.axa);
    P.out_y = D(O.oy);
    P.xp = D(O.xp);
    P.atyp = D(O.atyp);
    P.yp = D(O.yp);
    P.axp = D(O.axp);
    P.axan = D(O.axan);
    P.atyan = D(O.atyan);
    P.fr_x = D(O.fr[0]);
    P.fr_y = D(O.fr[1]);
    P.fr_ax = D(O.fr[2]);
    P.fa_x = D(O.fr[3]);
    P.fa_y = D(O.fr[4]);
    P.fa_ax = D(O.fr[5]);
    P.partials = D(O.part);
    P.sc = reinterpret_cast<Scalars*>(b + O.sc);
    P.trace = o.trace_cap > 0 ? D(O.tr) : nullptr;
    h->d_perm = I(O.perm);
    h->d_x0 = h->has_x0 ? D(O.x0) : nullptr;
    h->d_y0 = h->has_y0 ? D(O.y0) : nullptr;
    h->d_job = b + O.job;

    hipStream_t s = h->stream;
    const size_t sm = sizeof(double) * static_cast<size_t>(m), sn = sizeof(double) * static_cast<size_t>(n);
    const size_t si_nnz = sizeof(int32_t) * static_cast<size_t>(nnz), sd_nnz = sizeof(double) * static_cast<size_t>(nnz);
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_TRY(h, H2D(I(O.arp), rp, sizeof(int32_t) * (m + 1)));
    HIP_TRY(h, H2D(I(O.aci), ci, si_nnz));
    HIP_TRY(h, H2D(D(O.av), v, sd_nnz));
    HIP_TRY(h, H2D(I(O.at), Q.tA.data(), sizeof(int32_t) * Q.tA.size()));
    HIP_TRY(h, H2D(I(O.trp), Q.rpT.data(), sizeof(int32_t) * (n + 1)));
    HIP_TRY(h, H2D(I(O.tci), Q.ciT.data(), si_nnz));
    HIP_TRY(h, H2D(I(O.tt), Q.tAT.data(), sizeof(int32_t) * Q.tAT.size()));
    HIP_TRY(h, H2D(I(O.perm), Q.perm.data(), si_nnz));
    HIP_TRY(h, H2D(D(O.c), c, sn));
    HIP_TRY(h, H2D(D(O.xl), xl, sn));
    HIP_TRY(h, H2D(D(O.xu), xu, sn));
    if (m > 0) {
        HIP_TRY(h, H2D(D(O.bl), bl, sm));
        HIP_TRY(h, H2D(D(O.bu), bu, sm));
    }
    auto upload_layout = [&](const PanelLayoutHost& L, const size_t* off) -> hipError_t {
        hipError_t e = H2D(b + off[0], L.unit_row.data(), sizeof(int32_t) * L.unit_row.size());
        if (e == hipSuccess) e = H2D(b + off[1], L.unit_seg.data(), sizeof(int32_t) * L.unit_seg.size());
        if (e == hipSuccess) e = H2D(b + off[2], L.packed.data(), sizeof(uint32_t) * L.packed.size());
        if (e == hipSuccess) e = H2D(b + off[4], L.src.data(), sizeof(int32_t) * L.src.size());
        if (e == hipSuccess) e = H2D(b + off[5], L.long_rows.data(), sizeof(int32_t) * L.long_rows.size());
        if (e == hipSuccess) e = H2D(b + off[6], L.is_long.data(), L.is_long.size());
        return e;
    };
    if (panels) {
        HIP_TRY(h, upload_layout(Q.LA, O.pA));
        HIP_TRY(h, upload_layout(Q.LAT, O.pAT));
    }
    if (h->has_x0) HIP_TRY(h, H2D(h->d_x0, x0, sn));
    if (h->has_y0 && m > 0) HIP_TRY(h, H2D(h->d_y0, y0, sm));
    HIP_TRY(h, hipMemsetAsync(P.sc, 0, sizeof(Scalars), s));

    // a2: scaling, exact powers of two
    launch_fill(D(O.R), m, 1.0, s);
    launch_fill(D(O.C), n, 1.0, s);
    if (o.scaling) {
        for (int pass = 0; pass <= o.ruiz_passes; ++pass)
            launch_scale_pass(P, I(O.arp), I(O.aci), D(O.av), I(O.trp), h->d_perm, D(O.R), D(O.C), D(O.ax),
                              D(O.aty), pass == o.ruiz_passes ? 1 : 0, s);
    }
    launch_gather(h->d_perm, D(O.av), D(O.tv), nnz, s);
    if (panels) {  // panel values in packed order, from the scaled A
        launch_gather(I(O.pA[4]), D(O.av), D(O.pA[3]), Q.LA.nnz_packed, s);
        launch_gather(I(O.pAT[4]), D(O.av), D(O.pAT[3]), Q.LAT.nnz_packed, s);
    }
    if (fp32) {  // FP32 copies of the scaled values (rounded to nearest)
        launch_to_float(D(O.av), F(O.f32[13]), nnz, s);
        launch_to_float(D(O.tv), F(O.f32[14]), nnz, s);
        if (panels) {
            launch_to_float(D(O.pA[3]), F(O.pA32), Q.LA.nnz_packed, s);
            launch_to_float(D(O.pAT[3]), F(O.pAT32), Q.LAT.nnz_packed, s);
        }
    }
    launch_prepare(P, D(O.c), D(O.bl), D(O.bu), D(O.xl), D(O.xu), D(O.R), D(O.C), D(O.Ri), D(O.Ci), h->d_x0,
                   h->d_y0, s);
    // layout tuner: time both product layouts on this device and keep the faster one for
    // every product of the solve, the power iteration below included
    if (o.spmv_layout == 2) {
        if (Q.tuned.load() < 0) {
            if (int32_t rc = tune_layout(h, s)) return rc;
        }
        P.A.layout = P.AT.layout = Q.tuned.load();
        h->trial_us[0] = Q.trial_us[0];
        h->trial_us[1] = Q.trial_us[1];
    }
    // a3: ||A~||_2 by power iteration (x, A~x and A~^T y buffers are free at this point), in
    // chunks of pow_iters steps until a chunk's last step raises the estimate by at most
    // 1e-8 of it (it approaches ||A~||_2 from below and eta = 0.998 / estimate must keep
    // eta ||A~||_2 < 1), at most 25 chunks
    if (!(o.step_size > 0.0)) {
        launch_power_start(P, o.seed, P.x, s);
        for (int chunk = 0; chunk < 25; ++chunk) {
            launch_power_steps(P, o.pow_iters, P.x, P.ax, P.aty, s);
            if (chunk == 24) break;
            double sg[2];
            HIP_TRY(h, hipMemcpyAsync(sg, &P.sc->sigma_max, sizeof(sg), hipMemcpyDeviceToHost, s));
            HIP_TRY(h, hipStreamSynchronize(s));
            if (sg[0] - sg[1] <= 1e-8 * sg[0]) break;
        }
    }
    launch_finalize_setup(P, o.step_size, o.omega0, h->c0, s);
    if (int32_t rc = check_launch(h, "setup kernels")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (!h->ev[0])
        for (auto& e : h->ev) HIP_TRY(h, hipEventCreate(&e));
    h->on_device = true;
    return LP_OK;
}

// Device memory of a deferred handle: allocate and set up from the kept host data.
int32_t materialize(lp_handle* h) {
    if (h->on_device) return LP_OK;
    if (!h->deferred) return fail(h, LP_ERR_INTERNAL, "handle has no device data and no host copy");
    const HostData& R = *h->raw;
    return device_setup(h, R.rp.data(), R.ci.data(), R.v.data(), R.c.data(), R.bl.data(), R.bu.data(), R.xl.data(),
                        R.xu.data(), R.x0.data(), R.y0.data());
}


// ------------------------------------------------------------------ serving form

// A request's private handle: the problem's host data and layout are shared with the
// submitted handle (read-only), device state and result are its own.
lp_handle* clone_for_request(const lp_handle* t) {
    lp_handle* h = new lp_handle();
    h->opt = t->opt;
    h->opt.hip_stream = nullptr;
    h->device = t->device;
    h->m = t->m;
    h->n = t->n;
    h->nnz = t->nnz;
    h->c0 = t->c0;
    h->long_a = t->long_a;
    h->long_at = t->long_at;
    h->units_a = t->units_a;
    h->units_at = t->units_at;
    h->panels_a = t->panels_a;
    h->panels_at = t->panels_at;
    h->arena_bytes = t->arena_bytes;
    h->prep = t->prep;
    h->raw = t->raw;
    h->has_x0 = t->has_x0;
    h->has_y0 = t->has_y0;
    h->deferred = true;
    return h;
}

struct Ticket {
    uint64_t id;
    lp_handle* h;
    double t_submit, t_admit, t_done;
    int64_t counted;  // iterations already added to the server's work counters
    int32_t setup_rc; // result of the device set-up (materialize)
};

}  // namespace

struct lp_server {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t budget = 0;
    int max_slots = 1;
    lp_options opt{};
    std::chrono::steady_clock::time_point t0;
    std::thread worker;
    // Set-up thread: admits queued requests (arrival order, slot and budget permitting) and
    // sets them up on the device on its own stream while the worker runs rounds.
    std::thread setup_worker;
    hipStream_t setup_stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_idle, cv_setup;
    std::deque<Ticket> queue;
    std::deque<Ticket> ready;  // set up, waiting to join the running set
    int64_t live = 0;          // admitted and not yet completed (slots in use)
    std::vector<Ticket> running;
    std::vector<uint64_t> done;
    std::unordered_map<uint64_t, Ticket> finished;       // completed, result not fetched yet
    std::unordered_map<uint64_t, std::array<double, 3>> times;  // submit, admit, done
    std::unordered_set<uint64_t> cancels;  // admitted requests to stop at the end of the current round
    uint64_t next_ticket = 1;
    bool stop = false;
    lp_server_stats st{};
    lp_handle err_sink;  // receives error messages of the worker

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

void server_round(lp_server* S, DevMaps& run_maps, DevMaps& new_maps, bool& dirty) {
    hipStream_t s = S->stream;
    // requests the set-up thread has placed on the device join the running set
    std::vector<Ticket> newly;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        while (!S->ready.empty()) {
            newly.push_back(S->ready.front());
            S->ready.pop_front();
        }
    }
    std::vector<Ticket> failed;
    std::vector<Ticket> ok;
    for (Ticket& t : newly) {
        t.h->stream = S->stream;
        (t.setup_rc == LP_OK ? ok : failed).push_back(t);
    }
    if (!ok.empty()) {
        std::vector<lp_handle*> hs;
        for (Ticket& t : ok) hs.push_back(t.h);
        if (new_maps.build(hs, &S->opt, s, &S->err_sink) == LP_OK) {
            const MultiMaps& M = new_maps.M;
            launch_multi(M, MULTI_RESET, 0, s);
            launch_multi(M, MULTI_INIT, 0, s);
            launch_multi(M, MULTI_AX_ALL, 0, s);
            launch_multi(M, MULTI_ATY, 1, s);  // 1: products of the initial point
            launch_multi(M, MULTI_PARTIALS, 1, s);
            launch_multi(M, MULTI_DECIDE, 1, s);
            launch_multi(M, MULTI_REBASE_INIT, 0, s);
            (void)hipStreamSynchronize(s);
            std::unique_lock<std::mutex> lk(S->mu);
            for (Ticket& t : ok) S->running.push_back(t);
            S->st.running = static_cast<int64_t>(S->running.size());
            dirty = true;
        } else {
            for (Ticket& t : ok) failed.push_back(t);
        }
    }
    std::vector<Ticket> finished = failed;
    if (!S->running.empty() && dirty) {
        std::vector<lp_handle*> hs;
        for (Ticket& t : S->running) hs.push_back(t.h);
        if (run_maps.build(hs, &S->opt, s, &S->err_sink) == LP_OK) {
            dirty = false;
        } else {  // no launch maps for this set: its requests end as failed, not forgotten
            std::unique_lock<std::mutex> lk(S->mu);
            for (Ticket& t : S->running) {
                t.h->err = S->err_sink.err;
                finished.push_back(t);
                failed.push_back(t);
            }
            S->running.clear();
            S->st.running = 0;
        }
    }
    if (!S->running.empty()) {
        const MultiMaps& M = run_maps.M;
        run_round(run_maps, s, 1);
        (void)hipMemcpyAsync(run_maps.hstatus, M.active, sizeof(int) * M.count, hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        S->st.rounds++;
        std::vector<Ticket> still;
        int64_t work_it = 0;
        double work_nnz = 0.0;
        for (int i = 0; i < M.count; ++i) {
            Ticket& t = S->running[i];
            if (run_maps.hstatus[i] == kRunning) {
                t.counted += run_maps.E;
                work_it += run_maps.E;
                work_nnz += static_cast<double>(run_maps.E) * static_cast<double>(t.h->nnz);
                still.push_back(t);
                continue;
            }
            launch_extract(t.h->P, s);
            (void)hipMemcpyAsync(t.h->h_sc, t.h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s);
            finished.push_back(t);
        }
        if (finished.size() > failed.size()) {
            (void)hipStreamSynchronize(s);
            for (size_t k = failed.size(); k < finished.size(); ++k) {
                lp_handle* h = finished[k].h;
                fill_info(h);
                h->solved = true;
                const int64_t extra = h->info.iterations - finished[k].counted;
                work_it += extra;
                work_nnz += static_cast<double>(extra) * static_cast<double>(h->nnz);
            }
            std::unique_lock<std::mutex> lk(S->mu);
            S->st.lp_iterations += work_it;
            S->st.nnz_iterations += work_nnz;
            S->running = still;
            S->st.running = static_cast<int64_t>(S->running.size());
            dirty = true;
        } else {
            std::unique_lock<std::mutex> lk(S->mu);
            S->st.lp_iterations += work_it;
            S->st.nnz_iterations += work_nnz;
        }
    }
    // cancelled requests of the running set: stopped here, between rounds, with the statistics
    // and the point of their current iterate (the evaluation a host-side stop runs)
    std::vector<Ticket> cancelled;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        if (!S->cancels.empty() && !S->running.empty()) {
            std::vector<Ticket> keep;
            for (Ticket& t : S->running) (S->cancels.erase(t.id) ? cancelled : keep).push_back(t);
            if (!cancelled.empty()) {
                S->running = keep;
                S->st.running = static_cast<int64_t>(S->running.size());
            }
        }
    }
    if (!cancelled.empty()) {
        for (Ticket& t : cancelled) {
            set_form(t.h->P, S->opt);  // the form the server's launches ran it in
            launch_stop(t.h->P, LP_CANCELLED, s);
            launch_evaluate(t.h->P, 2, s);
            launch_extract(t.h->P, s);
            (void)hipMemcpyAsync(t.h->h_sc, t.h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s);
        }
        (void)hipStreamSynchronize(s);
        int64_t work_it = 0;
        double work_nnz = 0.0;
        for (Ticket& t : cancelled) {
            fill_info(t.h);
            t.h->solved = true;
            const int64_t extra = t.h->info.iterations - t.counted;
            work_it += extra;
            work_nnz += static_cast<double>(extra) * static_cast<double>(t.h->nnz);
            finished.push_back(t);
        }
        std::unique_lock<std::mutex> lk(S->mu);
        S->st.lp_iterations += work_it;
        S->st.nnz_iterations += work_nnz;
        dirty = true;
    }
    if (!finished.empty()) {
        for (Ticket& t : finished) {
            const int64_t fp = static_cast<int64_t>(t.h->arena_bytes);
            (void)release_device(t.h);
            t.t_done = S->now();
            std::unique_lock<std::mutex> lk(S->mu);
            S->st.bytes_in_use -= fp;
            S->live--;
            S->st.completed++;
            S->done.push_back(t.id);
            S->finished[t.id] = t;
            S->times[t.id] = {t.t_submit, t.t_admit, t.t_done};
        }
        S->cv_idle.notify_all();
        S->cv_setup.notify_one();  // memory and a slot are free again
    }
}

void setup_loop(lp_server* S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        Ticket t;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop) return;
                if (!S->queue.empty() && S->live < S->max_slots &&
                    S->st.bytes_in_use + static_cast<int64_t>(S->queue.front().h->arena_bytes) <= S->budget)
                    break;
                S->cv_setup.wait(lk);
            }
            t = S->queue.front();
            S->queue.pop_front();
            S->st.bytes_in_use += static_cast<int64_t>(t.h->arena_bytes);
            if (S->st.bytes_in_use > S->st.peak_bytes) S->st.peak_bytes = S->st.bytes_in_use;
            S->live++;
            S->st.admitted++;
            S->st.queued--;
            t.t_admit = S->now();
        }
        t.h->stream = S->setup_stream;
        t.h->own_stream = false;
        t.setup_rc = materialize(t.h);
        std::unique_lock<std::mutex> lk(S->mu);
        S->ready.push_back(t);
        S->cv_work.notify_one();
    }
}

void server_loop(lp_server* S) {
    (void)hipSetDevice(S->device);
    DevMaps run_maps, new_maps;
    bool dirty = true;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) break;
            if (S->ready.empty() && S->running.empty()) {
                S->cv_idle.notify_all();
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
        }
        server_round(S, run_maps, new_maps, dirty);
    }
    run_maps.free_all();
    new_maps.free_all();
}

}  // namespace

extern "C" {

int32_t lp_server_create(lp_server** out, int32_t device, int64_t hbm_budget_bytes, int32_t max_slots,
                         const lp_options* opt) {
    if (!out || hbm_budget_bytes <= 0 || max_slots < 1) return fail(nullptr, LP_ERR_INVALID_ARG, "bad server arguments");
    *out = nullptr;
    try {
        lp_options o;
        lp_default_options(&o);
        if (opt) o = *opt;
        std::string msg;
        if (int32_t rc = validate_options(o, &msg)) return fail(nullptr, rc, msg);
        lp_server* S = new (std::nothrow) lp_server();
        if (!S) return fail(nullptr, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
        S->device = device;
        S->budget = hbm_budget_bytes;
        S->max_slots = max_slots;
        S->opt = o;
        S->t0 = std::chrono::steady_clock::now();
        S->st.hbm_budget = hbm_budget_bytes;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            if (S->stream) (void)hipStreamDestroy(S->stream);
            delete S;
            return fail(nullptr, LP_ERR_DEVICE, std::string("server stream: ") + hipGetErrorString(e));
        }
        S->worker = std::thread(server_loop, S);
        S->setup_worker = std::thread(setup_loop, S);
        *out = S;
        return LP_OK;
    } catch (...) {
        return fail(nullptr, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_server_submit(lp_server* S, lp_handle* h, uint64_t* ticket) {
    if (!S || !h || !ticket) return fail(nullptr, LP_ERR_INVALID_ARG, "bad submit arguments");
    if (!h->deferred || !h->raw || !h->prep) return fail(h, LP_ERR_INVALID_ARG, "a served handle must be deferred");
    if (h->device != S->device) return fail(h, LP_ERR_INVALID_ARG, "handle and server on different devices");
    if (static_cast<int64_t>(h->arena_bytes) > S->budget)
        return fail(h, LP_ERR_INVALID_ARG, "footprint exceeds the server's HBM budget");
    lp_handle* r = nullptr;
    try {
        r = clone_for_request(h);
    } catch (...) {
        return fail(h, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    std::unique_lock<std::mutex> lk(S->mu);
    Ticket t{S->next_ticket++, r, S->now(), 0.0, 0.0, 0, LP_OK};
    S->queue.push_back(t);
    S->st.submitted++;
    S->st.queued++;
    *ticket = t.id;
    S->cv_setup.notify_one();
    return LP_OK;
}

int32_t lp_server_poll(lp_server* S, uint64_t* done_tickets, int32_t cap, int32_t* n_done) {
    if (!S || cap < 0 || (cap > 0 && !done_tickets) || !n_done) return fail(nullptr, LP_ERR_INVALID_ARG, "bad poll arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    const int32_t k = static_cast<int32_t>(std::min<size_t>(S->done.size(), static_cast<size_t>(cap)));
    for (int32_t i = 0; i < k; ++i) done_tickets[i] = S->done[i];
    S->done.erase(S->done.begin(), S->done.begin() + k);
    *n_done = k;
    return LP_OK;
}

int32_t lp_server_ticket_times(lp_server* S, uint64_t ticket, double* times) {
    if (!S || !times) return fail(nullptr, LP_ERR_INVALID_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->times.find(ticket);
    if (it == S->times.end()) return fail(nullptr, LP_ERR_NOT_SOLVED, "ticket not completed");
    for (int k = 0; k < 3; ++k) times[k] = it->second[k];
    return LP_OK;
}

int32_t lp_server_cancel(lp_server* S, uint64_t ticket) {
    if (!S) return fail(nullptr, LP_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
        if (it->id != ticket) continue;
        // not admitted yet: completed at once, without a point
        Ticket t = *it;
        S->queue.erase(it);
        lp_handle* h = t.h;
        h->info = lp_info{};
        h->info.status = LP_CANCELLED;
        const double nan = std::numeric_limits<double>::quiet_NaN();
        h->res_x.assign(static_cast<size_t>(h->n), nan);
        h->res_y.assign(static_cast<size_t>(h->m), nan);
        h->res_z.assign(static_cast<size_t>(h->n), nan);
        h->solved = true;
        t.t_done = S->now();
        S->st.queued--;
        S->st.completed++;
        S->done.push_back(t.id);
        S->finished[t.id] = t;
        S->times[t.id] = {t.t_submit, t.t_admit, t.t_done};
        S->cv_idle.notify_all();
        return LP_OK;
    }
    if (ticket == 0 || ticket >= S->next_ticket || S->times.count(ticket) || S->cancels.count(ticket))
        return fail(nullptr, LP_ERR_INVALID_ARG, "ticket is not pending (unknown, completed or already cancelled)");
    S->cancels.insert(ticket);  // admitted: the worker stops it after the current round
    S->cv_work.notify_one();
    return LP_OK;
}

int32_t lp_server_result(lp_server* S, uint64_t ticket, double* x, double* y, double* z, lp_info* info) {
    if (!S) return fail(nullptr, LP_ERR_INVALID_ARG, "server is NULL");
    lp_handle* h = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->finished.find(ticket);
        if (it == S->finished.end()) return fail(nullptr, LP_ERR_NOT_SOLVED, "ticket not completed (or already fetched)");
        h = it->second.h;
        S->finished.erase(it);
    }
    int32_t rc = LP_OK;
    if (h->solved) {
        rc = lp_get_solution(h, x, y, z, info);
    } else {
        rc = fail(nullptr, LP_ERR_DEVICE, "the request failed to start on the device: " + h->err);
    }
    lp_destroy(h);
    return rc;
}

int32_t lp_server_wait(lp_server* S, double timeout_s) {
    if (!S) return fail(nullptr, LP_ERR_INVALID_ARG, "server is NULL");
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9);
    std::unique_lock<std::mutex> lk(S->mu);
    // every submitted request has reached the finished table
    while (S->st.completed < S->st.submitted) {
        if (S->cv_idle.wait_until(lk, deadline) == std::cv_status::timeout && S->st.completed < S->st.submitted)
            return fail(nullptr, LP_ERR_INTERNAL, "server wait timed out");
    }
    return LP_OK;
}

int32_t lp_server_stats_get(lp_server* S, lp_server_stats* st) {
    if (!S || !st) return fail(nullptr, LP_ERR_INVALID_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    *st = S->st;
    return LP_OK;
}

void lp_server_destroy(lp_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_setup.notify_all();
    if (S->worker.joinable()) S->worker.join();
    if (S->setup_worker.joinable()) S->setup_worker.join();
    (void)hipSetDevice(S->device);
    (void)hipStreamSynchronize(S->stream);
    (void)hipStreamSynchronize(S->setup_stream);
    for (Ticket& t : S->running) lp_destroy(t.h);
    for (Ticket& t : S->ready) lp_destroy(t.h);
    for (Ticket& t : S->queue) lp_destroy(t.h);
    for (auto& kv : S->finished) lp_destroy(kv.second.h);
    (void)hipStreamDestroy(S->stream);
    (void)hipStreamDestroy(S->setup_stream);
    delete S;
}

}  // extern "C"

namespace {
}  // namespace

extern "C" {

void lp_default_options(lp_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps_rel = 1e-4;
    o->max_iters = 100000;
    o->time_limit_s = 0.0;
    o->eval_every = 64;
    o->precision = LP_PREC_FP64;
    o->scaling = 1;
    o->ruiz_passes = 10;
    o->pow_iters = 200;
    o->restarts = 1;
    o->step_size = 0.0;
    o->omega0 = 0.0;
    o->seed = 0x5EED0C0FFEEull;
    o->hip_stream = nullptr;
    o->device = 0;
    o->trace_cap = 4096;
    o->spmv_layout = 0;
    o->long_row_len = 256;
    o->units_per_cu = 4;
    o->batch_wg_per_cu = 3;
    o->batch_split_nnz = 20000;
    o->small_lp_lds = kSmallLpLdsMax;
    o->tile_nnz = 0;
    o->panel_slice_bytes = int64_t(1) << 19;
    o->x0 = nullptr;
    o->y0 = nullptr;
    o->eps_infeas = 1e-8;
    o->method = LP_METHOD_AVERAGED;
    o->reflection = 1.0;
    o->omega_steps = 0;
    o->pw_rule = LP_PW_DEFAULT;
    o->pid_kp = 0.7;
    o->pid_ki = 0.05;
    o->pid_kd = 0.2;
}

int32_t lp_preset_options(lp_options* o, int32_t preset) {
    if (!o || preset < LP_PRESET_DEFAULT || preset > LP_PRESET_SERVING)
        return fail(nullptr, LP_ERR_INVALID_ARG, "unknown preset or NULL options");
    lp_default_options(o);
    switch (preset) {
        case LP_PRESET_SMALL:
            o->spmv_layout = LP_LAYOUT_TILES;
            o->method = LP_METHOD_HALPERN;
            break;
        case LP_PRESET_LARGE:
            o->spmv_layout = LP_LAYOUT_PANELS;
            o->method = LP_METHOD_HALPERN;
            break;
        case LP_PRESET_LARGE_FP32:
            o->spmv_layout = LP_LAYOUT_PANELS;
            o->method = LP_METHOD_HALPERN;
            o->precision = LP_PREC_FP32_REFINED;
            break;
        case LP_PRESET_BATCH:
        case LP_PRESET_SERVING:
            o->spmv_layout = LP_LAYOUT_TILES;
            o->method = LP_METHOD_HALPERN;
            o->precision = LP_PREC_FP32_REFINED;
            o->deferred = preset == LP_PRESET_SERVING ? 1 : 0;
            break;
        default:
            break;
    }
    return LP_OK;
}

int32_t lp_check_word(int32_t device, uint32_t* word, int32_t* checked) {
    if (!word || !checked) return fail(nullptr, LP_ERR_INVALID_ARG, "word or checked NULL");
    *checked = kChecked ? 1 : 0;
    unsigned w = 0;
    if (read_check_word(device, &w) != 0) return fail(nullptr, LP_ERR_DEVICE, "reading the device check word failed");
    *word = w;
    return LP_OK;
}

const char* lp_error_string(int32_t code) {
    switch (code) {
        case LP_OK: return "ok";
        case LP_ERR_INVALID_ARG: return "invalid argument";
        case LP_ERR_INVALID_MATRIX: return "invalid CSR matrix";
        case LP_ERR_INCONSISTENT_BOUNDS: return "inconsistent bounds";
        case LP_ERR_NAN_INPUT: return "NaN or infinite input";
        case LP_ERR_OUT_OF_MEMORY: return "out of memory";
        case LP_ERR_DEVICE: return "HIP device error";
        case LP_ERR_NOT_SOLVED: return "not solved yet";
        case LP_ERR_INTERNAL: return "internal error";
        default: return "unknown error code";
    }
}

const char* lp_last_error(const lp_handle* h) { return h ? h->err.c_str() : g_last_error.c_str(); }

int32_t lp_create(lp_handle** out, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                  const double* vals, const double* c, double c0, const double* b_lo, const double* b_hi,
                  const double* x_lo, const double* x_hi, const lp_options* opt) {
    try {
        if (!out) return fail(nullptr, LP_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        std::string msg;
        int32_t rc = validate_lp(m, n, nnz, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi, &msg);
        if (rc) return fail(nullptr, rc, msg);
        lp_options o;
        lp_default_options(&o);
        if (opt) o = *opt;
        rc = validate_options(o, &msg);
        if (rc) return fail(nullptr, rc, msg);
        if (o.x0)
            for (int32_t j = 0; j < n; ++j)
                if (!std::isfinite(o.x0[j])) return fail(nullptr, LP_ERR_NAN_INPUT, "x0 is not finite");
        if (o.y0)
            for (int32_t i = 0; i < m; ++i)
                if (!std::isfinite(o.y0[i])) return fail(nullptr, LP_ERR_NAN_INPUT, "y0 is not finite");
        lp_handle* h = new (std::nothrow) lp_handle();
        if (!h) return fail(nullptr, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
        h->opt = o;
        h->device = o.device;
        h->m = m;
        h->n = n;
        h->nnz = nnz;
        h->c0 = c0;
        h->has_x0 = o.x0 != nullptr;
        h->has_y0 = o.y0 != nullptr && m > 0;
        h->deferred = o.deferred != 0;
        const auto t0 = std::chrono::steady_clock::now();
        rc = host_prep(h, row_ptr, col_idx);
        if (!rc && h->deferred) {
            h->raw = std::make_shared<HostData>();
            HostData& R = *h->raw;
            R.rp.assign(row_ptr, row_ptr + m + 1);
            R.ci.assign(col_idx, col_idx + nnz);
            R.v.assign(vals, vals + nnz);
            R.c.assign(c, c + n);
            if (m > 0) {
                R.bl.assign(b_lo, b_lo + m);
                R.bu.assign(b_hi, b_hi + m);
            }
            R.xl.assign(x_lo, x_lo + n);
            R.xu.assign(x_hi, x_hi + n);
            if (h->has_x0) R.x0.assign(o.x0, o.x0 + n);
            if (h->has_y0) R.y0.assign(o.y0, o.y0 + m);
            Offsets O;
            h->arena_bytes = arena_layout(h, &O);
        } else if (!rc) {
            rc = device_setup(h, row_ptr, col_idx, vals, c, b_lo, b_hi, x_lo, x_hi, o.x0, o.y0);
            h->prep.reset();  // uploaded; the host copy is no longer needed
        }
        if (rc) {
            g_last_error = h->err;
            destroy_device(h);
            delete h;
            return rc;
        }
        h->opt.x0 = nullptr;  // copied
        h->opt.y0 = nullptr;
        h->info.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = h;
        return LP_OK;
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(nullptr, LP_ERR_INTERNAL, "unexpected exception");
    }
}

}  // extern "C"

namespace {

// The solve loop of lp_solve from a scaled start point (x0s, y0s: device arrays or NULL for
// 0), stopping on E_rel (term_mode 0) or on one residual alone (1 primal, 2 dual: the
// polishing solves), with the set-up primal weight or omega0 > 0.
// lp_solve of an LP whose iteration arrays fit the small-LP LDS budget: one workgroup runs
// the whole loop from LDS (the persistent batched path with a batch of one), bit-identical to
// the kernel-per-phase loop with the same row tiles; the time limit is its device deadline.
int32_t solve_one_workgroup(lp_handle* h, size_t lds_need) {
    hipStream_t s = h->stream;
    const auto t0 = std::chrono::steady_clock::now();
    BatchJob J = make_job(h, nullptr);
    char* b = h->d_job;
    BatchJob* dj = reinterpret_cast<BatchJob*>(b);
    int32_t* dorder = reinterpret_cast<int32_t*>(b + kSoloJobAligned);
    int32_t* dcounter = reinterpret_cast<int32_t*>(b + kSoloJobAligned + 256);
    long long* dt0 = reinterpret_cast<long long*>(b + kSoloJobAligned + 512);
    J.t0 = dt0;
    const int32_t first = 0;
    HIP_TRY(h, hipMemcpyAsync(dj, &J, sizeof(BatchJob), hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipMemcpyAsync(dorder, &first, sizeof(first), hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipStreamSynchronize(s));  // J and `first` are on this stack frame
    launch_batch_start(dcounter, dt0, s);
    const int lds_cap = static_cast<int>((lds_need + 16383) / 16384 * 16384);
    launch_batch(dj, dorder, 1, dcounter, 1, s, lds_cap);
    if (int32_t rc = check_launch(h, "one-workgroup solve")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    fill_info(h);
    h->info.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->info.solve_path = 1;
    h->solved = true;
    return LP_OK;
}

int32_t run_periods(lp_handle* h, std::chrono::steady_clock::time_point t0, long long pause_k);

int32_t solve_from(lp_handle* h, const double* x0s, const double* y0s, int term_mode, double omega0,
                   long long pause_k = 0) {
    set_form(h->P, h->opt);
    hipStream_t s = h->stream;
    const DevLP& P = h->P;
    h->resumable = false;
    if (term_mode == 0 && omega0 == 0.0 && pause_k == 0 && x0s == h->d_x0 && y0s == h->d_y0 && !h->timing &&
        h->opt.small_lp_lds > 0) {
        const size_t need = small_lp_lds_bytes(P);
        if (need <= static_cast<size_t>(h->opt.small_lp_lds) && need <= static_cast<size_t>(kSmallLpLdsMax))
            return solve_one_workgroup(h, need);
    }
    const auto t0 = std::chrono::steady_clock::now();
    launch_reset(P, h->opt.eps_rel, h->opt.eps_infeas, h->opt.max_iters, h->opt.eval_every, h->opt.restarts,
                 h->opt.trace_cap, s, term_mode, omega0);
    launch_init_state(P, x0s, y0s, s);
    launch_evaluate(P, 1, s);
    if (int32_t rc = check_launch(h, "initial evaluation")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return run_periods(h, t0, pause_k);
}

// The period loop of lp_solve from the device state in P: evaluation periods until the
// status leaves "running", the host time limit, or (pause_k > 0) the first period that ends
// at or beyond iteration pause_k, whose decision and restart have then been applied; a pause
// leaves the iteration state untouched (the stop and the statistics of the returned point
// write only outputs), so lp_resume continues it bit for bit. Then the point is extracted.
int32_t run_periods(lp_handle* h, std::chrono::steady_clock::time_point t0, long long pause_k) {
    hipStream_t s = h->stream;
    const DevLP& P = h->P;
    bool paused = false;
    const bool use_graph = !h->timing;
    if (use_graph) capture_graph(h);
    const int timed_it = h->opt.eval_every / 2;
    while (h->h_sc->status == kRunning) {
        const long long k_before = h->h_sc->k;
        if (use_graph && h->gexec) {
            HIP_TRY(h, hipGraphLaunch(h->gexec, s));
        } else {
            record_bundle(h, h->timing ? timed_it : -1);
            if (int32_t rc = check_launch(h, "iteration kernels")) return rc;
        }
        HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        if (h->timing && k_before + timed_it < h->opt.max_iters) {
            float a = 0.f, b = 0.f;
            if (hipEventElapsedTime(&a, h->ev[0], h->ev[1]) == hipSuccess &&
                hipEventElapsedTime(&b, h->ev[1], h->ev[2]) == hipSuccess) {
                h->sum_p_ms += a;
                h->sum_d_ms += b;
                h->samples += 1;
            }
        }
        if (h->h_sc->status != kRunning) break;
        if (pause_k > 0 && h->h_sc->k >= pause_k) {
            launch_stop(P, LP_ITERATION_LIMIT, s);
            launch_evaluate(P, 2, s);
            paused = true;
            break;
        }
        if (h->opt.time_limit_s > 0.0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > h->opt.time_limit_s) {
            launch_stop(P, LP_TIME_LIMIT, s);
            launch_evaluate(P, 2, s);
            break;
        }
    }
    launch_extract(P, s);
    if (int32_t rc = check_launch(h, "extract")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    fill_info(h);
    h->info.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->solved = true;
    h->resumable = paused;
    if (paused) h->paused_opt = h->opt;
    return LP_OK;
}

// ---- state of a paused solve (checkpoint and resume) -------------------------------

// A device array that carries a solve from one evaluation period to the next.
struct StateSpan {
    void* p;
    size_t bytes;
};

// Every such array of the handle, in the order of a state buffer: the FP64 iterates,
// averages, anchors, the point of the previous evaluation and the products kept with them;
// in the FP32 form also the corrections, the rounded shifted data and the FP64 master point.
std::vector<StateSpan> state_spans(const lp_handle* h) {
    const DevLP& P = h->P;
    const size_t dn = sizeof(double) * static_cast<size_t>(h->n), dm = sizeof(double) * static_cast<size_t>(h->m);
    const size_t fn = sizeof(float) * static_cast<size_t>(h->n), fm = sizeof(float) * static_cast<size_t>(h->m);
    std::vector<StateSpan> v = {{P.x, dn},    {P.xa, dn},   {P.xan, dn},   {P.aty, dn},   {P.atya, dn},
                                {P.xp, dn},   {P.atyp, dn}, {P.atyan, dn}, {P.y, dm},     {P.ya, dm},
                                {P.yan, dm},  {P.ax, dm},   {P.axa, dm},   {P.yp, dm},    {P.axp, dm},
                                {P.axan, dm}, {P.fr_x, dn}, {P.fr_y, dm},  {P.fr_ax, dm}, {P.fa_x, dn},
                                {P.fa_y, dm}, {P.fa_ax, dm}};
    if (P.fp32) {
        const StateSpan f[] = {{P.dx, fn},   {P.dxa, fn},  {P.d32, fn},  {P.lo32, fn}, {P.hi32, fn},
                               {P.dy, fm},   {P.dya, fm},  {P.adx, fm},  {P.rl32, fm}, {P.ru32, fm},
                               {P.yh32, fm}, {P.xh, dn},   {P.yh, dm}};
        v.insert(v.end(), std::begin(f), std::end(f));
    }
    return v;
}

struct StateHeader {
    char magic[8];
    int32_t version, precision;
    int32_t m, n;
    int64_t nnz, trace_cap, n_records, total_bytes;
    int32_t method, eval_every, restarts, omega_steps, pw_rule, scalars_bytes, restart_metric, pad;
    double reflection, pid_kp, pid_ki, pid_kd;
    uint64_t fingerprint;
};
constexpr char kStateMagic[8] = {'L', 'P', 'S', 'T', 'A', 'T', 'E', 0};
constexpr int32_t kStateVersion = 1;

// Options that fix the iterations of a run: they must be the same when it is resumed.
bool same_form(const lp_options& a, const lp_options& b) {
    return a.eval_every == b.eval_every && a.restarts == b.restarts && a.method == b.method &&
           a.reflection == b.reflection && a.omega_steps == b.omega_steps && a.pw_rule == b.pw_rule &&
           a.pid_kp == b.pid_kp && a.pid_ki == b.pid_ki && a.pid_kd == b.pid_kd && a.restart_metric == b.restart_metric;
}

// FNV-1a over the scaled cost and the two scaling vectors: tells the LP of a state buffer
// from another one of the same sizes.
int32_t lp_fingerprint(lp_handle* h, uint64_t* out) {
    const size_t n = static_cast<size_t>(h->n), m = static_cast<size_t>(h->m);
    std::vector<double> buf(2 * n + m);
    hipStream_t s = h->stream;
    HIP_TRY(h, hipMemcpyAsync(buf.data(), h->P.c, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(buf.data() + n, h->P.C, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    if (m) HIP_TRY(h, hipMemcpyAsync(buf.data() + 2 * n, h->P.R, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    uint64_t f = 1469598103934665603ull;
    const unsigned char* p = reinterpret_cast<const unsigned char*>(buf.data());
    for (size_t i = 0; i < sizeof(double) * buf.size(); ++i) f = (f ^ p[i]) * 1099511628211ull;
    *out = f;
    return LP_OK;
}

StateHeader state_header(const lp_handle* h, int64_t n_records) {
    StateHeader H{};
    std::memcpy(H.magic, kStateMagic, sizeof(kStateMagic));
    H.version = kStateVersion;
    H.precision = h->opt.precision;
    H.m = h->m;
    H.n = h->n;
    H.nnz = h->nnz;
    H.trace_cap = h->opt.trace_cap;
    H.n_records = n_records;
    H.method = h->opt.method;
    H.eval_every = h->opt.eval_every;
    H.restarts = h->opt.restarts;
    H.omega_steps = h->opt.omega_steps;
    H.pw_rule = h->opt.pw_rule;
    H.restart_metric = h->opt.restart_metric;
    H.scalars_bytes = static_cast<int32_t>(sizeof(Scalars));
    H.reflection = h->opt.reflection;
    H.pid_kp = h->opt.pid_kp;
    H.pid_ki = h->opt.pid_ki;
    H.pid_kd = h->opt.pid_kd;
    int64_t total = static_cast<int64_t>(sizeof(StateHeader) + sizeof(Scalars));
    for (const StateSpan& sp : state_spans(h)) total += static_cast<int64_t>(sp.bytes);
    H.total_bytes = total + n_records * kTraceW * static_cast<int64_t>(sizeof(double));
    return H;
}

// The checked build's report after a call that ran kernels on `device`: LP_ERR_INTERNAL when
// a kernel met an index outside its array (the check word's bits in the message).
int32_t with_checks(lp_handle* h, int device, int32_t rc) {
    if (!kChecked || rc != LP_OK) return rc;
    unsigned w = 0;
    if (read_check_word(device, &w) != 0) return fail(h, LP_ERR_DEVICE, "reading the device check word failed");
    if (w) return fail(h, LP_ERR_INTERNAL, "device index check failed (bits " + std::to_string(w) + ")");
    return LP_OK;
}

// Statistics and extraction of the paused point (after a pause or a state import).
int32_t finish_paused(lp_handle* h) {
    hipStream_t s = h->stream;
    launch_evaluate(h->P, 2, s);
    launch_extract(h->P, s);
    if (int32_t rc = check_launch(h, "paused point")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    fill_info(h);
    h->info.solve_seconds = 0.0;
    h->info.polish_primal_iterations = h->info.polish_dual_iterations = 0;
    return LP_OK;
}

}  // namespace

extern "C" {

int32_t lp_solve(lp_handle* h) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        if (int32_t rc = materialize(h)) return rc;
        const int32_t rc = solve_from(h, h->d_x0, h->d_y0, 0, 0.0);
        h->info.polish_primal_iterations = h->info.polish_dual_iterations = 0;
        return with_checks(h, h->device, rc);
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_polish(lp_handle* h, double eps, int64_t max_iters) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (!(eps > 0.0) || max_iters < 0) return fail(h, LP_ERR_INVALID_ARG, "polish needs eps > 0 and max_iters >= 0");
    if (!h->solved || !h->on_device) return fail(h, LP_ERR_NOT_SOLVED, "lp_polish before lp_solve");
    const int st = h->info.status;
    if (st != LP_OPTIMAL && st != LP_ITERATION_LIMIT && st != LP_TIME_LIMIT)
        return fail(h, LP_ERR_INVALID_ARG, "lp_polish needs a solve that ended at a point, not a certificate");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        DevLP& P = h->P;
        hipStream_t s = h->stream;
        const size_t n = static_cast<size_t>(h->n), m = static_cast<size_t>(h->m);
        double* tmp = nullptr;
        HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&tmp), sizeof(double) * (4 * n + 3 * m + 1)));
        struct Free {
            double* p;
            ~Free() { (void)hipFree(p); }
        } release{tmp};
        // px, the objective's and the variable bounds' copies (n each); py, the row bounds' copies (m each)
        double *px = tmp, *cb = px + n, *xlb = cb + n, *xub = xlb + n, *py = xub + n, *blb = py + m, *bub = blb + m;
        double *c = const_cast<double*>(P.c), *xl = const_cast<double*>(P.xl), *xu = const_cast<double*>(P.xu);
        double *bl = const_cast<double*>(P.bl), *bu = const_cast<double*>(P.bu);
        auto D2D = [&](double* dst, const double* src, size_t count) {
            return count ? hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToDevice, s) : hipSuccess;
        };
        const lp_options saved = h->opt;
        const auto t0 = std::chrono::steady_clock::now();
        // the returned point, in the scaled space
        const int avg = h->h_sc->out_avg;
        HIP_TRY(h, D2D(px, avg ? P.xa : P.x, n));
        HIP_TRY(h, D2D(py, avg ? P.ya : P.y, m));
        h->opt.eps_rel = eps;
        h->opt.max_iters = max_iters;
        h->opt.eps_infeas = 0.0;
        // primal: objective removed, start (x, 0), stop on the primal residual
        HIP_TRY(h, D2D(cb, c, n));
        launch_fill(c, static_cast<long long>(n), 0.0, s);
        int32_t rc = solve_from(h, px, nullptr, 1, 1.0);
        HIP_TRY(h, D2D(c, cb, n));
        const int64_t pit = h->h_sc->k;
        if (!rc) HIP_TRY(h, D2D(px, h->h_sc->out_avg ? P.xa : P.x, n));
        // dual: every finite bound set to 0, start (0, y), stop on the dual residual
        if (!rc) {
            HIP_TRY(h, D2D(xlb, xl, n));
            HIP_TRY(h, D2D(xub, xu, n));
            HIP_TRY(h, D2D(blb, bl, m));
            HIP_TRY(h, D2D(bub, bu, m));
            launch_zero_finite(xl, static_cast<long long>(n), s);
            launch_zero_finite(xu, static_cast<long long>(n), s);
            launch_zero_finite(bl, static_cast<long long>(m), s);
            launch_zero_finite(bu, static_cast<long long>(m), s);
            rc = solve_from(h, nullptr, py, 2, 1.0);
            HIP_TRY(h, D2D(xl, xlb, n));
            HIP_TRY(h, D2D(xu, xub, n));
            HIP_TRY(h, D2D(bl, blb, m));
            HIP_TRY(h, D2D(bu, bub, m));
        }
        const int64_t dit = h->h_sc->k;
        h->opt = saved;
        if (rc) {
            (void)hipStreamSynchronize(s);
            return rc;
        }
        HIP_TRY(h, D2D(py, h->h_sc->out_avg ? P.ya : P.y, m));
        // the polished point (x of the primal solve, y of the dual one) and its statistics
        HIP_TRY(h, D2D(P.x, px, n));
        HIP_TRY(h, D2D(P.xa, px, n));
        HIP_TRY(h, D2D(P.y, py, m));
        HIP_TRY(h, D2D(P.ya, py, m));
        launch_evaluate_point(P, s);
        launch_extract(P, s);
        if (int32_t rc2 = check_launch(h, "polished point")) return rc2;
        HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        const double before = h->info.solve_seconds;
        fill_info(h);
        h->info.status = st;
        h->info.polish_primal_iterations = pit;
        h->info.polish_dual_iterations = dit;
        h->info.solve_seconds = before;
        h->info.polish_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return with_checks(h, h->device, LP_OK);
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_solve_until(lp_handle* h, int64_t k_pause) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (k_pause <= 0) return fail(h, LP_ERR_INVALID_ARG, "k_pause must be positive");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        if (int32_t rc = materialize(h)) return rc;
        const int32_t rc = solve_from(h, h->d_x0, h->d_y0, 0, 0.0, k_pause);
        h->info.polish_primal_iterations = h->info.polish_dual_iterations = 0;
        return with_checks(h, h->device, rc);
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_resume(lp_handle* h, int64_t k_pause) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (k_pause < 0) return fail(h, LP_ERR_INVALID_ARG, "k_pause must be >= 0");
    if (!h->on_device || !h->resumable) return fail(h, LP_ERR_NOT_SOLVED, "the handle holds no paused solve");
    if (!same_form(h->opt, h->paused_opt))
        return fail(h, LP_ERR_INVALID_ARG, "eval_every, restarts, the iteration form or the primal-weight rule changed");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        hipStream_t s = h->stream;
        HIP_TRY(h, hipMemcpyAsync(h->h_sc, h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        if (h->opt.max_iters <= h->h_sc->k) return LP_OK;  // nothing left to run: still paused
        const auto t0 = std::chrono::steady_clock::now();
        Scalars& sc = *h->h_sc;
        sc.status = kRunning;
        sc.eps_rel = h->opt.eps_rel;
        sc.eps_infeas = h->opt.eps_infeas;
        sc.max_iters = h->opt.max_iters;
        sc.out_avg = 0;
        sc.last_restart = 0;
        sc.deadline = 0;
        HIP_TRY(h, hipMemcpyAsync(h->P.sc, h->h_sc, sizeof(Scalars), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        set_form(h->P, h->opt);
        h->resumable = false;
        h->solved = false;
        const int32_t rc = run_periods(h, t0, k_pause);
        h->info.polish_primal_iterations = h->info.polish_dual_iterations = 0;
        return with_checks(h, h->device, rc);
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_export_state(lp_handle* h, void* buf, int64_t cap, int64_t* size) {
    if (!h || !size) return fail(h, LP_ERR_INVALID_ARG, "handle or size NULL");
    if (!h->on_device || !h->resumable) return fail(h, LP_ERR_NOT_SOLVED, "the handle holds no paused solve");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        hipStream_t s = h->stream;
        HIP_TRY(h, hipMemcpyAsync(h->h_sc, h->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        const long long nt = h->h_sc->n_trace;
        const int64_t n_records = h->P.trace ? (nt < h->opt.trace_cap ? nt : h->opt.trace_cap) : 0;
        StateHeader H = state_header(h, n_records);
        *size = H.total_bytes;
        if (!buf) return LP_OK;
        if (cap < H.total_bytes) return fail(h, LP_ERR_INVALID_ARG, "buffer smaller than the state");
        if (int32_t rc = lp_fingerprint(h, &H.fingerprint)) return rc;
        char* out = static_cast<char*>(buf);
        std::memcpy(out, &H, sizeof(H));
        std::memcpy(out + sizeof(H), h->h_sc, sizeof(Scalars));
        size_t off = sizeof(H) + sizeof(Scalars);
        for (const StateSpan& sp : state_spans(h)) {
            if (sp.bytes) HIP_TRY(h, hipMemcpyAsync(out + off, sp.p, sp.bytes, hipMemcpyDeviceToHost, s));
            off += sp.bytes;
        }
        const size_t tb = sizeof(double) * kTraceW * static_cast<size_t>(n_records);
        if (tb) HIP_TRY(h, hipMemcpyAsync(out + off, h->P.trace, tb, hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        return LP_OK;
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_import_state(lp_handle* h, const void* buf, int64_t size) {
    if (!h || !buf) return fail(h, LP_ERR_INVALID_ARG, "handle or buffer NULL");
    if (!h->on_device) return fail(h, LP_ERR_INVALID_ARG, "the handle holds no device memory (deferred)");
    StateHeader H;
    if (size < static_cast<int64_t>(sizeof(H) + sizeof(Scalars)))
        return fail(h, LP_ERR_INVALID_ARG, "buffer too small for a state");
    std::memcpy(&H, buf, sizeof(H));
    if (std::memcmp(H.magic, kStateMagic, sizeof(kStateMagic)) != 0 || H.version != kStateVersion ||
        H.scalars_bytes != static_cast<int32_t>(sizeof(Scalars)))
        return fail(h, LP_ERR_INVALID_ARG, "not a state buffer of this library");
    if (H.m != h->m || H.n != h->n || H.nnz != h->nnz || H.precision != h->opt.precision ||
        H.trace_cap != h->opt.trace_cap)
        return fail(h, LP_ERR_INVALID_ARG, "state of an LP of other sizes, precision or trace capacity");
    if (H.n_records < 0 || H.n_records > (h->opt.trace_cap > 0 ? h->opt.trace_cap : 0))
        return fail(h, LP_ERR_INVALID_ARG, "state with a bad trace length");
    const StateHeader E = state_header(h, H.n_records);
    if (H.total_bytes != size || E.total_bytes != size) return fail(h, LP_ERR_INVALID_ARG, "state buffer of another size");
    if (H.method != h->opt.method || H.eval_every != h->opt.eval_every || H.restarts != h->opt.restarts ||
        H.omega_steps != h->opt.omega_steps || H.pw_rule != h->opt.pw_rule || H.reflection != h->opt.reflection ||
        H.pid_kp != h->opt.pid_kp || H.pid_ki != h->opt.pid_ki || H.pid_kd != h->opt.pid_kd ||
        H.restart_metric != h->opt.restart_metric)
        return fail(h, LP_ERR_INVALID_ARG, "the handle's iteration form differs from the saved run's");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        uint64_t fp = 0;
        if (int32_t rc = lp_fingerprint(h, &fp)) return rc;
        if (fp != H.fingerprint) return fail(h, LP_ERR_INVALID_ARG, "state of another LP");
        const char* in = static_cast<const char*>(buf);
        Scalars sc;
        std::memcpy(&sc, in + sizeof(H), sizeof(Scalars));
        if (sc.status != LP_ITERATION_LIMIT || sc.n_trace < H.n_records || sc.k < 0 || sc.t < 0 ||
            sc.trace_cap != h->opt.trace_cap || sc.eval_every != h->opt.eval_every || sc.term_mode != 0)
            return fail(h, LP_ERR_INVALID_ARG, "state of a solve that is not paused");
        hipStream_t s = h->stream;
        *h->h_sc = sc;
        HIP_TRY(h, hipMemcpyAsync(h->P.sc, h->h_sc, sizeof(Scalars), hipMemcpyHostToDevice, s));
        size_t off = sizeof(H) + sizeof(Scalars);
        for (const StateSpan& sp : state_spans(h)) {
            if (sp.bytes) HIP_TRY(h, hipMemcpyAsync(sp.p, in + off, sp.bytes, hipMemcpyHostToDevice, s));
            off += sp.bytes;
        }
        const size_t tb = sizeof(double) * kTraceW * static_cast<size_t>(H.n_records);
        if (tb) HIP_TRY(h, hipMemcpyAsync(h->P.trace, in + off, tb, hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipStreamSynchronize(s));  // the copies read the caller's pageable buffer
        set_form(h->P, h->opt);
        if (int32_t rc = finish_paused(h)) return rc;
        h->solved = true;
        h->resumable = true;
        h->paused_opt = h->opt;
        return LP_OK;
    } catch (...) {
        return fail(h, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_solve_batch(lp_handle* const* hs, int32_t count, const lp_options* bo) {
    if (count < 0 || (count > 0 && !hs)) return fail(nullptr, LP_ERR_INVALID_ARG, "bad batch arguments");
    if (count == 0) return LP_OK;
    try {
        for (int32_t i = 0; i < count; ++i)
            if (!hs[i]) return fail(nullptr, LP_ERR_INVALID_ARG, "NULL handle in batch");
        const int dev = hs[0]->device;
        for (int32_t i = 1; i < count; ++i)
            if (hs[i]->device != dev) return fail(nullptr, LP_ERR_INVALID_ARG, "batch handles on different devices");
        std::string msg;
        if (bo && validate_options(*bo, &msg)) return fail(nullptr, LP_ERR_INVALID_ARG, msg);
        lp_handle* h0 = hs[0];
        HIP_TRY(h0, hipSetDevice(dev));
        for (int32_t i = 0; i < count; ++i) hs[i]->resumable = false;  // a batch restarts every LP
        const int64_t split = bo ? bo->batch_split_nnz : 20000;
        std::vector<lp_handle*> big, small;
        for (int32_t i = 0; i < count; ++i) (hs[i]->nnz > split ? big : small).push_back(hs[i]);
        const auto t0 = std::chrono::steady_clock::now();
        PersistentRun pr;
        if (!small.empty()) {
            if (int32_t rc = start_persistent(small, bo, pr)) {
                (void)finish_persistent(small, pr, false);
                return rc;
            }
        }
        if (!big.empty()) {
            if (int32_t rc = solve_block_diagonal(big, bo, small.empty() ? h0->stream : pr.s[2])) {
                if (!small.empty()) (void)finish_persistent(small, pr, false);
                return rc;
            }
        }
        if (!small.empty()) {
            if (int32_t rc = finish_persistent(small, pr, true)) return rc;
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int32_t i = 0; i < count; ++i) hs[i]->info.solve_seconds = secs;
        return with_checks(nullptr, dev, LP_OK);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(nullptr, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_solve_batch_static(lp_handle* const* hs, int32_t count, const lp_options* bo) {
    static_assert(LP_STATIC_BATCH_MAX == kStaticBatchMax, "the header's maximum is the scratch array's");
    if (count < 0 || (count > 0 && !hs)) return fail(nullptr, LP_ERR_INVALID_ARG, "bad batch arguments");
    if (count > LP_STATIC_BATCH_MAX)
        return fail(nullptr, LP_ERR_INVALID_ARG, "lp_solve_batch_static: more LPs than LP_STATIC_BATCH_MAX");
    if (count == 0) return LP_OK;
    try {
        for (int32_t i = 0; i < count; ++i) {
            if (!hs[i]) return fail(nullptr, LP_ERR_INVALID_ARG, "NULL handle in batch");
            if (!hs[i]->on_device)
                return fail(hs[i], LP_ERR_INVALID_ARG,
                            "lp_solve_batch_static: the handle holds no device memory (a deferred handle is placed "
                            "on the device by lp_solve or lp_solve_batch)");
            if (hs[i]->device != hs[0]->device)
                return fail(nullptr, LP_ERR_INVALID_ARG, "batch handles on different devices");
        }
        if (bo && (!(bo->eps_rel >= 0.0) || bo->max_iters < 0 || bo->eval_every < 1 || bo->batch_wg_per_cu < 0 ||
                   !(bo->eps_infeas >= 0.0) || bo->method < LP_METHOD_AVERAGED || bo->method > LP_METHOD_HALPERN ||
                   !(bo->reflection >= 0.0 && bo->reflection <= 1.0) || bo->omega_steps < 0 || bo->omega_steps > 8 ||
                   bo->pw_rule < LP_PW_DEFAULT || bo->pw_rule > LP_PW_PID || !(bo->pid_kp >= 0.0 && bo->pid_kp <= 2.0) ||
                   !(bo->pid_ki >= 0.0 && bo->pid_ki <= 2.0) || !(bo->pid_kd >= 0.0 && bo->pid_kd <= 2.0) ||
                   std::isnan(bo->time_limit_s)))
            return fail(nullptr, LP_ERR_INVALID_ARG, "invalid option value");
        lp_handle* h0 = hs[0];
        const int dev = h0->device;
        HIP_TRY(h0, hipSetDevice(dev));
        for (int32_t i = 0; i < count; ++i) hs[i]->resumable = false;  // a batch restarts every LP
        StaticBatchScratch S{};
        HIP_TRY(h0, static_batch_scratch(dev, &S));
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = h0->stream;
        // largest LP first (ties by position: a strict order, so the sort needs no buffer)
        int32_t order[LP_STATIC_BATCH_MAX];
        for (int32_t i = 0; i < count; ++i) order[i] = i;
        std::sort(order, order + count, [&](int32_t a, int32_t b) {
            return hs[a]->nnz != hs[b]->nnz ? hs[a]->nnz > hs[b]->nnz : a < b;
        });
        // job table through a small stack buffer, copied chunk by chunk on the stream
        constexpr int32_t kChunk = 16;
        BatchJob buf[kChunk];
        for (int32_t i = 0; i < count; i += kChunk) {
            const int32_t nb = std::min(kChunk, count - i);
            for (int32_t j = 0; j < nb; ++j) {
                buf[j] = make_job(hs[i + j], bo);
                buf[j].t0 = S.t0;
            }
            HIP_TRY(h0, hipMemcpyAsync(S.jobs + i, buf, sizeof(BatchJob) * nb, hipMemcpyHostToDevice, s));
            HIP_TRY(h0, hipStreamSynchronize(s));
        }
        HIP_TRY(h0, hipMemcpyAsync(S.order, order, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
        HIP_TRY(h0, hipStreamSynchronize(s));  // `order` is on this stack frame
        launch_batch_start(S.counter, S.t0, s);
        int cus = 256;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
        const int wpc = (bo && bo->batch_wg_per_cu > 0) ? bo->batch_wg_per_cu : 3;
        const int grid = std::min(cus * wpc, static_cast<int>(count));
        launch_batch(S.jobs, S.order, count, S.counter, grid, s);
        if (int32_t rc = check_launch(h0, "allocation-free batched solve")) return rc;
        HIP_TRY(h0, hipStreamSynchronize(s));
        for (int32_t i = 0; i < count; ++i)
            HIP_TRY(hs[i], hipMemcpyAsync(hs[i]->h_sc, hs[i]->P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h0, hipStreamSynchronize(s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int32_t i = 0; i < count; ++i) {
            fill_info(hs[i]);
            hs[i]->info.solve_seconds = secs;
            hs[i]->solved = true;
        }
        return with_checks(nullptr, dev, LP_OK);
    } catch (...) {
        return fail(nullptr, LP_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t lp_update_options(lp_handle* h, const lp_options* opt) {
    if (!h || !opt) return fail(h, LP_ERR_INVALID_ARG, "handle or options NULL");
    lp_options o = h->opt;
    o.eps_rel = opt->eps_rel;
    o.max_iters = opt->max_iters;
    o.time_limit_s = opt->time_limit_s;
    o.eval_every = opt->eval_every;
    o.restarts = opt->restarts;
    o.eps_infeas = opt->eps_infeas;
    o.method = opt->method;
    o.reflection = opt->reflection;
    o.omega_steps = opt->omega_steps;
    o.pw_rule = opt->pw_rule;
    o.pid_kp = opt->pid_kp;
    o.pid_ki = opt->pid_ki;
    o.pid_kd = opt->pid_kd;
    o.restart_metric = opt->restart_metric;
    std::string msg;
    if (int32_t rc = validate_options(o, &msg)) return fail(h, rc, msg);
    // the captured iteration bundle bakes in the period, the form, its reflection and the
    // primal-weight steps (the kernels take the solver state by value)
    if (o.eval_every != h->opt.eval_every || o.method != h->opt.method || o.reflection != h->opt.reflection ||
        o.omega_steps != h->opt.omega_steps || o.pw_rule != h->opt.pw_rule || o.pid_kp != h->opt.pid_kp ||
        o.pid_ki != h->opt.pid_ki || o.pid_kd != h->opt.pid_kd || o.restart_metric != h->opt.restart_metric) {
        if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        h->gexec = nullptr;
        h->graph = nullptr;
        h->graph_failed = false;
    }
    h->opt = o;
    return LP_OK;
}

int32_t lp_get_solution(lp_handle* h, double* x, double* y, double* z, lp_info* info) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (!h->solved) return fail(h, LP_ERR_NOT_SOLVED, "lp_get_solution before lp_solve");
    if (!h->on_device) {  // released by a server: the result was kept on the host
        if (x) std::memcpy(x, h->res_x.data(), sizeof(double) * h->n);
        if (y && h->m > 0) std::memcpy(y, h->res_y.data(), sizeof(double) * h->m);
        if (z) std::memcpy(z, h->res_z.data(), sizeof(double) * h->n);
        if (info) *info = h->info;
        return LP_OK;
    }
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = h->stream;
    if (x) HIP_TRY(h, hipMemcpyAsync(x, h->P.out_x, sizeof(double) * h->n, hipMemcpyDeviceToHost, s));
    if (y && h->m > 0) HIP_TRY(h, hipMemcpyAsync(y, h->P.out_y, sizeof(double) * h->m, hipMemcpyDeviceToHost, s));
    if (z) HIP_TRY(h, hipMemcpyAsync(z, h->P.out_z, sizeof(double) * h->n, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (info) *info = h->info;
    return LP_OK;
}

void lp_destroy(lp_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    destroy_device(h);
    delete h;
}

int32_t lp_get_iterates(lp_handle* h, double* x, double* y, double* x_avg, double* y_avg) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (!h->on_device) return fail(h, LP_ERR_NOT_SOLVED, "the handle holds no device data");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const size_t sn = sizeof(double) * h->n, sm = sizeof(double) * h->m;
    if (h->P.fp32) {
        launch_materialize(h->P, s);
        if (int32_t rc = check_launch(h, "materialize")) return rc;
    }
    if (x) HIP_TRY(h, hipMemcpyAsync(x, h->P.x, sn, hipMemcpyDeviceToHost, s));
    if (x_avg) HIP_TRY(h, hipMemcpyAsync(x_avg, h->P.xa, sn, hipMemcpyDeviceToHost, s));
    if (h->m > 0) {
        if (y) HIP_TRY(h, hipMemcpyAsync(y, h->P.y, sm, hipMemcpyDeviceToHost, s));
        if (y_avg) HIP_TRY(h, hipMemcpyAsync(y_avg, h->P.ya, sm, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(h, hipStreamSynchronize(s));
    return LP_OK;
}

int32_t lp_get_scaled(lp_handle* h, double* vals, double* R, double* C, int32_t* t_row_ptr, int32_t* t_col_idx,
                      double* t_vals) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    if (!h->on_device) return fail(h, LP_ERR_NOT_SOLVED, "the handle holds no device data");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const size_t nz = static_cast<size_t>(h->nnz);
    if (vals && nz) HIP_TRY(h, hipMemcpyAsync(vals, h->P.A.csr.v, sizeof(double) * nz, hipMemcpyDeviceToHost, s));
    if (R && h->m) HIP_TRY(h, hipMemcpyAsync(R, h->P.R, sizeof(double) * h->m, hipMemcpyDeviceToHost, s));
    if (C) HIP_TRY(h, hipMemcpyAsync(C, h->P.C, sizeof(double) * h->n, hipMemcpyDeviceToHost, s));
    if (t_row_ptr)
        HIP_TRY(h, hipMemcpyAsync(t_row_ptr, h->P.AT.csr.rp, sizeof(int32_t) * (h->n + 1), hipMemcpyDeviceToHost, s));
    if (t_col_idx && nz)
        HIP_TRY(h, hipMemcpyAsync(t_col_idx, h->P.AT.csr.ci, sizeof(int32_t) * nz, hipMemcpyDeviceToHost, s));
    if (t_vals && nz) HIP_TRY(h, hipMemcpyAsync(t_vals, h->P.AT.csr.v, sizeof(double) * nz, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return LP_OK;
}

int32_t lp_get_trace(lp_handle* h, double* out, int32_t cap, int32_t* n_records) {
    if (!h || cap < 0 || (cap > 0 && !out)) return fail(h, LP_ERR_INVALID_ARG, "bad trace arguments");
    if (!h->solved) return fail(h, LP_ERR_NOT_SOLVED, "lp_get_trace before lp_solve");
    if (!h->on_device || !h->h_sc) {
        if (n_records) *n_records = 0;
        return LP_OK;
    }
    const long long avail = h->h_sc->n_trace < h->opt.trace_cap ? h->h_sc->n_trace : h->opt.trace_cap;
    const long long k = avail < cap ? avail : cap;
    if (k > 0 && h->P.trace) {
        HIP_TRY(h, hipSetDevice(h->device));
        HIP_TRY(h, hipMemcpyAsync(out, h->P.trace, sizeof(double) * kTraceW * static_cast<size_t>(k),
                                  hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    if (n_records) *n_records = static_cast<int32_t>(avail);
    return LP_OK;
}

int32_t lp_set_kernel_timing(lp_handle* h, int32_t enable) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    h->timing = enable != 0;
    h->sum_p_ms = h->sum_d_ms = 0.0;
    h->samples = 0;
    return LP_OK;
}

int32_t lp_get_kernel_times(lp_handle* h, double* primal_ms, double* dual_ms, int64_t* samples) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    const double k = h->samples > 0 ? static_cast<double>(h->samples) : 1.0;
    if (primal_ms) *primal_ms = h->sum_p_ms / k;
    if (dual_ms) *dual_ms = h->sum_d_ms / k;
    if (samples) *samples = h->samples;
    return LP_OK;
}

int32_t lp_get_layout(lp_handle* h, int64_t* sizes, int32_t cap) {
    if (!h || !sizes || cap < 0) return fail(h, LP_ERR_INVALID_ARG, "bad layout arguments");
    const int64_t v[13] = {h->P.A.csr.ntiles, h->P.AT.csr.ntiles, h->long_a, h->long_at,
                           static_cast<int64_t>(h->arena_bytes), h->units_a, h->units_at, h->panels_a, h->panels_at,
                           h->on_device ? h->P.A.layout : -1,
                           static_cast<int64_t>(h->trial_us[0] * 1e3), static_cast<int64_t>(h->trial_us[1] * 1e3),
                           tile_nnz_of(h->tile_shape)};
    for (int32_t i = 0; i < cap && i < 13; ++i) sizes[i] = v[i];
    return LP_OK;
}

}  // extern "C"
