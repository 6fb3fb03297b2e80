// C ABI of the restarted-PDHG solver (include/lp.h): input validation, the one-time
// device setup (CSR transpose, scaling, norm estimate, step size) and the solve loop that
// replays hipGraph-captured bundles of iterations and reads one status word per bundle.
#include "lp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lp_device.h"
#include "lp_layout.h"

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

// Row tiles for the LDS-staged SpMV: consecutive rows while the tile holds at most kTileNnz
// nonzeros and kTileRows rows; a row longer than kTileNnz is a tile of its own.
std::vector<int32_t> build_tiles(int32_t rows, const int32_t* rp, int64_t* n_long) {
    std::vector<int32_t> t;
    t.reserve(static_cast<size_t>(rows) / 64 + 2);
    t.push_back(0);
    int64_t nl = 0;
    int32_t r = 0;
    while (r < rows) {
        const int32_t start = r;
        const int64_t len = rp[r + 1] - rp[r];
        if (len > kTileNnz) {
            ++r;
            ++nl;
        } else {
            int64_t nz = 0;
            while (r < rows && r - start < kTileRows) {
                const int64_t l = rp[r + 1] - rp[r];
                if (l > kTileNnz || nz + l > kTileNnz) break;
                nz += l;
                ++r;
            }
        }
        t.push_back(r);
    }
    *n_long = nl;
    return t;
}

}  // namespace

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
    char* arena = nullptr;
    size_t arena_bytes = 0;
    DevLP P{};
    int* d_perm = nullptr;
    double* d_x0 = nullptr;
    double* d_y0 = nullptr;
    Scalars* h_sc = nullptr;  // pinned host copy of the device scalars
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    bool solved = false;
    lp_info info{};
    std::string err;
    bool timing = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    double sum_p_ms = 0.0, sum_d_ms = 0.0;
    int64_t samples = 0;
};

namespace {

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

int32_t validate(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                 const double* c, double c0, const double* bl, const double* bu, const double* xl, const double* xu,
                 std::string* msg) {
    if (m < 0 || n < 1 || nnz < 0 || nnz > 0x7fffffffLL) {
        *msg = "sizes must satisfy m >= 0, n >= 1, 0 <= nnz < 2^31";
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

int32_t validate_options(const lp_options& o, std::string* msg) {
    if (!(o.eps_rel >= 0.0) || o.max_iters < 0 || o.eval_every < 1 || o.ruiz_passes < 0 || o.pow_iters < 0 ||
        o.trace_cap < 0 || o.precision < LP_PREC_FP64 || o.precision > LP_PREC_FP32_REFINED || o.spmv_layout < 0 || o.spmv_layout > 1 ||
        o.long_row_len < 0 || o.units_per_cu < 0 || o.batch_wg_per_cu < 0 || o.batch_split_nnz < 0 || o.panel_slice_bytes < 0 || std::isnan(o.step_size) || std::isnan(o.omega0) ||
        std::isnan(o.time_limit_s)) {
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
}


BatchJob make_job(lp_handle* h, const lp_options* bo) {
    const lp_options& o = bo ? *bo : h->opt;
    BatchJob J{};
    J.P = h->P;
    J.eps_rel = o.eps_rel;
    J.max_iters = o.max_iters;
    J.trace_cap = h->opt.trace_cap;
    J.eval_every = o.eval_every;
    J.restarts_on = o.restarts;
    J.x0 = h->d_x0;
    J.y0 = h->d_y0;
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

// LPs solved one per workgroup in a single persistent launch.
int32_t solve_persistent(const std::vector<lp_handle*>& hs, const lp_options* bo, hipStream_t s) {
    const int count = static_cast<int>(hs.size());
    lp_handle* h0 = hs[0];
    std::vector<BatchJob> jobs(static_cast<size_t>(count));
    std::vector<int32_t> order(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) {
        jobs[i] = make_job(hs[i], bo);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hs[a]->nnz > hs[b]->nnz; });
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h0->device) != hipSuccess || cus < 1)
        cus = 256;
    const int wpc = (bo && bo->batch_wg_per_cu > 0) ? bo->batch_wg_per_cu : 3;
    int grid = cus * wpc;
    if (grid > count) grid = count;
    const size_t bj = sizeof(BatchJob) * static_cast<size_t>(count), bo_ = sizeof(int32_t) * static_cast<size_t>(count);
    const size_t oc = (bj + bo_ + 255) / 256 * 256;
    char* buf = nullptr;
    HIP_TRY(h0, hipMalloc(reinterpret_cast<void**>(&buf), oc + 256));
    BatchJob* djobs = reinterpret_cast<BatchJob*>(buf);
    int32_t* dorder = reinterpret_cast<int32_t*>(buf + bj);
    int32_t* dcounter = reinterpret_cast<int32_t*>(buf + oc);
    hipError_t e = hipMemcpyAsync(djobs, jobs.data(), bj, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dorder, order.data(), bo_, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(dcounter, 0, sizeof(int32_t), s);
    if (e == hipSuccess) {
        launch_batch(djobs, dorder, count, dcounter, grid, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(h0, LP_ERR_DEVICE, std::string("batched solve: ") + hipGetErrorString(e));
    return finish_batch(hs, s);
}

// LPs advanced together as one block-diagonal problem, one launch per phase for all of
// them, evaluation periods replayed as a hipGraph.
int32_t solve_block_diagonal(const std::vector<lp_handle*>& hs, const lp_options* bo, hipStream_t s) {
    const int count = static_cast<int>(hs.size());
    lp_handle* h0 = hs[0];
    std::vector<BatchJob> jobs(static_cast<size_t>(count));
    std::vector<int2> ma, mat, mred, melem;
    int E = 0;
    for (int i = 0; i < count; ++i) {
        lp_handle* h = hs[i];
        jobs[i] = make_job(h, bo);
        if (E == 0) E = jobs[i].eval_every;
        if (jobs[i].eval_every != E)
            return fail(h0, LP_ERR_INVALID_ARG, "block-diagonal batch LPs must share eval_every");
        for (int t = 0; t < h->P.A.csr.ntiles; ++t) ma.push_back(make_int2(i, t));
        for (int t = 0; t < h->P.AT.csr.ntiles; ++t) mat.push_back(make_int2(i, t));
        for (int b = 0; b < h->P.nred; ++b) mred.push_back(make_int2(i, b));
        const int mx = h->m > h->n ? h->m : h->n;
        for (int b = 0; b < (mx + kBlock - 1) / kBlock; ++b) melem.push_back(make_int2(i, b));
    }
    Arena L;
    const size_t oj = L.add(sizeof(BatchJob) * jobs.size()), oa = L.add(sizeof(int2) * ma.size()),
                 oat = L.add(sizeof(int2) * mat.size()), ored = L.add(sizeof(int2) * mred.size()),
                 oel = L.add(sizeof(int2) * melem.size()), oact = L.add(sizeof(int));
    char* buf = nullptr;
    HIP_TRY(h0, hipMalloc(reinterpret_cast<void**>(&buf), L.off));
    int* hact = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&hact), sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(buf);
        return fail(h0, LP_ERR_OUT_OF_MEMORY, "pinned allocation failed");
    }
    MultiMaps M{};
    M.jobs = reinterpret_cast<const BatchJob*>(buf + oj);
    M.count = count;
    M.map_a = reinterpret_cast<const int2*>(buf + oa);
    M.n_a = static_cast<int>(ma.size());
    M.map_at = reinterpret_cast<const int2*>(buf + oat);
    M.n_at = static_cast<int>(mat.size());
    M.map_red = reinterpret_cast<const int2*>(buf + ored);
    M.n_red = static_cast<int>(mred.size());
    M.map_elem = reinterpret_cast<const int2*>(buf + oel);
    M.n_elem = static_cast<int>(melem.size());
    M.active = reinterpret_cast<int*>(buf + oact);
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    auto cleanup = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipHostFree(hact);
        (void)hipFree(buf);
    };
    auto H2D = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(buf + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    hipError_t e = H2D(oj, jobs.data(), sizeof(BatchJob) * jobs.size());
    if (e == hipSuccess) e = H2D(oa, ma.data(), sizeof(int2) * ma.size());
    if (e == hipSuccess) e = H2D(oat, mat.data(), sizeof(int2) * mat.size());
    if (e == hipSuccess) e = H2D(ored, mred.data(), sizeof(int2) * mred.size());
    if (e == hipSuccess) e = H2D(oel, melem.data(), sizeof(int2) * melem.size());
    if (e == hipSuccess) {
        launch_multi(M, MULTI_RESET, 0, s);
        launch_multi(M, MULTI_INIT, 0, s);
        launch_multi(M, MULTI_AX_ALL, 0, s);
        launch_multi(M, MULTI_ATY, 0, s);
        launch_multi(M, MULTI_PARTIALS, 1, s);
        launch_multi(M, MULTI_DECIDE, 1, s);
        launch_multi(M, MULTI_REBASE_INIT, 0, s);
        e = hipGetLastError();
    }
    auto bundle = [&]() {
        for (int it = 0; it < E; ++it) {
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
        launch_multi(M, MULTI_ACTIVE, 0, s);
    };
    if (e == hipSuccess) {
        hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
            bundle();
            ce = hipStreamEndCapture(s, &graph);
        }
        if (ce == hipSuccess) ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (ce != hipSuccess) {
            (void)hipGetLastError();
            if (graph) (void)hipGraphDestroy(graph);
            graph = nullptr;
            gexec = nullptr;
        }
    }
    long long max_bundles = 0;
    for (const BatchJob& J : jobs) {
        const long long b = J.max_iters / E + 2;
        if (b > max_bundles) max_bundles = b;
    }
    for (long long b = 0; e == hipSuccess && b < max_bundles; ++b) {
        if (gexec) e = hipGraphLaunch(gexec, s);
        else {
            bundle();
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(hact, M.active, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && *hact == 0) break;
    }
    if (e == hipSuccess) {
        launch_multi(M, MULTI_EXTRACT, 0, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return fail(h0, LP_ERR_DEVICE, std::string("block-diagonal batch: ") + hipGetErrorString(e));
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

int32_t setup(lp_handle* h, const int32_t* rp, const int32_t* ci, const double* v, const double* c,
              const double* bl, const double* bu, const double* xl, const double* xu) {
    const int32_t m = h->m, n = h->n;
    const int64_t nnz = h->nnz;
    const lp_options& o = h->opt;
    HIP_TRY(h, hipSetDevice(h->device));
    if (o.hip_stream) {
        h->stream = static_cast<hipStream_t>(o.hip_stream);
    } else {
        HIP_TRY(h, hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    // a1: transpose structure by a stable counting sort on the column index (integer work);
    // perm maps each entry of A^T to its entry of A so the values are moved on the device.
    std::vector<int32_t> rpT(static_cast<size_t>(n) + 1, 0), ciT(static_cast<size_t>(nnz)),
        perm(static_cast<size_t>(nnz));
    for (int64_t e = 0; e < nnz; ++e) rpT[ci[e] + 1]++;
    for (int32_t j = 0; j < n; ++j) rpT[j + 1] += rpT[j];
    {
        std::vector<int32_t> next(rpT.begin(), rpT.end() - 1);
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int32_t p = next[ci[e]]++;
                ciT[p] = i;
                perm[p] = e;
            }
    }
    int64_t dummy_long = 0;
    std::vector<int32_t> tA = build_tiles(m, rp, &dummy_long);
    std::vector<int32_t> tAT = build_tiles(n, rpT.data(), &dummy_long);
    const int32_t ntA = static_cast<int32_t>(tA.size()) - 1, ntAT = static_cast<int32_t>(tAT.size()) - 1;
    // panel-packed layouts of A (gathers x) and A^T (gathers y)
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    const int target_units = cus * (o.units_per_cu > 0 ? o.units_per_cu : 8);
    const int64_t slice = o.panel_slice_bytes > 0 ? o.panel_slice_bytes : (int64_t(1) << 20);
    const int long_len = o.long_row_len > 0 ? o.long_row_len : 256;
    const bool panels = o.spmv_layout == 0;
    PanelLayoutHost LA, LAT;
    if (panels) {
        LA = build_panel_layout(m, n, rp, ci, nullptr, choose_panels(n, slice), long_len, target_units, kUnitRowCap);
        LAT = build_panel_layout(n, m, rpT.data(), ciT.data(), perm.data(), choose_panels(m, slice), long_len,
                                 target_units, kUnitRowCap);
        h->long_a = static_cast<int64_t>(LA.long_rows.size());
        h->long_at = static_cast<int64_t>(LAT.long_rows.size());
        h->units_a = LA.units;
        h->units_at = LAT.units;
        h->panels_a = LA.panels;
        h->panels_at = LAT.panels;
    }

    int mx = m > n ? m : n;
    int nred = (mx + 1023) / 1024;
    if (nred < 1) nred = 1;
    if (nred > kMaxRedBlocks) nred = kMaxRedBlocks;

    const size_t sm = sizeof(double) * static_cast<size_t>(m), sn = sizeof(double) * static_cast<size_t>(n);
    const size_t si_nnz = sizeof(int32_t) * static_cast<size_t>(nnz), sd_nnz = sizeof(double) * static_cast<size_t>(nnz);
    Arena L;
    const size_t o_arp = L.add(sizeof(int32_t) * (m + 1)), o_aci = L.add(si_nnz), o_av = L.add(sd_nnz),
                 o_at = L.add(sizeof(int32_t) * tA.size());
    const size_t o_trp = L.add(sizeof(int32_t) * (n + 1)), o_tci = L.add(si_nnz), o_tv = L.add(sd_nnz),
                 o_tt = L.add(sizeof(int32_t) * tAT.size()), o_perm = L.add(si_nnz);
    const size_t o_c = L.add(sn), o_xl = L.add(sn), o_xu = L.add(sn), o_C = L.add(sn), o_Ci = L.add(sn);
    const size_t o_bl = L.add(sm), o_bu = L.add(sm), o_R = L.add(sm), o_Ri = L.add(sm);
    const size_t o_x = L.add(sn), o_xa = L.add(sn), o_xan = L.add(sn), o_aty = L.add(sn), o_atya = L.add(sn),
                 o_ox = L.add(sn), o_oz = L.add(sn);
    const size_t o_y = L.add(sm), o_ya = L.add(sm), o_yan = L.add(sm), o_ax = L.add(sm), o_axa = L.add(sm),
                 o_oy = L.add(sm);
    const size_t o_x0 = o.x0 ? L.add(sn) : 0, o_y0 = o.y0 ? L.add(sm) : 0;
    const bool fp32 = o.precision == LP_PREC_FP32_REFINED;
    const size_t fn = sizeof(float) * static_cast<size_t>(n), fm = sizeof(float) * static_cast<size_t>(m);
    size_t o32[16] = {0};
    if (fp32) {
        o32[0] = L.add(fn);   // dx
        o32[1] = L.add(fn);   // dxa
        o32[2] = L.add(fm);   // dy
        o32[3] = L.add(fm);   // dya
        o32[4] = L.add(fm);   // adx
        o32[5] = L.add(fn);   // d32
        o32[6] = L.add(fn);   // lo32
        o32[7] = L.add(fn);   // hi32
        o32[8] = L.add(fm);   // rl32
        o32[9] = L.add(fm);   // ru32
        o32[10] = L.add(fm);  // yh32
        o32[11] = L.add(sn);  // xh
        o32[12] = L.add(sm);  // yh
        o32[13] = L.add(sizeof(float) * static_cast<size_t>(nnz));  // A values
        o32[14] = L.add(sizeof(float) * static_cast<size_t>(nnz));  // A^T values
    }
    auto add_layout = [&](const PanelLayoutHost& Q, size_t* off) {
        off[0] = L.add(sizeof(int32_t) * Q.unit_row.size());
        off[1] = L.add(sizeof(int32_t) * Q.unit_seg.size());
        off[2] = L.add(sizeof(uint32_t) * Q.packed.size());
        off[3] = L.add(sizeof(double) * Q.packed.size());
        off[4] = L.add(sizeof(int32_t) * Q.src.size());
        off[5] = L.add(sizeof(int32_t) * Q.long_rows.size());
        off[6] = L.add(Q.is_long.size());
    };
    size_t offA[7] = {0}, offAT[7] = {0}, offA32 = 0, offAT32 = 0;
    if (panels) {
        add_layout(LA, offA);
        add_layout(LAT, offAT);
        if (fp32) {
            offA32 = L.add(sizeof(float) * LA.packed.size());
            offAT32 = L.add(sizeof(float) * LAT.packed.size());
        }
    }
    const size_t o_part = L.add(sizeof(double) * 2 * kNQ * kMaxRedBlocks), o_sc = L.add(sizeof(Scalars)),
                 o_tr = L.add(sizeof(double) * kTraceW * static_cast<size_t>(o.trace_cap > 0 ? o.trace_cap : 1));
    h->arena_bytes = L.off;
    HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->arena), h->arena_bytes));
    HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->h_sc), sizeof(Scalars), hipHostMallocDefault));
    std::memset(h->h_sc, 0, sizeof(Scalars));
    char* b = h->arena;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(b + off); };
    auto I = [&](size_t off) { return reinterpret_cast<int32_t*>(b + off); };

    DevLP& P = h->P;
    P.m = m;
    P.n = n;
    P.nnz = nnz;
    P.nred = nred;
    P.A = Mat{};
    P.AT = Mat{};
    P.A.csr = Csr{m, ntA, static_cast<int>(nnz), I(o_arp), I(o_aci), D(o_av), I(o_at), nullptr};
    P.AT.csr = Csr{n, ntAT, static_cast<int>(nnz), I(o_trp), I(o_tci), D(o_tv), I(o_tt), nullptr};
    P.A.layout = P.AT.layout = panels ? 0 : 1;
    auto bind_layout = [&](const PanelLayoutHost& Q, const size_t* off, Mat& M) {
        M.pan = Panels{Q.units, Q.panels, Q.col_bits, static_cast<int>(Q.nnz_packed), I(off[0]), I(off[1]),
                       reinterpret_cast<const unsigned*>(b + off[2]), D(off[3]),
                       Q.is_long.empty() ? nullptr : reinterpret_cast<const unsigned char*>(b + off[6])};
        M.nlong = static_cast<int>(Q.long_rows.size());
        M.longrows = M.nlong ? I(off[5]) : nullptr;
    };
    if (panels) {
        bind_layout(LA, offA, P.A);
        bind_layout(LAT, offAT, P.AT);
    }
    auto F = [&](size_t off) { return reinterpret_cast<float*>(b + off); };
    P.fp32 = fp32 ? 1 : 0;
    if (fp32) {
        P.dx = F(o32[0]);
        P.dxa = F(o32[1]);
        P.dy = F(o32[2]);
        P.dya = F(o32[3]);
        P.adx = F(o32[4]);
        P.d32 = F(o32[5]);
        P.lo32 = F(o32[6]);
        P.hi32 = F(o32[7]);
        P.rl32 = F(o32[8]);
        P.ru32 = F(o32[9]);
        P.yh32 = F(o32[10]);
        P.xh = D(o32[11]);
        P.yh = D(o32[12]);
        P.A.csr.v32 = F(o32[13]);
        P.AT.csr.v32 = F(o32[14]);
        if (panels) {
            P.A.pan.v32 = F(offA32);
            P.AT.pan.v32 = F(offAT32);
        }
    }
    P.c = D(o_c);
    P.xl = D(o_xl);
    P.xu = D(o_xu);
    P.C = D(o_C);
    P.Ci = D(o_Ci);
    P.bl = D(o_bl);
    P.bu = D(o_bu);
    P.R = D(o_R);
    P.Ri = D(o_Ri);
    P.x = D(o_x);
    P.xa = D(o_xa);
    P.xan = D(o_xan);
    P.aty = D(o_aty);
    P.atya = D(o_atya);
    P.out_x = D(o_ox);
    P.out_z = D(o_oz);
    P.y = D(o_y);
    P.ya = D(o_ya);
    P.yan = D(o_yan);
    P.ax = D(o_ax);
    P.axa = D(o_axa);
    P.out_y = D(o_oy);
    P.partials = D(o_part);
    P.sc = reinterpret_cast<Scalars*>(b + o_sc);
    P.trace = o.trace_cap > 0 ? D(o_tr) : nullptr;
    h->d_perm = I(o_perm);
    h->d_x0 = o.x0 ? D(o_x0) : nullptr;
    h->d_y0 = o.y0 ? D(o_y0) : nullptr;

    hipStream_t s = h->stream;
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_TRY(h, H2D(I(o_arp), rp, sizeof(int32_t) * (m + 1)));
    HIP_TRY(h, H2D(I(o_aci), ci, si_nnz));
    HIP_TRY(h, H2D(D(o_av), v, sd_nnz));
    HIP_TRY(h, H2D(I(o_at), tA.data(), sizeof(int32_t) * tA.size()));
    HIP_TRY(h, H2D(I(o_trp), rpT.data(), sizeof(int32_t) * (n + 1)));
    HIP_TRY(h, H2D(I(o_tci), ciT.data(), si_nnz));
    HIP_TRY(h, H2D(I(o_tt), tAT.data(), sizeof(int32_t) * tAT.size()));
    HIP_TRY(h, H2D(I(o_perm), perm.data(), si_nnz));
    HIP_TRY(h, H2D(D(o_c), c, sn));
    HIP_TRY(h, H2D(D(o_xl), xl, sn));
    HIP_TRY(h, H2D(D(o_xu), xu, sn));
    if (m > 0) {
        HIP_TRY(h, H2D(D(o_bl), bl, sm));
        HIP_TRY(h, H2D(D(o_bu), bu, sm));
    }
    auto upload_layout = [&](const PanelLayoutHost& Q, const size_t* off) -> hipError_t {
        hipError_t e = H2D(b + off[0], Q.unit_row.data(), sizeof(int32_t) * Q.unit_row.size());
        if (e == hipSuccess) e = H2D(b + off[1], Q.unit_seg.data(), sizeof(int32_t) * Q.unit_seg.size());
        if (e == hipSuccess) e = H2D(b + off[2], Q.packed.data(), sizeof(uint32_t) * Q.packed.size());
        if (e == hipSuccess) e = H2D(b + off[4], Q.src.data(), sizeof(int32_t) * Q.src.size());
        if (e == hipSuccess) e = H2D(b + off[5], Q.long_rows.data(), sizeof(int32_t) * Q.long_rows.size());
        if (e == hipSuccess) e = H2D(b + off[6], Q.is_long.data(), Q.is_long.size());
        return e;
    };
    if (panels) {
        HIP_TRY(h, upload_layout(LA, offA));
        HIP_TRY(h, upload_layout(LAT, offAT));
    }
    if (o.x0) HIP_TRY(h, H2D(h->d_x0, o.x0, sn));
    if (o.y0 && m > 0) HIP_TRY(h, H2D(h->d_y0, o.y0, sm));
    HIP_TRY(h, hipMemsetAsync(P.sc, 0, sizeof(Scalars), s));

    // a2: scaling, exact powers of two
    launch_fill(D(o_R), m, 1.0, s);
    launch_fill(D(o_C), n, 1.0, s);
    if (o.scaling) {
        for (int pass = 0; pass <= o.ruiz_passes; ++pass)
            launch_scale_pass(P, I(o_arp), I(o_aci), D(o_av), I(o_trp), h->d_perm, D(o_R), D(o_C), D(o_ax),
                              D(o_aty), pass == o.ruiz_passes ? 1 : 0, s);
    }
    launch_gather(h->d_perm, D(o_av), D(o_tv), nnz, s);
    if (panels) {  // panel values in packed order, from the scaled A
        launch_gather(I(offA[4]), D(o_av), D(offA[3]), LA.nnz_packed, s);
        launch_gather(I(offAT[4]), D(o_av), D(offAT[3]), LAT.nnz_packed, s);
    }
    if (fp32) {  // FP32 copies of the scaled values (rounded to nearest)
        launch_to_float(D(o_av), F(o32[13]), nnz, s);
        launch_to_float(D(o_tv), F(o32[14]), nnz, s);
        if (panels) {
            launch_to_float(D(offA[3]), F(offA32), LA.nnz_packed, s);
            launch_to_float(D(offAT[3]), F(offAT32), LAT.nnz_packed, s);
        }
    }
    launch_prepare(P, D(o_c), D(o_bl), D(o_bu), D(o_xl), D(o_xu), D(o_R), D(o_C), D(o_Ri), D(o_Ci), h->d_x0,
                   h->d_y0, s);
    // a3: ||A~||_2 by power iteration (x, A~x and A~^T y buffers are free at this point)
    if (!(o.step_size > 0.0)) launch_power_norm(P, o.pow_iters, o.seed, P.x, P.ax, P.aty, s);
    launch_finalize_setup(P, o.step_size, o.omega0, h->c0, s);
    if (int32_t rc = check_launch(h, "setup kernels")) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    for (auto& e : h->ev) HIP_TRY(h, hipEventCreate(&e));
    return LP_OK;
}

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
    o->units_per_cu = 8;
    o->batch_wg_per_cu = 3;
    o->batch_split_nnz = 20000;
    o->panel_slice_bytes = int64_t(1) << 20;
    o->x0 = nullptr;
    o->y0 = nullptr;
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
        int32_t rc = validate(m, n, nnz, row_ptr, col_idx, vals, c, c0, b_lo, b_hi, x_lo, x_hi, &msg);
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
        const auto t0 = std::chrono::steady_clock::now();
        rc = setup(h, row_ptr, col_idx, vals, c, b_lo, b_hi, x_lo, x_hi);
        if (rc) {
            g_last_error = h->err;
            destroy_device(h);
            delete h;
            return rc;
        }
        h->opt.x0 = nullptr;  // copied to the device
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

int32_t lp_solve(lp_handle* h) {
    if (!h) return fail(nullptr, LP_ERR_INVALID_ARG, "handle is NULL");
    try {
        HIP_TRY(h, hipSetDevice(h->device));
        hipStream_t s = h->stream;
        const DevLP& P = h->P;
        const auto t0 = std::chrono::steady_clock::now();
        launch_reset(P, h->opt.eps_rel, h->opt.max_iters, h->opt.eval_every, h->opt.restarts, h->opt.trace_cap, s);
        launch_init_state(P, h->d_x0, h->d_y0, s);
        launch_evaluate(P, 1, s);
        if (int32_t rc = check_launch(h, "initial evaluation")) return rc;
        HIP_TRY(h, hipMemcpyAsync(h->h_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
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
        const int64_t split = bo ? bo->batch_split_nnz : 20000;
        std::vector<lp_handle*> big, small;
        for (int32_t i = 0; i < count; ++i) (hs[i]->nnz > split ? big : small).push_back(hs[i]);
        const auto t0 = std::chrono::steady_clock::now();
        if (!big.empty()) {
            if (int32_t rc = solve_block_diagonal(big, bo, h0->stream)) return rc;
        }
        if (!small.empty()) {
            if (int32_t rc = solve_persistent(small, bo, h0->stream)) return rc;
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int32_t i = 0; i < count; ++i) hs[i]->info.solve_seconds = secs;
        return LP_OK;
    } catch (const std::bad_alloc&) {
        return fail(nullptr, LP_ERR_OUT_OF_MEMORY, "host allocation failed");
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
    std::string msg;
    if (int32_t rc = validate_options(o, &msg)) return fail(h, rc, msg);
    if (o.eval_every != h->opt.eval_every) {
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
    const int64_t v[9] = {h->P.A.csr.ntiles, h->P.AT.csr.ntiles, h->long_a, h->long_at,
                          static_cast<int64_t>(h->arena_bytes), h->units_a, h->units_at, h->panels_a, h->panels_at};
    for (int32_t i = 0; i < cap && i < 9; ++i) sizes[i] = v[i];
    return LP_OK;
}

}  // extern "C"
