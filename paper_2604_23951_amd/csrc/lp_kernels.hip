// HIP kernels of the restarted, averaged PDHG solver for gfx950 (MI355X).
//
// The method (the PDLP-family averaged PDHG that the paper's presolve feeds, Section 1 and
// Section 4 name it; the iteration itself is the published one) spends its time in two
// sparse products per iteration, A^T y and A x, each followed by an elementwise update.
// Both are HBM-bound: the products are streamed from CSR (values + int32 indices) with the
// nonzeros of a tile staged in LDS and the row sums formed from LDS, and the primal / dual
// updates are fused into the epilogue of the product that feeds them, so every vector is
// read and written once per iteration. No step is a dense contraction: no MFMA.
//
// Determinism: every row sum is formed sequentially in CSR order from the products
// (a_e * x_col(e) rounded, then added in order), which is also the plain definition of the
// sum; rows longer than one tile use a fixed-shape workgroup tree. All reductions use a
// fixed grid, fixed wave64 shuffles and a fixed-order second stage, so a solve is bitwise
// reproducible run to run.
#include "lp_device.h"

#include <math.h>

#include <mutex>

// Check word of the checked build (see lp_device.h); unused otherwise.
__device__ unsigned int lp_check_word;

namespace lpgpu {

namespace {

// An index into an array of n elements: itself, or, in the checked build when out of range,
// 0 with `bit` set in the check word.
template <class I>
__device__ inline I checked_index(I i, int n, unsigned bit) {
    if constexpr (kChecked) {
        if (static_cast<unsigned>(i) >= static_cast<unsigned>(n)) {
            atomicOr(&lp_check_word, bit);
            return I(0);
        }
    }
    return i;
}

__device__ inline double clampd(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

__device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the workgroup in a fixed order; the result is valid in thread 0. `red` holds
// kBlock / 64 doubles of LDS. Ends with a barrier so `red` may be reused.
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kBlock / 64; ++i) t += red[i];
    }
    __syncthreads();
    return t;
}

// Same, but every thread gets the total.
__device__ inline double block_sum_all(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

// Power-of-two stand-in for 1/sqrt(v): v = f 2^E with f in [1/2, 1) gives 2^(-floor(E/2)).
__device__ inline double pow2_rsqrt(double v) {
    if (!(v > 0.0) || !finite_d(v)) return 1.0;
    int e;
    frexp(v, &e);
    const int h = (e >= 0) ? e / 2 : -((1 - e) / 2);
    return ldexp(1.0, -h);
}

// SplitMix64 finaliser applied to seed + (k+1) * golden gamma, mapped to [-1/2, 1/2).
__device__ inline double splitmix_centered(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= (z >> 31);
    return static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

inline unsigned grid_for(long long n, int per_block = kBlock) {
    long long g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65535LL * 64) g = 65535LL * 64;
    return static_cast<unsigned>(g);
}

// ------------------------------------------------------------------ SpMV with epilogues

// One workgroup per tile. Short tiles (at most TN nonzeros, TN one of the row-tile shapes):
// every thread owns TN / kBlock nonzeros of the tile; it first issues all their index and value loads, then all
// the gathers of the vector entries, and stores the products to LDS, so each thread keeps
// kPerThread independent memory requests in flight. The epilogue operands of the rows a
// thread finishes are loaded before the barrier. After the barrier each thread forms the sum
// of one row from LDS in CSR order and runs the epilogue. A tile that is a single row longer
// than TN is reduced by the whole workgroup (fixed-shape tree).

// Matrix values in the arithmetic type of a kernel instance.
template <class T>
__device__ inline const T* vals_of(const Csr& M);
template <>
__device__ inline const double* vals_of<double>(const Csr& M) { return M.v; }
template <>
__device__ inline const float* vals_of<float>(const Csr& M) { return M.v32; }
template <class T>
__device__ inline const T* vals_of(const Panels& M);
template <>
__device__ inline const double* vals_of<double>(const Panels& M) { return M.v; }
template <>
__device__ inline const float* vals_of<float>(const Panels& M) { return M.v32; }

template <class T>
__device__ inline T block_sum_t(T v, double* red) {
    return static_cast<T>(block_sum(static_cast<double>(v), red));
}

// Row r reduced by the whole workgroup: thread t adds the products of entries t, t + kBlock,
// ... in order (TN / kBlock loads in flight per round; the order of the additions does not
// depend on TN), then a fixed-shape tree over the workgroup. Called by every thread.
template <int TN, class T, class Epi>
__device__ void row_tree_body(const Csr& M, int r, const T* __restrict__ xin, const Epi& epi, double* red) {
    constexpr int kPerThread = TN / kBlock;
    const int p0 = M.rp[r], p1 = M.rp[r + 1];
    const int tid = threadIdx.x;
    const int* __restrict__ ci = M.ci;
    const T* __restrict__ av = vals_of<T>(M);
    const int elast = M.nnz > 0 ? M.nnz - 1 : 0;
    const typename Epi::Pre pre = epi.load(r);
    T s = 0;
    for (int base = p0; base < p1; base += TN) {
        int col[kPerThread];
        T val[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = min(base + tid + k * kBlock, elast);
            col[k] = __builtin_nontemporal_load(ci + e);
            val[k] = __builtin_nontemporal_load(av + e);
        }
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
            if (base + tid + k * kBlock >= p1) col[k] = 0;
        T xv[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) xv[k] = xin[checked_index(col[k], M.cols, 8u)];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const T pr = val[k] * xv[k];
            if (base + tid + k * kBlock < p1) s += pr;
        }
    }
    s = block_sum_t(s, red);
    if (tid == 0) epi.finish(r, s, pre);
}

template <int TN, class T, class Epi>
__device__ void tile_body(const Csr& M, int b, const T* __restrict__ xin, const Epi& epi, T* prod, double* red) {
    constexpr int kPerThread = TN / kBlock;
    constexpr int kRowsPerThread = TN / 4 / kBlock;
    const int r0 = M.tiles[b], r1 = M.tiles[b + 1];
    const int p0 = M.rp[r0], p1 = M.rp[r1];
    const int tid = threadIdx.x;
    const int* __restrict__ ci = M.ci;
    const T* __restrict__ av = vals_of<T>(M);
    // Loads below are unconditional on clamped, in-bounds indices (every array holds at least
    // one element) so that they issue back to back; out-of-range lanes are masked afterwards.
    const int elast = M.nnz > 0 ? M.nnz - 1 : 0;
    if (p1 - p0 <= TN) {
        int col[kPerThread];
        T val[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int e = min(p0 + tid + k * kBlock, elast);
            col[k] = __builtin_nontemporal_load(ci + e);
            val[k] = __builtin_nontemporal_load(av + e);
        }
        typename Epi::Pre pre[kRowsPerThread];
        int q0[kRowsPerThread], q1[kRowsPerThread];
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) {
            const int r = min(r0 + tid + j * kBlock, r1 - 1);
            q0[j] = M.rp[r] - p0;
            q1[j] = M.rp[r + 1] - p0;
            pre[j] = epi.load(r);
        }
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
            if (p0 + tid + k * kBlock >= p1) col[k] = 0;
        T xv[kPerThread];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) xv[k] = xin[checked_index(col[k], M.cols, 4u)];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) prod[tid + k * kBlock] = val[k] * xv[k];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) {
            const int r = r0 + tid + j * kBlock;
            if (r < r1) {
                T s = 0;
                int q = q0[j];
                const int qe = q1[j];
                for (; q + 4 <= qe; q += 4) {
                    const T a0 = prod[q], a1 = prod[q + 1], a2 = prod[q + 2], a3 = prod[q + 3];
                    s += a0;
                    s += a1;
                    s += a2;
                    s += a3;
                }
                for (; q < qe; ++q) s += prod[q];
                epi.finish(r, s, pre[j]);
            }
        }
    } else {
        row_tree_body<TN, T>(M, r0, xin, epi, red);
    }
}

// The tile body of the LP's row-tile shape (Csr::shape; prod holds kTileNnzMax values).
template <class T, class Epi>
__device__ inline void tile_body_any(const Csr& M, int b, const T* __restrict__ xin, const Epi& epi, T* prod,
                                     double* red) {
    if (M.shape == 0) tile_body<tile_nnz_of(0)>(M, b, xin, epi, prod, red);
    else if (M.shape == 1) tile_body<tile_nnz_of(1)>(M, b, xin, epi, prod, red);
    else tile_body<tile_nnz_of(2)>(M, b, xin, epi, prod, red);
}

template <class T, class Epi, int TN>
__global__ __launch_bounds__(kBlock) void spmv_tiles_kernel(Csr M, const T* __restrict__ xin, Epi epi) {
    __shared__ T prod[TN];
    __shared__ double red[kBlock / 64];
    if (!epi.begin()) return;
    tile_body<TN>(M, static_cast<int>(blockIdx.x), xin, epi, prod, red);
}

// Panel-packed SpMV over wave units of rows. The entries of a unit are walked in packed order,
// panel by panel (all resident units do, so the slice of the gathered vector for the current
// panel stays in the L2 of each XCD), in chunks of 64 consecutive entries. Inside a panel
// segment the entries are sorted by row, so between two places where the row id drops (the
// start of a later segment) the rows of a chunk ascend and each row forms one run. The run's
// first lane adds the run's products, in order, to the row's accumulator in LDS; a chunk with
// drops is handled piece by piece, in order. Later runs of a row (later chunks, later panels)
// follow in column order, so every row sum is formed in CSR order. Rows listed as long have no
// packed entries; workgroups past the panel ones reduce them, one long row each (fixed-shape
// tree), in the same launch.
//
// Each unit has two waves: a producer that streams the entries, gathers the vector and writes
// each group's products and row ids to an LDS buffer, and a consumer that forms the run sums
// of the previous group from the other buffer. A workgroup holds kPanelUnits units; its waves
// meet at a barrier after every group step, so the two halves of the work overlap instead of
// taking turns in one wave. After the last group both waves of a unit finish its rows with
// the epilogue.
//
// Producer pipeline: the entries of kStreamDepth groups of kChunks chunks are loaded or in
// flight and the gathers of two groups are in flight: while group g is multiplied, the gathers
// of groups g + 1 and g + 2 and the entry loads of groups g + 3 and g + 4 are outstanding.
// Slots are indexed at compile time (the loop is unrolled by 12 = lcm(4, 3) steps) so that
// every group stays in registers.
constexpr int kPanelUnits = 2;  // wave units per workgroup (a producer and a consumer wave each)
static_assert(2 * kPanelUnits * 64 == kBlock, "a panel workgroup is one producer and one consumer wave per unit");

template <class T>
struct PanelGroups {
    unsigned pk[kStreamDepth][kChunks];
    T val[kStreamDepth][kChunks];
    T xv[3][kChunks];
};

// One group's products and row ids, handed from the producer to the consumer of a unit.
template <class T>
struct PanelBuf {
    T prod[2][kChunks * 64];
    int row[2][kChunks * 64];
};

struct PanelUnit {
    int s, e, last, lane, cb;
    int cols, rows;  // gathered vector length, accumulator rows (the checked build's bounds)
    unsigned cmask;
    __device__ int chunk_start(int g, int c) const { return s + (g * kChunks + c) * 64; }
};

template <class T>
__device__ inline void panel_load(PanelGroups<T>& G, int S, int g, const PanelUnit& U, const unsigned* __restrict__ pkp,
                                  const T* __restrict__ pvp) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int idx = min(U.chunk_start(g, c) + U.lane, U.last);
        G.pk[S][c] = __builtin_nontemporal_load(pkp + idx);
        G.val[S][c] = __builtin_nontemporal_load(pvp + idx);
    }
}

template <class T>
__device__ inline void panel_gather(PanelGroups<T>& G, int S, int X, int g, const PanelUnit& U,
                                    const T* __restrict__ xin) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const unsigned col = U.chunk_start(g, c) + U.lane < U.e ? (G.pk[S][c] & U.cmask) : 0u;
        G.xv[X][c] = xin[checked_index(col, U.cols, 1u)];
    }
}

// Row id of the previous lane (lane 0 gets -1): a DPP shift of the whole wave by one lane.
__device__ inline int prev_lane_row(int row) {
    return __builtin_amdgcn_update_dpp(-1, row, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}

// Adds the run that starts at this (head) lane to its row's accumulator, in order.
template <class T>
__device__ inline void add_run(T* acc, const T* prodc, int row, T own, int lane, unsigned long long heads, int nvalid) {
    const unsigned long long rest = lane < 63 ? (heads >> (lane + 1)) : 0ull;
    const int end = rest ? lane + 1 + __builtin_ctzll(rest) : nvalid;
    T a = acc[row] + own;
    int q = lane + 1;
    for (; q + 4 <= end; q += 4) {
        const T a0 = prodc[q], a1 = prodc[q + 1], a2 = prodc[q + 2], a3 = prodc[q + 3];
        a += a0;
        a += a1;
        a += a2;
        a += a3;
    }
    for (; q < end; ++q) a += prodc[q];
    acc[row] = a;
}

// Producer step K of the unrolled loop on group g (K = g mod 12): issue the gathers of group
// g + 2 and the entry loads of group g + 4, then write the products and row ids of group g.
// Steps past the end of the unit see empty chunks and do only masked work.
template <class T, int K>
__device__ inline void panel_produce(PanelGroups<T>& G, int g, const PanelUnit& U, const unsigned* __restrict__ pkp,
                                     const T* __restrict__ pvp, const T* __restrict__ xin, T* prod, int* rowb) {
    constexpr int S = K % kStreamDepth, X = K % 3;
    constexpr int S2 = (K + 2) % kStreamDepth, X2 = (K + 2) % 3;
    panel_gather(G, S2, X2, g + 2, U, xin);
    int row[kChunks];
    T v[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        row[c] = static_cast<int>(checked_index(G.pk[S][c] >> U.cb, U.rows, 2u));
        v[c] = G.val[S][c];
    }
    panel_load(G, S, g + kStreamDepth, U, pkp, pvp);
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        prod[c * 64 + U.lane] = v[c] * G.xv[X][c];
        rowb[c * 64 + U.lane] = row[c];
    }
}

// Consumer: the run sums of group g, chunk by chunk, from the producer's buffer.
template <class T>
__device__ inline void panel_consume(int g, const PanelUnit& U, const T* prod, const int* rowb, T* acc) {
    const int lane = U.lane;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int nvalid = min(64, U.e - U.chunk_start(g, c));
        if (nvalid <= 0) break;
        const int row = rowb[c * 64 + lane];
        const T own = prod[c * 64 + lane];
        const int prev = prev_lane_row(row);
        const bool valid = lane < nvalid;
        const bool head = valid && prev != row;
        const unsigned long long heads = __ballot(head);
        const unsigned long long drops = __ballot(valid && prev > row);
        if (drops == 0) {
            if (head) add_run(acc, prod + c * 64, row, own, lane, heads, nvalid);
        } else {
            const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
            const int piece = __popcll(drops & upto);
            const int npieces = __popcll(drops) + 1;
            for (int j = 0; j < npieces; ++j) {
                if (head && piece == j) add_run(acc, prod + c * 64, row, own, lane, heads, nvalid);
                __builtin_amdgcn_wave_barrier();
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <class T, class Epi>
__global__ __launch_bounds__(kBlock) void spmv_panel_kernel(Panels M, Csr L, int panel_blocks,
                                                            const T* __restrict__ xin, Epi epi) {
    extern __shared__ __align__(16) unsigned char panel_acc_lds[];  // kPanelUnits x M.max_rows of T
    __shared__ PanelBuf<T> bufs[kPanelUnits];
    __shared__ double red[kBlock / 64];
    if (!epi.begin()) return;
    if (static_cast<int>(blockIdx.x) >= panel_blocks) {
        const int r = L.rowlist[blockIdx.x - panel_blocks];
        row_tree_body<tile_nnz_of(1), T>(L, r, xin, epi, red);
        return;
    }
    // The wave index is the same on every lane; saying so keeps the unit's bookkeeping in
    // scalar registers and its branches scalar.
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int slot = w % kPanelUnits;
    const bool producer = w < kPanelUnits;
    const int u = blockIdx.x * kPanelUnits + slot;
    const bool active = u < M.units;
    // Group steps of the workgroup: those of its longest unit (the same value on every wave).
    int groups = 0;
#pragma unroll
    for (int k = 0; k < kPanelUnits; ++k) {
        const int uk = blockIdx.x * kPanelUnits + k;
        if (uk < M.units) {
            const int len = M.unit_seg[uk * (M.panels + 1) + M.panels] - M.unit_seg[uk * (M.panels + 1)];
            groups = max(groups, (len + kChunks * 64 - 1) / (kChunks * 64));
        }
    }
    const int r0 = active ? M.unit_row[u] : 0, nr = active ? M.unit_row[u + 1] - r0 : 0;
    T* acc = reinterpret_cast<T*>(panel_acc_lds) + slot * M.max_rows;
    PanelUnit U;
    U.s = active ? M.unit_seg[u * (M.panels + 1)] : 0;
    U.e = active ? M.unit_seg[u * (M.panels + 1) + M.panels] : 0;
    U.last = M.nnz > 0 ? M.nnz - 1 : 0;
    U.lane = lane;
    U.cb = M.col_bits;
    U.cmask = (1u << M.col_bits) - 1u;
    U.cols = M.cols;
    U.rows = M.max_rows;
    const unsigned* __restrict__ pkp = M.pk;
    const T* __restrict__ pvp = vals_of<T>(M);
    // Both roles run the same group steps with one barrier after each (the loops below have the
    // same shape): at step t the producers write group t and the consumers sum group t - 1.
    // The producer's steps are unconditional (steps past the end of its unit are masked), which
    // keeps its loads in flight across steps.
    static_assert(kStreamDepth == 4, "the loop below is unrolled for four entry slots and three gather slots");
    PanelBuf<T>& B = bufs[slot];
    if (active && producer) {
        PanelGroups<T> G;
#pragma unroll
        for (int S = 0; S < kStreamDepth; ++S) panel_load(G, S, S, U, pkp, pvp);
        panel_gather(G, 0, 0, 0, U, xin);
        panel_gather(G, 1, 1, 1, U, xin);
#define LP_PRODUCE(K)                                                                                \
    panel_produce<T, K>(G, t + K, U, pkp, pvp, xin, B.prod[(t + K) & 1], B.row[(t + K) & 1]); \
    __syncthreads();
        for (int t = 0; t <= groups; t += 12) {
            LP_PRODUCE(0) LP_PRODUCE(1) LP_PRODUCE(2) LP_PRODUCE(3) LP_PRODUCE(4) LP_PRODUCE(5)
            if (t + 6 > groups) break;
            LP_PRODUCE(6) LP_PRODUCE(7) LP_PRODUCE(8) LP_PRODUCE(9) LP_PRODUCE(10) LP_PRODUCE(11)
        }
#undef LP_PRODUCE
    } else {
        if (active)
            for (int r = lane; r < nr; r += 64) acc[r] = 0;
#define LP_CONSUME(K)                                                                    \
    if (active && t + K >= 1 && t + K <= groups)                                        \
        panel_consume<T>(t + K - 1, U, B.prod[(t + K - 1) & 1], B.row[(t + K - 1) & 1], acc); \
    __syncthreads();
        for (int t = 0; t <= groups; t += 12) {
            LP_CONSUME(0) LP_CONSUME(1) LP_CONSUME(2) LP_CONSUME(3) LP_CONSUME(4) LP_CONSUME(5)
            if (t + 6 > groups) break;
            LP_CONSUME(6) LP_CONSUME(7) LP_CONSUME(8) LP_CONSUME(9) LP_CONSUME(10) LP_CONSUME(11)
        }
#undef LP_CONSUME
    }
    // The last consumer step was followed by a barrier: every accumulator is complete.
    if (!active) return;
    constexpr int kEpiRows = 8;  // rows per lane whose epilogue operands are loaded together
    const int half = producer ? 0 : 1;
    for (int r = lane + half * kEpiRows * 64; r < nr; r += 2 * kEpiRows * 64) {
        typename Epi::Pre pre[kEpiRows];
        int rows[kEpiRows];
#pragma unroll
        for (int k = 0; k < kEpiRows; ++k) {
            rows[k] = r0 + min(r + k * 64, nr - 1);
            pre[k] = epi.load(rows[k]);
        }
#pragma unroll
        for (int k = 0; k < kEpiRows; ++k) {
            const int rl = r + k * 64;
            if (rl < nr && !(M.is_long && M.is_long[rows[k]])) epi.finish(rows[k], acc[rl], pre[k]);
        }
    }
}

struct NoPre {};

struct EpiStore {
    using Pre = NoPre;
    double* out;
    const Scalars* gate;
    __device__ bool begin() const { return gate == nullptr || gate->status == kRunning; }
    __device__ Pre load(int) const { return Pre{}; }
    __device__ void finish(int r, double s, const Pre&) const { out[r] = s; }
};

// Primal step on column j of A (row j of A^T), s = (A~^T y)_j:
//   x_j <- clamp(x_j - tau (c~_j - s), x~lo_j, x~hi_j);  running mean of x since the restart.
struct EpiPrimal {
    struct Pre {
        double c, lo, hi, x, xa;
    };
    const Scalars* sc;
    int it;
    const double *c, *xl, *xu;
    double *x, *xa;
    double tau, wt;
    bool first;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it + 1;
        tau = sc->tau;
        first = (t == 1);
        wt = 1.0 / static_cast<double>(t);
        return true;
    }
    __device__ Pre load(int j) const { return Pre{c[j], xl[j], xu[j], x[j], xa[j]}; }
    __device__ void finish(int j, double s, const Pre& p) const {
        const double g = p.c - s;
        const double xn = clampd(p.x - tau * g, p.lo, p.hi);
        x[j] = xn;
        xa[j] = first ? xn : p.xa + wt * (xn - p.xa);
    }
};

// Dual step on row i, s = (A~ x+)_i, with the extrapolation 2 A~x+ - A~x:
//   v = y_i - sigma (2 s - (A~x)_i),  y_i <- max(v + sigma b~lo_i, 0) + min(v + sigma b~hi_i, 0)
// (the closed-form proximal step of the row-bound term; it keeps y_i >= 0 where b_hi = +inf
// and y_i <= 0 where b_lo = -inf), running mean of y, and A~x <- A~x+ for the next step.
struct EpiDual {
    struct Pre {
        double y, bl, bu, ya, ax;
    };
    const Scalars* sc;
    int it;
    const double *bl, *bu;
    double *y, *ya, *ax;
    double sigma, wt;
    bool first;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it + 1;
        sigma = sc->sigma;
        first = (t == 1);
        wt = 1.0 / static_cast<double>(t);
        return true;
    }
    __device__ Pre load(int i) const { return Pre{y[i], bl[i], bu[i], ya[i], ax[i]}; }
    __device__ void finish(int i, double s, const Pre& p) const {
        const double w = 2.0 * s - p.ax;
        const double v = p.y - sigma * w;
        const double lo = v + sigma * p.bl;
        const double hi = v + sigma * p.bu;
        const double yn = (lo > 0.0 ? lo : 0.0) + (hi < 0.0 ? hi : 0.0);
        y[i] = yn;
        ya[i] = first ? yn : p.ya + wt * (yn - p.ya);
        ax[i] = s;
    }
};


// FP32 storage form. The loop runs on the correction around the FP64 master (xh, yh):
// x = xh + dx, y = yh + dy, which is the same PDHG in exact arithmetic; the data it needs
// from the master (reduced cost, shifted bounds) are recomputed in FP64 at every restart.
// Primal step on column j: dx_j <- clamp(dx_j - tau (d_j - (A~^T dy)_j), x~lo_j - xh_j, x~hi_j - xh_j).
struct EpiPrimal32 {
    struct Pre {
        float d, lo, hi, x, xa;
    };
    const Scalars* sc;
    int it;
    const float *d, *lo, *hi;
    float *x, *xa;
    float tau, wt;
    bool first;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it + 1;
        tau = static_cast<float>(sc->tau);
        first = (t == 1);
        wt = static_cast<float>(1.0 / static_cast<double>(t));
        return true;
    }
    __device__ Pre load(int j) const { return Pre{d[j], lo[j], hi[j], x[j], xa[j]}; }
    __device__ void finish(int j, float s, const Pre& p) const {
        const float g = p.d - s;
        float xn = p.x - tau * g;
        if (xn < p.lo) xn = p.lo;
        if (xn > p.hi) xn = p.hi;
        x[j] = xn;
        xa[j] = first ? xn : p.xa + wt * (xn - p.xa);
    }
};

// Dual step on row i, s = (A~ dx+)_i: v = dy_i - sigma (2 s - (A~ dx)_i) and, with
// a = v + sigma (b~lo_i - (A~xh)_i), b = v + sigma (b~hi_i - (A~xh)_i), the proximal step of
// y = yh + dy is yh + a if yh + a > 0, yh + b if yh + b < 0, and 0 otherwise.
struct EpiDual32 {
    struct Pre {
        float y, rl, ru, yh, ya, ax;
    };
    const Scalars* sc;
    int it;
    const float *rl, *ru, *yh;
    float *y, *ya, *ax;
    float sigma, wt;
    bool first;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it + 1;
        sigma = static_cast<float>(sc->sigma);
        first = (t == 1);
        wt = static_cast<float>(1.0 / static_cast<double>(t));
        return true;
    }
    __device__ Pre load(int i) const { return Pre{y[i], rl[i], ru[i], yh[i], ya[i], ax[i]}; }
    __device__ void finish(int i, float s, const Pre& p) const {
        const float w = 2.0f * s - p.ax;
        const float v = p.y - sigma * w;
        const float a = v + sigma * p.rl;
        const float b = v + sigma * p.ru;
        float yn;
        if (a > -p.yh) yn = a;
        else if (b < -p.yh) yn = b;
        else yn = -p.yh;
        y[i] = yn;
        ya[i] = first ? yn : p.ya + wt * (yn - p.ya);
        ax[i] = s;
    }
};

// Residual restarts: the iteration whose iterate's residual z - T(z) the next evaluation uses,
// the last one before it (period end or max_iters).
__device__ inline bool residual_at_last(const Scalars* sc, int it) {
    long long last = sc->k + sc->eval_every;
    if (last > sc->max_iters) last = sc->max_iters;
    return sc->k + it + 1 == last;
}

// Reflected Halpern form (a reading of the newer cuPDLPx-family iteration): with T the PDHG map
// above and the anchor z0 of the restart cycle, z <- w ((1 + rho) T(z) - rho z) + (1 - w) z0,
// w = (t + 1) / (t + 2), t the iterations of the cycle before this one. The primal half on
// column j, s = (A~^T y)_j: x+ = clamp(x - tau (c~ - s)), x <- w ((1 + rho) x+ - rho x) +
// (1 - w) x0, and x+ is kept in xa for the dual half and the evaluations.
struct EpiPrimalH {
    struct Pre {
        double c, lo, hi, x, xan;
    };
    const Scalars* sc;
    int it;
    const double *c, *xl, *xu, *xan;
    double *x, *xa;
    double *rx_c, *rx_a;  // residual restarts: x - T(z)_x of the last iterate / of the anchor (or null)
    double tau, w, wa, r1, rho;
    bool rec_c, rec_a;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it;
        tau = sc->tau;
        w = static_cast<double>(t + 1) / static_cast<double>(t + 2);
        wa = 1.0 - w;
        r1 = 1.0 + rho;
        rec_c = rx_c != nullptr && residual_at_last(sc, it);
        rec_a = rx_a != nullptr && t == 0;
        return true;
    }
    __device__ Pre load(int j) const { return Pre{c[j], xl[j], xu[j], x[j], xan[j]}; }
    __device__ void finish(int j, double s, const Pre& p) const {
        const double g = p.c - s;
        const double xp = clampd(p.x - tau * g, p.lo, p.hi);
        x[j] = w * (r1 * xp - rho * p.x) + wa * p.xan;
        xa[j] = xp;
        if (rec_c) rx_c[j] = p.x - xp;
        if (rec_a) rx_a[j] = p.x - xp;
    }
};

// Dual half on row i, s = (A~ x+)_i: y+ = prox of y - sigma (2 s - (A~x)_i) as in EpiDual;
// y <- w ((1 + rho) y+ - rho y) + (1 - w) y0, ya <- y+, axa <- s, and A~x of the new Halpern
// iterate by linearity: ax <- w ((1 + rho) s - rho ax) + (1 - w) A~x0.
struct EpiDualH {
    struct Pre {
        double y, bl, bu, ax, yan, axan;
    };
    const Scalars* sc;
    int it;
    const double *bl, *bu, *yan, *axan;
    double *y, *ya, *ax, *axa;
    double *ry_c, *rax_c, *ry_a, *rax_a;  // residual restarts: y and A~x parts of z - T(z) (or null)
    double sigma, w, wa, r1, rho;
    bool rec_c, rec_a;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it;
        sigma = sc->sigma;
        w = static_cast<double>(t + 1) / static_cast<double>(t + 2);
        wa = 1.0 - w;
        r1 = 1.0 + rho;
        rec_c = ry_c != nullptr && residual_at_last(sc, it);
        rec_a = ry_a != nullptr && t == 0;
        return true;
    }
    __device__ Pre load(int i) const { return Pre{y[i], bl[i], bu[i], ax[i], yan[i], axan[i]}; }
    __device__ void finish(int i, double s, const Pre& p) const {
        const double w2 = 2.0 * s - p.ax;
        const double v = p.y - sigma * w2;
        const double lo = v + sigma * p.bl;
        const double hi = v + sigma * p.bu;
        const double yp = (lo > 0.0 ? lo : 0.0) + (hi < 0.0 ? hi : 0.0);
        y[i] = w * (r1 * yp - rho * p.y) + wa * p.yan;
        ya[i] = yp;
        axa[i] = s;
        ax[i] = w * (r1 * s - rho * p.ax) + wa * p.axan;
        if (rec_c) {
            ry_c[i] = p.y - yp;
            rax_c[i] = p.ax - s;
        }
        if (rec_a) {
            ry_a[i] = p.y - yp;
            rax_a[i] = p.ax - s;
        }
    }
};

// Halpern form in the FP32 storage form: the anchor is the FP64 master point, so in correction
// space it is zero and the update is dz <- w ((1 + rho) T(dz) - rho dz).
struct EpiPrimal32H {
    struct Pre {
        float d, lo, hi, x;
    };
    const Scalars* sc;
    int it;
    const float *d, *lo, *hi;
    float *x, *xa;
    double *rx_c, *rx_a;  // residual restarts (FP64 copies of the FP32 differences, or null)
    float tau, w, r1, rho;
    bool rec_c, rec_a;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it;
        tau = static_cast<float>(sc->tau);
        w = static_cast<float>(static_cast<double>(t + 1) / static_cast<double>(t + 2));
        r1 = 1.0f + rho;
        rec_c = rx_c != nullptr && residual_at_last(sc, it);
        rec_a = rx_a != nullptr && t == 0;
        return true;
    }
    __device__ Pre load(int j) const { return Pre{d[j], lo[j], hi[j], x[j]}; }
    __device__ void finish(int j, float s, const Pre& p) const {
        const float g = p.d - s;
        float xp = p.x - tau * g;
        if (xp < p.lo) xp = p.lo;
        if (xp > p.hi) xp = p.hi;
        x[j] = w * (r1 * xp - rho * p.x);
        xa[j] = xp;
        if (rec_c) rx_c[j] = static_cast<double>(p.x) - static_cast<double>(xp);
        if (rec_a) rx_a[j] = static_cast<double>(p.x) - static_cast<double>(xp);
    }
};

struct EpiDual32H {
    struct Pre {
        float y, rl, ru, yh, ax;
    };
    const Scalars* sc;
    int it;
    const float *rl, *ru, *yh;
    float *y, *ya, *ax;
    double *ry_c, *rax_c, *ry_a, *rax_a;  // residual restarts (FP64 copies, or null)
    float sigma, w, r1, rho;
    bool rec_c, rec_a;
    __device__ bool begin() {
        if (sc->status != kRunning || sc->k + it >= sc->max_iters) return false;
        const long long t = sc->t + it;
        sigma = static_cast<float>(sc->sigma);
        w = static_cast<float>(static_cast<double>(t + 1) / static_cast<double>(t + 2));
        r1 = 1.0f + rho;
        rec_c = ry_c != nullptr && residual_at_last(sc, it);
        rec_a = ry_a != nullptr && t == 0;
        return true;
    }
    __device__ Pre load(int i) const { return Pre{y[i], rl[i], ru[i], yh[i], ax[i]}; }
    __device__ void finish(int i, float s, const Pre& p) const {
        const float w2 = 2.0f * s - p.ax;
        const float v = p.y - sigma * w2;
        const float a = v + sigma * p.rl;
        const float b = v + sigma * p.ru;
        float yp;
        if (a > -p.yh) yp = a;
        else if (b < -p.yh) yp = b;
        else yp = -p.yh;
        y[i] = w * (r1 * yp - rho * p.y);
        ya[i] = yp;
        ax[i] = w * (r1 * s - rho * p.ax);
        if (rec_c) {
            ry_c[i] = static_cast<double>(p.y) - static_cast<double>(yp);
            rax_c[i] = static_cast<double>(p.ax) - static_cast<double>(s);
        }
        if (rec_a) {
            ry_a[i] = static_cast<double>(p.y) - static_cast<double>(yp);
            rax_a[i] = static_cast<double>(p.ax) - static_cast<double>(s);
        }
    }
};

// Epilogues of the primal and dual halves for a solve's form and precision.
__host__ __device__ inline EpiPrimal epi_primal(const DevLP& P, const Scalars* sc, int it) {
    EpiPrimal e{};
    e.sc = sc;
    e.it = it;
    e.c = P.c;
    e.xl = P.xl;
    e.xu = P.xu;
    e.x = P.x;
    e.xa = P.xa;
    return e;
}
__host__ __device__ inline EpiDual epi_dual(const DevLP& P, const Scalars* sc, int it) {
    EpiDual e{};
    e.sc = sc;
    e.it = it;
    e.bl = P.bl;
    e.bu = P.bu;
    e.y = P.y;
    e.ya = P.ya;
    e.ax = P.ax;
    return e;
}
__host__ __device__ inline EpiPrimal32 epi_primal32(const DevLP& P, const Scalars* sc, int it) {
    EpiPrimal32 e{};
    e.sc = sc;
    e.it = it;
    e.d = P.d32;
    e.lo = P.lo32;
    e.hi = P.hi32;
    e.x = P.dx;
    e.xa = P.dxa;
    return e;
}
__host__ __device__ inline EpiDual32 epi_dual32(const DevLP& P, const Scalars* sc, int it) {
    EpiDual32 e{};
    e.sc = sc;
    e.it = it;
    e.rl = P.rl32;
    e.ru = P.ru32;
    e.yh = P.yh32;
    e.y = P.dy;
    e.ya = P.dya;
    e.ax = P.adx;
    return e;
}
__host__ __device__ inline EpiPrimalH epi_primal_h(const DevLP& P, const Scalars* sc, int it) {
    EpiPrimalH e{};
    e.sc = sc;
    e.it = it;
    e.c = P.c;
    e.xl = P.xl;
    e.xu = P.xu;
    e.xan = P.xan;
    e.x = P.x;
    e.xa = P.xa;
    e.rho = P.rho;
    e.rx_c = P.restart_metric == 1 ? P.fr_x : nullptr;
    e.rx_a = P.restart_metric == 1 ? P.fa_x : nullptr;
    return e;
}
__host__ __device__ inline EpiDualH epi_dual_h(const DevLP& P, const Scalars* sc, int it) {
    EpiDualH e{};
    e.sc = sc;
    e.it = it;
    e.bl = P.bl;
    e.bu = P.bu;
    e.yan = P.yan;
    e.axan = P.axan;
    e.y = P.y;
    e.ya = P.ya;
    e.ax = P.ax;
    e.axa = P.axa;
    e.rho = P.rho;
    if (P.restart_metric == 1) {
        e.ry_c = P.fr_y;
        e.rax_c = P.fr_ax;
        e.ry_a = P.fa_y;
        e.rax_a = P.fa_ax;
    }
    return e;
}
__host__ __device__ inline EpiPrimal32H epi_primal32_h(const DevLP& P, const Scalars* sc, int it) {
    EpiPrimal32H e{};
    e.sc = sc;
    e.it = it;
    e.d = P.d32;
    e.lo = P.lo32;
    e.hi = P.hi32;
    e.x = P.dx;
    e.xa = P.dxa;
    e.rho = static_cast<float>(P.rho);
    e.rx_c = P.restart_metric == 1 ? P.fr_x : nullptr;
    e.rx_a = P.restart_metric == 1 ? P.fa_x : nullptr;
    return e;
}
__host__ __device__ inline EpiDual32H epi_dual32_h(const DevLP& P, const Scalars* sc, int it) {
    EpiDual32H e{};
    e.sc = sc;
    e.it = it;
    e.rl = P.rl32;
    e.ru = P.ru32;
    e.yh = P.yh32;
    e.y = P.dy;
    e.ya = P.dya;
    e.ax = P.adx;
    e.rho = static_cast<float>(P.rho);
    if (P.restart_metric == 1) {
        e.ry_c = P.fr_y;
        e.rax_c = P.fr_ax;
        e.ry_a = P.fa_y;
        e.rax_a = P.fa_ax;
    }
    return e;
}

template <class T, class Epi>
void launch_tiles(const Csr& M, const T* xin, const Epi& epi, hipStream_t s) {
    if (M.ntiles <= 0) return;
    if (M.shape == 0)
        hipLaunchKernelGGL((spmv_tiles_kernel<T, Epi, tile_nnz_of(0)>), dim3(M.ntiles), dim3(kBlock), 0, s, M, xin, epi);
    else if (M.shape == 1)
        hipLaunchKernelGGL((spmv_tiles_kernel<T, Epi, tile_nnz_of(1)>), dim3(M.ntiles), dim3(kBlock), 0, s, M, xin, epi);
    else
        hipLaunchKernelGGL((spmv_tiles_kernel<T, Epi, tile_nnz_of(2)>), dim3(M.ntiles), dim3(kBlock), 0, s, M, xin, epi);
}

// One sparse product with its fused epilogue: one launch holding the panel-packed units and,
// after them, one workgroup per long row; or the row tiles when that layout is selected.
template <class T, class Epi>
void launch_spmv(const Mat& M, const T* xin, const Epi& epi, hipStream_t s) {
    if (M.layout == 1) {
        launch_tiles(M.csr, xin, epi, s);
        return;
    }
    Csr L = M.csr;
    L.rowlist = M.longrows;
    L.ntiles = M.nlong;
    const int pb = (M.pan.units + kPanelUnits - 1) / kPanelUnits;
    const int g = pb + M.nlong;
    const size_t lds = static_cast<size_t>(kPanelUnits) * (M.pan.max_rows > 0 ? M.pan.max_rows : 1) * sizeof(T);
    // Allow the largest accumulator block once per kernel instance (thread-safe static init).
    static const bool lds_attr = [] {
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&spmv_panel_kernel<T, Epi>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(kPanelUnits * kUnitRowCap * sizeof(T))) == hipSuccess;
    }();
    (void)lds_attr;
    if (g > 0)
        hipLaunchKernelGGL((spmv_panel_kernel<T, Epi>), dim3(g), dim3(kBlock), lds, s, M.pan, L, pb, xin, epi);
}

// ------------------------------------------------------------------- setup kernels

__global__ void fill_kernel(double* p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Row statistic of |A~| (max, or the sum in CSR order) turned into a power-of-two factor.
__global__ void scale_rowstat_kernel(int rows, const int* rp, const double* v, int use_sum, double* f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const double a = fabs(v[e]);
        if (use_sum) s += a;
        else if (a > s) s = a;
    }
    f[i] = pow2_rsqrt(s);
}

// Column statistic through the transpose permutation (entries of a column in ascending row).
__global__ void scale_colstat_kernel(int cols, const int* rpT, const int* perm, const double* v, int use_sum,
                                     double* f) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    double s = 0.0;
    for (int p = rpT[j]; p < rpT[j + 1]; ++p) {
        const double a = fabs(v[perm[p]]);
        if (use_sum) s += a;
        else if (a > s) s = a;
    }
    f[j] = pow2_rsqrt(s);
}

__global__ void scale_apply_rows_kernel(int rows, const int* rp, const int* ci, double* v, const double* rf,
                                        const double* cf, double* R) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const double r = rf[i];
    for (int e = rp[i]; e < rp[i + 1]; ++e) v[e] = v[e] * r * cf[ci[e]];
    R[i] *= r;
}

__global__ void scale_apply_cols_kernel(int cols, const double* cf, double* C) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    C[j] *= cf[j];
}

__global__ void gather_kernel(const int* perm, const double* src, double* dst, long long nnz) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nnz;
         p += (long long)gridDim.x * blockDim.x)
        dst[p] = src[perm[p]];
}

// Scaled data: c~ = C c, b~ = R b, x~bounds = x bounds / C, inverse factors, warm start.
__global__ void prepare_kernel(int m, int n, double* c, double* bl, double* bu, double* xl, double* xu,
                               const double* R, const double* C, double* Ri, double* Ci, double* x0, double* y0) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) {
        const double cc = C[g], ci = 1.0 / cc;
        Ci[g] = ci;
        c[g] = c[g] * cc;
        xl[g] = xl[g] * ci;
        xu[g] = xu[g] * ci;
        if (x0) x0[g] = x0[g] * ci;
    }
    if (g < m) {
        const double r = R[g], ri = 1.0 / r;
        Ri[g] = ri;
        bl[g] = bl[g] * r;
        bu[g] = bu[g] * r;
        if (y0) y0[g] = y0[g] * ri;
    }
}

// Partial sums of ||c||^2, ||q||^2 (original data, recovered exactly from the scaled data)
// and ||c~||^2, ||q~||^2 (scaled data). q_i = max finite |row bound|.
__global__ __launch_bounds__(kBlock) void norms_kernel(DevLP P) {
    __shared__ double red[kBlock / 64];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P.n; j += stride) {
        const double cs = P.c[j], co = cs * P.Ci[j];
        a0 += co * co;
        a2 += cs * cs;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.m; i += stride) {
        const double bl = P.bl[i], bu = P.bu[i], ri = P.Ri[i];
        double qs = 0.0;
        if (finite_d(bl) && fabs(bl) > qs) qs = fabs(bl);
        if (finite_d(bu) && fabs(bu) > qs) qs = fabs(bu);
        double qo = 0.0;
        const double blo = bl * ri, buo = bu * ri;
        if (finite_d(blo) && fabs(blo) > qo) qo = fabs(blo);
        if (finite_d(buo) && fabs(buo) > qo) qo = fabs(buo);
        a1 += qo * qo;
        a3 += qs * qs;
    }
    const double s0 = block_sum(a0, red), s1 = block_sum(a1, red), s2 = block_sum(a2, red), s3 = block_sum(a3, red);
    if (threadIdx.x == 0) {
        double* out = P.partials + blockIdx.x * 4;
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
        out[3] = s3;
    }
}

// Power iteration pieces. Start vector v_k = U[-1/2, 1/2)(seed, k).
__global__ void power_init_kernel(int n, unsigned long long seed, double* v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = splitmix_centered(seed, (unsigned long long)k);
}

// Partial sums of sum(a^2) over [0, na) and sum(b^2) over [0, nb) -> partials[blk*2 + {0,1}].
__global__ __launch_bounds__(kBlock) void sumsq2_kernel(const double* a, int na, const double* b, int nb,
                                                        double* partials) {
    __shared__ double red[kBlock / 64];
    double sa = 0.0, sb = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) sa += a[i] * a[i];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) sb += b[i] * b[i];
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 2] = sa;
        partials[blockIdx.x * 2 + 1] = sb;
    }
}

// dst = src / sqrt(sum of partial slot `slot`) when that norm is positive (every block
// forms the same total in the same order). Optionally records sqrt(slot 0) as sigma_max.
__global__ __launch_bounds__(kBlock) void normalize_kernel(const double* src, double* dst, int n,
                                                           const double* partials, int nparts, int slot,
                                                           Scalars* sc) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) s += partials[b * 2 + slot];
    s = block_sum_all(s, red);
    double s0 = 0.0;
    if (sc) {
        for (int b = threadIdx.x; b < nparts; b += kBlock) s0 += partials[b * 2];
        s0 = block_sum_all(s0, red);
    }
    const double nrm = sqrt(s);
    if (sc && blockIdx.x == 0 && threadIdx.x == 0) {
        sc->sigma_prev = sc->sigma_max;
        sc->sigma_max = sqrt(s0);
    }
    if (!(nrm > 0.0)) return;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) dst[k] = src[k] / nrm;
}

__global__ __launch_bounds__(kBlock) void finalize_setup_kernel(DevLP P, int nparts, double eta_override,
                                                                double omega_override, double c0) {
    __shared__ double red[kBlock / 64];
    double s[4];
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kBlock) v += P.partials[b * 4 + q];
        s[q] = block_sum(v, red);
    }
    if (threadIdx.x != 0) return;
    Scalars* sc = P.sc;
    sc->c0 = c0;
    sc->cnorm = sqrt(s[0]);
    sc->qnorm = sqrt(s[1]);
    const double cs = sqrt(s[2]), qs = sqrt(s[3]);
    double eta = eta_override;
    if (!(eta > 0.0)) eta = sc->sigma_max > 0.0 ? 0.998 / sc->sigma_max : 1.0;
    else sc->sigma_max = 0.0;
    double omega = omega_override;
    if (!(omega > 0.0)) omega = (cs > 1e-10 && qs > 1e-10) ? cs / qs : 1.0;
    sc->eta = eta;
    sc->omega0 = omega;
}

// ------------------------------------------------------------------- solve kernels

__global__ void reset_kernel(Scalars* sc, double eps_rel, double eps_infeas, long long max_iters, int eval_every,
                             int restarts_on, long long trace_cap, int term_mode, double omega_override) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc->omega = omega_override > 0.0 ? omega_override : sc->omega0;
    sc->term_mode = term_mode;
    sc->deadline = 0;  // lp_solve checks its time limit on the host between evaluation periods
    sc->tau = sc->eta / sc->omega;
    sc->sigma = sc->eta * sc->omega;
    sc->eps_rel = eps_rel;
    sc->eps_infeas = eps_infeas;
    sc->ray_scale = 0.0;
    sc->ray_src = 0;
    sc->max_iters = max_iters;
    sc->eval_every = eval_every;
    sc->restarts_on = restarts_on;
    sc->trace_cap = trace_cap;
    sc->k = 0;
    sc->t = 0;
    sc->restarts = 0;
    sc->n_trace = 0;
    sc->status = kRunning;
    sc->out_avg = 0;
    sc->last_restart = 0;
    sc->kkt_prev = __builtin_inf();
    sc->pid_int = 0.0;
    sc->pid_prev = 0.0;
}

__device__ inline void init_state_at(const DevLP& P, int g, const double* x0, const double* y0) {
    if (g < P.n) {
        const double v = clampd(x0 ? x0[g] : 0.0, P.xl[g], P.xu[g]);
        P.x[g] = v;
        P.xa[g] = v;
        P.xan[g] = v;
    }
    if (g < P.m) {
        const double v = y0 ? y0[g] : 0.0;
        P.y[g] = v;
        P.ya[g] = v;
        P.yan[g] = v;
    }
}

__global__ void init_state_kernel(DevLP P, const double* x0, const double* y0) {
    init_state_at(P, blockIdx.x * blockDim.x + threadIdx.x, x0, y0);
}

// Residual and objective terms of one row for a candidate (A~x~, y~); see the evaluation
// kernel for the definitions. acc: 0 rp2, 1 rps2, 2 rd2, 3 rds2, 4 pobj, 5 dobj, 6 dx2, 7 dy2.
__device__ inline void row_terms(const DevLP& P, int i, const double* ax, const double* y, double* acc) {
    const double bl = P.bl[i], bu = P.bu[i], R = P.R[i], Ri = P.Ri[i];
    const double v = ax[i];
    const double rs = v - clampd(v, bl, bu);
    const double ro = rs * Ri;
    acc[1] += rs * rs;
    acc[0] += ro * ro;
    const double yv = y[i];
    const double yo = yv * R;
    const double blo = bl * Ri, buo = bu * Ri;
    if (yo > 0.0 && finite_d(blo)) acc[5] += blo * yo;
    if (yo < 0.0 && finite_d(buo)) acc[5] += buo * yo;
    double vs = 0.0;
    if (bl == -__builtin_inf() && yv > 0.0) vs += yv;
    if (bu == __builtin_inf() && yv < 0.0) vs -= yv;
    const double vo = vs * R;
    acc[3] += vs * vs;
    acc[2] += vo * vo;
    const double dy = yv - P.yan[i];
    acc[7] += dy * dy;
}

__device__ inline void col_terms(const DevLP& P, int j, const double* x, const double* aty, double* acc) {
    const double cs = P.c[j], lo = P.xl[j], hi = P.xu[j], Cj = P.C[j], Ci = P.Ci[j];
    const double ls = cs - aty[j];
    const bool flo = finite_d(lo), fhi = finite_d(hi);
    double zs = ls;
    if (!flo && !fhi) zs = 0.0;
    else if (flo && !fhi) zs = ls > 0.0 ? ls : 0.0;
    else if (!flo && fhi) zs = ls < 0.0 ? ls : 0.0;
    const double rds = ls - zs;
    const double zo = zs * Ci;
    const double rdo = rds * Ci;
    acc[3] += rds * rds;
    acc[2] += rdo * rdo;
    const double xv = x[j];
    const double xo = xv * Cj;
    acc[4] += (cs * Ci) * xo;
    if (zo > 0.0) acc[5] += (lo * Cj) * zo;
    if (zo < 0.0) acc[5] += (hi * Cj) * zo;
    const double dx = xv - P.xan[j];
    acc[6] += dx * dx;
}

// Candidate rays for the infeasibility certificates: the difference of two points (y~, A~x~)
// minus (y~b, A~x~b) on the original scale: the displacement of the evaluated point since the
// previous evaluation (base: the saved previous point), or the averaged point minus the
// restart anchor. acc: 0 rd2, 1 D, 2 rp2, 3 G, where
//   dual ray y^ = R (y~ - y~b), lambda = -C^-1 (A~^T y~ - A~^T y~b), z^ = lambda projected on
//   the sign cone of eq. 2: rd2 = ||lambda - z^||^2 + ||sign violations of y^||^2,
//   D = sum_i (b_lo y^+ - b_hi y^-) + sum_k (x_lo z^+ - x_hi z^-) over finite bounds;
//   primal ray x^ = C (x~ - x~b), A x^ = R^-1 (A~x~ - A~x~b): rp2 = squared parts of A x^ and
//   x^ outside the recession cones of the row and variable bounds, G = -c^T x^.
__device__ inline void row_ray_terms(const DevLP& P, int i, const double* y, const double* ax, const double* yb,
                                     const double* axb, double* acc) {
    const double dy = (y[i] - yb[i]) * P.R[i];
    const double v = (ax[i] - axb[i]) * P.Ri[i];
    const double bl = P.bl[i], bu = P.bu[i], Ri = P.Ri[i];
    const bool flo = finite_d(bl), fhi = finite_d(bu);
    if (dy > 0.0 && flo) acc[1] += (bl * Ri) * dy;
    if (dy < 0.0 && fhi) acc[1] += (bu * Ri) * dy;
    double vs = 0.0;
    if (!flo && dy > 0.0) vs += dy;
    if (!fhi && dy < 0.0) vs -= dy;
    acc[0] += vs * vs;
    double w = 0.0;
    if (flo && fhi) w = v;
    else if (flo) w = v < 0.0 ? v : 0.0;
    else if (fhi) w = v > 0.0 ? v : 0.0;
    acc[2] += w * w;
}

__device__ inline void col_ray_terms(const DevLP& P, int j, const double* x, const double* aty, const double* xb,
                                     const double* atyb, double* acc) {
    const double lam = -(aty[j] - atyb[j]) * P.Ci[j];
    const double lo = P.xl[j], hi = P.xu[j], Cj = P.C[j];
    const bool flo = finite_d(lo), fhi = finite_d(hi);
    double zs = lam;
    if (!flo && !fhi) zs = 0.0;
    else if (flo && !fhi) zs = lam > 0.0 ? lam : 0.0;
    else if (!flo && fhi) zs = lam < 0.0 ? lam : 0.0;
    const double r = lam - zs;
    acc[0] += r * r;
    if (zs > 0.0) acc[1] += (lo * Cj) * zs;
    if (zs < 0.0) acc[1] += (hi * Cj) * zs;
    const double xh = (x[j] - xb[j]) * Cj;
    acc[3] -= (P.c[j] * P.Ci[j]) * xh;
    double w = 0.0;
    if (flo && fhi) w = xh;
    else if (flo) w = xh < 0.0 ? xh : 0.0;
    else if (fhi) w = xh > 0.0 ? xh : 0.0;
    acc[2] += w * w;
}

// Per-thread sums of one evaluation over rows and columns start, start + stride, ...
// Averaged form, mode 0: the current iterate (slots 0..7), the running average (8..15), the
// displacement ray of the current iterate (16..19) and the anchored ray of the average
// (20..23). Halpern form, mode 0: the PDHG output (xa, ya) in slots 0..7 and its two rays.
// Modes 1 and 2: the current iterate only.
__device__ inline void eval_terms(const DevLP& P, int mode, int start, int stride, double* acc) {
    const bool both = mode == 0 && !P.method;
    const bool cand = (mode == 0 || mode == 2) && P.method;
    const bool rays = mode == 0 && P.xp != nullptr;
    const double* ex = cand ? P.xa : P.x;
    const double* ey = cand ? P.ya : P.y;
    const double* eax = cand ? P.axa : P.ax;
    const double* eaty = cand ? P.atya : P.aty;
    for (int i = start; i < P.m; i += stride) {
        row_terms(P, i, eax, ey, acc);
        if (both) row_terms(P, i, P.axa, P.ya, acc + kNQ);
        if (rays) {
            row_ray_terms(P, i, ey, eax, P.yp, P.axp, acc + 2 * kNQ);
            row_ray_terms(P, i, P.ya, P.axa, P.yan, P.axan, acc + 2 * kNQ + 4);
        }
    }
    for (int j = start; j < P.n; j += stride) {
        col_terms(P, j, ex, eaty, acc);
        if (both) col_terms(P, j, P.xa, P.atya, acc + kNQ);
        if (rays) {
            col_ray_terms(P, j, ex, eaty, P.xp, P.atyp, acc + 2 * kNQ);
            col_ray_terms(P, j, P.xa, P.atya, P.xan, P.atyan, acc + 2 * kNQ + 4);
        }
    }
}

// Residual restarts (Halpern form, restart_metric 1): whether they are on, and their sums over
// rows and columns start, start + stride, ...: ||dx||^2, <dy, A~dx>, ||dy||^2 of the last
// iterate's z - T(z) (0..2) and of the anchor's (3..5).
__device__ inline bool residual_restarts(const DevLP& P) { return P.method != 0 && P.restart_metric == 1; }

__device__ inline void residual_terms(const DevLP& P, int start, int stride, double* acc) {
    for (int i = start; i < P.m; i += stride) {
        const double dc = P.fr_y[i], da = P.fa_y[i];
        acc[1] += dc * P.fr_ax[i];
        acc[2] += dc * dc;
        acc[4] += da * P.fa_ax[i];
        acc[5] += da * da;
    }
    for (int j = start; j < P.n; j += stride) {
        const double dc = P.fr_x[j], da = P.fa_x[j];
        acc[0] += dc * dc;
        acc[3] += da * da;
    }
}

// Partial sums of the evaluation quantities (see eval_terms) of one block. mode 1 (initial point) and
// mode 2 (final point after a stop) evaluate the current iterate only; mode 2 runs whatever
// the status.
__device__ void kkt_partials_body(const DevLP& P, int mode, int blk, int nblk) {
    __shared__ double red[kBlock / 64][kNT];
    if (mode != 2 && P.sc->status != kRunning) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    {
        constexpr int kMain = kNT - kNF;
        double acc[kMain];
#pragma unroll
        for (int q = 0; q < kMain; ++q) acc[q] = 0.0;
        eval_terms(P, mode, blk * kBlock + threadIdx.x, nblk * kBlock, acc);
#pragma unroll
        for (int q = 0; q < kMain; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red[w][q] = v;
        }
    }
    {
        double acc[kNF];
#pragma unroll
        for (int q = 0; q < kNF; ++q) acc[q] = 0.0;
        if (mode == 0 && residual_restarts(P)) residual_terms(P, blk * kBlock + threadIdx.x, nblk * kBlock, acc);
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red[w][kNT - kNF + q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kNT) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += red[k][threadIdx.x];
        P.partials[blk * kNT + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void kkt_partials_kernel(DevLP P, int mode) {
    kkt_partials_body(P, mode, static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
}

struct Kkt {
    double rp2, rps2, rd2, rds2, pobj, dobj, dx2, dy2;
    double rel_p, rel_d, rel_gap, erel;
};

__device__ inline Kkt make_kkt(const double* q, const Scalars* sc) {
    Kkt K;
    K.rp2 = q[0];
    K.rps2 = q[1];
    K.rd2 = q[2];
    K.rds2 = q[3];
    K.pobj = q[4];
    K.dobj = q[5];
    K.dx2 = q[6];
    K.dy2 = q[7];
    const double p = K.pobj + sc->c0, d = K.dobj + sc->c0;
    K.rel_p = sqrt(K.rp2) / (1.0 + sc->qnorm);
    K.rel_d = sqrt(K.rd2) / (1.0 + sc->cnorm);
    K.rel_gap = fabs(p - d) / (1.0 + fabs(p) + fabs(d));
    double e = K.rel_p;
    if (K.rel_d > e) e = K.rel_d;
    if (K.rel_gap > e) e = K.rel_gap;
    if (isnan(K.rel_p) || isnan(K.rel_d) || isnan(K.rel_gap)) e = __builtin_nan("");
    K.erel = e;
    return K;
}

// The quantity termination compares with eps_rel: E_rel, or (polishing) one residual alone.
__device__ inline double term_value(const Kkt& K, int mode) {
    if (isnan(K.erel)) return K.erel;
    return mode == 1 ? K.rel_p : mode == 2 ? K.rel_d : K.erel;
}

// KKT error in the primal-weighted norm on the scaled problem (the restart metric).
__device__ inline double kkt_w(double rps2, double rds2, double gap, double omega) {
    const double w2 = omega * omega;
    return sqrt(w2 * rps2 + rds2 / w2 + gap * gap);
}

__device__ inline void set_output(Scalars* sc, const Kkt& K, int avg) {
    sc->out_avg = avg;
    sc->out_pobj = K.pobj + sc->c0;
    sc->out_dobj = K.dobj + sc->c0;
    sc->out_rel_p = K.rel_p;
    sc->out_rel_d = K.rel_d;
    sc->out_rel_gap = K.rel_gap;
    sc->out_erel = K.erel;
}

// Evaluation and decision, one workgroup:
//  E_rel = max(||r_p||/(1+||q||), ||r_d||/(1+||c||), |p-d|/(1+|p|+|d|)) on the original data;
//  termination when E_rel(current) <= eps (then the average), or at max_iters the better one;
//  restart candidate = average if its KKT_w is strictly smaller; restart on
//  (1) KKT_c <= 0.2 KKT_anchor, (2) KKT_c <= 0.8 KKT_anchor and KKT_c > KKT_prev,
//  (3) t >= 0.36 k; on restart, when dx, dy > 1e-10, omega <- sqrt(omega dy / dx),
//  omega_steps times, or the PID rule (log omega -= kp e + ki I + kd (e - e_prev) with
//  e = log(omega dx / dy), I the sum of the errors so far).
// Thread-0 part of the evaluation: tot holds the summed KKT quantities of the current
// iterate (0..7) and, in mode 0, of the average (8..15).
__device__ void decide_logic(const DevLP& P, Scalars* sc, const double* tot, int mode) {
    const Kkt cur = make_kkt(tot, sc);
    if (mode == 2) {  // statistics of the returned point after a host-side stop
        set_output(sc, cur, P.method ? 1 : 0);
        return;
    }
    if (mode == 1) {
        sc->anc_rps2 = cur.rps2;
        sc->anc_rds2 = cur.rds2;
        sc->anc_gap = cur.pobj - cur.dobj;
        sc->kkt_anchor = kkt_w(cur.rps2, cur.rds2, cur.pobj - cur.dobj, sc->omega);
        sc->kkt_prev = __builtin_inf();
        if (isnan(cur.erel)) sc->status = 3;
        else if (term_value(cur, sc->term_mode) <= sc->eps_rel) sc->status = 0;
        else if (sc->max_iters <= 0) sc->status = 1;
        if (sc->status != kRunning) {
            set_output(sc, cur, 0);
            sc->done_clock = static_cast<long long>(wall_clock64());
        }
        return;
    }
    // Halpern form: the PDHG output is the only candidate (slots 0..7), returned as "average"
    const bool halpern = P.method != 0;
    const Kkt avg = halpern ? cur : make_kkt(tot + kNQ, sc);
    long long ex = sc->max_iters - sc->k;
    if (ex > sc->eval_every) ex = sc->eval_every;
    const long long k = sc->k + ex;
    long long t = sc->t + ex;
    const double omega = sc->omega;
    double kc = kkt_w(cur.rps2, cur.rds2, cur.pobj - cur.dobj, omega);
    double ka = kkt_w(avg.rps2, avg.rds2, avg.pobj - avg.dobj, omega);
    if (residual_restarts(P)) {
        // the restart tests compare fixed-point residuals in the norm of the PDHG map:
        // r^2 = omega ||dx||^2 + 2 eta <dy, A~dx> + ||dy||^2 / omega
        const double* f = tot + 2 * kNQ + kNR;
        const double rc2 = omega * f[0] + 2.0 * sc->eta * f[1] + f[2] / omega;
        const double ra2 = omega * f[3] + 2.0 * sc->eta * f[4] + f[5] / omega;
        kc = ka = sqrt(rc2 > 0.0 ? rc2 : 0.0);
        sc->kkt_anchor = sqrt(ra2 > 0.0 ? ra2 : 0.0);
    }
    double rec[kTraceW];
    for (int f = 0; f < kTraceW; ++f) rec[f] = 0.0;
    rec[0] = (double)k;
    rec[1] = (double)t;
    rec[2] = kc;
    rec[3] = ka;
    rec[4] = cur.erel;
    rec[5] = avg.erel;
    rec[9] = sc->kkt_anchor;
    rec[10] = sc->kkt_prev;
    int status = kRunning, out_avg = 0;
    if (isnan(cur.erel) || isnan(avg.erel)) {
        status = 3;
    } else if (term_value(cur, sc->term_mode) <= sc->eps_rel) {
        status = 0;
        out_avg = halpern;
    } else if (term_value(avg, sc->term_mode) <= sc->eps_rel) {
        status = 0;
        out_avg = 1;
    } else {
        if (sc->eps_infeas > 0.0 && P.xp != nullptr) {
            // the displacement ray first, then the anchored ray of the average
            for (int src = 1; src <= 2 && status == kRunning; ++src) {
                const double* ray = tot + 2 * kNQ + 4 * (src - 1);  // rd2, D, rp2, G
                if (ray[1] > 0.0 && sqrt(ray[0]) <= sc->eps_infeas * ray[1]) {
                    status = 4;
                    sc->ray_scale = 1.0 / ray[1];
                } else if (ray[3] > 0.0 && sqrt(ray[2]) <= sc->eps_infeas * ray[3]) {
                    status = 5;
                    sc->ray_scale = 1.0 / ray[3];
                }
                if (status != kRunning) sc->ray_src = src;
            }
        }
        if (status != kRunning) out_avg = halpern;
        if (status == kRunning && k >= sc->max_iters) {
            status = 1;
            out_avg = halpern ? 1 : term_value(avg, sc->term_mode) < term_value(cur, sc->term_mode);
        }
        // time limit: the evaluated point is returned, as after a stop between evaluations
        if (status == kRunning && sc->deadline > 0 && static_cast<long long>(wall_clock64()) >= sc->deadline) {
            status = 2;
            out_avg = halpern;
        }
    }
    sc->k = k;
    if (status != kRunning) {
        sc->t = t;
        sc->status = status;
        sc->done_clock = static_cast<long long>(wall_clock64());
        sc->last_restart = 0;
        set_output(sc, out_avg ? avg : cur, out_avg);
        rec[6] = out_avg;
        rec[8] = omega;
        rec[11] = __builtin_inf();
    } else {
        const int use_avg = halpern ? 1 : ka < kc;
        const double kcand = use_avg ? ka : kc;
        const double anc = sc->kkt_anchor, prev = sc->kkt_prev;
        double margin = fabs(ka - kc) / fmax(fmax(ka, kc), 1e-300);
        int why = 0;
        if (sc->restarts_on) {
            const double mi = fabs(kcand - 0.2 * anc) / fmax(anc, 1e-300);
            const double mii = fabs(kcand - 0.8 * anc) / fmax(anc, 1e-300);
            const double mprev = finite_d(prev) ? fabs(kcand - prev) / fmax(prev, 1e-300) : __builtin_inf();
            const double miii = fabs((double)t - 0.36 * (double)k) / (double)k;
            margin = fmin(margin, fmin(fmin(mi, mii), fmin(mprev, miii)));
            if (kcand <= 0.2 * anc) why = 1;
            else if (kcand <= 0.8 * anc && kcand > prev) why = 2;
            else if ((double)t >= 0.36 * (double)k) why = 3;
        }
        rec[6] = use_avg;
        rec[7] = why;
        rec[11] = margin;
        double om = omega;
        if (why) {
            const Kkt& cd = use_avg ? avg : cur;
            const double dx = sqrt(cd.dx2), dy = sqrt(cd.dy2);
            if (dx > 1e-10 && dy > 1e-10) {
                if (P.pw_rule == 2) {
                    // PID controller on the log imbalance of the weighted distances
                    const double e = log((om * dx) / dy);
                    sc->pid_int += e;
                    const double u = P.kp * e + P.ki * sc->pid_int + P.kd * (e - sc->pid_prev);
                    sc->pid_prev = e;
                    om = om * exp(-u);
                } else {
                    for (int q = 0; q < P.omega_steps; ++q) om = sqrt((om * dy) / dx);
                }
            }
            sc->omega = om;
            sc->tau = sc->eta / om;
            sc->sigma = sc->eta * om;
            sc->anc_rps2 = cd.rps2;
            sc->anc_rds2 = cd.rds2;
            sc->anc_gap = cd.pobj - cd.dobj;
            sc->kkt_anchor = kkt_w(cd.rps2, cd.rds2, cd.pobj - cd.dobj, om);
            sc->kkt_prev = __builtin_inf();
            sc->last_restart = use_avg ? 2 : 1;
            sc->restarts += 1;
            t = 0;
        } else {
            sc->kkt_prev = kcand;
            sc->last_restart = 0;
        }
        sc->t = t;
        rec[8] = om;
        // keep the latest statistics of both candidates for a host-side stop
        set_output(sc, (avg.erel < cur.erel) ? avg : cur, avg.erel < cur.erel);
    }
    const long long nt = sc->n_trace;
    if (P.trace && nt < sc->trace_cap) {
        for (int f = 0; f < kTraceW; ++f) P.trace[nt * kTraceW + f] = rec[f];
    }
    sc->n_trace = nt + 1;
}

__device__ void decide_body(const DevLP& P, int mode) {
    __shared__ double red[kBlock / 64];
    __shared__ double tot[kNT];
    Scalars* sc = P.sc;
    if (mode != 2 && sc->status != kRunning) return;
    const int nq = (mode == 0) ? (residual_restarts(P) ? kNT : kNT - kNF) : kNQ;
    for (int q = 0; q < nq; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < P.nred; b += kBlock) v += P.partials[b * kNT + q];
        v = block_sum(v, red);
        if (threadIdx.x == 0) tot[q] = v;
    }
    if (threadIdx.x != 0) return;
    decide_logic(P, P.sc, tot, mode);
}

__global__ __launch_bounds__(kBlock) void decide_kernel(DevLP P, int mode) { decide_body(P, mode); }

// Restart: the candidate becomes the iterate, the anchor and the average.
__device__ inline void apply_restart_at(const DevLP& P, int lr, int g) {
    if (g < P.n) {
        double v;
        if (lr == 2) {
            v = P.xa[g];
            P.x[g] = v;
        } else {
            v = P.x[g];
            P.xa[g] = v;
        }
        P.xan[g] = v;
        P.atyan[g] = lr == 2 ? P.atya[g] : P.aty[g];
    }
    if (g < P.m) {
        double v;
        if (lr == 2) {
            v = P.ya[g];
            P.y[g] = v;
            P.ax[g] = P.axa[g];
            P.axan[g] = P.axa[g];
        } else {
            v = P.y[g];
            P.ya[g] = v;
            P.axan[g] = P.ax[g];
        }
        P.yan[g] = v;
    }
}

// The point the next evaluation's rays start from: the current iterate, or the average when
// this evaluation restarts there (lr == 2).
// In the Halpern form the evaluated point is always the PDHG output; after the initial
// evaluation (init) it equals the start, whose products A~x, A~^T y also seed axa, atya and
// the anchor's A~x.
__device__ inline void save_prev_at(const DevLP& P, int lr, bool init, int g) {
    if (init) {  // the start is the first anchor
        if (g < P.n) {
            P.atyan[g] = P.aty[g];
            if (P.method) P.atya[g] = P.aty[g];
        }
        if (g < P.m) {
            P.axan[g] = P.ax[g];
            if (P.method) P.axa[g] = P.ax[g];
        }
    }
    if (P.xp == nullptr) return;
    const bool avg = lr == 2 || (P.method && !init);
    if (g < P.n) {
        P.xp[g] = avg ? P.xa[g] : P.x[g];
        P.atyp[g] = avg ? P.atya[g] : P.aty[g];
    }
    if (g < P.m) {
        P.yp[g] = avg ? P.ya[g] : P.y[g];
        P.axp[g] = avg ? P.axa[g] : P.ax[g];
    }
}

__global__ void save_prev_kernel(DevLP P, int init) {
    if (P.sc->status != kRunning) return;
    save_prev_at(P, init ? 0 : P.sc->last_restart, init != 0, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void apply_restart_kernel(DevLP P) {
    const int lr = P.sc->last_restart;
    if (lr == 0) return;
    apply_restart_at(P, lr, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void stop_kernel(Scalars* sc, int status) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && sc->status == kRunning) {
        sc->status = status;
        sc->done_clock = static_cast<long long>(wall_clock64());
        sc->out_avg = 0;
        sc->last_restart = 0;
    }
}

// Returned point on the original scale: x = C x~, y = R y~, z = projected reduced cost.
// With a certificate (status 4: primal infeasible, 5: dual infeasible) the ray replaces the
// dual pair (y, z) or the primal x, scaled by `scale` so that its ray objective is 1.
__device__ inline void extract_at(const DevLP& P, int avg, int status, double scale, int src, int g) {
    const double* xs = avg ? P.xa : P.x;
    const double* ys = avg ? P.ya : P.y;
    const double* at = avg ? P.atya : P.aty;
    const bool dual_ray = status == 4 && P.xp != nullptr;
    const bool primal_ray = status == 5 && P.xp != nullptr;
    // a ray is the evaluated point ((x, y), or in the Halpern form the PDHG output) minus the
    // previous evaluation's point, or (src 2) the averaged point minus the anchor
    const bool anch = src == 2;
    const double* rx = (P.method || anch) ? P.xa : P.x;
    const double* ry = (P.method || anch) ? P.ya : P.y;
    const double* raty = (P.method || anch) ? P.atya : P.aty;
    const double* bx = anch ? P.xan : P.xp;
    const double* by = anch ? P.yan : P.yp;
    const double* baty = anch ? P.atyan : P.atyp;
    if (g < P.n) {
        P.out_x[g] = primal_ray ? ((rx[g] - bx[g]) * P.C[g]) * scale : xs[g] * P.C[g];
        const bool flo = finite_d(P.xl[g]), fhi = finite_d(P.xu[g]);
        if (dual_ray) {
            const double lam = -(raty[g] - baty[g]) * P.Ci[g];
            double zs = lam;
            if (!flo && !fhi) zs = 0.0;
            else if (flo && !fhi) zs = lam > 0.0 ? lam : 0.0;
            else if (!flo && fhi) zs = lam < 0.0 ? lam : 0.0;
            P.out_z[g] = zs * scale;
        } else {
            const double ls = P.c[g] - at[g];
            double zs = ls;
            if (!flo && !fhi) zs = 0.0;
            else if (flo && !fhi) zs = ls > 0.0 ? ls : 0.0;
            else if (!flo && fhi) zs = ls < 0.0 ? ls : 0.0;
            P.out_z[g] = zs * P.Ci[g];
        }
    }
    if (g < P.m) P.out_y[g] = dual_ray ? ((ry[g] - by[g]) * P.R[g]) * scale : ys[g] * P.R[g];
}

__global__ void extract_kernel(DevLP P) {
    extract_at(P, P.sc->out_avg, P.sc->status, P.sc->ray_scale, P.sc->ray_src, blockIdx.x * blockDim.x + threadIdx.x);
}


// FP64 values of the current and average iterate of the FP32 form: x = xh + dx, ...
__device__ inline void materialize_at(const DevLP& P, int g) {
    if (g < P.n) {
        const double h = P.xh[g];
        P.x[g] = h + static_cast<double>(P.dx[g]);
        P.xa[g] = h + static_cast<double>(P.dxa[g]);
    }
    if (g < P.m) {
        const double h = P.yh[g];
        P.y[g] = h + static_cast<double>(P.dy[g]);
        P.ya[g] = h + static_cast<double>(P.dya[g]);
    }
}

__global__ void materialize_kernel(DevLP P) { materialize_at(P, blockIdx.x * blockDim.x + threadIdx.x); }

// Refinement (FP32 form): after the initial evaluation (mode 1) or a restart decided by
// the evaluation (mode 0: last_restart 1 current, 2 average), the chosen point becomes the
// FP64 master and the anchor, and the correction data are recomputed in FP64 from the
// products A~x, A~^T y that the evaluation just formed.
__device__ inline void rebase_at(const DevLP& P, int lr, int g) {
    const bool avg = lr == 2;
    if (g < P.n) {
        const double xc = avg ? P.xa[g] : P.x[g];
        const double at = avg ? P.atya[g] : P.aty[g];
        P.xh[g] = xc;
        P.xan[g] = xc;
        P.atyan[g] = at;
        P.d32[g] = static_cast<float>(P.c[g] - at);
        P.lo32[g] = static_cast<float>(P.xl[g] - xc);
        P.hi32[g] = static_cast<float>(P.xu[g] - xc);
        P.dx[g] = 0.0f;
        P.dxa[g] = 0.0f;
    }
    if (g < P.m) {
        const double yc = avg ? P.ya[g] : P.y[g];
        const double ax = avg ? P.axa[g] : P.ax[g];
        P.yh[g] = yc;
        P.yan[g] = yc;
        P.axan[g] = ax;
        P.yh32[g] = static_cast<float>(yc);
        P.rl32[g] = static_cast<float>(P.bl[g] - ax);
        P.ru32[g] = static_cast<float>(P.bu[g] - ax);
        P.dy[g] = 0.0f;
        P.dya[g] = 0.0f;
        P.adx[g] = 0.0f;
    }
}

__global__ void rebase_kernel(DevLP P, int mode) {
    const int lr = mode == 1 ? 1 : P.sc->last_restart;
    if (lr == 0) return;
    if (mode == 1 && P.sc->status != kRunning) return;
    rebase_at(P, lr, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void to_float_kernel(const double* src, float* dst, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = static_cast<float>(src[i]);
}


// ------------------------------------------------------------------ batched form

// Sparse product by one workgroup: every row tile of M in turn.
template <class T, class Epi>
__device__ void wg_spmv(const Csr& M, const T* xin, const Epi& epi, double* lds, double* red) {
    T* prod = reinterpret_cast<T*>(lds);
    for (int b = 0; b < M.ntiles; ++b) {
        tile_body_any(M, b, xin, epi, prod, red);
        __syncthreads();
    }
}

// One half-iteration by one workgroup: the epilogue's begin() sets its scalars (it always
// runs here: the workgroup only iterates while the LP is running below max_iters).
template <class T, class Epi>
__device__ void wg_step(const Csr& M, const T* xin, Epi e, double* lds, double* red) {
    e.begin();
    wg_spmv(M, xin, e, lds, red);
}

// KKT quantities of the current iterate (and of the average in mode 0, of the candidate rays
// in mode 0) summed over the whole LP by one workgroup in a fixed order; tot[] in LDS afterwards.
__device__ void wg_kkt(const DevLP& P, int mode, double* tot, double* red16) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    {
        constexpr int kMain = kNT - kNF;
        double acc[kMain];
#pragma unroll
        for (int q = 0; q < kMain; ++q) acc[q] = 0.0;
        eval_terms(P, mode, threadIdx.x, kBlock, acc);
#pragma unroll
        for (int q = 0; q < kMain; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red16[w * kNT + q] = v;
        }
    }
    // the residual-restart sums in a pass of their own (their slots stay 0 when off)
    {
        double acc[kNF];
#pragma unroll
        for (int q = 0; q < kNF; ++q) acc[q] = 0.0;
        if (mode == 0 && residual_restarts(P)) residual_terms(P, threadIdx.x, kBlock, acc);
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) red16[w * kNT + kNT - kNF + q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kNT) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += red16[k * kNT + threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
}

// One LP solved by one workgroup: the same restarted, averaged PDHG as the multi-kernel
// path (same kernels' epilogues, evaluation and decision logic), with the scalar state in
// LDS and a workgroup barrier between the phases.
__device__ void wg_solve(const DevLP& P, const BatchJob& J, Scalars* ssc, double* lds, double* red, double* red16,
                         double* tot) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        *ssc = *P.sc;
        ssc->omega = ssc->omega0;
        ssc->tau = ssc->eta / ssc->omega;
        ssc->sigma = ssc->eta * ssc->omega;
        ssc->eps_rel = J.eps_rel;
        ssc->eps_infeas = J.eps_infeas;
        ssc->max_iters = J.max_iters;
        ssc->eval_every = J.eval_every;
        ssc->restarts_on = J.restarts_on;
        ssc->trace_cap = J.trace_cap;
        ssc->k = 0;
        ssc->t = 0;
        ssc->restarts = 0;
        ssc->n_trace = 0;
        ssc->status = kRunning;
        ssc->out_avg = 0;
        ssc->last_restart = 0;
        ssc->kkt_prev = __builtin_inf();
        ssc->pid_int = 0.0;
        ssc->pid_prev = 0.0;
        ssc->term_mode = 0;
        ssc->ray_src = 0;
        ssc->deadline = J.limit_ticks > 0
                            ? (J.t0 ? *J.t0 : static_cast<long long>(wall_clock64())) + J.limit_ticks
                            : 0;
    }
    __syncthreads();
    const int mx = P.m > P.n ? P.m : P.n;
    for (int g = tid; g < mx; g += kBlock) init_state_at(P, g, J.x0, J.y0);
    __syncthreads();
    if (P.m > 0) wg_spmv(P.A.csr, static_cast<const double*>(P.x), EpiStore{P.ax, nullptr}, lds, red);
    wg_spmv(P.AT.csr, static_cast<const double*>(P.y), EpiStore{P.aty, nullptr}, lds, red);
    wg_kkt(P, 1, tot, red16);
    if (tid == 0) decide_logic(P, ssc, tot, 1);
    __syncthreads();
    if (ssc->status == kRunning) {
        for (int g = tid; g < mx; g += kBlock) save_prev_at(P, 0, true, g);
        __syncthreads();
    }
    if (P.fp32 && ssc->status == kRunning) {
        for (int g = tid; g < mx; g += kBlock) rebase_at(P, 1, g);
        __syncthreads();
    }
    while (ssc->status == kRunning) {
        const int E = ssc->eval_every;
        for (int it = 0; it < E; ++it) {
            if (ssc->k + it >= ssc->max_iters) break;
            if (P.fp32) {
                const float* dy = static_cast<const float*>(P.dy);
                if (P.method) wg_step(P.AT.csr, dy, epi_primal32_h(P, ssc, it), lds, red);
                else wg_step(P.AT.csr, dy, epi_primal32(P, ssc, it), lds, red);
                if (P.m > 0) {
                    if (P.method) wg_step(P.A.csr, static_cast<const float*>(P.dxa), epi_dual32_h(P, ssc, it), lds, red);
                    else wg_step(P.A.csr, static_cast<const float*>(P.dx), epi_dual32(P, ssc, it), lds, red);
                }
            } else {
                const double* y = static_cast<const double*>(P.y);
                if (P.method) wg_step(P.AT.csr, y, epi_primal_h(P, ssc, it), lds, red);
                else wg_step(P.AT.csr, y, epi_primal(P, ssc, it), lds, red);
                if (P.m > 0) {
                    if (P.method) wg_step(P.A.csr, static_cast<const double*>(P.xa), epi_dual_h(P, ssc, it), lds, red);
                    else wg_step(P.A.csr, static_cast<const double*>(P.x), epi_dual(P, ssc, it), lds, red);
                }
            }
        }
        if (P.fp32) {
            for (int g = tid; g < mx; g += kBlock) materialize_at(P, g);
            __syncthreads();
            if (P.m > 0 && !P.method) wg_spmv(P.A.csr, static_cast<const double*>(P.x), EpiStore{P.ax, nullptr}, lds, red);
        }
        if (!P.method) wg_spmv(P.AT.csr, static_cast<const double*>(P.y), EpiStore{P.aty, nullptr}, lds, red);
        if (P.m > 0 && (!P.method || P.fp32))
            wg_spmv(P.A.csr, static_cast<const double*>(P.xa), EpiStore{P.axa, nullptr}, lds, red);
        wg_spmv(P.AT.csr, static_cast<const double*>(P.ya), EpiStore{P.atya, nullptr}, lds, red);
        wg_kkt(P, 0, tot, red16);
        if (tid == 0) decide_logic(P, ssc, tot, 0);
        __syncthreads();
        const int lr = ssc->last_restart;
        if (ssc->status == kRunning) {
            for (int g = tid; g < mx; g += kBlock) save_prev_at(P, lr, false, g);
            __syncthreads();
        }
        if (lr) {
            for (int g = tid; g < mx; g += kBlock) {
                if (P.fp32) rebase_at(P, lr, g);
                else apply_restart_at(P, lr, g);
            }
            __syncthreads();
        }
    }
    for (int g = tid; g < mx; g += kBlock) extract_at(P, ssc->out_avg, ssc->status, ssc->ray_scale, ssc->ray_src, g);
    __syncthreads();
    if (tid == 0) *P.sc = *ssc;
}

// ------------------------------------------------------------- small LPs held in LDS
// For an LP that fits, the arrays its iterations touch are copied into the workgroup's LDS
// for the whole solve and a copy of its DevLP points at them (generic pointers, so the same
// code reads LDS or global memory): both matrices (row pointers, column indices, row tiles and
// the values of the iteration's precision) and the iteration vectors (FP64 form: c~, x
// bounds, x, x_avg, x anchor, b~ bounds, y, y_avg, A~x, y anchor, A~x of the anchor,
// A~x_avg; FP32 form: the correction data and iterates). Everything else (the FP64 values in
// the FP32 form, the scale factors, the evaluation products, the saved previous point, the
// outputs, the trace) stays in global memory. The copy is exact and the operations are the
// same, so the result is bit-identical to the solve from global memory; only the latency of
// the hot accesses changes. At the end the iterates the host can inspect are copied back.
struct LdsCarve {
    char* base;
    size_t off;
    template <class T>
    __host__ __device__ T* take(long long count) {
        T* p = reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(base) + off);
        off += (static_cast<size_t>(count > 0 ? count : 1) * sizeof(T) + 15) & ~size_t(15);
        return p;
    }
};

// Lays the staged arrays of G out from `base` and writes their pointers into *L (a copy of
// G); with base == nullptr only the size is computed. Returns the bytes needed.
__host__ __device__ inline size_t carve_small_lp(const DevLP& G, DevLP* L, char* base) {
    LdsCarve c{base, 0};
    const long long m = G.m, n = G.n, nnz = G.nnz;
    DevLP D = G;
    auto mat = [&](Csr& M, long long rows) {
        M.rp = c.take<int>(rows + 1);
        M.ci = c.take<int>(nnz);
        M.tiles = c.take<int>(M.ntiles + 1);
        if (G.fp32) M.v32 = c.take<float>(nnz);
        else M.v = c.take<double>(nnz);
    };
    mat(D.A.csr, m);
    mat(D.AT.csr, n);
    if (G.fp32) {
        D.d32 = c.take<float>(n);
        D.lo32 = c.take<float>(n);
        D.hi32 = c.take<float>(n);
        D.dx = c.take<float>(n);
        D.dxa = c.take<float>(n);
        D.rl32 = c.take<float>(m);
        D.ru32 = c.take<float>(m);
        D.yh32 = c.take<float>(m);
        D.dy = c.take<float>(m);
        D.dya = c.take<float>(m);
        D.adx = c.take<float>(m);
    } else {
        D.c = c.take<double>(n);
        D.xl = c.take<double>(n);
        D.xu = c.take<double>(n);
        D.x = c.take<double>(n);
        D.xa = c.take<double>(n);
        D.xan = c.take<double>(n);
        D.bl = c.take<double>(m);
        D.bu = c.take<double>(m);
        D.y = c.take<double>(m);
        D.ya = c.take<double>(m);
        D.ax = c.take<double>(m);
        D.yan = c.take<double>(m);
        D.axan = c.take<double>(m);
        D.axa = c.take<double>(m);
    }
    if (L) *L = D;
    return c.off;
}

template <class T>
__device__ inline void lds_copy(T* dst, const T* src, long long count) {
    for (long long i = threadIdx.x; i < count; i += kBlock) dst[i] = src[i];
}

// Called by every thread; ends with a barrier. The read-only arrays are copied in; the
// iteration vectors are written by the solve's own start (initial point, first products,
// the FP32 form's first refinement) before they are read.
__device__ void stage_small_lp(const DevLP& G, DevLP* L, char* buf) {
    if (threadIdx.x == 0) carve_small_lp(G, L, buf);
    __syncthreads();
    const long long m = G.m, n = G.n, nnz = G.nnz;
    lds_copy(const_cast<int*>(L->A.csr.rp), G.A.csr.rp, m + 1);
    lds_copy(const_cast<int*>(L->A.csr.ci), G.A.csr.ci, nnz);
    lds_copy(const_cast<int*>(L->A.csr.tiles), G.A.csr.tiles, G.A.csr.ntiles + 1);
    lds_copy(const_cast<int*>(L->AT.csr.rp), G.AT.csr.rp, n + 1);
    lds_copy(const_cast<int*>(L->AT.csr.ci), G.AT.csr.ci, nnz);
    lds_copy(const_cast<int*>(L->AT.csr.tiles), G.AT.csr.tiles, G.AT.csr.ntiles + 1);
    if (G.fp32) {
        lds_copy(const_cast<float*>(L->A.csr.v32), G.A.csr.v32, nnz);
        lds_copy(const_cast<float*>(L->AT.csr.v32), G.AT.csr.v32, nnz);
    } else {
        lds_copy(const_cast<double*>(L->A.csr.v), G.A.csr.v, nnz);
        lds_copy(const_cast<double*>(L->AT.csr.v), G.AT.csr.v, nnz);
        lds_copy(const_cast<double*>(L->c), G.c, n);
        lds_copy(const_cast<double*>(L->xl), G.xl, n);
        lds_copy(const_cast<double*>(L->xu), G.xu, n);
        lds_copy(const_cast<double*>(L->bl), G.bl, m);
        lds_copy(const_cast<double*>(L->bu), G.bu, m);
    }
    __syncthreads();
}

// The iterates lp_get_iterates reads, back to global memory. Ends with a barrier.
__device__ void unstage_small_lp(const DevLP& L, const DevLP& G) {
    if (G.fp32) {
        lds_copy(G.dx, L.dx, G.n);
        lds_copy(G.dxa, L.dxa, G.n);
        lds_copy(G.dy, L.dy, G.m);
        lds_copy(G.dya, L.dya, G.m);
    } else {
        lds_copy(G.x, L.x, G.n);
        lds_copy(G.xa, L.xa, G.n);
        lds_copy(G.y, L.y, G.m);
        lds_copy(G.ya, L.ya, G.m);
    }
    __syncthreads();
}

// Persistent batched solve. Every workgroup loops: take the next LP from the counter,
// solve it, until the counter passes `count`; then all of its waves return together. With
// `lds_cap` > 0 the launch holds that many bytes of dynamic LDS per workgroup and an LP
// whose staged arrays fit is solved from LDS.
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchJob* jobs, const int* order, int count,
                                                        int* counter, int lds_cap) {
    extern __shared__ __align__(16) char small_lp_lds[];
    __shared__ double lds[kTileNnzMax];
    __shared__ double red[kBlock / 64];
    __shared__ double red16[(kBlock / 64) * kNT];
    __shared__ double tot[kNT];
    __shared__ Scalars ssc;
    __shared__ DevLP staged;
    __shared__ int job;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) job = atomicAdd(counter, 1);
        __syncthreads();
        const int j = job;
        if (j >= count) return;
        const BatchJob& J = jobs[order[j]];
        if (lds_cap > 0 && carve_small_lp(J.P, nullptr, nullptr) <= static_cast<size_t>(lds_cap)) {
            stage_small_lp(J.P, &staged, small_lp_lds);
            wg_solve(staged, J, &ssc, lds, red, red16, tot);
            unstage_small_lp(staged, J.P);
        } else {
            wg_solve(J.P, J, &ssc, lds, red, red16, tot);
        }
    }
}


// ------------------------------------------------ block-diagonal batch (many LPs per launch)
// One launch covers the row tiles (or reduction blocks, or vector blocks) of every LP of a
// batch; map[b] = (LP, tile-or-block of that LP). Each LP keeps its own scalars, so every
// LP follows exactly the trajectory of its own single-LP solve, bundles are graph-captured
// for the whole batch, and a converged LP's blocks return at once.
enum MultiKind { MK_PRIMAL = 0, MK_DUAL, MK_AX_ALL, MK_AX_FP32, MK_ATY, MK_AXA, MK_ATYA };

// One row tile with an epilogue whose begin() may decline the work (LP stopped).
template <int TN, class T, class Epi>
__device__ inline void run_tile(const Csr& M, int b, const T* xin, Epi e, T* prod, double* red) {
    if (!e.begin()) return;
    tile_body<TN>(M, b, xin, e, prod, red);
}

// FORM = 2 * fp32 + method for the iteration kinds (one instance per form: the four fused
// epilogues in one kernel would hold the registers of the largest and halve occupancy), -1
// for the evaluation products; TN the row-tile shape of the LPs of the launch.
template <int KIND, int FORM, int TN>
__global__ __launch_bounds__(kBlock) void multi_tiles_kernel(const BatchJob* jobs, const int2* map, int it) {
    __shared__ double lds[TN];
    __shared__ double red[kBlock / 64];
    const int2 mt = map[blockIdx.x];
    const DevLP& P = jobs[mt.x].P;
    float* lds32 = reinterpret_cast<float*>(lds);
    if constexpr (KIND == MK_PRIMAL) {
        if constexpr (FORM == 3) run_tile<TN>(P.AT.csr, mt.y, static_cast<const float*>(P.dy), epi_primal32_h(P, P.sc, it), lds32, red);
        else if constexpr (FORM == 2) run_tile<TN>(P.AT.csr, mt.y, static_cast<const float*>(P.dy), epi_primal32(P, P.sc, it), lds32, red);
        else if constexpr (FORM == 1) run_tile<TN>(P.AT.csr, mt.y, static_cast<const double*>(P.y), epi_primal_h(P, P.sc, it), lds, red);
        else run_tile<TN>(P.AT.csr, mt.y, static_cast<const double*>(P.y), epi_primal(P, P.sc, it), lds, red);
    } else if constexpr (KIND == MK_DUAL) {
        if constexpr (FORM == 3) run_tile<TN>(P.A.csr, mt.y, static_cast<const float*>(P.dxa), epi_dual32_h(P, P.sc, it), lds32, red);
        else if constexpr (FORM == 2) run_tile<TN>(P.A.csr, mt.y, static_cast<const float*>(P.dx), epi_dual32(P, P.sc, it), lds32, red);
        else if constexpr (FORM == 1) run_tile<TN>(P.A.csr, mt.y, static_cast<const double*>(P.xa), epi_dual_h(P, P.sc, it), lds, red);
        else run_tile<TN>(P.A.csr, mt.y, static_cast<const double*>(P.x), epi_dual(P, P.sc, it), lds, red);
    } else {
        if (P.sc->status != kRunning) return;
        if (KIND == MK_AX_FP32 && (!P.fp32 || P.method)) return;
        // the Halpern form evaluates only T(z): no A~^T y of the iterate, and in FP64 the
        // dual half already left A~ xa in axa
        if (KIND == MK_ATY && P.method && it == 0) return;  // it == 1: the initial point
        if (KIND == MK_AXA && P.method && !P.fp32) return;
        const bool onA = KIND == MK_AX_ALL || KIND == MK_AX_FP32 || KIND == MK_AXA;
        const double* xin = KIND == MK_ATY ? P.y : KIND == MK_ATYA ? P.ya : KIND == MK_AXA ? P.xa : P.x;
        double* out = KIND == MK_ATY ? P.aty : KIND == MK_ATYA ? P.atya : KIND == MK_AXA ? P.axa : P.ax;
        tile_body<TN>(onA ? P.A.csr : P.AT.csr, mt.y, xin, EpiStore{out, nullptr}, lds, red);
    }
}

__global__ __launch_bounds__(kBlock) void multi_partials_kernel(const BatchJob* jobs, const int2* map, int mode) {
    const int2 mt = map[blockIdx.x];
    const DevLP& P = jobs[mt.x].P;
    kkt_partials_body(P, mode, mt.y, P.nred);
}

__global__ __launch_bounds__(kBlock) void multi_decide_kernel(const BatchJob* jobs, int mode) {
    decide_body(jobs[blockIdx.x].P, mode);
}

enum ElemOp { EO_INIT = 0, EO_REBASE_INIT, EO_MATERIALIZE, EO_APPLY, EO_EXTRACT };

template <int OP>
__global__ __launch_bounds__(kBlock) void multi_elem_kernel(const BatchJob* jobs, const int2* map) {
    const int2 mt = map[blockIdx.x];
    const BatchJob& J = jobs[mt.x];
    const DevLP& P = J.P;
    const int g = mt.y * kBlock + threadIdx.x;
    const Scalars* sc = P.sc;
    if (OP == EO_INIT) {
        init_state_at(P, g, J.x0, J.y0);
    } else if (OP == EO_REBASE_INIT) {
        if (sc->status != kRunning) return;
        save_prev_at(P, 0, true, g);
        if (P.fp32) rebase_at(P, 1, g);
    } else if (OP == EO_MATERIALIZE) {
        if (P.fp32 && sc->status == kRunning) materialize_at(P, g);
    } else if (OP == EO_APPLY) {
        if (sc->status != kRunning) return;
        const int lr = sc->last_restart;
        save_prev_at(P, lr, false, g);
        if (lr == 0) return;
        if (P.fp32) rebase_at(P, lr, g);
        else apply_restart_at(P, lr, g);
    } else {
        extract_at(P, sc->out_avg, sc->status, sc->ray_scale, sc->ray_src, g);
    }
}

__global__ void multi_reset_kernel(const BatchJob* jobs, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const BatchJob& J = jobs[i];
    Scalars* sc = J.P.sc;
    sc->omega = sc->omega0;
    sc->tau = sc->eta / sc->omega;
    sc->sigma = sc->eta * sc->omega;
    sc->eps_rel = J.eps_rel;
    sc->eps_infeas = J.eps_infeas;
    sc->max_iters = J.max_iters;
    sc->eval_every = J.eval_every;
    sc->restarts_on = J.restarts_on;
    sc->trace_cap = J.trace_cap;
    sc->k = 0;
    sc->t = 0;
    sc->restarts = 0;
    sc->n_trace = 0;
    sc->status = kRunning;
    sc->out_avg = 0;
    sc->last_restart = 0;
    sc->kkt_prev = __builtin_inf();
    sc->pid_int = 0.0;
    sc->pid_prev = 0.0;
    sc->term_mode = 0;
    sc->ray_src = 0;
    sc->deadline = J.limit_ticks > 0 ? (J.t0 ? *J.t0 : static_cast<long long>(wall_clock64())) + J.limit_ticks : 0;
}

__global__ void multi_status_kernel(const BatchJob* jobs, int count, int* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) status[i] = jobs[i].P.sc->status;
}

// Number of LPs still running, summed by one workgroup in a fixed order.
__global__ __launch_bounds__(kBlock) void multi_active_kernel(const BatchJob* jobs, int count, int* active) {
    __shared__ double red[kBlock / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) a += jobs[i].P.sc->status == kRunning ? 1.0 : 0.0;
    a = block_sum(a, red);
    if (threadIdx.x == 0) *active = static_cast<int>(a);
}

}  // namespace

// ---------------------------------------------------------------------- launchers

void launch_fill(double* p, long long n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n) > 4096 ? 4096 : grid_for(n)), dim3(kBlock), 0, s, p, n, v);
}

void launch_scale_pass(const DevLP& P, int* A_rp, int* A_ci, double* A_v, const int* AT_rp, const int* perm,
                       double* R, double* C, double* rf, double* cf, int use_sum, hipStream_t s) {
    if (P.m > 0)
        hipLaunchKernelGGL(scale_rowstat_kernel, dim3(grid_for(P.m)), dim3(kBlock), 0, s, P.m, A_rp, A_v, use_sum,
                           rf);
    hipLaunchKernelGGL(scale_colstat_kernel, dim3(grid_for(P.n)), dim3(kBlock), 0, s, P.n, AT_rp, perm, A_v,
                       use_sum, cf);
    if (P.m > 0)
        hipLaunchKernelGGL(scale_apply_rows_kernel, dim3(grid_for(P.m)), dim3(kBlock), 0, s, P.m, A_rp, A_ci, A_v,
                           rf, cf, R);
    hipLaunchKernelGGL(scale_apply_cols_kernel, dim3(grid_for(P.n)), dim3(kBlock), 0, s, P.n, cf, C);
}

void launch_gather(const int* perm, const double* src, double* dst, long long nnz, hipStream_t s) {
    if (nnz <= 0) return;
    unsigned g = grid_for(nnz);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(kBlock), 0, s, perm, src, dst, nnz);
}

void launch_prepare(const DevLP& P, double* c, double* bl, double* bu, double* xl, double* xu, double* R, double* C,
                    double* Ri, double* Ci, double* x0, double* y0, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    hipLaunchKernelGGL(prepare_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P.m, P.n, c, bl, bu, xl, xu, R, C,
                       Ri, Ci, x0, y0);
}

void launch_norms(const DevLP& P, hipStream_t s) {
    hipLaunchKernelGGL(norms_kernel, dim3(P.nred), dim3(kBlock), 0, s, P);
}

void launch_power_start(const DevLP& P, unsigned long long seed, double* v, hipStream_t s) {
    hipLaunchKernelGGL(power_init_kernel, dim3(grid_for(P.n)), dim3(kBlock), 0, s, P.n, seed, v);
    hipLaunchKernelGGL(sumsq2_kernel, dim3(P.nred), dim3(kBlock), 0, s, v, P.n, v, 0, P.partials);
    unsigned gn = grid_for(P.n);
    if (gn > 2048) gn = 2048;
    hipLaunchKernelGGL(normalize_kernel, dim3(gn), dim3(kBlock), 0, s, v, v, P.n, P.partials, P.nred, 0,
                       (Scalars*)nullptr);
    static_assert(offsetof(Scalars, sigma_prev) == offsetof(Scalars, sigma_max) + sizeof(double),
                  "sigma_max and sigma_prev are cleared together");
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(2), 0, s, &P.sc->sigma_max, 2LL, 0.0);
}

void launch_power_steps(const DevLP& P, int iters, double* v, double* u, double* w, hipStream_t s) {
    unsigned gn = grid_for(P.n);
    if (gn > 2048) gn = 2048;
    for (int it = 0; it < iters; ++it) {
        if (P.m > 0) launch_spmv_store(P.A, v, u, nullptr, s);
        if (P.m > 0) launch_spmv_store(P.AT, u, w, nullptr, s);
        else launch_fill(w, P.n, 0.0, s);
        hipLaunchKernelGGL(sumsq2_kernel, dim3(P.nred), dim3(kBlock), 0, s, u, P.m, w, P.n, P.partials);
        hipLaunchKernelGGL(normalize_kernel, dim3(gn), dim3(kBlock), 0, s, w, v, P.n, P.partials, P.nred, 1, P.sc);
    }
}

void launch_finalize_setup(const DevLP& P, double eta_override, double omega_override, double c0, hipStream_t s) {
    launch_norms(P, s);
    hipLaunchKernelGGL(finalize_setup_kernel, dim3(1), dim3(kBlock), 0, s, P, P.nred, eta_override, omega_override,
                       c0);
}

void launch_reset(const DevLP& P, double eps_rel, double eps_infeas, long long max_iters, int eval_every,
                  int restarts_on, long long trace_cap, hipStream_t s, int term_mode, double omega_override) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, P.sc, eps_rel, eps_infeas, max_iters, eval_every,
                       restarts_on, trace_cap, term_mode, omega_override);
}

__global__ void zero_finite_kernel(double* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        if (finite_d(p[i])) p[i] = 0.0;
}

void launch_zero_finite(double* p, long long n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = grid_for(n);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(zero_finite_kernel, dim3(g), dim3(kBlock), 0, s, p, n);
}

void launch_evaluate_point(const DevLP& P, hipStream_t s) {
    if (P.m > 0) {
        launch_spmv_store(P.A, P.x, P.ax, nullptr, s);
        launch_spmv_store(P.A, P.xa, P.axa, nullptr, s);
    }
    launch_spmv_store(P.AT, P.y, P.aty, nullptr, s);
    launch_spmv_store(P.AT, P.ya, P.atya, nullptr, s);
    hipLaunchKernelGGL(kkt_partials_kernel, dim3(P.nred), dim3(kBlock), 0, s, P, 2);
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(kBlock), 0, s, P, 2);
}

void launch_init_state(const DevLP& P, const double* x0, const double* y0, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    hipLaunchKernelGGL(init_state_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P, x0, y0);
}

void launch_spmv_store(const Mat& M, const double* xin, double* out, const Scalars* gate, hipStream_t s) {
    EpiStore e{out, gate};
    launch_spmv(M, xin, e, s);
}

void launch_layout_trial(const DevLP& P, int layout, int reps, hipStream_t s) {
    Mat A = P.A, AT = P.AT;
    A.layout = AT.layout = layout;
    for (int r = 0; r < reps; ++r) {
        if (P.fp32) {
            if (P.m > 0) launch_spmv(A, static_cast<const float*>(P.dx), EpiStore{P.ax, nullptr}, s);
            launch_spmv(AT, static_cast<const float*>(P.dy), EpiStore{P.aty, nullptr}, s);
        } else {
            if (P.m > 0) launch_spmv(A, static_cast<const double*>(P.x), EpiStore{P.ax, nullptr}, s);
            launch_spmv(AT, static_cast<const double*>(P.y), EpiStore{P.aty, nullptr}, s);
        }
    }
}

// With no rows every row of A^T is empty and the product still carries the primal update.
void launch_primal(const DevLP& P, int it, hipStream_t s) {
    const float* dy = static_cast<const float*>(P.dy);
    if (P.fp32) {
        if (P.method) launch_spmv(P.AT, dy, epi_primal32_h(P, P.sc, it), s);
        else launch_spmv(P.AT, dy, epi_primal32(P, P.sc, it), s);
    } else if (P.method) {
        launch_spmv(P.AT, static_cast<const double*>(P.y), epi_primal_h(P, P.sc, it), s);
    } else {
        launch_spmv(P.AT, static_cast<const double*>(P.y), epi_primal(P, P.sc, it), s);
    }
}

// The dual half gathers x+ : the updated x (averaged form) or the PDHG output xa (Halpern).
void launch_dual(const DevLP& P, int it, hipStream_t s) {
    if (P.m == 0) return;
    if (P.fp32) {
        if (P.method) launch_spmv(P.A, static_cast<const float*>(P.dxa), epi_dual32_h(P, P.sc, it), s);
        else launch_spmv(P.A, static_cast<const float*>(P.dx), epi_dual32(P, P.sc, it), s);
    } else if (P.method) {
        launch_spmv(P.A, static_cast<const double*>(P.xa), epi_dual_h(P, P.sc, it), s);
    } else {
        launch_spmv(P.A, static_cast<const double*>(P.x), epi_dual(P, P.sc, it), s);
    }
}

void launch_materialize(const DevLP& P, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    hipLaunchKernelGGL(materialize_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P);
}

// Evaluation (mode 0 periodic, 1 initial point, 2 final point after a host-side stop): the
// products the evaluated point needs, the fixed-order reductions, the decision, and the point
// the next evaluation's rays start from. The Halpern form evaluates the PDHG output only.
void launch_evaluate(const DevLP& P, int mode, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    const Scalars* gate = mode == 2 ? nullptr : P.sc;
    const bool cand = P.method && mode != 1;
    if (P.fp32 && mode != 1) {
        // FP64 iterates from the master and the FP32 correction, then FP64 products on A~
        launch_materialize(P, s);
        if (cand) {
            if (P.m > 0) launch_spmv_store(P.A, P.xa, P.axa, gate, s);
            launch_spmv_store(P.AT, P.ya, P.atya, gate, s);
        } else {
            if (P.m > 0) launch_spmv_store(P.A, P.x, P.ax, gate, s);
            launch_spmv_store(P.AT, P.y, P.aty, gate, s);
            if (mode == 0) {
                if (P.m > 0) launch_spmv_store(P.A, P.xa, P.axa, gate, s);
                launch_spmv_store(P.AT, P.ya, P.atya, gate, s);
            }
        }
    } else if (mode == 1) {
        if (P.m > 0) launch_spmv_store(P.A, P.x, P.ax, P.sc, s);
        launch_spmv_store(P.AT, P.y, P.aty, P.sc, s);
    } else if (cand) {
        launch_spmv_store(P.AT, P.ya, P.atya, gate, s);  // A~ xa is left in axa by the dual half
    } else if (mode == 0) {
        launch_spmv_store(P.AT, P.y, P.aty, P.sc, s);
        if (P.m > 0) launch_spmv_store(P.A, P.xa, P.axa, P.sc, s);
        launch_spmv_store(P.AT, P.ya, P.atya, P.sc, s);
    } else {
        launch_spmv_store(P.AT, P.y, P.aty, nullptr, s);
    }
    hipLaunchKernelGGL(kkt_partials_kernel, dim3(P.nred), dim3(kBlock), 0, s, P, mode);
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(kBlock), 0, s, P, mode);
    if (mode != 2) hipLaunchKernelGGL(save_prev_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P, mode == 1 ? 1 : 0);
    if (P.fp32 && mode == 1) hipLaunchKernelGGL(rebase_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P, 1);
}

void launch_apply_restart(const DevLP& P, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    if (P.fp32) {
        hipLaunchKernelGGL(rebase_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P, 0);
        return;
    }
    hipLaunchKernelGGL(apply_restart_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P);
}


// Tile launches of one kind: one per group of the maps (form v = 2 * fp32 + method and
// row-tile shape h, group g = 3 v + h), each with the kernel instance of its form and shape.
template <int KIND, int FORM>
void multi_tiles_group(const MultiMaps& M, int g, bool on_a, int it_or_mode, hipStream_t s) {
    const int n = on_a ? M.cnt_a[g] : M.cnt_at[g];
    if (n <= 0) return;
    const int2* map = on_a ? M.map_a + M.off_a[g] : M.map_at + M.off_at[g];
    switch (g % kTileShapes) {
        case 0: hipLaunchKernelGGL((multi_tiles_kernel<KIND, FORM, tile_nnz_of(0)>), dim3(n), dim3(kBlock), 0, s, M.jobs, map, it_or_mode); break;
        case 1: hipLaunchKernelGGL((multi_tiles_kernel<KIND, FORM, tile_nnz_of(1)>), dim3(n), dim3(kBlock), 0, s, M.jobs, map, it_or_mode); break;
        default: hipLaunchKernelGGL((multi_tiles_kernel<KIND, FORM, tile_nnz_of(2)>), dim3(n), dim3(kBlock), 0, s, M.jobs, map, it_or_mode); break;
    }
}

template <int KIND>
void multi_tiles_iter(const MultiMaps& M, bool on_a, int it, hipStream_t s) {
    for (int h = 0; h < kTileShapes; ++h) {
        multi_tiles_group<KIND, 0>(M, 0 * kTileShapes + h, on_a, it, s);
        multi_tiles_group<KIND, 1>(M, 1 * kTileShapes + h, on_a, it, s);
        multi_tiles_group<KIND, 2>(M, 2 * kTileShapes + h, on_a, it, s);
        multi_tiles_group<KIND, 3>(M, 3 * kTileShapes + h, on_a, it, s);
    }
}

template <int KIND>
void multi_tiles_eval(const MultiMaps& M, bool on_a, int mode, hipStream_t s) {
    for (int g = 0; g < kMapGroups; ++g) multi_tiles_group<KIND, -1>(M, g, on_a, mode, s);
}

void launch_multi(const MultiMaps& M, int kind, int it_or_mode, hipStream_t s) {
    switch (kind) {
        case MULTI_PRIMAL: multi_tiles_iter<MK_PRIMAL>(M, false, it_or_mode, s); break;
        case MULTI_DUAL: multi_tiles_iter<MK_DUAL>(M, true, it_or_mode, s); break;
        case MULTI_AX_ALL: multi_tiles_eval<MK_AX_ALL>(M, true, it_or_mode, s); break;
        case MULTI_AX_FP32: multi_tiles_eval<MK_AX_FP32>(M, true, it_or_mode, s); break;
        case MULTI_ATY: multi_tiles_eval<MK_ATY>(M, false, it_or_mode, s); break;
        case MULTI_AXA: multi_tiles_eval<MK_AXA>(M, true, it_or_mode, s); break;
        case MULTI_ATYA: multi_tiles_eval<MK_ATYA>(M, false, it_or_mode, s); break;
        case MULTI_PARTIALS:
            if (M.n_red > 0)
                hipLaunchKernelGGL(multi_partials_kernel, dim3(M.n_red), dim3(kBlock), 0, s, M.jobs, M.map_red,
                                   it_or_mode);
            break;
        case MULTI_DECIDE:
            hipLaunchKernelGGL(multi_decide_kernel, dim3(M.count), dim3(kBlock), 0, s, M.jobs, it_or_mode);
            break;
        case MULTI_INIT: hipLaunchKernelGGL(multi_elem_kernel<EO_INIT>, dim3(M.n_elem), dim3(kBlock), 0, s, M.jobs, M.map_elem); break;
        case MULTI_REBASE_INIT: hipLaunchKernelGGL(multi_elem_kernel<EO_REBASE_INIT>, dim3(M.n_elem), dim3(kBlock), 0, s, M.jobs, M.map_elem); break;
        case MULTI_MATERIALIZE: hipLaunchKernelGGL(multi_elem_kernel<EO_MATERIALIZE>, dim3(M.n_elem), dim3(kBlock), 0, s, M.jobs, M.map_elem); break;
        case MULTI_APPLY: hipLaunchKernelGGL(multi_elem_kernel<EO_APPLY>, dim3(M.n_elem), dim3(kBlock), 0, s, M.jobs, M.map_elem); break;
        case MULTI_EXTRACT: hipLaunchKernelGGL(multi_elem_kernel<EO_EXTRACT>, dim3(M.n_elem), dim3(kBlock), 0, s, M.jobs, M.map_elem); break;
        case MULTI_RESET:
            hipLaunchKernelGGL(multi_reset_kernel, dim3((M.count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M.jobs, M.count);
            break;
        case MULTI_ACTIVE:
            hipLaunchKernelGGL(multi_active_kernel, dim3(1), dim3(kBlock), 0, s, M.jobs, M.count, M.active);
            break;
        case MULTI_STATUS:
            hipLaunchKernelGGL(multi_status_kernel, dim3((M.count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M.jobs,
                               M.count, M.active);
            break;
        default: break;
    }
}

void launch_batch(const BatchJob* jobs, const int* order, int count, int* counter, int grid, hipStream_t s,
                  int lds_cap) {
    if (count <= 0 || grid <= 0) return;
    if (lds_cap > 0) {
        static const bool attr = [] {
            return hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLpLdsMax) == hipSuccess;
        }();
        if (!attr) lds_cap = 0;
    }
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kBlock), static_cast<size_t>(lds_cap), s, jobs, order, count,
                       counter, lds_cap);
}

size_t small_lp_lds_bytes(const DevLP& P) { return carve_small_lp(P, nullptr, nullptr); }

// ------------------------------------------------------ allocation-free batched form
// Scratch of lp_solve_batch_static: job table, LP order, work counter. Host code never takes
// the array's name as an address (in host code it is only a stand-in for the symbol); the
// device address comes from hipGetSymbolAddress, once per device with that device current.
constexpr size_t kStaticJobsBytes = (sizeof(BatchJob) * kStaticBatchMax + 255) / 256 * 256;
constexpr size_t kStaticOrderBytes = (sizeof(int) * kStaticBatchMax + 255) / 256 * 256;
constexpr size_t kStaticScratchBytes = kStaticJobsBytes + kStaticOrderBytes + 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

__global__ void batch_start_kernel(int* counter, long long* t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *counter = 0;
        *t0 = static_cast<long long>(wall_clock64());
    }
}
}  // namespace

hipError_t static_batch_scratch(int device, StaticBatchScratch* out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = static_cast<char*>(ptr);
    }
    char* b = g_scratch_addr[device];
    out->jobs = reinterpret_cast<BatchJob*>(b);
    out->order = reinterpret_cast<int*>(b + kStaticJobsBytes);
    out->counter = reinterpret_cast<int*>(b + kStaticJobsBytes + kStaticOrderBytes);
    out->t0 = reinterpret_cast<long long*>(b + kStaticJobsBytes + kStaticOrderBytes + 128);
    return hipSuccess;
}

size_t static_batch_scratch_bytes() { return kStaticScratchBytes; }

void launch_batch_start(int* counter, long long* t0, hipStream_t s) {
    hipLaunchKernelGGL(batch_start_kernel, dim3(1), dim3(64), 0, s, counter, t0);
}

void launch_to_float(const double* src, float* dst, long long n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = grid_for(n);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(to_float_kernel, dim3(g), dim3(kBlock), 0, s, src, dst, n);
}

void launch_stop(const DevLP& P, int status, hipStream_t s) {
    hipLaunchKernelGGL(stop_kernel, dim3(1), dim3(1), 0, s, P.sc, status);
}

void launch_extract(const DevLP& P, hipStream_t s) {
    const int mx = P.m > P.n ? P.m : P.n;
    hipLaunchKernelGGL(extract_kernel, dim3(grid_for(mx)), dim3(kBlock), 0, s, P);
}

}  // namespace lpgpu

namespace lpgpu {

int read_check_word(int device, unsigned* word) {
    *word = 0;
    if (!kChecked) return 0;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMemcpyFromSymbol(word, HIP_SYMBOL(lp_check_word), sizeof(unsigned), 0, hipMemcpyDeviceToHost);
    const unsigned zero = 0;
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(lp_check_word), &zero, sizeof(unsigned), 0, hipMemcpyHostToDevice);
    return static_cast<int>(e);
}

}  // namespace lpgpu
