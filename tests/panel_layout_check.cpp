// Host check of the panel-packed layout (built by the library's own builder, lp_layout.cpp)
// and of the order in which the panel SpMV kernel forms its row sums. Random CSR matrices with
// short and long rows are packed with random panel counts, long-row thresholds, unit targets
// and row caps; each unit is then walked the way the kernel walks it: 64-entry chunks from the
// unit's first entry, each split into pieces where the row id drops (a later panel segment
// starts), each run of a row inside a piece added by its first entry, in order, to the row's
// accumulator. Every row that is not listed as long must come out bit-identical to its plain
// CSR-order sum. Also checked: packed entries are in range, rows never exceed the unit's
// row cap, and the unit count does not exceed its target whenever the row cap allows that.
// Prints "ok <trials> <chunks> <multi-piece chunks>" and exits 0 on success.
#include "lp_layout.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <set>
#include <vector>

using lpgpu::PanelLayoutHost;

static int fail(int trial, const char* what) {
    std::printf("trial %d: %s\n", trial, what);
    return 1;
}

int main() {
    long long chunks = 0, multi = 0;
    const int trials = 300;
    for (int trial = 0; trial < trials; ++trial) {
        std::mt19937 g(static_cast<unsigned>(trial) * 7u + 1u);
        std::uniform_real_distribution<double> U(-1.0, 1.0);
        const int rows = 1 + static_cast<int>(g() % 3000), cols = 1 + static_cast<int>(g() % 5000);
        std::vector<int> rp(rows + 1, 0), ci;
        std::vector<double> v;
        for (int r = 0; r < rows; ++r) {
            int len = (g() % 10 == 0) ? static_cast<int>(g() % 400) : static_cast<int>(g() % 12);
            len = std::min(len, cols);
            std::set<int> cs;
            while (static_cast<int>(cs.size()) < len) cs.insert(static_cast<int>(g() % cols));
            for (int c : cs) {
                ci.push_back(c);
                v.push_back(U(g));
            }
            rp[r + 1] = static_cast<int>(ci.size());
        }
        std::vector<double> x(cols);
        for (double& t : x) t = U(g);
        const int panels = 1 + static_cast<int>(g() % 64), long_len = 1 + static_cast<int>(g() % 300);
        const int target = 1 + static_cast<int>(g() % 2000), cap = (g() % 2) ? 512 : 2048;
        const PanelLayoutHost L =
            lpgpu::build_panel_layout(rows, cols, rp.data(), ci.data(), nullptr, panels, long_len, target, cap);

        if (L.units < 1 || L.unit_row.front() != 0 || L.unit_row.back() != rows) return fail(trial, "unit rows");
        for (int u = 0; u < L.units; ++u) {
            const int nr = L.unit_row[u + 1] - L.unit_row[u];
            if (nr < 1 || nr > L.unit_rows_cap || nr > L.max_unit_rows) return fail(trial, "unit row count");
        }
        if ((rows + L.unit_rows_cap - 1) / L.unit_rows_cap <= target && L.units > target)
            return fail(trial, "more units than the target");

        std::vector<double> ref(rows, 0.0);
        for (int r = 0; r < rows; ++r) {
            double s = 0.0;
            for (int e = rp[r]; e < rp[r + 1]; ++e) s += v[e] * x[ci[e]];
            ref[r] = s;
        }
        const int P = L.panels;
        const unsigned cmask = (1u << L.col_bits) - 1u;
        const int last = L.nnz_packed > 0 ? static_cast<int>(L.nnz_packed) - 1 : 0;
        std::vector<double> out(rows, 0.0);
        std::vector<char> done(rows, 0);
        for (int u = 0; u < L.units; ++u) {
            const int r0 = L.unit_row[u], nr = L.unit_row[u + 1] - r0;
            std::vector<double> acc(nr, 0.0);
            const int s = L.unit_seg[static_cast<size_t>(u) * (P + 1)];
            const int e = L.unit_seg[static_cast<size_t>(u) * (P + 1) + P];
            for (int st = s; st < e; st += 64) {
                const int nvalid = std::min(64, e - st);
                ++chunks;
                int row[64], piece[64];
                double prod[64];
                bool head[64];
                for (int l = 0; l < 64; ++l) {
                    const int idx = std::min(st + l, last);
                    const unsigned pk = L.packed[idx];
                    const unsigned col = l < nvalid ? (pk & cmask) : 0u;
                    if (l < nvalid && (static_cast<int>(col) >= cols || static_cast<int>(pk >> L.col_bits) >= nr))
                        return fail(trial, "packed entry out of range");
                    row[l] = static_cast<int>(pk >> L.col_bits);
                    prod[l] = v[L.src[idx]] * x[col];
                }
                int npieces = 0;
                for (int l = 0; l < 64; ++l) {
                    const int prev = l ? row[l - 1] : -1;
                    const bool valid = l < nvalid;
                    if (valid && prev > row[l]) ++npieces;
                    piece[l] = npieces;
                    head[l] = valid && prev != row[l];
                }
                if (npieces) ++multi;
                for (int j = 0; j <= npieces; ++j) {
                    std::set<int> seen;
                    for (int l = 0; l < nvalid; ++l) {
                        if (!head[l] || piece[l] != j) continue;
                        if (!seen.insert(row[l]).second) return fail(trial, "row with two runs in one piece");
                        int end = l + 1;
                        while (end < nvalid && !head[end]) ++end;
                        double a = acc[row[l]] + prod[l];
                        for (int q = l + 1; q < end; ++q) a += prod[q];
                        acc[row[l]] = a;
                    }
                }
            }
            for (int r = 0; r < nr; ++r) {
                const int R = r0 + r;
                if (L.is_long.empty() || !L.is_long[R]) {
                    out[R] = acc[r];
                    done[R] = 1;
                }
            }
        }
        for (int r = 0; r < rows; ++r) {
            const bool is_long = !L.is_long.empty() && L.is_long[r];
            if (is_long != (rp[r + 1] - rp[r] > long_len)) return fail(trial, "long-row flag");
            if (is_long) continue;
            if (!done[r] || std::memcmp(&out[r], &ref[r], sizeof(double)) != 0) return fail(trial, "row sum differs");
        }
    }
    std::printf("ok %d %lld %lld\n", trials, chunks, multi);
    return 0;
}
