#include "lp_layout.h"

#include <algorithm>
#include <stdexcept>

namespace lpgpu {

int choose_panels(int cols, int64_t slice_bytes) {
    if (slice_bytes <= 0) slice_bytes = 1 << 19;
    const int64_t bytes = static_cast<int64_t>(cols) * 8;
    int64_t p = (bytes + slice_bytes - 1) / slice_bytes;
    if (p < 1) p = 1;
    if (p > 64) p = 64;
    return static_cast<int>(p);
}

PanelLayoutHost build_panel_layout(int rows, int cols, const int32_t* rp, const int32_t* ci,
                                   const int32_t* val_index, int panels, int long_len, int target_units,
                                   int unit_rows_max) {
    PanelLayoutHost L;
    L.rows = rows;
    L.cols = cols;
    L.panels = panels < 1 ? 1 : panels;
    int cb = 1;
    while ((1LL << cb) < static_cast<int64_t>(cols)) ++cb;
    L.col_bits = cb;
    const int row_bits = 32 - cb;
    int64_t cap = row_bits >= 31 ? (1LL << 30) : (1LL << row_bits);
    if (cap > unit_rows_max) cap = unit_rows_max;
    if (cap < 1) throw std::runtime_error("matrix too wide for the packed layout");
    L.unit_rows_cap = static_cast<int>(cap);

    // long rows
    int64_t nnz_short = 0;
    for (int r = 0; r < rows; ++r) {
        const int64_t len = rp[r + 1] - rp[r];
        if (len > long_len) {
            L.long_rows.push_back(r);
        } else {
            nnz_short += len;
        }
    }
    if (!L.long_rows.empty()) {
        L.is_long.assign(static_cast<size_t>(rows), 0);
        for (int r : L.long_rows) L.is_long[r] = 1;
    }

    // units: contiguous rows, balanced by short nonzeros, at most `cap` rows each. The greedy
    // split can leave more units than the target (rows do not divide evenly); the share per
    // unit is then raised, in small steps first and by bisection after that, until it does
    // not, so that the units fit the resident wave slots the target was sized for (one launch
    // round). A larger share never gives more units, and the share of all short nonzeros
    // gives the fewest the row cap allows.
    if (target_units < 1) target_units = 1;
    auto split = [&](int64_t share) -> int64_t {
        L.unit_row.assign(1, 0);
        int r = 0;
        while (r < rows) {
            const int start = r;
            int64_t nz = 0;
            while (r < rows && r - start < cap) {
                const int64_t len = L.is_long.empty() || !L.is_long[r] ? rp[r + 1] - rp[r] : 0;
                if (nz > 0 && nz + len > share) break;
                nz += len;
                ++r;
            }
            L.unit_row.push_back(r);
        }
        return static_cast<int64_t>(L.unit_row.size()) - 1;
    };
    int64_t per_unit = std::max<int64_t>(64, (nnz_short + target_units - 1) / target_units);
    int64_t nunits = split(per_unit);
    for (int attempt = 0; nunits > target_units && attempt < 32; ++attempt) {
        per_unit += std::max<int64_t>(1, per_unit / 128);
        nunits = split(per_unit);
    }
    if (nunits > target_units) {
        int64_t lo = per_unit, hi = std::max(per_unit, nnz_short);
        if (split(hi) <= target_units) {
            while (hi - lo > 1) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (split(mid) <= target_units) hi = mid;
                else lo = mid;
            }
        }
        split(hi);
    }
    L.units = static_cast<int>(L.unit_row.size()) - 1;
    for (int u = 0; u < L.units; ++u) L.max_unit_rows = std::max(L.max_unit_rows, L.unit_row[u + 1] - L.unit_row[u]);

    // panel-major packing
    const int P = L.panels;
    const int64_t width = (static_cast<int64_t>(cols) + P - 1) / P;
    L.packed.resize(static_cast<size_t>(nnz_short));
    L.src.resize(static_cast<size_t>(nnz_short));
    L.unit_seg.resize(static_cast<size_t>(L.units) * (P + 1));
    std::vector<int32_t> cursor;
    int64_t out = 0;
    for (int u = 0; u < L.units; ++u) {
        const int r0 = L.unit_row[u], r1 = L.unit_row[u + 1];
        cursor.assign(rp + r0, rp + r1);
        for (int p = 0; p < P; ++p) {
            L.unit_seg[static_cast<size_t>(u) * (P + 1) + p] = static_cast<int32_t>(out);
            const int64_t hi = (p + 1) * width;
            for (int r = r0; r < r1; ++r) {
                if (!L.is_long.empty() && L.is_long[r]) continue;
                int32_t& e = cursor[r - r0];
                const int32_t end = rp[r + 1];
                while (e < end && ci[e] < hi) {
                    L.packed[out] = (static_cast<uint32_t>(r - r0) << cb) | static_cast<uint32_t>(ci[e]);
                    L.src[out] = val_index ? val_index[e] : e;
                    ++out;
                    ++e;
                }
            }
        }
        L.unit_seg[static_cast<size_t>(u) * (P + 1) + P] = static_cast<int32_t>(out);
    }
    if (out != nnz_short) throw std::runtime_error("panel packing lost entries");
    L.nnz_packed = nnz_short;
    return L;
}

}  // namespace lpgpu
