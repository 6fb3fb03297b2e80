// Host-side construction of the panel-packed SpMV layout (integer work done once per LP).
//
// A CSR matrix with R rows and N columns is cut into P column panels of equal width and
// into "units" of contiguous rows, each swept by one wave64 (with a second wave that sums
// its products). The nonzeros of a unit are stored panel by panel (inside a panel: by row,
// then column), so a wave sweeps the panels in order and, while all resident waves do the
// same, the slice of the gathered vector that
// belongs to the current panel stays in the L2 of each XCD. Each entry keeps its column in
// the low `col_bits` of a 32-bit word and its row inside the unit in the high bits; the
// unit's row count is capped so that both fit. Because columns inside a row ascend, the
// panel-major order visits each row's entries in CSR order.
//
// Rows longer than `long_len` are not packed; they are listed separately and reduced by a
// whole workgroup each.
#pragma once

#include <cstdint>
#include <vector>

namespace lpgpu {

struct PanelLayoutHost {
    int rows = 0, cols = 0, panels = 1, col_bits = 0, units = 0, unit_rows_cap = 0, max_unit_rows = 0;
    int64_t nnz_packed = 0;
    std::vector<int32_t> unit_row;   // [units + 1] first row of each unit
    std::vector<int32_t> unit_seg;   // [units * (panels + 1)] entry offset of each (unit, panel) segment
    std::vector<uint32_t> packed;    // [nnz_packed] (local row << col_bits) | column
    std::vector<int32_t> src;        // [nnz_packed] index of the entry in the source value array
    std::vector<int32_t> long_rows;  // rows reduced by the long-row kernel
    std::vector<uint8_t> is_long;    // [rows] 1 for a long row (empty when there are none)
};

// val_index maps an entry of the CSR (position in col_idx order) to the value array it is
// gathered from on the device (identity for A, the transpose permutation for A^T).
PanelLayoutHost build_panel_layout(int rows, int cols, const int32_t* rp, const int32_t* ci,
                                   const int32_t* val_index, int panels, int long_len, int target_units,
                                   int unit_rows_max);

// Panel count for a gathered vector of `cols` doubles so that one panel slice is about
// `slice_bytes`.
int choose_panels(int cols, int64_t slice_bytes);

}  // namespace lpgpu
