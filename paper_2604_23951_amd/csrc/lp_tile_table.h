// Row-tile shape per LP class, as measured on the device by paper_2604_23951_amd/tune_tiles.py
// (which rewrites this file). An LP takes the first rule that matches its precision, the mean
// row length of A (nnz / m) and its nonzero count.
#pragma once

#include <cstdint>

namespace lpgpu {

struct TileRule {
    int fp32;             // 0 FP64, 1 FP32 storage form
    double max_row_len;   // the rule applies when nnz / m <= max_row_len
    int64_t max_nnz;      // and nnz <= max_nnz
    int shape;            // 0: 1024, 1: 2048, 2: 4096 nonzeros per tile
};

// TUNED-TABLE-BEGIN (generated; a class the sweep did not measure takes shape 1)
constexpr TileRule kTileRules[] = {
    {0, 6.0, 20000, 2},  // 1024: 117.5 ms, 2048: 85.0 ms, 4096: 72.9 ms
    {0, 6.0, 500000, 0},  // 1024: 17.4 ms, 2048: 17.7 ms, 4096: 17.8 ms
    {0, 6.0, INT64_MAX, 0},  // 1024: 7.8 ms, 2048: 8.0 ms, 4096: 8.1 ms
    {0, 12.0, 20000, 2},  // 1024: 67.2 ms, 2048: 53.1 ms, 4096: 45.7 ms
    {0, 12.0, 500000, 0},  // 1024: 8.0 ms, 2048: 8.3 ms, 4096: 9.4 ms
    {0, 12.0, INT64_MAX, 1},  // 1024: 4.7 ms, 2048: 4.6 ms, 4096: 5.2 ms
    {0, 24.0, 20000, 2},  // 1024: 61.8 ms, 2048: 44.0 ms, 4096: 35.8 ms
    {0, 24.0, 500000, 0},  // 1024: 7.0 ms, 2048: 7.2 ms, 4096: 8.1 ms
    {0, 24.0, INT64_MAX, 0},  // 1024: 3.4 ms, 2048: 3.5 ms, 4096: 3.5 ms
    {0, 1e300, 20000, 2},  // 1024: 66.2 ms, 2048: 44.3 ms, 4096: 32.7 ms
    {0, 1e300, 500000, 1},  // 1024: 7.8 ms, 2048: 7.3 ms, 4096: 7.8 ms
    {0, 1e300, INT64_MAX, 1},  // 1024: 4.2 ms, 2048: 3.9 ms, 4096: 4.2 ms
    {1, 6.0, 20000, 2},  // 1024: 99.4 ms, 2048: 70.9 ms, 4096: 56.9 ms
    {1, 6.0, 500000, 1},  // 1024: 9.3 ms, 2048: 8.7 ms, 4096: 9.6 ms
    {1, 6.0, INT64_MAX, 1},  // 1024: 6.6 ms, 2048: 6.5 ms, 4096: 6.6 ms
    {1, 12.0, 20000, 2},  // 1024: 57.1 ms, 2048: 41.3 ms, 4096: 34.5 ms
    {1, 12.0, 500000, 1},  // 1024: 5.5 ms, 2048: 5.3 ms, 4096: 5.8 ms
    {1, 12.0, INT64_MAX, 1},  // 1024: 3.6 ms, 2048: 3.6 ms, 4096: 4.0 ms
    {1, 24.0, 20000, 2},  // 1024: 50.0 ms, 2048: 35.5 ms, 4096: 29.4 ms
    {1, 24.0, 500000, 1},  // 1024: 6.2 ms, 2048: 5.7 ms, 4096: 6.3 ms
    {1, 24.0, INT64_MAX, 1},  // 1024: 3.8 ms, 2048: 3.3 ms, 4096: 3.6 ms
    {1, 1e300, 20000, 2},  // 1024: 63.8 ms, 2048: 40.8 ms, 4096: 29.7 ms
    {1, 1e300, 500000, 1},  // 1024: 5.0 ms, 2048: 4.8 ms, 4096: 5.6 ms
    {1, 1e300, INT64_MAX, 1},  // 1024: 3.7 ms, 2048: 3.2 ms, 4096: 3.4 ms
};
constexpr const char* kTileTableSource = "tune_tiles.py on AMD Radeon Graphics, 2026-12-03";
// TUNED-TABLE-END

inline int tuned_tile_shape(bool fp32, int64_t m, int64_t n, int64_t nnz) {
    (void)n;
    const double row_len = m > 0 ? static_cast<double>(nnz) / static_cast<double>(m) : 0.0;
    for (const TileRule& r : kTileRules)
        if (r.fp32 == (fp32 ? 1 : 0) && row_len <= r.max_row_len && nnz <= r.max_nnz) return r.shape;
    return 1;
}

}  // namespace lpgpu
