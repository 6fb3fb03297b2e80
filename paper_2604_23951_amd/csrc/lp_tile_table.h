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
    {0, 6.0, 1024, 1},  // 1024: 19.9 ms, 2048: 16.2 ms, 4096: 16.8 ms
    {0, 6.0, 2048, 2},  // 1024: 30.1 ms, 2048: 27.2 ms, 4096: 26.9 ms
    {0, 6.0, 20000, 2},  // 1024: 123.2 ms, 2048: 89.3 ms, 4096: 78.5 ms
    {0, 6.0, 500000, 1},  // 1024: 12.4 ms, 2048: 11.7 ms, 4096: 12.8 ms
    {0, 6.0, INT64_MAX, 0},  // 1024: 5.9 ms, 2048: 6.4 ms, 4096: 6.6 ms
    {0, 12.0, 1024, 0},  // 1024: 11.7 ms, 2048: 11.8 ms, 4096: 15.4 ms
    {0, 12.0, 2048, 1},  // 1024: 17.9 ms, 2048: 16.9 ms, 4096: 17.4 ms
    {0, 12.0, 20000, 2},  // 1024: 59.4 ms, 2048: 43.1 ms, 4096: 38.5 ms
    {0, 12.0, 500000, 2},  // 1024: 11.8 ms, 2048: 11.5 ms, 4096: 11.2 ms
    {0, 12.0, INT64_MAX, 0},  // 1024: 4.7 ms, 2048: 5.2 ms, 4096: 5.1 ms
    {0, 24.0, 1024, 0},  // 1024: 9.6 ms, 2048: 11.5 ms, 4096: 15.4 ms
    {0, 24.0, 2048, 1},  // 1024: 16.4 ms, 2048: 12.4 ms, 4096: 16.1 ms
    {0, 24.0, 20000, 2},  // 1024: 53.6 ms, 2048: 36.1 ms, 4096: 33.2 ms
    {0, 24.0, 500000, 2},  // 1024: 9.9 ms, 2048: 10.0 ms, 4096: 9.6 ms
    {0, 24.0, INT64_MAX, 1},  // 1024: 5.3 ms, 2048: 5.0 ms, 4096: 5.2 ms
    {0, 1e300, 1024, 0},  // 1024: 9.6 ms, 2048: 11.8 ms, 4096: 15.7 ms
    {0, 1e300, 2048, 1},  // 1024: 18.1 ms, 2048: 12.5 ms, 4096: 16.6 ms
    {0, 1e300, 20000, 2},  // 1024: 63.7 ms, 2048: 43.9 ms, 4096: 34.0 ms
    {0, 1e300, 500000, 2},  // 1024: 8.4 ms, 2048: 8.6 ms, 4096: 7.8 ms
    {0, 1e300, INT64_MAX, 0},  // 1024: 3.7 ms, 2048: 3.9 ms, 4096: 4.1 ms
    {1, 6.0, 1024, 2},  // 1024: 15.2 ms, 2048: 13.7 ms, 4096: 13.3 ms
    {1, 6.0, 2048, 2},  // 1024: 25.2 ms, 2048: 21.1 ms, 4096: 20.2 ms
    {1, 6.0, 20000, 2},  // 1024: 100.0 ms, 2048: 68.8 ms, 4096: 56.3 ms
    {1, 6.0, 500000, 1},  // 1024: 6.7 ms, 2048: 6.6 ms, 4096: 6.9 ms
    {1, 6.0, INT64_MAX, 0},  // 1024: 5.0 ms, 2048: 5.1 ms, 4096: 5.5 ms
    {1, 12.0, 1024, 0},  // 1024: 8.6 ms, 2048: 9.8 ms, 4096: 12.6 ms
    {1, 12.0, 2048, 1},  // 1024: 14.3 ms, 2048: 10.7 ms, 4096: 13.2 ms
    {1, 12.0, 20000, 2},  // 1024: 55.6 ms, 2048: 40.5 ms, 4096: 33.7 ms
    {1, 12.0, 500000, 1},  // 1024: 8.4 ms, 2048: 7.8 ms, 4096: 8.2 ms
    {1, 12.0, INT64_MAX, 1},  // 1024: 4.7 ms, 2048: 4.3 ms, 4096: 4.5 ms
    {1, 24.0, 1024, 0},  // 1024: 9.1 ms, 2048: 10.4 ms, 4096: 12.9 ms
    {1, 24.0, 2048, 1},  // 1024: 15.2 ms, 2048: 10.7 ms, 4096: 13.3 ms
    {1, 24.0, 20000, 2},  // 1024: 59.3 ms, 2048: 39.4 ms, 4096: 31.8 ms
    {1, 24.0, 500000, 1},  // 1024: 5.6 ms, 2048: 4.7 ms, 4096: 5.3 ms
    {1, 24.0, INT64_MAX, 1},  // 1024: 3.8 ms, 2048: 3.5 ms, 4096: 3.8 ms
    {1, 1e300, 1024, 0},  // 1024: 9.6 ms, 2048: 10.6 ms, 4096: 12.8 ms
    {1, 1e300, 2048, 1},  // 1024: 16.5 ms, 2048: 11.4 ms, 4096: 14.0 ms
    {1, 1e300, 20000, 2},  // 1024: 61.3 ms, 2048: 39.0 ms, 4096: 30.0 ms
    {1, 1e300, 500000, 1},  // 1024: 6.5 ms, 2048: 5.5 ms, 4096: 5.9 ms
    {1, 1e300, INT64_MAX, 1},  // 1024: 3.4 ms, 2048: 3.4 ms, 4096: 3.5 ms
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
