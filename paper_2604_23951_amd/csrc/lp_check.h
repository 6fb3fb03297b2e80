// Input validation shared by lp_create and lp_presolve (host code).
#pragma once

#include <cstdint>
#include <string>

namespace lpgpu {

// Checks the LP data of eq. 1 (sizes, CSR structure with strictly increasing columns per row,
// finite matrix values and costs, NaN-free consistent bounds). Returns an lp_error code and
// sets *msg on failure.
int32_t validate_lp(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                    const double* c, double c0, const double* bl, const double* bu, const double* xl,
                    const double* xu, std::string* msg);

// Message returned by lp_last_error(NULL) on this thread.
void set_last_error(const std::string& msg);

}  // namespace lpgpu
