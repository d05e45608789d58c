// Diagnostics over the macroscopic fields (separate unit from the step
// kernels): the enstrophy of a periodic velocity field.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbm {

// Launches the enstrophy reduction on stream s: sum over the nodes of
// |curl u|^2, with central differences of half-width m (order 2m) whose
// coefficients over the spacing are coef[0..m-1], written to result[0] (a
// device double).  u is [D][nz][ny][nx], double if f64 else float;
// partial holds max_blocks doubles of block sums.
hipError_t launch_enstrophy(const void* u, bool f64, const int64_t n[3], int D, int m, const double* coef,
                            double* partial, int max_blocks, double* result, hipStream_t s);

}  // namespace lbm
