// Multi-vector product Y = A X on scalar CSR handles (row-major X and Y).
#pragma once

#include <hip/hip_runtime.h>

#include "matrix.h"

namespace spmvlib {

// Launches on `st`: every row tile of the handle's plan plus its long rows.
// X holds n_cols x k doubles, Y n_rows x k, both row-major with leading
// dimension k.
hipError_t launch_spmm(const spmv_matrix *A, const double *X, double *Y, int k, hipStream_t st);

}  // namespace spmvlib
