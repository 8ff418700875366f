// The opaque handle behind spmv_matrix* (host-side bookkeeping).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "device.h"
#include "spmv.h"

struct spmv_matrix {
    spmvlib::DevMatrix M;
    spmv_info info{};
    int device = 0;
    int64_t bytes = 0;
    std::vector<void *> allocs;
    int32_t n_win_tiles = 0;       // ring-window tiles (all blocks)
    int32_t max_tile_entries = 0;  // stored entries of the largest row tile
};

namespace spmvlib {
// Maps a HIP error to SPMV_ENOMEM / SPMV_EDEVICE with a message.
int hip_fail(hipError_t e, const char *what);

// cg_solve on an explicit stream; pinned_state (optional) is a caller-owned
// pinned host buffer of at least 256 bytes for the solver's scalar mirror.
int cg_run(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter, int32_t mode,
           cg_info *info, hipStream_t s, void *pinned_state);
}  // namespace spmvlib
