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
};

namespace spmvlib {
// Maps a HIP error to SPMV_ENOMEM / SPMV_EDEVICE with a message.
int hip_fail(hipError_t e, const char *what);
}  // namespace spmvlib
