// Calibration: the rate at which a plain streaming kernel reads HBM on this
// part, the practical ceiling the products are also reported against (the
// published 8 TB/s is the nominal one).  Each lane reads 16-byte pieces in
// a grid-stride loop with non-temporal loads (measured on a 4 GiB buffer:
// 7.09 TB/s at 2048 workgroups, against 6.38 with ordinary loads and at
// most 6.27 with four loads in flight per lane), and the workgroup's sum is
// stored so that no load can be dropped.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "matrix.h"

namespace spmvlib {

__global__ __launch_bounds__(kBlock) void k_read_stream(const f64x2 *__restrict__ p, int64_t n2,
                                                        double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    f64x2 s{0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += stride)
        s += __builtin_nontemporal_load(p + i);
    const double sum = block_sum(s[0] + s[1], sh);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

}  // namespace spmvlib

using namespace spmvlib;

extern "C" int spmv_calibrate_read(const double *buf, int64_t n, double *partials, int32_t n_blocks, void *stream) {
    clear_error();
    if (n < 0 || n_blocks < 1) return fail(SPMV_EINVAL, "n = %lld, n_blocks = %d", (long long)n, n_blocks);
    if (n % 2 != 0 || (reinterpret_cast<uintptr_t>(buf) & 15) != 0)
        return fail(SPMV_EINVAL, "the buffer must be 16-byte aligned and hold an even number of doubles");
    if (!partials || (n > 0 && !buf)) return fail(SPMV_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_read_stream, dim3(n_blocks), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const f64x2 *>(buf), n / 2, partials);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "read calibration launch");
    return SPMV_OK;
}
