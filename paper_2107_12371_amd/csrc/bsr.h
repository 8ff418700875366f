// 3x3 block-CSR product: tile limits, argument block, launcher (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace spmvlib {

constexpr int kBsrRows = 84;     // block rows per tile (3 lanes each: 21 per wavefront)
constexpr int kBsrBlocks = 510;  // stored 3x3 blocks staged in LDS per tile

template <typename V, typename T> struct BsrArgs {
    const int32_t *brow_ptr;
    const int32_t *col;
    const V *val;      // 9 values per block, row-major
    const T *X;        // (3 n_cols) x ldx, row-major
    T *Y;              // (3 n_rows) x ldy, row-major
    const int32_t *tiles;  // n_tiles + 1 block-row boundaries
    int32_t n_tiles;
    int32_t per_xcd;
    int32_t chunk_log2;     // XCD assignment of tiles (xcd_tile)
    int32_t ldx, ldy, off;  // leading dimensions and first column of this launch
};

// Y = A X for a 3x3 block-CSR handle, k right-hand sides (row-major).
template <typename V, typename T>
hipError_t launch_bsr3(const DevMatrix &M, const V *val, int k, const T *X, T *Y, hipStream_t st);

}  // namespace spmvlib
