// Kernel argument blocks and launcher declarations (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace spmvlib {

template <typename V, typename X, typename Y> struct SpmvArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const V *val;
    const X *x;
    Y *y;
    const Y *b;             // EPI_RESID: right-hand side
    double *part;           // EPI_DOT / EPI_RESID: one partial per segment
    const TileDesc *desc;   // tiles of this launch
    int32_t n_list;         // number of tiles
    int32_t per_xcd;        // > 0: XCD grouping of tiles (xcd_tile), 0: tile = workgroup
    int32_t chunk_log2;     // XCD grouping: -1 contiguous range per XCD, c: chunks of 2^c tiles
    int32_t wg_per_xcd;     // pipelined kernel: workgroups per XCD
    const int *done;        // optional: non-zero makes the launch a no-op (CG)
    const int32_t *win_blk_ptr;
    int32_t ring_words;
    const int32_t *runs;    // compact windows
    const uint16_t *lidx;
    const uint32_t *lidx12;
    const int32_t *sell_perm;  // sliced ELLPACK
    const uint8_t *sell_len;
    const int32_t *sell_ptr;
    int32_t n_slices;
    double *long_ws;        // optional: one double per long-row piece (several workgroups per row)
};

// y = A x over all segments of M (direct tiles, long rows, window blocks),
// launched on `st`.  V: stored value type (double, float, uint16_t = bf16),
// X/Y: vector types, A: accumulation type.  `part` must hold M.n_seg doubles
// when epi != EPI_PLAIN.  `long_ws` (optional) holds M.n_long_pieces doubles:
// then the pieces of the long rows run on a workgroup each (same bits).
template <typename V, typename X, typename Y, typename A>
hipError_t launch_spmv(const DevMatrix &M, const V *val, const X *x, Y *y, int epi, const Y *b,
                       double *part, const int *done, hipStream_t st, double *long_ws = nullptr);

// y[0..n) = 0 with a fill kernel (never a memset node, so a product on a
// matrix without stored entries stays capturable like any other); the
// products take this path when nnz = 0 and never touch x then.
template <typename T> hipError_t launch_zero_fill(T *y, int64_t n, hipStream_t st);

// Opts every window-kernel instantiation into up to 8192 ring words of
// dynamic LDS.  Called once when a matrix with window blocks is created.
hipError_t prepare_window_kernels();

// Caches the device's CU count and each kernel's occupancy so no runtime
// query is made later (for example while a CG graph is being captured).
void prepare_launch_queries();

}  // namespace spmvlib
