// Y = A X for a scalar CSR handle with k right-hand sides, X and Y row-major
// (the k values of one row contiguous), so one gather of X's row c brings
// all the columns a lane works on.
//
// One workgroup per row tile of the handle's plan (direct, compact-window
// and ring tiles alike; only the tile's rows and stored entries are used).
// The tile's values and column indices are staged in LDS with coalesced
// loads; then the lanes take (row, column group) tasks: a lane walks its
// row's entries in ascending order, U entries per round with all their
// gathers of KC adjacent values of X issued before any is used, and adds
// the rounded products one by one starting from zero, exactly as the
// single-vector product sums a row, so column j of Y equals the
// single-vector product of column j of X bit for bit.  A row longer than a
// tile is summed as the single-vector product sums it (pieces of 16,384
// entries): one workgroup per (piece, column) with the pieces' sums in Y's
// rows of the longest run without a long row, or, without room there, one
// workgroup per (row, column) walking the pieces.
// The values are read once for all k columns, which is what the batched
// requests of a serving workload need.  One column goes to the
// single-vector product.  Measured on the 16M-row mesh matrix: 1.10 ms
// (k = 4), 1.65 ms (8), 2.69 ms (16) against 0.52-0.54 ms for one column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "launch.h"
#include "spmm.h"
#include "tile.h"

namespace spmvlib {

__device__ __forceinline__ double add_rounded_product(double sum, double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    return sum + p;
}

// KC adjacent columns j0.. of row c of X (clamped into the row: columns at
// or beyond k read a valid word and are discarded by the caller); VEC: k is
// even and X 16-byte aligned, so pairs of columns move in 16-byte pieces.
template <int KC, bool VEC>
__device__ __forceinline__ void load_cols(const double *__restrict__ xr, int j0, int k, double (&o)[KC]) {
    if constexpr (VEC && KC >= 2) {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int p = 0; p < KC / 2; ++p) {
            const d2 v = *reinterpret_cast<const d2 *>(xr + min(j0 + 2 * p, k - 2));
            o[2 * p] = v[0];
            o[2 * p + 1] = v[1];
        }
    } else {
#pragma unroll
        for (int j = 0; j < KC; ++j) o[j] = xr[min(j0 + j, k - 1)];
    }
}

// Tasks are (row, group of KC columns); a lane takes U entries of its row
// per round: U column indices and values from LDS, then all U x KC gathers,
// then the additions in ascending entry order (slots past the row's end
// re-read its last entry and are discarded by a select).
template <int KC, int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_spmm_tiles(const TileDesc *__restrict__ desc, int n_list, int per_xcd,
                                                       int chunk_log2,
                                                       const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val, const double *__restrict__ X,
                                                       double *__restrict__ Y, int k, int cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *sv = reinterpret_cast<double *>(smem);
    int32_t *sc = reinterpret_cast<int32_t *>(sv + cap);
    const int li = xcd_tile(blockIdx.x, per_xcd, chunk_log2);
    if (li >= n_list) return;
    const TileDesc d = desc[li];
    const int n = min(d.e - d.s, cap);  // the host sizes cap to the largest tile
    for (int i = (int)threadIdx.x; i < n; i += kBlock) {
        sv[i] = val[d.s + i];
        sc[i] = col[d.s + i];
    }
    __syncthreads();
    const int groups = (k + KC - 1) / KC;
    const int tasks = (d.r1 - d.r0) * groups;
    for (int t = (int)threadIdx.x; t < tasks; t += kBlock) {
        const int r = d.r0 + t / groups;
        const int j0 = (t % groups) * KC;
        const int a = row_ptr[r] - d.s, z = min(row_ptr[r + 1] - d.s, n);
        double acc[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = 0.0;
        for (int q = a; q < z; q += U) {
            double v[U];
            double xv[U][KC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int qq = min(q + u, z - 1);
                v[u] = sv[qq];
                load_cols<KC, VEC>(X + (size_t)sc[qq] * k, j0, k, xv[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in_row = q + u < z;
#pragma unroll
                for (int j = 0; j < KC; ++j) {
                    const double s = add_rounded_product(acc[j], v[u], xv[u][j]);
                    acc[j] = in_row ? s : acc[j];
                }
            }
        }
        double *__restrict__ yr = Y + (size_t)r * k + j0;
#pragma unroll
        for (int j = 0; j < KC; ++j)
            if (j0 + j < k) yr[j] = acc[j];
    }
}

// Row d.r0 (longer than a tile), column blockIdx.y: the single-vector
// long-row sum (its pieces in order) with x read from column j of X.
__global__ __launch_bounds__(kBlock) void k_spmm_long(const TileDesc *__restrict__ desc,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val, const double *__restrict__ X,
                                                      double *__restrict__ Y, int k) {
    __shared__ double sh[kBlock / kWave];
    const TileDesc d = desc[blockIdx.x];
    const int j = (int)blockIdx.y;
    const auto gx = [X, k, j](int c) { return X[(size_t)c * k + j]; };
    double tot = 0.0;
    for (int ps = d.s; ps < d.e; ps += kLongPiece) {
        const double t = long_piece_sum<double>(val, col, ps, min(d.e, ps + kLongPiece), gx, sh);
        tot = ps == d.s ? t : tot + t;
        __syncthreads();
    }
    if (threadIdx.x == 0) Y[(size_t)d.r0 * k + j] = tot;
}

// Several workgroups per long row: one per (piece, column), its sum to
// ws[piece * k + column] ...
__global__ __launch_bounds__(kBlock) void k_spmm_long_pieces(const TileDesc *__restrict__ desc,
                                                             const int32_t *__restrict__ piece_long,
                                                             const int32_t *__restrict__ piece_ptr,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val,
                                                             const double *__restrict__ X, double *__restrict__ ws,
                                                             int k) {
    __shared__ double sh[kBlock / kWave];
    const int pc = (int)blockIdx.x, j = (int)blockIdx.y;
    const int li = piece_long[pc];
    const TileDesc d = desc[li];
    const int ps = d.s + (pc - piece_ptr[li]) * kLongPiece;
    const auto gx = [X, k, j](int c) { return X[(size_t)c * k + j]; };
    const double t = long_piece_sum<double>(val, col, ps, min(d.e, ps + kLongPiece), gx, sh);
    if (threadIdx.x == 0) ws[(size_t)pc * k + j] = t;
}

// ... then one wavefront per (long row, column) adds them in piece order,
// 64 sums per load round trip, as the single-vector combine does.
__global__ __launch_bounds__(kBlock) void k_spmm_long_combine(const TileDesc *__restrict__ desc,
                                                              const int32_t *__restrict__ piece_ptr,
                                                              const double *__restrict__ ws, double *__restrict__ Y,
                                                              int n_long, int k) {
    const int li = (int)(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);
    if (li >= n_long) return;  // the same for every lane of the wavefront
    const int j = (int)blockIdx.y;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int p0 = piece_ptr[li], p1 = piece_ptr[li + 1];
    double tot = 0.0;
    for (int b = p0; b < p1; b += kWave) {
        const int n = min(kWave, p1 - b);
        const double v = lane < n ? ws[(size_t)(b + lane) * k + j] : 0.0;
        for (int i = 0; i < n; ++i) {
            const double w = __shfl(v, i, kWave);
            tot = b == p0 && i == 0 ? w : tot + w;
        }
    }
    if (lane == 0) Y[(size_t)desc[li].r0 * k + j] = tot;
}

template <int KC, int U>
static void launch_tiles(const TileDesc *desc, int n, bool remap, const DevMatrix &M, const double *X, double *Y,
                         int k, int cap, hipStream_t st) {
    const int per_xcd = remap && n >= 16 ? (n + 7) / 8 : 0;
    const int chunk_log2 = M.xcd_chunk_log2;
    const int grid = xcd_grid(n, per_xcd, chunk_log2);
    const size_t lds = (size_t)cap * (sizeof(double) + sizeof(int32_t));
    const bool vec = KC >= 2 && k % 2 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_spmm_tiles<KC, U, true>), dim3(grid), dim3(kBlock), lds, st, desc, n, per_xcd,
                           chunk_log2, M.row_ptr, M.col, M.val64, X, Y, k, cap);
    else
        hipLaunchKernelGGL((k_spmm_tiles<KC, U, false>), dim3(grid), dim3(kBlock), lds, st, desc, n, per_xcd,
                           chunk_log2, M.row_ptr, M.col, M.val64, X, Y, k, cap);
}

hipError_t launch_spmm(const spmv_matrix *A, const double *X, double *Y, int k, hipStream_t st) {
    const DevMatrix &M = A->M;
    // one column: the single-vector product itself (compact windows where
    // the plan has them), which is the same sum
    if (k == 1) return launch_spmv<double, double, double, double>(M, M.val64, X, Y, EPI_PLAIN, nullptr, nullptr,
                                                                   nullptr, st);
    const int cap = std::max(A->max_tile_entries, 1);
    if (M.n_long > 0) {
        // first: the pieces' sums can live in Y's rows of the longest run
        // without a long row, which the row tiles below write afterwards
        if (M.piece_long && M.long_split && M.y_ws_rows >= M.n_long_pieces) {
            double *ws = Y + (size_t)M.y_ws_row * k;
            hipLaunchKernelGGL(k_spmm_long_pieces, dim3(M.n_long_pieces, k), dim3(kBlock), 0, st, M.long_desc,
                               M.piece_long, M.long_piece_ptr, M.col, M.val64, X, ws, k);
            constexpr int kRowsPerWg = kBlock / kWave;
            hipLaunchKernelGGL(k_spmm_long_combine, dim3((M.n_long + kRowsPerWg - 1) / kRowsPerWg, k), dim3(kBlock), 0,
                               st, M.long_desc, M.long_piece_ptr, ws, Y, M.n_long, k);
        } else {
            hipLaunchKernelGGL(k_spmm_long, dim3(M.n_long, k), dim3(kBlock), 0, st, M.long_desc, M.col, M.val64, X,
                               Y, k);
        }
    }
    const struct {
        const TileDesc *desc;
        int n;
    } lists[3] = {{M.stream_desc, M.n_stream}, {M.cwin_desc, M.n_cwin}, {M.win_desc, A->n_win_tiles}};
    for (const auto &l : lists) {
        if (l.n <= 0) continue;
        // two columns per lane for every k: the lanes sharing a row gather
        // its X row in 16-byte pieces side by side, so one gather
        // instruction touches half as many cache lines as with four
        // columns per lane (16M-row mesh matrix, k = 4 / 8 / 16: 1.10 /
        // 1.65 / 2.69 ms against 1.32 / 1.87 / 2.86 ms)
        launch_tiles<2, 8>(l.desc, l.n, M.xcd_remap, M, X, Y, k, cap, st);
    }
    return hipGetLastError();
}

}  // namespace spmvlib
