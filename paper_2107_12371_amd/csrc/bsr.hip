// 3x3 block-CSR product with k right-hand sides: Y = A X.
//
// A couples three unknowns per cell (u, v, w of the momentum equations,
// paper Sec. 2), so each stored entry is a dense 3x3 block and block row i
// holds cell i's neighbour blocks.  X and Y are row-major (3 n) x k, so the
// k values of one scalar row sit contiguously and one gather brings all k.
//
// One workgroup per tile of up to 85 block rows and 512 stored blocks:
// pass 1 stages the tile's block values (9 per block) and block columns in
// LDS with coalesced streaming loads; pass 2 gives each (block row, scalar
// row r) pair one lane, which walks the row's blocks in ascending order and
// accumulates its k outputs:  Y[3i+r][j] += sum_c a_rc * X[3 col + c][j].
// A block row with more than 512 blocks forms its own tile and reads its
// values straight from global memory.  Tiles go to XCDs in contiguous runs
// as in the scalar kernels.
#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"

namespace spmvlib {

template <typename V, typename T, int K>
__global__ __launch_bounds__(kBlock) void k_bsr3(BsrArgs<V, T> g) {
    __shared__ V sval[kBsrBlocks * 9];
    __shared__ int32_t scol[kBsrBlocks];
    const int b = blockIdx.x;
    const int li = g.per_xcd ? (b & 7) * g.per_xcd + (b >> 3) : b;
    if (li >= g.n_tiles) return;
    const int R0 = g.tiles[li], R1 = g.tiles[li + 1];
    const int q0 = g.brow_ptr[R0], q1 = g.brow_ptr[R1];
    const bool staged = (q1 - q0) <= kBsrBlocks;
    if (staged) {
        const V *__restrict__ src = g.val + 9 * (size_t)q0;
        const int nv = 9 * (q1 - q0);
        for (int i = (int)threadIdx.x; i < nv; i += kBlock) sval[i] = __builtin_nontemporal_load(src + i);
        for (int i = (int)threadIdx.x; i < q1 - q0; i += kBlock) scol[i] = __builtin_nontemporal_load(g.col + q0 + i);
    }
    __syncthreads();
    const int t = (int)threadIdx.x;
    if (t >= 3 * (R1 - R0)) return;
    const int br = R0 + t / 3, r = t % 3;
    T acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = T(0);
    const int a = g.brow_ptr[br], z = g.brow_ptr[br + 1];
    for (int q = a; q < z; ++q) {
        int bc;
        T v[3];
        if (staged) {
            bc = scol[q - q0];
            const V *s = sval + 9 * (q - q0) + 3 * r;
            v[0] = static_cast<T>(s[0]);
            v[1] = static_cast<T>(s[1]);
            v[2] = static_cast<T>(s[2]);
        } else {
            bc = g.col[q];
            const V *s = g.val + 9 * (size_t)q + 3 * r;
            v[0] = static_cast<T>(s[0]);
            v[1] = static_cast<T>(s[1]);
            v[2] = static_cast<T>(s[2]);
        }
        const T *__restrict__ xr = g.X + (size_t)(3 * bc) * g.ldx + g.off;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int j = 0; j < K; ++j) acc[j] += v[c] * xr[(size_t)c * g.ldx + j];
        }
    }
    T *__restrict__ yr = g.Y + (size_t)(3 * br + r) * g.ldy + g.off;
#pragma unroll
    for (int j = 0; j < K; ++j) yr[j] = acc[j];
}

template <typename V, typename T, int K>
static void launch_k(const DevMatrix &M, BsrArgs<V, T> g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_bsr3<V, T, K>), dim3(grid), dim3(kBlock), 0, st, g);
}

template <typename V, typename T>
hipError_t launch_bsr3(const DevMatrix &M, const V *val, int k, const T *X, T *Y, hipStream_t st) {
    if (M.n_bsr_tiles == 0 || k == 0) return hipSuccess;
    BsrArgs<V, T> g{};
    g.brow_ptr = M.row_ptr;
    g.col = M.col;
    g.val = val;
    g.X = X;
    g.Y = Y;
    g.tiles = M.bsr_tiles;
    g.n_tiles = M.n_bsr_tiles;
    g.ldx = k;
    g.ldy = k;
    int grid = M.n_bsr_tiles;
    g.per_xcd = 0;
    if (M.xcd_remap && M.n_bsr_tiles >= 16) {
        g.per_xcd = (M.n_bsr_tiles + 7) / 8;
        grid = 8 * g.per_xcd;
    }
    // right-hand sides in chunks of 8, 4, 2, 1 columns
    int off = 0;
    while (off < k) {
        const int rem = k - off;
        g.off = off;
        if (rem >= 8) { launch_k<V, T, 8>(M, g, grid, st); off += 8; }
        else if (rem >= 4) { launch_k<V, T, 4>(M, g, grid, st); off += 4; }
        else if (rem >= 2) { launch_k<V, T, 2>(M, g, grid, st); off += 2; }
        else { launch_k<V, T, 1>(M, g, grid, st); off += 1; }
    }
    return hipGetLastError();
}

template hipError_t launch_bsr3<double, double>(const DevMatrix &, const double *, int, const double *, double *,
                                                hipStream_t);
template hipError_t launch_bsr3<float, float>(const DevMatrix &, const float *, int, const float *, float *,
                                              hipStream_t);

}  // namespace spmvlib
