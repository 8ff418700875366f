// 3x3 block-CSR product with k right-hand sides: Y = A X.
//
// A couples three unknowns per cell (u, v, w of the momentum equations,
// paper Sec. 2), so each stored entry is a dense 3x3 block and block row i
// holds cell i's neighbour blocks.  X and Y are row-major (3 n) x k, so the
// k values of one scalar row sit contiguously and one gather brings all k.
//
// One workgroup per tile of up to 85 block rows and 510 stored blocks (the
// staged values of four tiles fill one CU's LDS).
// Pass 1 stages the tile's block values (9 per block) and block columns in
// LDS: every lane issues all of its 16-byte loads (fixed count, addresses
// clamped to the tile) before the first LDS store, so the loads overlap.
// Pass 2 gives each (scalar row, column group) one lane: JL lanes share a
// scalar row 3i+r and each owns K/JL adjacent columns of Y, so the JL lanes
// read one contiguous piece of each gathered X row.  A lane walks its row's
// blocks U at a time: U column indices and 3U values from LDS, then all 3U
// gathers of X, then the accumulation in ascending block order, so only
// ceil(len/U) gather latencies are serial.  Out-of-row slots of the last
// group re-read the row's last block (valid addresses) and are discarded
// by a select, never by multiplying with zero, so Inf/NaN in X behave as
// in the definition.  A block row with more than 510 blocks forms its own
// tile and reads its values straight from global memory.  Tiles go to XCDs
// in contiguous runs as in the scalar kernels.
//
// Per output the sum is sum over blocks (ascending) of a_r0 x0 + a_r1 x1 +
// a_r2 x2, left to right, whatever K, JL and U are: a column of a k-column
// product equals the one-column product of that column bit for bit.
#include <hip/hip_runtime.h>

#include "device.h"
#include "bsr.h"
#include "launch.h"

namespace spmvlib {

template <typename V> struct BsrStage {
    static constexpr int kVe = 16 / (int)sizeof(V);                           // values per 16-byte load
    static constexpr int kVecs = (kBsrBlocks * 9 + kVe - 1) / kVe + 1;        // + 1: unaligned start
    static constexpr int kTrips = (kVecs + kBlock - 1) / kBlock;
    static constexpr int kColVecs = (kBsrBlocks + 3) / 4 + 1;                // + 1: unaligned start
    static_assert(kColVecs <= kBlock, "one column load per lane");
};

// Pass-2 shapes (blocks per gather round U, lanes per scalar row JL) for
// k = 1, 2, 4, 8 columns per launch.
constexpr int kBsrU1 = 6, kBsrU2 = 4, kBsrU4 = 4, kBsrJL4 = 4, kBsrU8 = 4, kBsrJL8 = 4;

// Pass 2 for lanes [t] of one tile; VP/CP point into LDS (staged) or global.
template <typename V, typename T, int K, int JL, int U, typename VP, typename CP>
__device__ __forceinline__ void bsr_rows(const BsrArgs<V, T> &g, int R0, int R1, int q0, VP vals, CP cols) {
    constexpr int KC = K / JL;             // columns per lane
    constexpr int kPairsPerPass = kBlock / JL;
    const int t = (int)threadIdx.x;
    const int jl = t % JL;
    const int npairs = 3 * (R1 - R0);
    for (int pr = t / JL; pr < npairs; pr += kPairsPerPass) {
        const int br = R0 + pr / 3, r = pr % 3;
        const int a = g.brow_ptr[br], z = g.brow_ptr[br + 1];
        T acc[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = T(0);
        const size_t xoff = (size_t)g.off + (size_t)jl * KC;
        for (int q = a; q < z; q += U) {
            int bc[U];
            T v[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int qq = min(q + u, z - 1) - q0;
                bc[u] = cols[qq];
#pragma unroll
                for (int c = 0; c < 3; ++c) v[u][c] = static_cast<T>(vals[9 * (size_t)qq + 3 * r + c]);
            }
            T xv[U][3][KC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T *__restrict__ xr = g.X + (size_t)(3 * bc[u] + c) * g.ldx + xoff;
#pragma unroll
                    for (int j = 0; j < KC; ++j) xv[u][c][j] = xr[j];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in_row = q + u < z;
#pragma unroll
                for (int j = 0; j < KC; ++j) {
                    T s = acc[j];
                    s += v[u][0] * xv[u][0][j];
                    s += v[u][1] * xv[u][1][j];
                    s += v[u][2] * xv[u][2][j];
                    acc[j] = in_row ? s : acc[j];
                }
            }
        }
        T *__restrict__ yr = g.Y + (size_t)(3 * br + r) * g.ldy + xoff;
#pragma unroll
        for (int j = 0; j < KC; ++j) yr[j] = acc[j];
    }
}

template <typename V, typename T, int K, int JL, int U>
__global__ __launch_bounds__(kBlock) void k_bsr3(BsrArgs<V, T> g) {
    using S = BsrStage<V>;
    __shared__ i32x4 sval_raw[S::kTrips * kBlock];
    __shared__ i32x4 scol_raw[S::kColVecs];
    const int b = blockIdx.x;
    const int li = g.per_xcd ? (b & 7) * g.per_xcd + (b >> 3) : b;
    if (li >= g.n_tiles) return;
    const int t = (int)threadIdx.x;
    const int R0 = g.tiles[li], R1 = g.tiles[li + 1];
    const int q0 = g.brow_ptr[R0], q1 = g.brow_ptr[R1];
    if (q1 - q0 > kBsrBlocks) {  // one long block row: values from global memory
        bsr_rows<V, T, K, JL, U>(g, R0, R1, q0, g.val + 9 * (size_t)q0, g.col + q0);
        return;
    }
    // Pass 1.  The arrays carry 16 elements of padding past the last block,
    // so the rounded-up last vector stays inside the allocation; rounding
    // the start down stays inside because allocations are 256-byte aligned.
    const V *vbase = g.val + 9 * (size_t)q0;
    const int vshift = (int)(((uintptr_t)vbase & 15) / sizeof(V));
    const i32x4 *vsrc = reinterpret_cast<const i32x4 *>(vbase - vshift);
    const int nvv = max((9 * (q1 - q0) + vshift + S::kVe - 1) / S::kVe, 1);
    const int32_t *cbase = g.col + q0;
    const int cshift = (int)(((uintptr_t)cbase & 15) / 4);
    const i32x4 *csrc = reinterpret_cast<const i32x4 *>(cbase - cshift);
    const int ncv = max((q1 - q0 + cshift + 3) / 4, 1);
    i32x4 tv[S::kTrips];
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) tv[i] = __builtin_nontemporal_load(vsrc + min(t + i * kBlock, nvv - 1));
    const i32x4 tc = __builtin_nontemporal_load(csrc + min(t, ncv - 1));
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) sval_raw[t + i * kBlock] = tv[i];
    if (t < S::kColVecs) scol_raw[t] = tc;
    __syncthreads();
    const V *sval = reinterpret_cast<const V *>(sval_raw) + vshift;
    const int32_t *scol = reinterpret_cast<const int32_t *>(scol_raw) + cshift;
    bsr_rows<V, T, K, JL, U>(g, R0, R1, q0, sval, scol);
}

template <typename V, typename T, int K, int JL, int U>
static void launch_k(BsrArgs<V, T> g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_bsr3<V, T, K, JL, U>), dim3(grid), dim3(kBlock), 0, st, g);
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
        if (rem >= 8) { launch_k<V, T, 8, kBsrJL8, kBsrU8>(g, grid, st); off += 8; }
        else if (rem >= 4) { launch_k<V, T, 4, kBsrJL4, kBsrU4>(g, grid, st); off += 4; }
        else if (rem >= 2) { launch_k<V, T, 2, 2, kBsrU2>(g, grid, st); off += 2; }
        else { launch_k<V, T, 1, 1, kBsrU1>(g, grid, st); off += 1; }
    }
    return hipGetLastError();
}

template hipError_t launch_bsr3<double, double>(const DevMatrix &, const double *, int, const double *, double *,
                                                hipStream_t);
template hipError_t launch_bsr3<float, float>(const DevMatrix &, const float *, int, const float *, float *,
                                              hipStream_t);

}  // namespace spmvlib
