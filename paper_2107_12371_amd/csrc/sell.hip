// Sliced ELLPACK (SELL-C-sigma, C = 64): one wavefront per slice and one
// lane per row, the paper's column-wise slices (Sec. 4.2, 5.2) mapped onto a
// wavefront instead of an FPGA pipeline.  Entry j of lane l sits at
// slice_ptr[s] + 64 j + l, so every step of j is one coalesced 256-byte
// column load and one value load of 64 entries per wavefront.
//
// A lane walks j in groups of U with clamped addresses.  The loop is
// software-pipelined: the next group's column and value loads are issued
// before the current group's gathers are consumed, so the matrix stream
// stays in flight behind the gathers.  Each product is added in ascending j
// only while j < the row's length: padding is masked, never multiplied, so
// Inf/NaN in x behave as in the definition.  Products are rounded before
// they are added (no fused multiply-add), the arithmetic of the CSR row
// tiles, so a SELL handle gives the same bits as a CSR handle.
#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"
#include "sell.h"
#include "tile.h"

namespace spmvlib {

template <typename A> __device__ __forceinline__ A add_product(A sum, A a, A b) {
#pragma clang fp contract(off)
    const A p = a * b;
    return sum + p;
}

template <typename V, int U> struct SellGroup {
    int c[U];
    V v[U];
    __device__ __forceinline__ void load(const int32_t *__restrict__ col, const V *__restrict__ val, int base,
                                         int j, int width, int lane) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = base + min(j + u, width - 1) * kWave + lane;
            c[u] = stream_load<StreamNT<V>::value>(col + k);
            v[u] = stream_load<StreamNT<V>::value>(val + k);
        }
    }
};

template <typename V, typename X, typename Y, typename A, int EPI>
__global__ __launch_bounds__(kBlock) void k_sell(SpmvArgs<V, X, Y> g) {
    __shared__ double sh[kBlock / kWave];
    if (g.done && *g.done) return;
    const int li = xcd_tile(blockIdx.x, g.per_xcd, g.chunk_log2);
    if (li >= g.n_list) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int sl = li * (kBlock / kWave) + (int)threadIdx.x / kWave;
    double dot = 0.0;
    if (sl < g.n_slices) {
        const int slot = sl * kWave + lane;
        const int row = g.sell_perm[slot];
        const int len = g.sell_len[slot];
        const int base = g.sell_ptr[sl];
        const int width = (g.sell_ptr[sl + 1] - base) / kWave;
        const int rr = row >= 0 ? row : 0;
        Y op = Y(0);
        if (EPI == EPI_DOT) op = static_cast<Y>(g.x[rr]);
        else if (EPI == EPI_RESID) op = g.b[rr];
        A sum = A(0);
        constexpr int U = 8;
        if (width > 0) {
            SellGroup<V, U> cur;
            cur.load(g.col, g.val, base, 0, width, lane);
            for (int j = 0; j < width; j += U) {
                A xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) xv[u] = static_cast<A>(g.x[cur.c[u]]);
                // next group's stream (past the end it re-reads the last group: L1 hits)
                SellGroup<V, U> nxt;
                nxt.load(g.col, g.val, base, j + U, width, lane);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const A t = add_product<A>(sum, to_acc<A>(cur.v[u]), xv[u]);
                    sum = j + u < len ? t : sum;
                }
                cur = nxt;
            }
        }
        if (row >= 0) {
            if (EPI == EPI_RESID) {
                const Y res = static_cast<Y>(op - static_cast<Y>(sum));
                g.y[row] = res;
                dot = static_cast<double>(res) * static_cast<double>(res);
            } else {
                g.y[row] = static_cast<Y>(sum);
                if (EPI == EPI_DOT) dot = static_cast<double>(sum) * static_cast<double>(op);
            }
        }
    }
    if (EPI != EPI_PLAIN) {
        const double t = block_sum(dot, sh);
        if (threadIdx.x == 0) g.part[li] = t;
    }
}

template <typename V, typename X, typename Y, typename A>
void launch_sell_slices(const DevMatrix &M, SpmvArgs<V, X, Y> g, int epi, hipStream_t st) {
    SpmvArgs<V, X, Y> a = g;
    a.n_list = M.n_sell_wg;
    a.sell_perm = M.sell_perm;
    a.sell_len = M.sell_len;
    a.sell_ptr = M.sell_ptr;
    a.n_slices = M.n_slices;
    a.per_xcd = M.xcd_remap && M.n_sell_wg >= 16 ? (M.n_sell_wg + 7) / 8 : 0;
    a.chunk_log2 = M.xcd_chunk_log2;
    const int grid = xcd_grid(M.n_sell_wg, a.per_xcd, a.chunk_log2);
    switch (epi) {
        case EPI_DOT: hipLaunchKernelGGL((k_sell<V, X, Y, A, EPI_DOT>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case EPI_RESID: hipLaunchKernelGGL((k_sell<V, X, Y, A, EPI_RESID>), dim3(grid), dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL((k_sell<V, X, Y, A, EPI_PLAIN>), dim3(grid), dim3(kBlock), 0, st, a); break;
    }
}

template void launch_sell_slices<double, double, double, double>(const DevMatrix &,
                                                                 SpmvArgs<double, double, double>, int,
                                                                 hipStream_t);
template void launch_sell_slices<float, float, float, float>(const DevMatrix &, SpmvArgs<float, float, float>,
                                                             int, hipStream_t);
template void launch_sell_slices<float, double, double, double>(const DevMatrix &,
                                                                SpmvArgs<float, double, double>, int,
                                                                hipStream_t);
template void launch_sell_slices<uint16_t, float, float, float>(const DevMatrix &,
                                                                SpmvArgs<uint16_t, float, float>, int,
                                                                hipStream_t);

}  // namespace spmvlib
