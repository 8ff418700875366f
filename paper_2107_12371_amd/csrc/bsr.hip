// 3x3 block-CSR product with k right-hand sides: Y = A X.
//
// A couples three unknowns per cell (u, v, w of the momentum equations,
// paper Sec. 2), so each stored entry is a dense 3x3 block and block row i
// holds cell i's neighbour blocks.  X and Y are row-major (3 n) x k, so the
// k values of one scalar row sit contiguously and one gather brings all k.
//
// One workgroup per tile of up to 84 block rows and 510 stored blocks (the
// staged values of four tiles fill one CU's LDS).
// Pass 1 stages the tile's block values (9 per block) and block columns in
// LDS: every lane issues all of its 16-byte loads (fixed count, addresses
// clamped to the tile) before the first LDS store, so the loads overlap.
// Pass 2, one column (k_bsr3_one): each lane owns one scalar row 3i+r, and
// the X gathers are issued while the value loads are in flight.  Pass 2, k >= 2
// columns: each lane owns a block row and K/JL adjacent columns of Y (JL
// lanes share the block row) and computes all three scalar rows, so every
// gathered X row is read once, in 8- or 16-byte pieces when aligned.  A
// lane walks its row's blocks U at a time: U column indices from LDS, then
// all gathers of X for those U blocks, then the accumulation in ascending
// block order, so only ceil(len/U) gather latencies are serial.  Out-of-row
// slots of the last group re-read the row's last block (valid addresses)
// and are discarded by a select, never by multiplying with zero, so Inf/NaN
// in X behave as in the definition.  A block row with more than 510 blocks
// forms its own tile and reads its values straight from global memory.
// Tiles go to XCDs in chunks as in the scalar kernels.
//
// Per output the sum is sum over blocks (ascending) of a_r0 x0 + a_r1 x1 +
// a_r2 x2, left to right, whatever K, JL and U are: a column of a k-column
// product equals the one-column product of that column bit for bit.
#include <hip/hip_runtime.h>

#include "bsr.h"
#include "device.h"

namespace spmvlib {

template <typename V> struct BsrStage {
    static constexpr int kVe = 16 / (int)sizeof(V);                           // values per 16-byte load
    static constexpr int kVecs = (kBsrBlocks * 9 + kVe - 1) / kVe + 1;        // + 1: unaligned start
    static constexpr int kTrips = (kVecs + kBlock - 1) / kBlock;
    static constexpr int kColVecs = (kBsrBlocks + 3) / 4 + 1;                // + 1: unaligned start
    static_assert(kColVecs <= kBlock, "one column load per lane");
};

// Pass-2 shape for K columns per launch: ROWS selects one lane per (block
// row, column group) computing all three scalar rows (K >= 2: each gathered
// X row is read once, with 16-byte loads when aligned) instead of one lane
// per (scalar row, column group); JL lanes share a row, U blocks per round.
// Measured on the 4M-block-row operator (FP64 / FP32 ms, k = 1, 4, 8):
// 0.643 / 0.402, 0.813 / 0.413, 1.199 / 0.588.
template <typename T, int K> struct BsrShape;
template <> struct BsrShape<double, 1> { static constexpr bool ROWS = false; static constexpr int JL = 1, U = 6, P = 12; };
template <> struct BsrShape<double, 2> { static constexpr bool ROWS = true; static constexpr int JL = 1, U = 3; };
template <> struct BsrShape<double, 4> { static constexpr bool ROWS = true; static constexpr int JL = 2, U = 4; };
template <> struct BsrShape<double, 8> { static constexpr bool ROWS = true; static constexpr int JL = 4, U = 2; };
template <> struct BsrShape<float, 1> { static constexpr bool ROWS = false; static constexpr int JL = 1, U = 4, P = 12; };
template <> struct BsrShape<float, 2> { static constexpr bool ROWS = true; static constexpr int JL = 1, U = 4; };
template <> struct BsrShape<float, 4> { static constexpr bool ROWS = true; static constexpr int JL = 4, U = 6; };
template <> struct BsrShape<float, 8> { static constexpr bool ROWS = true; static constexpr int JL = 8, U = 6; };

// KC adjacent values of one X or Y row; VEC: the address is aligned to the
// vector width (checked at launch), so they move in 8- or 16-byte pieces.
template <typename T, int KC, bool VEC> struct RowChunk {
    static constexpr int W = (VEC && KC > 1) ? (KC * (int)sizeof(T) >= 16 ? 16 / (int)sizeof(T) : KC) : 1;
    typedef T vt __attribute__((ext_vector_type(W)));
    __device__ __forceinline__ static void load(const T *p, T (&o)[KC]) {
        if constexpr (W == 1) {
#pragma unroll
            for (int j = 0; j < KC; ++j) o[j] = p[j];
        } else {
#pragma unroll
            for (int i = 0; i < KC; i += W) {
                const vt v = *reinterpret_cast<const vt *>(p + i);
#pragma unroll
                for (int w = 0; w < W; ++w) o[i + w] = v[w];
            }
        }
    }
    __device__ __forceinline__ static void store(T *p, const T (&o)[KC]) {
        if constexpr (W == 1) {
#pragma unroll
            for (int j = 0; j < KC; ++j) p[j] = o[j];
        } else {
#pragma unroll
            for (int i = 0; i < KC; i += W) {
                vt v;
#pragma unroll
                for (int w = 0; w < W; ++w) v[w] = o[i + w];
                *reinterpret_cast<vt *>(p + i) = v;
            }
        }
    }
};

// Pass 2, one lane per (scalar row, column group), for lanes [t] of one
// tile; VP/CP point into LDS (staged) or global memory.
template <typename V, typename T, int K, int JL, int U, typename VP, typename CP>
__device__ __forceinline__ void bsr_pairs(const BsrArgs<V, T> &g, int R0, int R1, int q0, VP vals, CP cols) {
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

// Pass 2, one column: three adjacent lanes (a triad) per block row, lane r
// computing scalar row 3 br + r.  Each lane gathers only x[3 bc + r] of a
// block and takes the block's other two x values from its triad siblings
// by lane shuffle, so a block costs one gather per lane instead of three
// (the three lanes used to fetch the same three words each).  A wavefront
// holds 21 triads (lane 63 idles), so a triad never straddles two
// wavefronts; its three lanes share the block row, hence the loop bounds,
// and take every shuffle together.  Same per-output sum as bsr_pairs.
template <typename V, typename T, int U, typename VP, typename CP>
__device__ __forceinline__ void bsr_triads(const BsrArgs<V, T> &g, int R0, int R1, int q0, VP vals, CP cols) {
    constexpr int kTriads = kWave / 3;                  // 21 per wavefront
    constexpr int kRowsPerPass = kTriads * (kBlock / kWave);
    const int lane = (int)threadIdx.x & (kWave - 1), wave = (int)threadIdx.x / kWave;
    const int r = lane % 3, first = lane - r;           // lane 63: r = 0, a triad of its own, never stored
    const int nbr = R1 - R0;
    for (int brl0 = wave * kTriads; brl0 < nbr; brl0 += kRowsPerPass) {
        const int brl = brl0 + lane / 3;
        const bool live = lane < 3 * kTriads && brl < nbr;
        const int br = R0 + min(brl, nbr - 1);
        const int a = g.brow_ptr[br], z = g.brow_ptr[br + 1];
        T acc = T(0);
        for (int q = a; q < z; q += U) {
            int qq[U];
            T xo[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                qq[u] = min(q + u, z - 1) - q0;
                xo[u] = g.X[(size_t)(3 * cols[qq[u]] + r) * g.ldx + g.off];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const T x0 = __shfl(xo[u], first, kWave);
                const T x1 = __shfl(xo[u], first + 1, kWave);
                const T x2 = __shfl(xo[u], first + 2, kWave);
                const T a0 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r]);
                const T a1 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r + 1]);
                const T a2 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r + 2]);
                const bool in_row = q + u < z;
                T s = acc;
                s += a0 * x0;
                s += a1 * x1;
                s += a2 * x2;
                acc = in_row ? s : acc;
            }
        }
        if (live) g.Y[(size_t)(3 * br + r) * g.ldy + g.off] = acc;
    }
}

// Pass 2, one lane per (block row, column group): the lane gathers each X
// row once and accumulates the three scalar rows of its block row.  Same
// per-output summation order as bsr_pairs.
template <typename V, typename T, int K, int JL, int U, bool VEC, typename VP, typename CP>
__device__ __forceinline__ void bsr_blockrows(const BsrArgs<V, T> &g, int R0, int R1, int q0, VP vals, CP cols) {
    constexpr int KC = K / JL;
    constexpr int kRowsPerPass = kBlock / JL;
    using RC = RowChunk<T, KC, VEC>;
    const int t = (int)threadIdx.x;
    const size_t xoff = (size_t)g.off + (size_t)(t % JL) * KC;
    for (int brl = t / JL; brl < R1 - R0; brl += kRowsPerPass) {
        const int br = R0 + brl;
        const int a = g.brow_ptr[br], z = g.brow_ptr[br + 1];
        T acc[3][KC];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int j = 0; j < KC; ++j) acc[r][j] = T(0);
        for (int q = a; q < z; q += U) {
            int qq[U];
            T xv[U][3][KC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                qq[u] = min(q + u, z - 1) - q0;
                const int bc = cols[qq[u]];
#pragma unroll
                for (int c = 0; c < 3; ++c) RC::load(g.X + (size_t)(3 * bc + c) * g.ldx + xoff, xv[u][c]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in_row = q + u < z;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const T a0 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r]);
                    const T a1 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r + 1]);
                    const T a2 = static_cast<T>(vals[9 * (size_t)qq[u] + 3 * r + 2]);
#pragma unroll
                    for (int j = 0; j < KC; ++j) {
                        T s = acc[r][j];
                        s += a0 * xv[u][0][j];
                        s += a1 * xv[u][1][j];
                        s += a2 * xv[u][2][j];
                        acc[r][j] = in_row ? s : acc[r][j];
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) RC::store(g.Y + (size_t)(3 * br + r) * g.ldy + xoff, acc[r]);
    }
}

template <typename V, typename T, int K, bool VEC, typename VP, typename CP>
__device__ __forceinline__ void bsr_pass2(const BsrArgs<V, T> &g, int R0, int R1, int q0, VP vals, CP cols) {
    using Sh = BsrShape<T, K>;
    static_assert(K % Sh::JL == 0, "column groups must split K");
    if constexpr (Sh::ROWS) bsr_blockrows<V, T, K, Sh::JL, Sh::U, VEC>(g, R0, R1, q0, vals, cols);
    else if constexpr (K == 1) bsr_triads<V, T, Sh::U>(g, R0, R1, q0, vals, cols);
    else bsr_pairs<V, T, K, Sh::JL, Sh::U>(g, R0, R1, q0, vals, cols);
}

template <typename V, typename T, int K, bool VEC>
__global__ __launch_bounds__(kBlock) void k_bsr3(BsrArgs<V, T> g) {
    using S = BsrStage<V>;
    __shared__ i32x4 sval_raw[S::kTrips * kBlock];
    __shared__ i32x4 scol_raw[S::kColVecs];
    const int li = xcd_tile(blockIdx.x, g.per_xcd, g.chunk_log2);
    if (li >= g.n_tiles) return;
    const int t = (int)threadIdx.x;
    const int R0 = g.tiles[li], R1 = g.tiles[li + 1];
    const int q0 = g.brow_ptr[R0], q1 = g.brow_ptr[R1];
    if (q1 - q0 > kBsrBlocks) {  // one long block row: values from global memory
        bsr_pass2<V, T, K, VEC>(g, R0, R1, q0, g.val + 9 * (size_t)q0, g.col + q0);
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
    // the block-column load first, taken while the value loads are still in
    // flight (loads complete in issue order)
    i32x4 tc = __builtin_nontemporal_load(csrc + min(t, ncv - 1));
    i32x4 tv[S::kTrips];
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) tv[i] = __builtin_nontemporal_load(vsrc + min(t + i * kBlock, nvv - 1));
    asm volatile("" : "+v"(tc));
    if (t < S::kColVecs) scol_raw[t] = tc;
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) sval_raw[t + i * kBlock] = tv[i];
    __syncthreads();
    const V *sval = reinterpret_cast<const V *>(sval_raw) + vshift;
    const int32_t *scol = reinterpret_cast<const int32_t *>(scol_raw) + cshift;
    bsr_pass2<V, T, K, VEC>(g, R0, R1, q0, sval, scol);
}

// One column, gathers in flight with the value stream.  Every lane issues
// its block row's bounds, then the tile's block-column load, then its value
// loads; as soon as the columns are in LDS (one barrier, values still in
// flight) each triad lane issues the X gathers of its row's first P blocks
// and only then waits for the values, so the gathers' round trip overlaps
// the stream instead of following it.  Blocks past the first P are
// gathered afterwards, U at a time.  Same per-output sum as bsr_triads.
template <typename V, typename T>
__global__ __launch_bounds__(kBlock) void k_bsr3_one(BsrArgs<V, T> g) {
    using S = BsrStage<V>;
    constexpr int P = BsrShape<T, 1>::P, U = BsrShape<T, 1>::U;
    constexpr int kTriads = kWave / 3;
    static_assert(kTriads * (kBlock / kWave) >= kBsrRows, "one triad per block row of a tile");
    __shared__ i32x4 sval_raw[S::kTrips * kBlock];
    __shared__ i32x4 scol_raw[S::kColVecs];
    const int li = xcd_tile(blockIdx.x, g.per_xcd, g.chunk_log2);
    if (li >= g.n_tiles) return;
    const int t = (int)threadIdx.x;
    const int lane = t & (kWave - 1);
    const int r = lane % 3, first = lane - r;  // lane 63: r = 0, a triad of its own, never stored
    const int R0 = g.tiles[li], R1 = g.tiles[li + 1];
    const int nbr = R1 - R0;
    const int brl = (t / kWave) * kTriads + lane / 3;
    const bool live = lane < 3 * kTriads && brl < nbr;
    const int br = R0 + min(brl, nbr - 1);
    const int q0 = g.brow_ptr[R0], q1 = g.brow_ptr[R1];
    if (q1 - q0 > kBsrBlocks) {  // one long block row: values from global memory
        bsr_triads<V, T, U>(g, R0, R1, q0, g.val + 9 * (size_t)q0, g.col + q0);
        return;
    }
    T *const yr = g.Y + (size_t)(3 * br + r) * g.ldy + g.off;
    if (q1 == q0) {  // only empty block rows
        if (live) *yr = T(0);
        return;
    }
    // Pass 1, issued in this order: row bounds, block columns, values (the
    // padding and alignment rules of k_bsr3 apply).
    int a = g.brow_ptr[br], z = g.brow_ptr[br + 1];
    const int32_t *cbase = g.col + q0;
    const int cshift = (int)(((uintptr_t)cbase & 15) / 4);
    const i32x4 *csrc = reinterpret_cast<const i32x4 *>(cbase - cshift);
    const int ncv = max((q1 - q0 + cshift + 3) / 4, 1);
    i32x4 tc = __builtin_nontemporal_load(csrc + min(t, ncv - 1));
    const V *vbase = g.val + 9 * (size_t)q0;
    const int vshift = (int)(((uintptr_t)vbase & 15) / sizeof(V));
    const i32x4 *vsrc = reinterpret_cast<const i32x4 *>(vbase - vshift);
    const int nvv = max((9 * (q1 - q0) + vshift + S::kVe - 1) / S::kVe, 1);
    i32x4 tv[S::kTrips];
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) tv[i] = __builtin_nontemporal_load(vsrc + min(t + i * kBlock, nvv - 1));
    // Take the bounds and columns here, with the value loads still in flight
    // (loads complete in issue order, so this waits for the first two only).
    asm volatile("" : "+v"(a), "+v"(z), "+v"(tc));
    if (t < S::kColVecs) scol_raw[t] = tc;
    __syncthreads();
    const int32_t *scol = reinterpret_cast<const int32_t *>(scol_raw) + cshift;
    // Gathers of the first P blocks.  An empty row reads the tile's first
    // block (valid, discarded below); past the row's end the last block.
    const int lo = z > a ? a - q0 : 0, hi = z > a ? z - 1 - q0 : 0;
    T xo[P];
#pragma unroll
    for (int u = 0; u < P; ++u) xo[u] = g.X[(size_t)(3 * scol[min(lo + u, hi)] + r) * g.ldx + g.off];
#pragma unroll
    for (int i = 0; i < S::kTrips; ++i) sval_raw[t + i * kBlock] = tv[i];
    __syncthreads();
    const V *sval = reinterpret_cast<const V *>(sval_raw) + vshift;
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int qq = min(lo + u, hi);
        const T x0 = __shfl(xo[u], first, kWave);
        const T x1 = __shfl(xo[u], first + 1, kWave);
        const T x2 = __shfl(xo[u], first + 2, kWave);
        const T a0 = static_cast<T>(sval[9 * qq + 3 * r]);
        const T a1 = static_cast<T>(sval[9 * qq + 3 * r + 1]);
        const T a2 = static_cast<T>(sval[9 * qq + 3 * r + 2]);
        const bool in_row = a + u < z;
        T s = acc;
        s += a0 * x0;
        s += a1 * x1;
        s += a2 * x2;
        acc = in_row ? s : acc;
    }
    // the rest of a row longer than P blocks (a triad's lanes share it)
    for (int q = a + P; q < z; q += U) {
        int qq[U];
        T xg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            qq[u] = min(q + u, z - 1) - q0;
            xg[u] = g.X[(size_t)(3 * scol[qq[u]] + r) * g.ldx + g.off];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T x0 = __shfl(xg[u], first, kWave);
            const T x1 = __shfl(xg[u], first + 1, kWave);
            const T x2 = __shfl(xg[u], first + 2, kWave);
            const T a0 = static_cast<T>(sval[9 * qq[u] + 3 * r]);
            const T a1 = static_cast<T>(sval[9 * qq[u] + 3 * r + 1]);
            const T a2 = static_cast<T>(sval[9 * qq[u] + 3 * r + 2]);
            const bool in_row = q + u < z;
            T s = acc;
            s += a0 * x0;
            s += a1 * x1;
            s += a2 * x2;
            acc = in_row ? s : acc;
        }
    }
    if (live) *yr = acc;
}

template <typename V, typename T, int K>
static void launch_k(BsrArgs<V, T> g, int grid, hipStream_t st) {
    // vector moves of X/Y rows need 16-byte aligned rows and column offsets
    constexpr int kW = 16 / (int)sizeof(T);
    if constexpr (K > 1) {
        const bool vec = ((reinterpret_cast<uintptr_t>(g.X) | reinterpret_cast<uintptr_t>(g.Y)) & 15) == 0 &&
                         g.ldx % kW == 0 && g.ldy % kW == 0 && g.off % kW == 0;
        if (vec) {
            hipLaunchKernelGGL((k_bsr3<V, T, K, true>), dim3(grid), dim3(kBlock), 0, st, g);
            return;
        }
    }
    if constexpr (K == 1) hipLaunchKernelGGL((k_bsr3_one<V, T>), dim3(grid), dim3(kBlock), 0, st, g);
    else hipLaunchKernelGGL((k_bsr3<V, T, K, false>), dim3(grid), dim3(kBlock), 0, st, g);
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
    g.per_xcd = M.xcd_remap && M.n_bsr_tiles >= 16 ? (M.n_bsr_tiles + 7) / 8 : 0;
    g.chunk_log2 = M.xcd_chunk_log2;
    const int grid = xcd_grid(M.n_bsr_tiles, g.per_xcd, g.chunk_log2);
    // right-hand sides in chunks of 8, 4, 2, 1 columns
    int off = 0;
    while (off < k) {
        const int rem = k - off;
        g.off = off;
        if (rem >= 8) { launch_k<V, T, 8>(g, grid, st); off += 8; }
        else if (rem >= 4) { launch_k<V, T, 4>(g, grid, st); off += 4; }
        else if (rem >= 2) { launch_k<V, T, 2>(g, grid, st); off += 2; }
        else { launch_k<V, T, 1>(g, grid, st); off += 1; }
    }
    return hipGetLastError();
}

template hipError_t launch_bsr3<double, double>(const DevMatrix &, const double *, int, const double *, double *,
                                                hipStream_t);
template hipError_t launch_bsr3<float, float>(const DevMatrix &, const float *, int, const float *, float *,
                                              hipStream_t);

}  // namespace spmvlib
