// Row-tile building blocks shared by the SpMV kernels and the server's
// multi-matrix kernel: streaming a tile's entries into registers, gathering
// x, writing products to LDS, and the per-row sums with their epilogues.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace spmvlib {

template <typename A, typename V> __device__ __forceinline__ A to_acc(V v) { return static_cast<A>(v); }
template <> __device__ __forceinline__ float to_acc<float, uint16_t>(uint16_t v) {
    return __uint_as_float(static_cast<unsigned>(v) << 16);
}

// A tile's stored entries [s, e) held in registers: each lane owns 4
// consecutive entries per pass (16-byte loads), s4 = s & ~3 aligns the
// first pass.  The code is straight-line on purpose: a lane whose group
// lies past the tile re-reads the tile's last group (an L1 hit) and every
// gather is issued unconditionally (every padded column index is valid), so
// the compiler can count outstanding loads exactly and keep all of a lane's
// loads, then all of its gathers, in flight at once.
template <typename V, int NT, int LANES = kBlock> struct TileRegs {
    static constexpr int kPass = kEntriesPerLane * LANES;
    // the plan keeps e - s4 <= NT (at most NT - 3 entries per tile)
    static constexpr int kMaxPass = NT / kPass;
    static_assert(NT % kPass == 0, "tile capacity must be a whole number of passes");
    i32x4 c[kMaxPass];
    Val4<V> v[kMaxPass];

    __device__ __forceinline__ void load(const int32_t *__restrict__ col, const V *__restrict__ val, int s, int e) {
        const int s4 = s & ~3;
        const int last = e > s4 ? ((e - 1) & ~3) : s4;  // last group of the tile
        const int lane0 = kEntriesPerLane * (threadIdx.x & (LANES - 1));
        // column indices of every pass first: the gathers depend only on
        // them, and loads complete in issue order, so the gathers can start
        // while the values are still streaming in
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) c[p] = load_col4<V>(col + min(s4 + p * kPass + lane0, last));
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) v[p].load(val + min(s4 + p * kPass + lane0, last));
    }

    // x[c] for every loaded entry (entries outside [s, e) are never used)
    template <typename A, class Gather>
    __device__ __forceinline__ void gather(Gather g, A (&xv)[kMaxPass][4]) const {
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[p][j] = static_cast<A>(g(c[p][j]));
        }
    }

    // products a_k * x[c_k] into prod[p * kPass + 4 * lane + j] = prod[k - s4]
    // for every loaded entry; prod holds kProd entries, so the stores need no
    // predicate (a predicate would let the compiler sink the gathers into it).
    // Positions outside [s - s4, e - s4) hold junk that pass 2 never reads.
    static constexpr int kProd = kMaxPass * kPass;
    template <typename A>
    __device__ __forceinline__ void products(const A (&xv)[kMaxPass][4], A *__restrict__ prod) const {
        const int lane0 = kEntriesPerLane * (threadIdx.x & (LANES - 1));
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
            A *d = prod + p * kPass + lane0;
            d[0] = to_acc<A>(v[p].template get<0>()) * xv[p][0];
            d[1] = to_acc<A>(v[p].template get<1>()) * xv[p][1];
            d[2] = to_acc<A>(v[p].template get<2>()) * xv[p][2];
            d[3] = to_acc<A>(v[p].template get<3>()) * xv[p][3];
        }
    }
};

// A compact-window tile's stored entries: 16-bit window positions (8 bytes
// per 4 entries) and values, streamed like TileRegs with clamped addresses.
template <typename V, int NT> struct WinTileRegs {
    static constexpr int kPass = kEntriesPerLane * kBlock;
    static constexpr int kMaxPass = NT / kPass;
    static constexpr int kProd = kMaxPass * kPass;
    static_assert(NT % kPass == 0, "tile capacity must be a whole number of passes");
    u32x2 w[kMaxPass];
    Val4<V> v[kMaxPass];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ lidx, const uint32_t *__restrict__ /*lidx12*/,
                                         const V *__restrict__ val, int /*tile*/, int s, int e) {
        const int s4 = s & ~3;
        const int last = e > s4 ? ((e - 1) & ~3) : s4;
        const int lane0 = kEntriesPerLane * threadIdx.x;
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p)
            w[p] = stream_load<StreamNT<V>::value>(
                reinterpret_cast<const u32x2 *>(lidx + min(s4 + p * kPass + lane0, last)));
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) v[p].load(val + min(s4 + p * kPass + lane0, last));
    }

    // products a_k * win[pos_k] (window in LDS) into registers.  Entries
    // outside [s, e) belong to other tiles and read position 0 instead, so
    // every LDS read stays inside this tile's window.
    template <typename A>
    __device__ __forceinline__ void products(int s, int e, const A *__restrict__ win,
                                             A (&pr)[kMaxPass][4]) const {
        const int s4 = s & ~3;
        const int lane0 = kEntriesPerLane * threadIdx.x;
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
            const int k = s4 + p * kPass + lane0;
            const unsigned pos[4] = {w[p][0] & 0xffffu, w[p][0] >> 16, w[p][1] & 0xffffu, w[p][1] >> 16};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = k + j >= s && k + j < e;
                pr[p][j] = to_acc<A>(v[p].get_dyn(j)) * win[in ? pos[j] : 0u];
            }
        }
    }

    template <typename A>
    __device__ __forceinline__ void store(const A (&pr)[kMaxPass][4], A *__restrict__ prod) const {
        const int lane0 = kEntriesPerLane * threadIdx.x;
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
            A *d = prod + p * kPass + lane0;
            d[0] = pr[p][0];
            d[1] = pr[p][1];
            d[2] = pr[p][2];
            d[3] = pr[p][3];
        }
    }
};

// Compact-window positions for 2048-entry tiles packed in 12 bits each (a
// window holds at most 2048 words): lane l of the t-th window tile owns the
// positions of its 8 entries (2 passes x 4) in the three 32-bit words at
// lidx12[3 * (t * 256 + l)], entry m in bits [12m, 12m + 12) of the 96.
// 1.5 instead of 2 bytes per entry; the layout is indexed by tile, not by
// entry, so an entry outside the tile owns no bits and reads position 0.
template <typename V> struct WinTileRegs12 {
    static constexpr int kPass = kEntriesPerLane * kBlock;
    static constexpr int kMaxPass = 2;
    static constexpr int kProd = kMaxPass * kPass;
    uint32_t w0, w1, w2;
    Val4<V> v[kMaxPass];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ /*lidx*/, const uint32_t *__restrict__ lidx12,
                                         const V *__restrict__ val, int tile, int s, int e) {
        const int s4 = s & ~3;
        const int last = e > s4 ? ((e - 1) & ~3) : s4;
        const int lane0 = kEntriesPerLane * threadIdx.x;
        // positions are read once per product: non-temporal (measured 0.6%
        // faster on the 16M-row mesh matrix; the values non-temporal were
        // 10% slower, so they keep the type's policy)
        const uint32_t *q = lidx12 + 3 * ((size_t)tile * kBlock + threadIdx.x);
        w0 = stream_load<true>(q);
        w1 = stream_load<true>(q + 1);
        w2 = stream_load<true>(q + 2);
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) v[p].load(val + min(s4 + p * kPass + lane0, last));
    }

    template <int M> __device__ __forceinline__ unsigned pos() const {
        if constexpr (M < 5) {
            const uint64_t a = (uint64_t)w0 | ((uint64_t)w1 << 32);
            return (unsigned)(a >> (12 * M)) & 0xfffu;
        } else {
            const uint64_t b = (uint64_t)w1 | ((uint64_t)w2 << 32);
            return (unsigned)(b >> (12 * M - 32)) & 0xfffu;
        }
    }

    template <typename A>
    __device__ __forceinline__ void products(int s, int e, const A *__restrict__ win,
                                             A (&pr)[kMaxPass][4]) const {
        const unsigned ps[8] = {pos<0>(), pos<1>(), pos<2>(), pos<3>(), pos<4>(), pos<5>(), pos<6>(), pos<7>()};
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
#pragma unroll
            for (int j = 0; j < 4; ++j) pr[p][j] = to_acc<A>(v[p].get_dyn(j)) * win[ps[4 * p + j]];
        }
    }

    template <typename A>
    __device__ __forceinline__ void store(const A (&pr)[kMaxPass][4], A *__restrict__ prod) const {
        const int lane0 = kEntriesPerLane * threadIdx.x;
#pragma unroll
        for (int p = 0; p < kMaxPass; ++p) {
            A *d = prod + p * kPass + lane0;
            d[0] = pr[p][0];
            d[1] = pr[p][1];
            d[2] = pr[p][2];
            d[3] = pr[p][3];
        }
    }
};

// The compact-window register set of a tile capacity: packed 12-bit
// positions for 2048-entry tiles, 16-bit positions otherwise.
template <typename V, int NT> struct CwinRegsSel { using type = WinTileRegs<V, NT>; };
template <typename V> struct CwinRegsSel<V, 2048> { using type = WinTileRegs12<V>; };

// Pass 2 inputs, loaded early (before the gathers and any prefetch, so
// waiting for them never drains loads issued later): each lane's rows
// r0 + lane and r0 + lane + 256 (tiles hold at most 512 rows), their entry
// ranges relative to s4 and the epilogue operand (x_r for the p.q partial,
// b_r for the residual).  Indices are clamped into the tile so the loads are
// unconditional.
template <typename Y, int EPI, int LANES = kBlock> struct RowPre {
    int a[2], z[2];
    Y op[2];

    template <typename X>
    __device__ __forceinline__ void load(const int32_t *__restrict__ row_ptr, const X *__restrict__ x,
                                         const Y *__restrict__ b, int r0, int r1, int s4) {
        const int lane = threadIdx.x & (LANES - 1);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = min(r0 + lane + i * LANES, r1 - 1);
            a[i] = row_ptr[r] - s4;
            z[i] = row_ptr[r + 1] - s4;
            if (EPI == EPI_DOT) op[i] = static_cast<Y>(x[r]);
            else if (EPI == EPI_RESID) op[i] = b[r];
            else op[i] = Y(0);
        }
    }
};

// Pass 2: per-row sums of the tile's rows [r0, r1) in ascending entry
// order, epilogue, optional per-tile partial (fixed-shape reduction).
// Row sums for a tile worked by LANES lanes (256: a workgroup, reduced with
// block_sum; 64: one wavefront, reduced with wave_sum, sh unused).
template <typename Y, typename A, int EPI, int LANES = kBlock>
__device__ __forceinline__ void tile_rows(const RowPre<Y, EPI, LANES> &pre, int r0, int r1,
                                          const A *__restrict__ prod, Y *__restrict__ y,
                                          double *__restrict__ part, int seg, double *sh) {
    const int lane = threadIdx.x & (LANES - 1);
    double dot = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int r = r0 + lane + i * LANES;
        if (r < r1) {
            // ascending order; reads issued 8 at a time so LDS latency overlaps
            A sum = A(0);
            int k = pre.a[i];
            const int z = pre.z[i];
            for (; k + 8 <= z; k += 8) {
                A q[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) q[u] = prod[k + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) sum += q[u];
            }
            if (k + 4 <= z) {
                A q[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) q[u] = prod[k + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) sum += q[u];
                k += 4;
            }
            for (; k < z; ++k) sum += prod[k];
            if (EPI == EPI_RESID) {
                const Y res = static_cast<Y>(pre.op[i] - static_cast<Y>(sum));
                y[r] = res;
                dot += static_cast<double>(res) * static_cast<double>(res);
            } else {
                y[r] = static_cast<Y>(sum);
                if (EPI == EPI_DOT) dot += static_cast<double>(sum) * static_cast<double>(pre.op[i]);
            }
        }
    }
    if (EPI != EPI_PLAIN) {
        if constexpr (LANES == kWave) {
            const double t = wave_sum(dot);
            if (lane == 0) part[seg] = t;
        } else {
            const double t = block_sum(dot, sh);
            if (threadIdx.x == 0) part[seg] = t;
        }
    }
}

__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Rows longer than a tile are summed in pieces of kLongPiece stored entries.
// One piece [s, e): lane t adds a_k * x[c_k] for k = s + t, s + t + kBlock,
// ... in ascending k with fused multiply-adds into an accumulator of type A
// (eight columns, then eight values, then eight gathers in flight per lane),
// and block_sum adds the lanes' sums in double; the result is valid in
// thread 0.  A row's sum is its pieces' sums added in piece order, in double,
// then rounded to A: the same bits whether one workgroup walks the pieces or
// each piece has a workgroup of its own.  `sh` is block_sum's scratch; the
// caller separates two calls with a barrier.
template <typename A, typename V, class Gather>
__device__ __forceinline__ double long_piece_sum(const V *__restrict__ val, const int32_t *__restrict__ col, int s,
                                                 int e, Gather gather, double *sh) {
    constexpr int U = 8;
    A acc = A(0);
    int k = s + (int)threadIdx.x;
    for (; k + (U - 1) * kBlock < e; k += U * kBlock) {
        int32_t c[U];
        A v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = col[k + u * kBlock];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = to_acc<A>(val[k + u * kBlock]);
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = static_cast<A>(gather(c[u]));
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma_acc(v[u], xv[u], acc);
    }
    for (; k < e; k += kBlock) acc = fma_acc(to_acc<A>(val[k]), static_cast<A>(gather(col[k])), acc);
    return block_sum(static_cast<double>(acc), sh);
}

}  // namespace spmvlib
