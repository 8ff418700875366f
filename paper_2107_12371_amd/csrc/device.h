// Device-side helpers and the resident-matrix layout shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spmvlib {

constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts of 64)
constexpr int kWave = 64;
constexpr int kEntriesPerLane = 4; // stored entries a lane streams per pass
constexpr int kPad = 16;           // padding entries after col/val arrays
constexpr int kCwinMaxRunsDev = 64; // compact windows: runs per tile (plan limit)
// Rows longer than a tile are summed in pieces of this many stored entries
// (one workgroup's share when the pieces of a row run side by side).
constexpr int kLongPiece = 16384;

// Epilogues of the row-tile kernels.
enum Epilogue : int {
    EPI_PLAIN = 0,  // y_i = (A x)_i
    EPI_DOT = 1,    // y_i = (A x)_i and per-tile partial of sum_i x_i y_i (CG's p.q)
    EPI_RESID = 2   // y_i = b_i - (A x)_i and per-tile partial of sum_i y_i^2
};

// Per-tile launch descriptor (one 32-byte scalar load per tile).
struct TileDesc {
    int32_t r0, r1;   // rows [r0, r1)
    int32_t s, e;     // stored entries [s, e) = [row_ptr[r0], row_ptr[r1])
    int32_t seg;      // segment id (index of the tile's dot-product partial)
    int32_t woff;     // ring tiles: first x word staged; compact tiles: first run
    int32_t wcnt;     // ring tiles: x words staged; compact tiles: number of runs
    int32_t width;    // compact tiles: staged window words
};

// Kernel variants for the direct-gather tiles.
enum KernelVariant : int32_t { KV_AUTO = 0, KV_ONE_TILE = 1, KV_PIPELINED = 2, KV_WAVE = 3 };

// Resident matrix and its plan in device memory.  Owned by spmv_matrix.
struct DevMatrix {
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;
    int32_t tile_nnz = 0;
    int32_t *row_ptr = nullptr;      // n_rows + 1
    int32_t *col = nullptr;          // nnz + padding (padding columns are 0)
    double *val64 = nullptr;         // nnz + padding
    float *val32 = nullptr;          // optional FP32 copy
    uint16_t *val16 = nullptr;       // optional BF16 copy (upper half of an FP32)
    int32_t n_seg = 0;
    int32_t n_stream = 0;
    TileDesc *stream_desc = nullptr; // direct-gather tiles, in row order
    int32_t n_long = 0;
    TileDesc *long_desc = nullptr;   // rows longer than a tile
    int32_t n_long_pieces = 0;       // pieces of kLongPiece entries over the long rows
    int32_t *long_piece_ptr = nullptr;  // n_long + 1 offsets into the pieces (only when
                                        // some long row has more than one piece)
    int32_t *piece_long = nullptr;      // per piece: its long row (index into long_desc)
    bool long_split = true;             // pieces on a workgroup each where scratch exists
    int32_t y_ws_row = 0, y_ws_rows = 0;  // longest run of rows without a long row
    int32_t n_blk = 0;
    int32_t *win_blk_ptr = nullptr;  // n_blk + 1 offsets into win_desc
    TileDesc *win_desc = nullptr;    // window tiles, grouped by block
    int32_t ring_words = 0;
    int32_t n_cwin = 0;
    TileDesc *cwin_desc = nullptr;   // compact-window tiles: woff = first run, wcnt = runs, pad = width
    int32_t *runs = nullptr;         // (first column, window position) per run
    uint16_t *lidx = nullptr;        // window-relative column per stored entry (+ padding)
    uint32_t *lidx12 = nullptr;      // 2048-entry tiles: packed 12-bit positions per tile and lane
    bool xcd_remap = true;
    int32_t xcd_chunk_log2 = -1;     // XCD assignment (xcd_tile): -1 one contiguous range per XCD
    int32_t kernel = KV_AUTO;        // direct-gather kernel variant
    int32_t block = 1;                // 1: scalar CSR, 3: 3x3 block CSR
    int32_t n_bsr_tiles = 0;
    int32_t *bsr_tiles = nullptr;     // block-row tile boundaries (block CSR)
    // sliced ELLPACK handles: col / val* hold the slices (then the long rows)
    int32_t format = 0;               // SPMV_FORMAT_CSR or SPMV_FORMAT_SELL
    int32_t n_slices = 0;
    int32_t n_sell_wg = 0;            // workgroups of 4 slices; long rows follow in n_seg
    int32_t *sell_perm = nullptr;     // row per slot (-1: empty)
    uint8_t *sell_len = nullptr;      // entries per slot
    int32_t *sell_ptr = nullptr;      // n_slices + 1 entry offsets
};

// Tile taken by workgroup b.  The dispatcher deals workgroups to the 8 XCDs
// in turn (b mod 8); the j-th workgroup of an XCD (j = b / 8) takes
//  - chunk_log2 < 0: tile xcd * per_xcd + j, one contiguous range per XCD
//    (each XCD's L2 walks its own band of x);
//  - chunk_log2 = c >= 0: tile j mod 2^c of chunk (j >> c) * 8 + xcd, i.e.
//    chunks of 2^c consecutive tiles dealt to the XCDs in turn, so that all
//    XCDs work near the same rows and share one band of x in the MALL;
//  - per_xcd = 0: tile b (no XCD grouping).
__device__ __forceinline__ int xcd_tile(int b, int per_xcd, int chunk_log2) {
    if (per_xcd == 0) return b;
    const int x = b & 7, j = b >> 3;
    if (chunk_log2 < 0) return x * per_xcd + j;
    return ((((j >> chunk_log2) << 3) + x) << chunk_log2) + (j & ((1 << chunk_log2) - 1));
}

// Workgroups that cover n tiles under xcd_tile (some past n exit at once).
inline int xcd_grid(int n, int per_xcd, int chunk_log2) {
    if (per_xcd == 0) return n;
    if (chunk_log2 < 0) return 8 * per_xcd;
    const int c = 1 << chunk_log2;
    const int groups = ((n + c - 1) / c + 7) / 8;
    return groups * 8 * c;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Stream-load policy per value type, chosen by measurement on the 16M-row
// mesh matrix: binary64 tiles stream faster with ordinary cached loads
// (4.81 vs 4.37 TB/s effective), FP32/BF16 tiles with non-temporal loads
// (4.90 vs 4.75 TB/s).  Column indices follow their tile's values.
template <typename V> struct StreamNT { static constexpr bool value = true; };
template <> struct StreamNT<double> { static constexpr bool value = false; };

template <bool NTL, typename T> __device__ __forceinline__ T stream_load(const T *p) {
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}

// Four consecutive stored values (16 bytes or less per lane).
template <typename V> struct Val4;
template <> struct Val4<double> {
    f64x2 a, b;
    __device__ __forceinline__ void load(const double *p) {
        a = stream_load<StreamNT<double>::value>(reinterpret_cast<const f64x2 *>(p));
        b = stream_load<StreamNT<double>::value>(reinterpret_cast<const f64x2 *>(p + 2));
    }
    __device__ __forceinline__ void zero() { a = f64x2{0.0, 0.0}; b = a; }
    template <int J> __device__ __forceinline__ double get() const { return J < 2 ? a[J & 1] : b[J & 1]; }
    __device__ __forceinline__ double get_dyn(int j) const { return j < 2 ? a[j & 1] : b[j & 1]; }
};
template <> struct Val4<float> {
    f32x4 a;
    __device__ __forceinline__ void load(const float *p) {
        a = stream_load<StreamNT<float>::value>(reinterpret_cast<const f32x4 *>(p));
    }
    __device__ __forceinline__ void zero() { a = f32x4{0.f, 0.f, 0.f, 0.f}; }
    template <int J> __device__ __forceinline__ float get() const { return a[J]; }
    __device__ __forceinline__ float get_dyn(int j) const { return a[j]; }
};
template <> struct Val4<uint16_t> {  // bfloat16 bit patterns
    u32x2 a;
    __device__ __forceinline__ void load(const uint16_t *p) {
        a = stream_load<StreamNT<uint16_t>::value>(reinterpret_cast<const u32x2 *>(p));
    }
    __device__ __forceinline__ void zero() { a = u32x2{0u, 0u}; }
    template <int J> __device__ __forceinline__ float get() const {
        unsigned w = a[J >> 1];
        unsigned bits = (J & 1) ? (w & 0xffff0000u) : (w << 16);
        return __uint_as_float(bits);
    }
    __device__ __forceinline__ float get_dyn(int j) const {
        unsigned w = a[j >> 1];
        unsigned bits = (j & 1) ? (w & 0xffff0000u) : (w << 16);
        return __uint_as_float(bits);
    }
};

template <typename V> __device__ __forceinline__ i32x4 load_col4(const int32_t *p) {
    return stream_load<StreamNT<V>::value>(reinterpret_cast<const i32x4 *>(p));
}

// Fixed-shape wavefront sum: a butterfly over lane distances 32..1.  Lane 0's
// result depends only on the inputs' lane positions, never on timing.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Workgroup sum in a fixed order (waves' lane-0 results added in wave order).
// Valid in thread 0.  `sh` holds kBlock / kWave doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / kWave; ++i) t += sh[i];
    return t;
}

}  // namespace spmvlib
