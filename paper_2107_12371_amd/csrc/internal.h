// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "spmv.h"

namespace spmvlib {

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int fail(int code, const char *fmt, ...);
void clear_error();
const char *last_error();

// Serialises the library's stream captures with its synchronous runtime
// work (device and pinned allocations and frees, blocking copies, graph
// teardown).  HIP rejects some of that work from other threads while a
// stream of the device is being captured, and the rejected call also
// invalidates the capture; holding this lock on both sides keeps them apart.
std::mutex &capture_gate();

// Largest accepted number of stored entries (scalar CSR): 2^31 - 2^16, so
// that every 32-bit entry offset a kernel forms (at most a 4096-entry tile,
// or a 510-block tile of 9 values, past the last entry) stays below 2^31.
constexpr int64_t kMaxNnz = (int64_t(1) << 31) - (int64_t(1) << 16);

// Host-side CSR validation (paper Sec. 4.2 storage: int32 columns, row
// pointers).  Returns SPMV_OK or SPMV_EINVAL with a message.
int validate_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                 const int32_t *col_idx);

// Segment kinds of the analysis plan.
enum SegKind : int32_t { SEG_STREAM = 0, SEG_LONG = 1, SEG_WINDOW = 2, SEG_CWIN = 3 };

// The wavefront-tile kernel's number in spmv_params.kernel (its tiles are planned
// differently: 1024-entry capacity, at most 128 rows).
constexpr int KV_WAVE_PLAN = 3;

// The default XCD assignment of tiles (spmv_params.xcd_chunk = 0): a matrix
// that does not fit the 256 MB memory-side cache is dealt to the XCDs in
// chunks of 16 tiles, so that all XCDs stream near the same rows and share
// one band of x there (16M-row mesh matrix, 3.2 GB: 0.518 against 0.567 ms
// with one contiguous range per XCD; 3x3 blocks with 8 columns, 2.7 GB:
// 0.98 against 1.18 ms); a smaller one keeps one contiguous range per XCD,
// whose private L2 then holds that range's band (2M-row kNN matrix, 165 MB,
// warm: 30.2 against 34.7 us with chunks).
constexpr int kDefaultXcdChunk = 16, kDefaultXcdChunkLog2 = 4;
constexpr int64_t kXcdChunkMinBytes = int64_t(256) << 20;
inline int default_xcd_chunk(int64_t matrix_bytes) { return matrix_bytes >= kXcdChunkMinBytes ? kDefaultXcdChunk : -2; }

// Compact per-tile windows: at most this many words and runs per tile.
constexpr int kCwinMaxRuns = 64;  // must equal the kernels' kCwinMaxRunsDev

// Stored entries per piece of a long row (must equal the kernels' kLongPiece).
constexpr int kLongPieceHost = 16384;
inline int32_t long_row_pieces(int64_t len) { return (int32_t)((len + kLongPieceHost - 1) / kLongPieceHost); }

// Analysis plan built once per matrix (the matrix is constant, so its
// preprocessing is amortised -- paper Sec. 2).
struct Plan {
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;
    int32_t tile_nnz = 0, tile_rows = 0;
    int32_t window_mode = 0, ring_words = 0, window_block = 0, kernel = 0;
    int32_t xcd_chunk = 0;           // spmv_params.xcd_chunk (validated; 0 replaced by the default)
    std::vector<int32_t> seg_bound;  // n_seg + 1 row boundaries
    std::vector<int32_t> seg_kind;   // SegKind per segment
    std::vector<int32_t> win_off;    // first staged x word (window segments)
    std::vector<int32_t> win_cnt;    // staged x words (window segments)
    std::vector<int32_t> win_block;  // window block id or -1
    std::vector<int32_t> stream_list;  // segment ids on the direct-gather path
    std::vector<int32_t> long_list;    // segment ids of long rows
    std::vector<int32_t> win_list;     // window segment ids, grouped by block
    std::vector<int32_t> win_blk_ptr;  // n_blocks + 1 offsets into win_list
    int64_t window_words = 0;
    // compact windows (SEG_CWIN): per tile, runs of columns staged in LDS;
    // win_off/win_cnt hold the tile's first run and run count, cwin_width its
    // staged words; runs are (first column, window position) pairs and lidx
    // holds each stored entry's window position (16-bit, relative).
    std::vector<int32_t> cwin_list;
    std::vector<int32_t> cwin_width;   // per segment
    std::vector<int32_t> runs;         // 2 per run
    std::vector<uint16_t> lidx;        // per stored entry (compact tiles only)
    // 2048-entry tiles: the same positions packed 12 bits each, per tile of
    // cwin_list and per lane (256 lanes x 8 entries = 3 words per lane)
    std::vector<uint32_t> lidx12;
    int32_t n_seg() const { return (int32_t)seg_kind.size(); }
};

constexpr int kPackTileNnz = 2048;  // tile capacity with packed 12-bit positions
constexpr int kPackLanes = 256;     // lanes per workgroup; each lane owns 4 entries per 1024-entry pass

// Sliced ELLPACK with sigma sorting (SELL-C-sigma; the paper's sliced
// ELLPACK storage, Sec. 4.2, with C = 64 rows per slice, one per lane of a
// wavefront).  Rows of at most kSellMaxLen entries are sorted by length
// (descending, ties by row) within windows of sigma consecutive such rows and
// cut into slices of 64; a slice stores its rows column-major, padded to its
// longest row.  Longer rows are appended after the slices in CSR order and
// take the long-row path.
constexpr int kSellC = 64;
constexpr int kSellMaxLen = 255;

struct SellPlan {
    int32_t sigma = 0;
    int32_t n_slices = 0;
    int64_t n_entries = 0;           // padded slice entries (64 * width per slice)
    std::vector<int32_t> perm;       // 64 * n_slices slots: row, or -1 for an empty slot
    std::vector<uint8_t> len;        // per slot: the row's stored entries (0 for empty)
    std::vector<int32_t> slice_ptr;  // n_slices + 1 entry offsets
    std::vector<int32_t> long_rows;  // rows longer than kSellMaxLen, ascending
    std::vector<int64_t> long_off;   // their first entry, after the slices
};

int build_sell_plan(int32_t n_rows, const int32_t *row_ptr, int32_t sigma, SellPlan &S);

// SELL columns from CSR (n_entries + long-row entries).  A padding slot
// repeats its row's last column (column 0 for an empty row), so every
// gather address is valid; kernels mask padding by row length.
void sell_fill_cols(const SellPlan &S, const int32_t *row_ptr, const int32_t *col_idx, int32_t *col_out);

// SELL values from CSR, converted by `cvt`; padding slots hold zero.
template <typename O, typename F>
void sell_fill_vals(const SellPlan &S, const int32_t *row_ptr, const double *val, O *out, F cvt) {
    for (int32_t sl = 0; sl < S.n_slices; ++sl) {
        const int64_t base = S.slice_ptr[sl];
        const int width = (int)((S.slice_ptr[sl + 1] - base) / kSellC);
        for (int lane = 0; lane < kSellC; ++lane) {
            const int64_t slot = (int64_t)sl * kSellC + lane;
            const int32_t r = S.perm[slot];
            const int len = S.len[slot];
            for (int j = 0; j < width; ++j)
                out[base + (int64_t)j * kSellC + lane] = (r >= 0 && j < len) ? cvt(val[(int64_t)row_ptr[r] + j]) : cvt(0.0);
        }
    }
    for (size_t i = 0; i < S.long_rows.size(); ++i) {
        const int32_t r = S.long_rows[i];
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) out[S.long_off[i] + (k - row_ptr[r])] = cvt(val[k]);
    }
}

// Tiles of consecutive block rows for the 3x3 block kernel: at most
// max_rows block rows and max_blocks stored blocks per tile; a longer block
// row forms a tile of its own.  Returns n_tiles + 1 boundaries.
std::vector<int32_t> build_bsr_tiles(int32_t n_block_rows, const int32_t *brow_ptr, int max_rows,
                                     int max_blocks);

int build_plan(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
               const int32_t *col_idx, const spmv_params *params, Plan &plan);

}  // namespace spmvlib
