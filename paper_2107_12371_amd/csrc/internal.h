// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "spmv.h"

namespace spmvlib {

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int fail(int code, const char *fmt, ...);
void clear_error();

// Host-side CSR validation (paper Sec. 4.2 storage: int32 columns, row
// pointers).  Returns SPMV_OK or SPMV_EINVAL with a message.
int validate_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                 const int32_t *col_idx);

// Segment kinds of the analysis plan.
enum SegKind : int32_t { SEG_STREAM = 0, SEG_LONG = 1, SEG_WINDOW = 2, SEG_CWIN = 3 };

// The wavefront-tile kernel's number in spmv_params.kernel (its tiles are planned
// differently: 1024-entry capacity, at most 128 rows).
constexpr int KV_WAVE_PLAN = 3;

// Compact per-tile windows: at most this many words and runs per tile.
constexpr int kCwinMaxRuns = 64;  // must equal the kernels' kCwinMaxRunsDev

// Analysis plan built once per matrix (the matrix is constant, so its
// preprocessing is amortised -- paper Sec. 2).
struct Plan {
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;
    int32_t tile_nnz = 0, tile_rows = 0;
    int32_t window_mode = 0, ring_words = 0, window_block = 0, kernel = 0;
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

// Tiles of consecutive block rows for the 3x3 block kernel: at most
// max_rows block rows and max_blocks stored blocks per tile; a longer block
// row forms a tile of its own.  Returns n_tiles + 1 boundaries.
std::vector<int32_t> build_bsr_tiles(int32_t n_block_rows, const int32_t *brow_ptr, int max_rows,
                                     int max_blocks);

int build_plan(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
               const int32_t *col_idx, const spmv_params *params, Plan &plan);

}  // namespace spmvlib
