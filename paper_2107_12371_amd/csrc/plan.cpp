// Host-side analysis plan: row tiles, long-row bin and the LDS x-window
// metadata.  Pure C++ (no HIP calls) so it runs and is tested on the CPU.
//
// Tiles.  Rows are cut into consecutive tiles holding at most tile_nnz
// stored entries and tile_rows rows; one workgroup streams a tile's values
// and column indices with coalesced loads (the paper's slices of S rows,
// Sec. 5.1, sized here for a 256-lane workgroup instead of an FPGA pipeline).
// A row longer than tile_nnz becomes its own segment on the long-row path.
//
// Window.  For each tile the first and last column it touches are the
// paper's col_start_i / col_end_i (Sec. 5.1).  A window workgroup walks a
// block of adjacent tiles in order and keeps x[...] in an LDS ring of
// ring_words entries (word w in slot w mod ring_words, the paper's circular
// list).  Before tile i it stages only the words not yet resident: the
// range (colend_{i-1}, colend_i], i.e. count_i = colend_i - colend_{i-1} words
// starting at offset colend_{i-1} + 1, the paper's per-block metadata
// (Sec. 5.1; we read "offset_i = colend_{i-1}" as the last resident word, so
// loading starts one past it).  When a tile needs a word that has already
// been overwritten (or lies below the block's first tile), the ring restarts
// with the tile's full range [col_start_i, col_end_i].
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"

#include <thread>

namespace spmvlib {

static thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

const char *last_error() { return g_err; }

std::mutex &capture_gate() {
    static std::mutex m;
    return m;
}

int validate_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                 const int32_t *col_idx) {
    if (n_rows < 0 || n_cols < 0) return fail(SPMV_EINVAL, "negative dimension (%d x %d)", n_rows, n_cols);
    // the kernels index entries with 32-bit offsets up to a tile (or a
    // 3x3-block tile) past the last one, so nnz keeps 2^16 of headroom
    if (nnz < 0 || nnz > kMaxNnz)
        return fail(SPMV_EINVAL, "nnz = %lld outside [0, 2^31 - 2^16]", (long long)nnz);
    if (!row_ptr) return fail(SPMV_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && !col_idx) return fail(SPMV_EINVAL, "col_idx is NULL with nnz > 0");
    if (row_ptr[0] != 0) return fail(SPMV_EINVAL, "row_ptr[0] = %d, expected 0", row_ptr[0]);
    for (int32_t i = 0; i < n_rows; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return fail(SPMV_EINVAL, "row_ptr decreases at row %d (%d -> %d)", i, row_ptr[i], row_ptr[i + 1]);
    if ((int64_t)row_ptr[n_rows] != nnz)
        return fail(SPMV_EINVAL, "row_ptr[n_rows] = %d differs from nnz = %lld", row_ptr[n_rows], (long long)nnz);
    for (int64_t k = 0; k < nnz; ++k)
        if (col_idx[k] < 0 || col_idx[k] >= n_cols)
            return fail(SPMV_EINVAL, "col_idx[%lld] = %d outside [0, %d)", (long long)k, col_idx[k], n_cols);
    return SPMV_OK;
}

std::vector<int32_t> build_bsr_tiles(int32_t n_block_rows, const int32_t *brow_ptr, int max_rows,
                                     int max_blocks) {
    std::vector<int32_t> t;
    int32_t r = 0;
    while (r < n_block_rows) {
        t.push_back(r);
        int32_t r1 = r + 1;
        int64_t acc = (int64_t)brow_ptr[r + 1] - brow_ptr[r];
        while (r1 < n_block_rows && r1 - r < max_rows) {
            int64_t l = (int64_t)brow_ptr[r1 + 1] - brow_ptr[r1];
            if (acc + l > max_blocks) break;
            acc += l;
            ++r1;
        }
        r = r1;
    }
    t.push_back(n_block_rows);
    return t;
}

static int default_tile_nnz(int64_t nnz) {
    // Enough tiles to give every CU several workgroups (256 CUs on MI355X).
    if (nnz >= (int64_t)4096 * 4096) return 4096;
    if (nnz >= (int64_t)2048 * 2048) return 2048;
    return 1024;
}

static int build_plan_once(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, const spmv_params &p, int tnz, Plan &P);

int build_plan(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
               const int32_t *col_idx, const spmv_params *params, Plan &P) {
    spmv_params p{};
    if (params) p = *params;
    if (p.tile_nnz || p.kernel == KV_WAVE_PLAN || p.window_mode != SPMV_WINDOW_AUTO)
        return build_plan_once(n_rows, n_cols, nnz, row_ptr, col_idx, p, p.tile_nnz ? p.tile_nnz : default_tile_nnz(nnz), P);
    // AUTO with the default capacity: compact windows on 2048-entry tiles
    // (measured fastest on the 16M-row mesh matrix: 0.64 ms with packed
    // 12-bit positions vs 0.738 ms for the best direct-gather tiling; 4096-
    // and 1024-entry windows were slower), unless the windows cover under
    // half of the tiles (scattered orderings), then direct gathers on the
    // default capacity.
    // Compact windows pay only when the matrix streams from HBM: below about
    // twice the 256 MB last-level (MALL) cache the direct gathers hit cache
    // and the windows' staging is pure overhead (measured: 41.5 vs 30.4 us on a
    // 205 MB matrix).
    if (default_tile_nnz(nnz) < 2048 || nnz * 12 < ((int64_t)512 << 20)) {
        spmv_params q = p;
        q.window_mode = SPMV_WINDOW_OFF;
        int rc = build_plan_once(n_rows, n_cols, nnz, row_ptr, col_idx, q, default_tile_nnz(nnz), P);
        P.window_mode = SPMV_WINDOW_AUTO;
        return rc;
    }
    int rc = build_plan_once(n_rows, n_cols, nnz, row_ptr, col_idx, p, 2048, P);
    if (rc) return rc;
    int64_t windowed = 0;
    for (int32_t sg : P.cwin_list) windowed += P.win_cnt[sg] > 0 ? 1 : 0;
    if (2 * windowed >= (int64_t)P.seg_kind.size()) return SPMV_OK;
    spmv_params q = p;
    q.window_mode = SPMV_WINDOW_OFF;
    rc = build_plan_once(n_rows, n_cols, nnz, row_ptr, col_idx, q, default_tile_nnz(nnz), P);
    P.window_mode = SPMV_WINDOW_AUTO;
    return rc;
}

// Window positions of 2048-entry tiles, 12 bits each, in the order the
// window kernel's lanes own the entries: lane l covers entries
// s4 + pass*1024 + 4l + j (s4 = tile start rounded down to a multiple of 4,
// pass < 2, j < 4), entry m = 4*pass + j in bits [12m, 12m+12) of the lane's
// three words.  Entries outside the tile keep position 0.
static void pack_lidx12(const int32_t *row_ptr, Plan &P) {
    const size_t nt = P.cwin_list.size();
    P.lidx12.assign(nt * kPackLanes * 3, 0u);
    const int nth = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    auto work = [&](int t) {
        for (size_t i = t; i < nt; i += nth) {
            const int32_t sg = P.cwin_list[i];
            if (P.win_cnt[sg] == 0) continue;   // direct tile: no window
            const int64_t s = row_ptr[P.seg_bound[sg]], e = row_ptr[P.seg_bound[sg + 1]];
            const int64_t s4 = s & ~(int64_t)3;
            for (int l = 0; l < kPackLanes; ++l) {
                uint32_t *w = &P.lidx12[(i * kPackLanes + l) * 3];
                for (int m = 0; m < 8; ++m) {
                    const int64_t k = s4 + (m / 4) * (4 * kPackLanes) + 4 * l + (m % 4);
                    if (k < s || k >= e) continue;
                    const uint32_t v = P.lidx[k] & 0xfffu;
                    const int bit = 12 * m, word = bit / 32, sh = bit % 32;
                    w[word] |= v << sh;
                    if (sh + 12 > 32) w[word + 1] |= v >> (32 - sh);
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
}

static int build_plan_once(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, const spmv_params &p, int tnz, Plan &P) {
    if (tnz != 1024 && tnz != 2048 && tnz != 4096)
        return fail(SPMV_EINVAL, "tile_nnz = %d must be 1024, 2048 or 4096", tnz);
    int trows = p.tile_rows ? p.tile_rows : 512;
    if (trows < 1 || trows > 512) return fail(SPMV_EINVAL, "tile_rows = %d outside [1, 512]", trows);
    int wmode = p.window_mode;
    if (wmode < SPMV_WINDOW_AUTO || wmode > SPMV_WINDOW_RING)
        return fail(SPMV_EINVAL, "window_mode = %d unknown", wmode);
    const int gap = p.window_gap ? p.window_gap : 64;
    if (gap < 0 || gap > 4096) return fail(SPMV_EINVAL, "window_gap = %d outside [0, 4096]", gap);
    int ring = p.ring_words ? p.ring_words : 4096;
    if (ring < 256 || ring > 8192 || (ring & (ring - 1)))
        return fail(SPMV_EINVAL, "ring_words = %d must be a power of two in [256, 8192]", ring);
    if (p.window_block < 0) return fail(SPMV_EINVAL, "window_block = %d < 0", p.window_block);
    if (p.kernel < 0 || p.kernel > 3) return fail(SPMV_EINVAL, "kernel = %d unknown", p.kernel);
    if (p.xcd_chunk < -2 || p.xcd_chunk > 4096 || (p.xcd_chunk > 0 && (p.xcd_chunk & (p.xcd_chunk - 1))))
        return fail(SPMV_EINVAL, "xcd_chunk = %d must be -2, -1, 0 or a power of two <= 4096", p.xcd_chunk);
    if (p.long_rows != 0 && p.long_rows != 1) return fail(SPMV_EINVAL, "long_rows = %d must be 0 or 1", p.long_rows);
    if (p.kernel == KV_WAVE_PLAN) {
        // wavefront tiles: 1024-entry capacity, two rows per lane
        if (p.tile_nnz && p.tile_nnz != 1024)
            return fail(SPMV_EINVAL, "kernel 3 (wavefront tiles) needs tile_nnz = 1024");
        if (p.tile_rows > 128) return fail(SPMV_EINVAL, "kernel 3 (wavefront tiles) allows at most 128 rows");
        tnz = 1024;
        trows = p.tile_rows ? p.tile_rows : 128;
    }

    P = Plan{};
    P.n_rows = n_rows; P.n_cols = n_cols; P.nnz = nnz;
    P.tile_nnz = tnz; P.tile_rows = trows; P.window_mode = wmode; P.ring_words = ring;
    // A tile's first entry may sit up to 3 past a 4-aligned boundary and the
    // kernels stream whole aligned groups, so a tile holds at most tnz - 3
    // entries (its aligned span then fits tnz exactly).
    const int cap = tnz - 3;
    P.kernel = p.kernel;
    P.xcd_chunk = p.xcd_chunk ? p.xcd_chunk : default_xcd_chunk(12 * nnz + 4 * (int64_t)n_rows);

    // ---- segmentation into stream tiles and long rows
    int32_t r = 0;
    while (r < n_rows) {
        int64_t len = (int64_t)row_ptr[r + 1] - row_ptr[r];
        if (len > cap) {
            P.seg_bound.push_back(r);
            P.seg_kind.push_back(SEG_LONG);
            ++r;
            continue;
        }
        int32_t r1 = r;
        int64_t acc = 0;
        while (r1 < n_rows && r1 - r < trows) {
            int64_t l = (int64_t)row_ptr[r1 + 1] - row_ptr[r1];
            if (l > cap || acc + l > cap) break;
            acc += l;
            ++r1;
        }
        P.seg_bound.push_back(r);
        P.seg_kind.push_back(SEG_STREAM);
        r = r1;
    }
    P.seg_bound.push_back(n_rows);
    const int32_t nseg = P.n_seg();
    P.win_off.assign(nseg, 0);
    P.win_cnt.assign(nseg, 0);
    P.win_block.assign(nseg, -1);

    // ---- ring-window analysis (circular LDS cache over blocks of tiles)
    if (wmode == SPMV_WINDOW_RING && nseg > 0) {
        std::vector<int32_t> cmin(nseg, INT32_MAX), cmax(nseg, -1);
        int32_t n_stream = 0;
        for (int32_t s = 0; s < nseg; ++s) {
            if (P.seg_kind[s] != SEG_STREAM) continue;
            ++n_stream;
            for (int64_t k = row_ptr[P.seg_bound[s]]; k < row_ptr[P.seg_bound[s + 1]]; ++k) {
                cmin[s] = std::min(cmin[s], col_idx[k]);
                cmax[s] = std::max(cmax[s], col_idx[k]);
            }
        }
        int B = p.window_block;
        if (B == 0) B = std::max(1, std::min(64, n_stream / 512));
        P.window_block = B;
        int32_t blk_id = 0;
        int32_t s = 0;
        while (s < nseg) {
            if (P.seg_kind[s] != SEG_STREAM) { ++s; continue; }
            // a chunk of up to B consecutive stream segments
            int32_t e = s;
            while (e < nseg && e - s < B && P.seg_kind[e] == SEG_STREAM) ++e;
            bool ok = true;
            int64_t staged = 0, entries = 0;
            int64_t H = -1, vlo = 0;
            bool first = true;
            std::vector<int32_t> off(e - s, 0), cnt(e - s, 0);
            for (int32_t t = s; t < e; ++t) {
                int64_t ent = (int64_t)row_ptr[P.seg_bound[t + 1]] - row_ptr[P.seg_bound[t]];
                entries += ent;
                if (ent == 0) continue;
                int64_t lo = cmin[t], hi = cmax[t], span = hi - lo + 1;
                if (span > ring) { ok = false; break; }
                int64_t Hn = std::max(H, hi);
                if (!first && lo >= std::max(vlo, Hn - ring + 1)) {
                    off[t - s] = (int32_t)(H + 1);
                    cnt[t - s] = (int32_t)(Hn - H);
                    H = Hn;
                } else {
                    off[t - s] = (int32_t)lo;
                    cnt[t - s] = (int32_t)span;
                    vlo = lo;
                    H = hi;
                    first = false;
                }
                staged += cnt[t - s];
            }
            bool use = ok && !first;
            if (use) {
                P.win_blk_ptr.push_back((int32_t)P.win_list.size());
                for (int32_t t = s; t < e; ++t) {
                    P.seg_kind[t] = SEG_WINDOW;
                    P.win_off[t] = off[t - s];
                    P.win_cnt[t] = cnt[t - s];
                    P.win_block[t] = blk_id;
                    P.win_list.push_back(t);
                }
                P.window_words += staged;
                ++blk_id;
            }
            s = e;
        }
        if (!P.win_list.empty()) P.win_blk_ptr.push_back((int32_t)P.win_list.size());
    }
    // ---- compact windows (default): per tile, the distinct columns merged
    // into runs (gaps up to `gap` words are staged too), at most
    // tile-capacity words and kCwinMaxRuns runs; entries get 16-bit
    // positions in the tile's window.  Tiles that do not fit keep direct
    // gathers.
    P.cwin_width.assign(nseg, 0);
    if (wmode == SPMV_WINDOW_AUTO && nseg > 0) {
        std::vector<int32_t> cand;
        for (int32_t s = 0; s < nseg; ++s)
            if (P.seg_kind[s] == SEG_STREAM) cand.push_back(s);
        P.lidx.assign((size_t)nnz, 0);
        const int nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
        std::vector<std::vector<int32_t>> runs_t(nth);
        std::vector<int32_t> run_first(nseg, 0), run_cnt(nseg, 0), ok(nseg, 0);
        auto work = [&](int t) {
            std::vector<int32_t> u;
            std::vector<int32_t> rx, rp;
            for (size_t ci = t; ci < cand.size(); ci += nth) {
                const int32_t sg = cand[ci];
                const int64_t a = row_ptr[P.seg_bound[sg]], b = row_ptr[P.seg_bound[sg + 1]];
                if (b == a) continue;
                u.assign(col_idx + a, col_idx + b);
                std::sort(u.begin(), u.end());
                u.erase(std::unique(u.begin(), u.end()), u.end());
                bool fit = false;
                for (int g : {gap, gap / 4, 0}) {
                    rx.clear();
                    rp.clear();
                    int32_t width = 0, lo = u[0], hi = u[0];
                    for (size_t i = 1; i <= u.size(); ++i) {
                        if (i == u.size() || u[i] - hi - 1 > g) {
                            rx.push_back(lo);
                            rp.push_back(width);
                            width += hi - lo + 1;
                            if (i < u.size()) lo = hi = u[i];
                        } else {
                            hi = u[i];
                        }
                    }
                    if (width <= tnz && (int)rx.size() <= kCwinMaxRuns) {
                        fit = true;
                        P.cwin_width[sg] = width;
                        break;
                    }
                }
                if (!fit) continue;
                for (int64_t k = a; k < b; ++k) {
                    const int32_t c = col_idx[k];
                    const int r = (int)(std::upper_bound(rx.begin(), rx.end(), c) - rx.begin()) - 1;
                    P.lidx[k] = (uint16_t)(rp[r] + (c - rx[r]));
                }
                run_cnt[sg] = (int32_t)rx.size();
                run_first[sg] = (int32_t)(runs_t[t].size() / 2);   // local, fixed up below
                for (size_t r = 0; r < rx.size(); ++r) {
                    runs_t[t].push_back(rx[r]);
                    runs_t[t].push_back(rp[r]);
                }
                ok[sg] = t + 1;
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nth; ++t) th.emplace_back(work, t);
        work(0);
        for (auto &x : th) x.join();
        std::vector<int64_t> base(nth, 0);
        int64_t tot = 0;
        for (int t = 0; t < nth; ++t) {
            base[t] = tot;
            tot += (int64_t)runs_t[t].size() / 2;
        }
        P.runs.reserve((size_t)tot * 2);
        for (int t = 0; t < nth; ++t) P.runs.insert(P.runs.end(), runs_t[t].begin(), runs_t[t].end());
        int64_t n_fit = 0;
        for (int32_t sg : cand) n_fit += ok[sg] ? 1 : 0;
        if (n_fit == 0) {
            P.lidx.clear();
        } else {
            // One launch does the whole product: tiles whose window does not
            // fit ride along in the window kernel as direct-gather tiles (no
            // runs), in row order with the others.
            for (int32_t sg : cand) {
                P.seg_kind[sg] = SEG_CWIN;
                if (ok[sg]) {
                    P.win_off[sg] = (int32_t)(base[ok[sg] - 1] + run_first[sg]);
                    P.win_cnt[sg] = run_cnt[sg];
                    P.window_words += P.cwin_width[sg];
                } else {
                    P.win_off[sg] = 0;
                    P.win_cnt[sg] = 0;
                    P.cwin_width[sg] = 0;
                }
                P.cwin_list.push_back(sg);
            }
        }
    }
    for (int32_t s = 0; s < nseg; ++s) {
        if (P.seg_kind[s] == SEG_STREAM) P.stream_list.push_back(s);
        else if (P.seg_kind[s] == SEG_LONG) P.long_list.push_back(s);
    }
    if (tnz == kPackTileNnz && !P.cwin_list.empty()) pack_lidx12(row_ptr, P);
    return SPMV_OK;
}

}  // namespace spmvlib

extern "C" const char *spmv_last_error(void) { return spmvlib::last_error(); }

extern "C" int spmv_plan_inspect(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                                 const int32_t *col_idx, const spmv_params *params, int32_t *n_tiles_out,
                                 int32_t *seg_bound, int32_t *seg_kind, int32_t *win_off, int32_t *win_cnt,
                                 int32_t *win_block, int32_t *runs, uint16_t *lidx, uint32_t *lidx12,
                                 spmv_info *info) {
    using namespace spmvlib;
    clear_error();
    int rc = validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    if (rc) return rc;
    if (params && params->format != SPMV_FORMAT_CSR)
        return fail(SPMV_EINVAL, "spmv_plan_inspect covers CSR row tiles; use spmv_sell_inspect");
    Plan P;
    rc = build_plan(n_rows, n_cols, nnz, row_ptr, col_idx, params, P);
    if (rc) return rc;
    const int32_t ns = P.n_seg();
    if (n_tiles_out) *n_tiles_out = ns;
    if (seg_bound) std::memcpy(seg_bound, P.seg_bound.data(), sizeof(int32_t) * (ns + 1));
    if (seg_kind && ns) std::memcpy(seg_kind, P.seg_kind.data(), sizeof(int32_t) * ns);
    if (win_off && ns) std::memcpy(win_off, P.win_off.data(), sizeof(int32_t) * ns);
    if (win_cnt && ns) std::memcpy(win_cnt, P.win_cnt.data(), sizeof(int32_t) * ns);
    if (win_block && ns) std::memcpy(win_block, P.win_block.data(), sizeof(int32_t) * ns);
    if (runs && !P.runs.empty()) std::memcpy(runs, P.runs.data(), sizeof(int32_t) * P.runs.size());
    if (lidx && !P.lidx.empty()) std::memcpy(lidx, P.lidx.data(), sizeof(uint16_t) * P.lidx.size());
    if (lidx12 && !P.lidx12.empty()) std::memcpy(lidx12, P.lidx12.data(), sizeof(uint32_t) * P.lidx12.size());
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->n_rows = n_rows; info->n_cols = n_cols; info->nnz = nnz;
        info->tile_nnz = P.tile_nnz; info->tile_rows = P.tile_rows;
        info->n_tiles = ns;
        info->n_stream_tiles = (int32_t)P.stream_list.size();
        info->n_long_rows = (int32_t)P.long_list.size();
        int32_t nw = (int32_t)P.win_list.size();
        for (int32_t sg : P.cwin_list) nw += P.win_cnt[sg] > 0 ? 1 : 0;
        info->n_window_tiles = nw;
        info->n_window_blocks = P.win_blk_ptr.empty() ? 0 : (int32_t)P.win_blk_ptr.size() - 1;
        info->ring_words = P.ring_words;
        info->window_words = P.window_words;
        info->n_runs = (int64_t)P.runs.size() / 2;
        info->block_size = 1;
        int32_t pieces = 0;
        for (int32_t sg : P.long_list)
            pieces += long_row_pieces((int64_t)row_ptr[P.seg_bound[sg + 1]] - row_ptr[P.seg_bound[sg]]);
        info->n_long_pieces = pieces;
        info->workspace_bytes = pieces > (int32_t)P.long_list.size() ? (int64_t)sizeof(double) * pieces : 0;
    }
    return SPMV_OK;
}
