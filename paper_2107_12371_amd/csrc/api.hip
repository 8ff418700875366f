// C ABI: matrix handles (create / destroy / info) and the product entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"
#include "bsr.h"
#include "launch.h"
#include "matrix.h"
#include "spmm.h"

namespace spmvlib {

namespace {

// Restores the caller's current device on scope exit.
// Makes `dev` current for the guard's scope (and restores the caller's
// device); err is the failure to switch, if any.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err != hipSuccess || prev == dev) {
            prev = -1;
            return;
        }
        err = hipSetDevice(dev);
        if (err != hipSuccess) prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// round-to-nearest-even FP32 -> BF16 bit pattern (NaN kept quiet)
uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!na || !nb) return false;
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? SPMV_ENOMEM : SPMV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// The device side of one matrix creation.  It holds the capture gate for
// its lifetime and copies through a private non-blocking stream, never the
// legacy default stream (HIP refuses legacy-stream work while any stream is
// being captured).
struct Uploader {
    spmv_matrix *A;
    std::lock_guard<std::mutex> lock{capture_gate()};
    hipStream_t s = nullptr;
    hipError_t init = hipSuccess;

    explicit Uploader(spmv_matrix *A_) : A(A_) { init = hipStreamCreateWithFlags(&s, hipStreamNonBlocking); }
    ~Uploader() {
        if (s) (void)hipStreamDestroy(s);
    }
    Uploader(const Uploader &) = delete;
    Uploader &operator=(const Uploader &) = delete;

    // Allocates max(alloc_n, n, 1) elements, zero-fills the tail beyond n and
    // copies n elements from the host; the copy has completed on return, so
    // the host source may be released.
    template <typename T> int put(T **dst, const T *src, size_t n, size_t alloc_n) {
        if (alloc_n < n) alloc_n = n;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, sizeof(T) * (alloc_n ? alloc_n : 1));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        A->allocs.push_back(p);
        A->bytes += (int64_t)(sizeof(T) * (alloc_n ? alloc_n : 1));
        if (alloc_n > n) {
            e = hipMemsetAsync(static_cast<T *>(p) + n, 0, sizeof(T) * (alloc_n - n), s);
            if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        }
        if (n) {
            e = hipMemcpyAsync(p, src, sizeof(T) * n, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "upload");
        *dst = static_cast<T *>(p);
        return SPMV_OK;
    }

    // Releases what was allocated so far (failed creation).
    void release_all() {
        for (void *q : A->allocs) (void)hipFree(q);
        A->allocs.clear();
    }
};

static_assert(kLongPiece == kLongPieceHost, "long-row piece size differs between host and kernels");

// The pieces of the long rows (d: their descriptors, in long_desc order).
// The piece tables go to the device only when some row has more than one
// piece; otherwise every product walks each long row on one workgroup.
static int upload_long_pieces(Uploader &U, DevMatrix &M, const std::vector<TileDesc> &d) {
    std::vector<int32_t> ptr(d.size() + 1, 0);
    for (size_t i = 0; i < d.size(); ++i) ptr[i + 1] = ptr[i] + long_row_pieces((int64_t)d[i].e - d[i].s);
    M.n_long_pieces = ptr.back();
    // the longest run of rows without a long row (the long rows come in
    // ascending order): a product's own output rows there are scratch for
    // the pieces' sums until its row tiles write them
    int32_t prev = -1;
    M.y_ws_row = 0;
    M.y_ws_rows = 0;
    for (size_t i = 0; i <= d.size(); ++i) {
        const int32_t next = i < d.size() ? d[i].r0 : M.n_rows;
        if (next - (prev + 1) > M.y_ws_rows) {
            M.y_ws_row = prev + 1;
            M.y_ws_rows = next - (prev + 1);
        }
        prev = next;
    }
    if (M.n_long_pieces <= M.n_long) return SPMV_OK;
    std::vector<int32_t> owner((size_t)M.n_long_pieces);
    for (size_t i = 0; i < d.size(); ++i)
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) owner[(size_t)p] = (int32_t)i;
    int rc = U.put(&M.long_piece_ptr, ptr.data(), ptr.size(), 0);
    if (!rc) rc = U.put(&M.piece_long, owner.data(), owner.size(), 0);
    return rc;
}

static int64_t workspace_bytes_of(const DevMatrix &M) {
    return M.piece_long ? (int64_t)sizeof(double) * M.n_long_pieces : 0;
}

static int check_apply(const spmv_matrix *A, const void *x, size_t xs, const void *y, size_t ys) {
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    if (A->M.n_rows > 0 && !y) return fail(SPMV_EINVAL, "y is NULL");
    if (A->M.n_rows > 0 && A->M.nnz > 0 && !x) return fail(SPMV_EINVAL, "x is NULL");
    if (x && y && overlaps(x, xs * (size_t)A->M.n_cols, y, ys * (size_t)A->M.n_rows))
        return fail(SPMV_EINVAL, "x and y overlap");
    return SPMV_OK;
}

template <typename V, typename X, typename Y, typename Acc>
static int apply_typed(const spmv_matrix *A, const V *val, const X *x, Y *y, void *stream,
                       double *long_ws = nullptr) {
    clear_error();
    int rc = check_apply(A, x, sizeof(X), y, sizeof(Y));
    if (rc) return rc;
    if (A->M.n_rows == 0) return SPMV_OK;
    DeviceGuard g(A->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "making the matrix's device current");
    if (A->M.nnz == 0) {
        // no stored entry: y = 0 without reading x (which may be NULL or empty)
        const hipError_t z = launch_zero_fill<Y>(y, A->M.n_rows, static_cast<hipStream_t>(stream));
        return z == hipSuccess ? SPMV_OK : hip_fail(z, "zero fill");
    }
    hipError_t e = launch_spmv<V, X, Y, Acc>(A->M, val, x, y, EPI_PLAIN, nullptr, nullptr, nullptr,
                                             static_cast<hipStream_t>(stream), long_ws);
    if (e != hipSuccess) return hip_fail(e, "spmv launch");
    return SPMV_OK;
}

// SPMV_DEVICE_PTRS: copies n elements of a caller's device array into a
// host vector (the plan is built on the host).  A pointer that the runtime
// does not know as device or managed memory is SPMV_EINVAL.
template <typename T> static int fetch_device(const T *src, size_t n, std::vector<T> &dst, const char *what) {
    dst.resize(n);
    if (n == 0) return SPMV_OK;
    if (!src) return fail(SPMV_EINVAL, "%s is NULL", what);
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, src) != hipSuccess ||
        (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return fail(SPMV_EINVAL, "%s is not device memory (SPMV_DEVICE_PTRS)", what);
    }
    std::lock_guard<std::mutex> lock(capture_gate());
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemcpyAsync(dst.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) return hip_fail(e, what);
    return SPMV_OK;
}

// A sliced-ELLPACK handle (SPMV_FORMAT_SELL): slices and long rows in one
// column array and one array per value precision.
static int create_sell(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                       const int32_t *col_idx, const double *values, uint32_t flags, const spmv_params &p,
                       spmv_matrix **out) {
    if (p.xcd_chunk < -2 || p.xcd_chunk > 4096 || (p.xcd_chunk > 0 && (p.xcd_chunk & (p.xcd_chunk - 1))))
        return fail(SPMV_EINVAL, "xcd_chunk = %d must be -2, -1, 0 or a power of two <= 4096", p.xcd_chunk);
    if (p.long_rows != 0 && p.long_rows != 1) return fail(SPMV_EINVAL, "long_rows = %d must be 0 or 1", p.long_rows);
    SellPlan S;
    int rc = build_sell_plan(n_rows, row_ptr, p.sell_sigma, S);
    if (rc) return rc;
    auto *A = new (std::nothrow) spmv_matrix();
    if (!A) return fail(SPMV_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) {
        delete A;
        return hip_fail(e, "hipGetDevice");
    }
    Uploader U(A);
    if (U.init != hipSuccess) {
        delete A;
        return hip_fail(U.init, "upload stream");
    }
    DevMatrix &M = A->M;
    M.format = SPMV_FORMAT_SELL;
    M.long_split = p.long_rows == 0;
    M.n_rows = n_rows;
    M.n_cols = n_cols;
    M.nnz = nnz;
    const int chunk = p.xcd_chunk ? p.xcd_chunk : default_xcd_chunk(12 * nnz + 4 * (int64_t)n_rows);
    M.xcd_remap = !(flags & SPMV_NO_XCD_REMAP) && chunk != -1;
    M.xcd_chunk_log2 = -1;  // -2: one contiguous range per XCD
    for (int c = 0; c <= 12; ++c)
        if (chunk == (1 << c)) M.xcd_chunk_log2 = c;
    int64_t total = S.n_entries;
    for (size_t i = 0; i < S.long_rows.size(); ++i) total += row_ptr[S.long_rows[i] + 1] - row_ptr[S.long_rows[i]];
    const size_t tot = (size_t)total, tot_pad = tot + kPad;
    {
        std::vector<int32_t> c(tot);
        sell_fill_cols(S, row_ptr, col_idx, c.data());
        rc = U.put(&M.col, c.data(), tot, tot_pad);
    }
    if (!rc) {
        std::vector<double> v(tot);
        sell_fill_vals(S, row_ptr, values, v.data(), [](double d) { return d; });
        rc = U.put(&M.val64, v.data(), tot, tot_pad);
    }
    if (!rc && (flags & SPMV_VALUES_FP32)) {
        std::vector<float> v(tot);
        sell_fill_vals(S, row_ptr, values, v.data(), [](double d) { return (float)d; });
        rc = U.put(&M.val32, v.data(), tot, tot_pad);
    }
    if (!rc && (flags & SPMV_VALUES_BF16)) {
        std::vector<uint16_t> v(tot);
        sell_fill_vals(S, row_ptr, values, v.data(), [](double d) { return to_bf16((float)d); });
        rc = U.put(&M.val16, v.data(), tot, tot_pad);
    }
    M.n_slices = S.n_slices;
    M.n_sell_wg = (S.n_slices + kBlock / kWave - 1) / (kBlock / kWave);
    if (!rc) rc = U.put(&M.sell_perm, S.perm.data(), S.perm.size(), 0);
    if (!rc) rc = U.put(&M.sell_len, S.len.data(), S.len.size(), 0);
    if (!rc) rc = U.put(&M.sell_ptr, S.slice_ptr.data(), S.slice_ptr.size(), 0);
    M.n_long = (int32_t)S.long_rows.size();
    if (!rc && M.n_long) {
        std::vector<TileDesc> d(M.n_long);
        for (int32_t i = 0; i < M.n_long; ++i) {
            const int32_t r = S.long_rows[i];
            d[i] = TileDesc{};
            d[i].r0 = r;
            d[i].r1 = r + 1;
            d[i].s = (int32_t)S.long_off[i];
            d[i].e = (int32_t)(S.long_off[i] + (row_ptr[r + 1] - row_ptr[r]));
            d[i].seg = M.n_sell_wg + i;
        }
        rc = U.put(&M.long_desc, d.data(), d.size(), 0);
        if (!rc) rc = upload_long_pieces(U, M, d);
    }
    M.n_seg = M.n_sell_wg + M.n_long;
    if (!rc) prepare_launch_queries();
    if (rc) {
        U.release_all();
        delete A;
        return rc;
    }
    spmv_info &I = A->info;
    std::memset(&I, 0, sizeof I);
    I.n_rows = n_rows;
    I.n_cols = n_cols;
    I.nnz = nnz;
    I.n_tiles = M.n_seg;
    I.n_long_rows = M.n_long;
    I.has_fp32 = M.val32 != nullptr;
    I.has_bf16 = M.val16 != nullptr;
    I.device_bytes = A->bytes;
    I.block_size = 1;
    I.format = SPMV_FORMAT_SELL;
    I.n_slices = S.n_slices;
    I.sell_entries = S.n_entries;
    I.n_long_pieces = M.n_long_pieces;
    I.workspace_bytes = workspace_bytes_of(M);
    I.y_scratch_ok = M.piece_long && M.long_split && (int64_t)M.y_ws_rows >= M.n_long_pieces;
    *out = A;
    return SPMV_OK;
}

}  // namespace spmvlib

using namespace spmvlib;

extern "C" int spmv_create(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, const double *values, uint32_t flags,
                           const spmv_params *params, spmv_matrix **out) {
    clear_error();
    if (!out) return fail(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(SPMV_VALUES_FP32 | SPMV_VALUES_BF16 | SPMV_NO_XCD_REMAP | SPMV_DEVICE_PTRS))
        return fail(SPMV_EINVAL, "unknown flags 0x%x", flags);
    if (flags & SPMV_DEVICE_PTRS) {
        if (n_rows < 0 || nnz < 0) return fail(SPMV_EINVAL, "n_rows = %d, nnz = %lld", n_rows, (long long)nnz);
        std::vector<int32_t> rp, ci;
        std::vector<double> va;
        int rc = fetch_device(row_ptr, (size_t)n_rows + 1, rp, "row_ptr");
        if (!rc) rc = fetch_device(col_idx, (size_t)nnz, ci, "col_idx");
        if (!rc) rc = fetch_device(values, (size_t)nnz, va, "values");
        if (rc) return rc;
        return spmv_create(n_rows, n_cols, nnz, rp.data(), nnz ? ci.data() : nullptr, nnz ? va.data() : nullptr,
                           flags & ~SPMV_DEVICE_PTRS, params, out);
    }
    int rc = validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    if (rc) return rc;
    if (nnz > 0 && !values) return fail(SPMV_EINVAL, "values is NULL with nnz > 0");
    if (params && params->format != SPMV_FORMAT_CSR) {
        if (params->format != SPMV_FORMAT_SELL) return fail(SPMV_EINVAL, "format = %d unknown", params->format);
        return create_sell(n_rows, n_cols, nnz, row_ptr, col_idx, values, flags, *params, out);
    }
    Plan P;
    rc = build_plan(n_rows, n_cols, nnz, row_ptr, col_idx, params, P);
    if (rc) return rc;

    auto *A = new (std::nothrow) spmv_matrix();
    if (!A) return fail(SPMV_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) {
        delete A;
        return hip_fail(e, "hipGetDevice");
    }
    Uploader U(A);
    if (U.init != hipSuccess) {
        delete A;
        return hip_fail(U.init, "upload stream");
    }
    DevMatrix &M = A->M;
    M.long_split = !params || params->long_rows == 0;
    M.n_rows = n_rows;
    M.n_cols = n_cols;
    M.nnz = nnz;
    M.tile_nnz = P.tile_nnz;
    M.ring_words = P.ring_words;
    M.xcd_remap = !(flags & SPMV_NO_XCD_REMAP) && P.xcd_chunk != -1;
    M.xcd_chunk_log2 = -1;  // -2: one contiguous range per XCD
    for (int c = 0; c <= 12; ++c)
        if (P.xcd_chunk == (1 << c)) M.xcd_chunk_log2 = c;
    const size_t nz = (size_t)nnz, nz_pad = ((nz + 3) & ~(size_t)3) + kPad;
    rc = U.put(&M.row_ptr, row_ptr, (size_t)n_rows + 1, (size_t)n_rows + 1);
    if (!rc) rc = U.put(&M.col, col_idx, nz, nz_pad);
    if (!rc) rc = U.put(&M.val64, values, nz, nz_pad);
    if (!rc && (flags & SPMV_VALUES_FP32)) {
        std::vector<float> v32(nz);
        for (size_t k = 0; k < nz; ++k) v32[k] = (float)values[k];
        rc = U.put(&M.val32, v32.data(), nz, nz_pad);
    }
    if (!rc && (flags & SPMV_VALUES_BF16)) {
        std::vector<uint16_t> v16(nz);
        for (size_t k = 0; k < nz; ++k) v16[k] = to_bf16((float)values[k]);
        rc = U.put(&M.val16, v16.data(), nz, nz_pad);
    }
    M.n_seg = P.n_seg();
    M.kernel = P.kernel;
    auto desc_of = [&](int32_t sg) {
        TileDesc d{};
        d.r0 = P.seg_bound[sg];
        d.r1 = P.seg_bound[sg + 1];
        d.s = row_ptr[d.r0];
        d.e = row_ptr[d.r1];
        d.seg = sg;
        d.woff = P.win_off[sg];
        d.wcnt = P.win_cnt[sg];
        d.width = P.cwin_width.empty() ? 0 : P.cwin_width[sg];
        return d;
    };
    auto upload_descs = [&](const std::vector<int32_t> &list, TileDesc **dst) {
        std::vector<TileDesc> v;
        v.reserve(list.size());
        for (int32_t sg : list) v.push_back(desc_of(sg));
        return U.put(dst, v.data(), v.size(), 0);
    };
    M.n_stream = (int32_t)P.stream_list.size();
    if (!rc && M.n_stream) rc = upload_descs(P.stream_list, &M.stream_desc);
    M.n_long = (int32_t)P.long_list.size();
    if (!rc && M.n_long) {
        std::vector<TileDesc> d;
        for (int32_t sg : P.long_list) d.push_back(desc_of(sg));
        rc = U.put(&M.long_desc, d.data(), d.size(), 0);
        if (!rc) rc = upload_long_pieces(U, M, d);
    }
    M.n_blk = P.win_blk_ptr.empty() ? 0 : (int32_t)P.win_blk_ptr.size() - 1;
    if (!rc && M.n_blk) {
        rc = upload_descs(P.win_list, &M.win_desc);
        if (!rc) rc = U.put(&M.win_blk_ptr, P.win_blk_ptr.data(), P.win_blk_ptr.size(), 0);
    }
    M.n_cwin = (int32_t)P.cwin_list.size();
    if (!rc && M.n_cwin) {
        rc = upload_descs(P.cwin_list, &M.cwin_desc);
        if (!rc) rc = U.put(&M.runs, P.runs.data(), P.runs.size(), 0);
        // 2048-entry tiles read packed 12-bit positions; other capacities 16-bit
        if (!rc && !P.lidx12.empty()) rc = U.put(&M.lidx12, P.lidx12.data(), P.lidx12.size(), 0);
        else if (!rc) rc = U.put(&M.lidx, P.lidx.data(), P.lidx.size(), nz_pad);
    }
    A->n_win_tiles = (int32_t)P.win_list.size();
    for (int32_t sg = 0; sg < P.n_seg(); ++sg)
        if (P.seg_kind[sg] != SEG_LONG)
            A->max_tile_entries = std::max(A->max_tile_entries,
                                           row_ptr[P.seg_bound[sg + 1]] - row_ptr[P.seg_bound[sg]]);
    if (!rc) prepare_launch_queries();
    if (!rc && M.n_blk) {
        hipError_t e2 = prepare_window_kernels();
        if (e2 != hipSuccess) rc = hip_fail(e2, "window kernel LDS opt-in");
    }
    if (rc) {
        U.release_all();
        delete A;
        return rc;
    }
    spmv_info &I = A->info;
    std::memset(&I, 0, sizeof I);
    I.n_rows = n_rows;
    I.n_cols = n_cols;
    I.nnz = nnz;
    I.tile_nnz = P.tile_nnz;
    I.tile_rows = P.tile_rows;
    I.n_tiles = P.n_seg();
    I.n_stream_tiles = M.n_stream;
    I.n_long_rows = M.n_long;
    I.n_window_tiles = (int32_t)P.win_list.size();
    for (int32_t sg : P.cwin_list) I.n_window_tiles += P.win_cnt[sg] > 0 ? 1 : 0;
    I.n_runs = (int64_t)P.runs.size() / 2;
    I.n_window_blocks = M.n_blk;
    I.ring_words = P.ring_words;
    I.window_words = P.window_words;
    I.has_fp32 = M.val32 != nullptr;
    I.has_bf16 = M.val16 != nullptr;
    I.device_bytes = A->bytes;
    I.block_size = 1;
    I.n_long_pieces = M.n_long_pieces;
    I.workspace_bytes = workspace_bytes_of(M);
    I.y_scratch_ok = M.piece_long && M.long_split && (int64_t)M.y_ws_rows >= M.n_long_pieces;
    *out = A;
    return SPMV_OK;
}

extern "C" int spmv_destroy(spmv_matrix *A) {
    clear_error();
    if (!A) return SPMV_OK;
    int rc = SPMV_OK;
    {
        DeviceGuard g(A->device);   // frees are attempted even if the switch failed
        if (g.err != hipSuccess) rc = hip_fail(g.err, "making the matrix's device current");
        std::lock_guard<std::mutex> lock(capture_gate());
        for (void *p : A->allocs) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess && rc == SPMV_OK) rc = hip_fail(e, "hipFree");
        }
    }
    delete A;
    return rc;
}

extern "C" int spmv_spmm(const spmv_matrix *A, int32_t k, const double *X, double *Y, void *stream) {
    clear_error();
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    if (A->M.block != 1) return fail(SPMV_ENOTSUP, "spmv_spmm needs a scalar CSR handle (use bsr3_spmm)");
    if (A->M.format != SPMV_FORMAT_CSR) return fail(SPMV_ENOTSUP, "spmv_spmm needs a CSR-format handle");
    if (k < 1) return fail(SPMV_EINVAL, "k = %d must be >= 1", k);
    if ((int64_t)A->max_tile_entries * 12 > 65536)
        return fail(SPMV_ENOTSUP, "tiles of %d entries exceed the product's LDS staging", A->max_tile_entries);
    if (A->M.n_rows == 0) return SPMV_OK;
    if (!Y) return fail(SPMV_EINVAL, "Y is NULL");
    if (A->M.nnz > 0 && !X) return fail(SPMV_EINVAL, "X is NULL");
    if (X && overlaps(X, sizeof(double) * (size_t)k * (size_t)A->M.n_cols, Y,
                      sizeof(double) * (size_t)k * (size_t)A->M.n_rows))
        return fail(SPMV_EINVAL, "X and Y overlap");
    DeviceGuard g(A->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "making the matrix's device current");
    if (A->M.nnz == 0) {
        const hipError_t z = launch_zero_fill<double>(Y, (int64_t)k * A->M.n_rows, static_cast<hipStream_t>(stream));
        return z == hipSuccess ? SPMV_OK : hip_fail(z, "zero fill");
    }
    const hipError_t e = launch_spmm(A, X, Y, k, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "spmm launch");
    return SPMV_OK;
}

extern "C" int spmv_get_info(const spmv_matrix *A, spmv_info *info) {
    clear_error();
    if (!A || !info) return fail(SPMV_EINVAL, "NULL argument");
    *info = A->info;
    return SPMV_OK;
}

template <typename V, typename T>
static int spmm_typed(const spmv_matrix *A, const V *val, int32_t k, const T *X, T *Y, void *stream) {
    clear_error();
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    if (A->M.block != 3) return fail(SPMV_ENOTSUP, "not a 3x3 block-CSR handle");
    if (k < 1) return fail(SPMV_EINVAL, "k = %d must be >= 1", k);
    const size_t nx = (size_t)3 * A->M.n_cols * k, ny = (size_t)3 * A->M.n_rows * k;
    if (ny && !Y) return fail(SPMV_EINVAL, "Y is NULL");
    if (ny && A->M.nnz && !X) return fail(SPMV_EINVAL, "X is NULL");
    if (X && Y && overlaps(X, nx * sizeof(T), Y, ny * sizeof(T))) return fail(SPMV_EINVAL, "X and Y overlap");
    if (ny == 0) return SPMV_OK;
    DeviceGuard g(A->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "making the matrix's device current");
    if (A->M.nnz == 0) {
        const hipError_t z = launch_zero_fill<T>(Y, (int64_t)ny, static_cast<hipStream_t>(stream));
        return z == hipSuccess ? SPMV_OK : hip_fail(z, "zero fill");
    }
    hipError_t e = launch_bsr3<V, T>(A->M, val, k, X, Y, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "bsr3 launch");
    return SPMV_OK;
}

extern "C" int spmv_apply(const spmv_matrix *A, const double *x, double *y, void *stream) {
    if (A && A->M.block == 3) return spmm_typed<double, double>(A, A->M.val64, 1, x, y, stream);
    return apply_typed<double, double, double, double>(A, A ? A->M.val64 : nullptr, x, y, stream);
}

extern "C" int spmv_workspace_bytes(const spmv_matrix *A, size_t *bytes) {
    clear_error();
    if (!A || !bytes) return fail(SPMV_EINVAL, "NULL argument");
    *bytes = (size_t)workspace_bytes_of(A->M);
    return SPMV_OK;
}

extern "C" int spmv_apply_ws(const spmv_matrix *A, const double *x, double *y, void *ws, size_t ws_bytes,
                             void *stream) {
    clear_error();
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    const size_t need = (size_t)workspace_bytes_of(A->M);
    if (ws_bytes < need)
        return fail(SPMV_EINVAL, "ws_bytes = %zu below the %zu bytes the long rows' pieces need", ws_bytes, need);
    if (need && !ws) return fail(SPMV_EINVAL, "ws is NULL");
    if (need && (reinterpret_cast<uintptr_t>(ws) & 7)) return fail(SPMV_EINVAL, "ws is not 8-byte aligned");
    if (need && x && overlaps(ws, need, x, sizeof(double) * (size_t)A->M.n_cols))
        return fail(SPMV_EINVAL, "ws and x overlap");
    if (need && y && overlaps(ws, need, y, sizeof(double) * (size_t)A->M.n_rows))
        return fail(SPMV_EINVAL, "ws and y overlap");
    if (A->M.block == 3) return spmm_typed<double, double>(A, A->M.val64, 1, x, y, stream);
    return apply_typed<double, double, double, double>(A, A->M.val64, x, y, stream,
                                                       need ? static_cast<double *>(ws) : nullptr);
}

extern "C" int spmv_apply_f32(const spmv_matrix *A, const float *x, float *y, void *stream) {
    if (A && !A->M.val32) return fail(SPMV_ENOTSUP, "matrix has no FP32 copy (create with SPMV_VALUES_FP32)");
    if (A && A->M.block == 3) return spmm_typed<float, float>(A, A->M.val32, 1, x, y, stream);
    return apply_typed<float, float, float, float>(A, A ? A->M.val32 : nullptr, x, y, stream);
}

extern "C" int spmv_apply_f32v(const spmv_matrix *A, const double *x, double *y, void *stream) {
    if (A && A->M.block == 3) return fail(SPMV_ENOTSUP, "not available for block-CSR handles");
    if (A && !A->M.val32) return fail(SPMV_ENOTSUP, "matrix has no FP32 copy (create with SPMV_VALUES_FP32)");
    return apply_typed<float, double, double, double>(A, A ? A->M.val32 : nullptr, x, y, stream);
}

extern "C" int spmv_apply_bf16(const spmv_matrix *A, const float *x, float *y, void *stream) {
    if (A && A->M.block == 3) return fail(SPMV_ENOTSUP, "not available for block-CSR handles");
    if (A && !A->M.val16) return fail(SPMV_ENOTSUP, "matrix has no BF16 copy (create with SPMV_VALUES_BF16)");
    return apply_typed<uint16_t, float, float, float>(A, A ? A->M.val16 : nullptr, x, y, stream);
}

extern "C" int bsr3_spmm(const spmv_matrix *A, int32_t k, const double *X, double *Y, void *stream) {
    return spmm_typed<double, double>(A, A ? A->M.val64 : nullptr, k, X, Y, stream);
}

extern "C" int bsr3_spmm_f32(const spmv_matrix *A, int32_t k, const float *X, float *Y, void *stream) {
    if (A && A->M.block == 3 && !A->M.val32)
        return fail(SPMV_ENOTSUP, "matrix has no FP32 copy (create with SPMV_VALUES_FP32)");
    return spmm_typed<float, float>(A, A ? A->M.val32 : nullptr, k, X, Y, stream);
}

extern "C" int spmv_create_bsr3(int32_t n_block_rows, int32_t n_block_cols, int64_t nnz_blocks,
                                const int32_t *brow_ptr, const int32_t *bcol_idx, const double *bvalues,
                                uint32_t flags, spmv_matrix **out) {
    clear_error();
    if (!out) return fail(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(SPMV_VALUES_FP32 | SPMV_NO_XCD_REMAP | SPMV_DEVICE_PTRS | SPMV_XCD_CONTIGUOUS))
        return fail(SPMV_EINVAL, "unknown flags 0x%x", flags);
    if (nnz_blocks > kMaxNnz / 9) return fail(SPMV_EINVAL, "nnz_blocks = %lld exceeds (2^31 - 2^16) / 9", (long long)nnz_blocks);
    if (flags & SPMV_DEVICE_PTRS) {
        if (n_block_rows < 0 || nnz_blocks < 0)
            return fail(SPMV_EINVAL, "n_block_rows = %d, nnz_blocks = %lld", n_block_rows, (long long)nnz_blocks);
        std::vector<int32_t> rp, ci;
        std::vector<double> va;
        int rc = fetch_device(brow_ptr, (size_t)n_block_rows + 1, rp, "brow_ptr");
        if (!rc) rc = fetch_device(bcol_idx, (size_t)nnz_blocks, ci, "bcol_idx");
        if (!rc) rc = fetch_device(bvalues, 9 * (size_t)nnz_blocks, va, "bvalues");
        if (rc) return rc;
        return spmv_create_bsr3(n_block_rows, n_block_cols, nnz_blocks, rp.data(), nnz_blocks ? ci.data() : nullptr,
                                nnz_blocks ? va.data() : nullptr, flags & ~SPMV_DEVICE_PTRS, out);
    }
    int rc = validate_csr(n_block_rows, n_block_cols, nnz_blocks, brow_ptr, bcol_idx);
    if (rc) return rc;
    if ((int64_t)n_block_rows * 3 > INT32_MAX || (int64_t)n_block_cols * 3 > INT32_MAX)
        return fail(SPMV_EINVAL, "scalar dimension exceeds int32");
    if (nnz_blocks > 0 && !bvalues) return fail(SPMV_EINVAL, "bvalues is NULL with nnz_blocks > 0");
    std::vector<int32_t> tiles = build_bsr_tiles(n_block_rows, brow_ptr, kBsrRows, kBsrBlocks);
    auto *A = new (std::nothrow) spmv_matrix();
    if (!A) return fail(SPMV_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) {
        delete A;
        return hip_fail(e, "hipGetDevice");
    }
    Uploader U(A);
    if (U.init != hipSuccess) {
        delete A;
        return hip_fail(U.init, "upload stream");
    }
    DevMatrix &M = A->M;
    M.block = 3;
    M.n_rows = n_block_rows;
    M.n_cols = n_block_cols;
    M.nnz = nnz_blocks;
    M.xcd_remap = !(flags & SPMV_NO_XCD_REMAP);
    M.xcd_chunk_log2 = (flags & SPMV_XCD_CONTIGUOUS) || default_xcd_chunk(76 * nnz_blocks + 4 * (int64_t)n_block_rows) < 0
                           ? -1 : kDefaultXcdChunkLog2;
    const size_t nb = (size_t)nnz_blocks;
    rc = U.put(&M.row_ptr, brow_ptr, (size_t)n_block_rows + 1, 0);
    if (!rc) rc = U.put(&M.col, bcol_idx, nb, nb + kPad);
    if (!rc) rc = U.put(&M.val64, bvalues, 9 * nb, 9 * nb + kPad);
    if (!rc && (flags & SPMV_VALUES_FP32)) {
        std::vector<float> v32(9 * nb);
        for (size_t k = 0; k < 9 * nb; ++k) v32[k] = (float)bvalues[k];
        rc = U.put(&M.val32, v32.data(), 9 * nb, 9 * nb + kPad);
    }
    M.n_bsr_tiles = (int32_t)tiles.size() - 1;
    if (!rc) rc = U.put(&M.bsr_tiles, tiles.data(), tiles.size(), 0);
    if (rc) {
        U.release_all();
        delete A;
        return rc;
    }
    spmv_info &I = A->info;
    std::memset(&I, 0, sizeof I);
    I.n_rows = n_block_rows;
    I.n_cols = n_block_cols;
    I.nnz = nnz_blocks;
    I.n_tiles = M.n_bsr_tiles;
    I.n_stream_tiles = M.n_bsr_tiles;
    I.has_fp32 = M.val32 != nullptr;
    I.device_bytes = A->bytes;
    I.block_size = 3;
    *out = A;
    return SPMV_OK;
}
