// Host-side plan of the sliced ELLPACK (SELL-C-sigma) storage: the paper's
// slices of rows stored column-wise and padded to the slice's longest row
// (Sec. 4.2, 5.2), with C = 64 rows per slice so that one wavefront lane owns
// one row, and rows sorted by length inside windows of sigma rows so a
// slice's rows have similar lengths and little padding (Kreutzer et al.,
// SIAM J. Sci. Comput. 36(5), 2014).  Pure C++ (no HIP), tested on the CPU.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace spmvlib {

int build_sell_plan(int32_t n_rows, const int32_t *row_ptr, int32_t sigma, SellPlan &S) {
    if (sigma == 0) sigma = 4096;
    if (sigma < kSellC || sigma % kSellC != 0 || sigma > (1 << 24))
        return fail(SPMV_EINVAL, "sell_sigma = %d must be a multiple of %d in [%d, 2^24]", sigma, kSellC, kSellC);
    S = SellPlan{};
    S.sigma = sigma;
    std::vector<int32_t> rows;
    rows.reserve((size_t)n_rows);
    for (int32_t r = 0; r < n_rows; ++r) {
        if (row_ptr[r + 1] - row_ptr[r] > kSellMaxLen) S.long_rows.push_back(r);
        else rows.push_back(r);
    }
    // sigma sorting: inside each window of sigma consecutive short rows,
    // longest first, ties by row index (a fixed order, so plans are reproducible)
    for (size_t w0 = 0; w0 < rows.size(); w0 += (size_t)sigma) {
        const size_t w1 = std::min(rows.size(), w0 + (size_t)sigma);
        std::stable_sort(rows.begin() + w0, rows.begin() + w1, [&](int32_t a, int32_t b) {
            return row_ptr[a + 1] - row_ptr[a] > row_ptr[b + 1] - row_ptr[b];
        });
    }
    S.n_slices = (int32_t)((rows.size() + kSellC - 1) / kSellC);
    S.perm.assign((size_t)S.n_slices * kSellC, -1);
    S.len.assign((size_t)S.n_slices * kSellC, 0);
    S.slice_ptr.assign((size_t)S.n_slices + 1, 0);
    int64_t off = 0;
    for (int32_t sl = 0; sl < S.n_slices; ++sl) {
        int width = 0;
        for (int lane = 0; lane < kSellC; ++lane) {
            const size_t i = (size_t)sl * kSellC + lane;
            if (i >= rows.size()) break;
            const int32_t r = rows[i];
            const int l = row_ptr[r + 1] - row_ptr[r];
            S.perm[i] = r;
            S.len[i] = (uint8_t)l;
            width = std::max(width, l);
        }
        S.slice_ptr[sl] = (int32_t)off;
        off += (int64_t)width * kSellC;
        if (off > (int64_t)INT32_MAX - (1 << 20))
            return fail(SPMV_EINVAL, "SELL storage (%lld padded entries) exceeds 32-bit offsets", (long long)off);
    }
    S.slice_ptr[S.n_slices] = (int32_t)off;
    S.n_entries = off;
    int64_t tail = off;
    for (int32_t r : S.long_rows) {
        S.long_off.push_back(tail);
        tail += row_ptr[r + 1] - row_ptr[r];
    }
    if (tail > (int64_t)INT32_MAX - (1 << 20))
        return fail(SPMV_EINVAL, "SELL storage (%lld entries) exceeds 32-bit offsets", (long long)tail);
    return SPMV_OK;
}

void sell_fill_cols(const SellPlan &S, const int32_t *row_ptr, const int32_t *col_idx, int32_t *out) {
    for (int32_t sl = 0; sl < S.n_slices; ++sl) {
        const int64_t base = S.slice_ptr[sl];
        const int width = (int)((S.slice_ptr[sl + 1] - base) / kSellC);
        for (int lane = 0; lane < kSellC; ++lane) {
            const int64_t slot = (int64_t)sl * kSellC + lane;
            const int32_t r = S.perm[slot];
            const int len = S.len[slot];
            const int32_t pad = (r >= 0 && len > 0) ? col_idx[(int64_t)row_ptr[r] + len - 1] : 0;
            for (int j = 0; j < width; ++j)
                out[base + (int64_t)j * kSellC + lane] = j < len ? col_idx[(int64_t)row_ptr[r] + j] : pad;
        }
    }
    for (size_t i = 0; i < S.long_rows.size(); ++i) {
        const int32_t r = S.long_rows[i];
        std::memcpy(out + S.long_off[i], col_idx + row_ptr[r], sizeof(int32_t) * (size_t)(row_ptr[r + 1] - row_ptr[r]));
    }
}

}  // namespace spmvlib

using namespace spmvlib;

extern "C" int spmv_sell_inspect(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                                 const int32_t *col_idx, int32_t sigma, int32_t *n_slices_out,
                                 int64_t *n_entries_out, int32_t *n_long_out, int32_t *perm, uint8_t *len,
                                 int32_t *slice_ptr, int32_t *col, int32_t *long_rows) {
    clear_error();
    int rc = validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    if (rc) return rc;
    SellPlan S;
    rc = build_sell_plan(n_rows, row_ptr, sigma, S);
    if (rc) return rc;
    if (n_slices_out) *n_slices_out = S.n_slices;
    if (n_entries_out) *n_entries_out = S.n_entries;
    if (n_long_out) *n_long_out = (int32_t)S.long_rows.size();
    if (perm && !S.perm.empty()) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * S.perm.size());
    if (len && !S.len.empty()) std::memcpy(len, S.len.data(), S.len.size());
    if (slice_ptr) std::memcpy(slice_ptr, S.slice_ptr.data(), sizeof(int32_t) * S.slice_ptr.size());
    if (col) sell_fill_cols(S, row_ptr, col_idx, col);
    if (long_rows && !S.long_rows.empty())
        std::memcpy(long_rows, S.long_rows.data(), sizeof(int32_t) * S.long_rows.size());
    return SPMV_OK;
}
