// The opaque handle behind spmv_matrix* (host-side bookkeeping).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <vector>

#include "device.h"
#include "spmv.h"

namespace spmvlib {
// A number no other handle of the process carries (caches key on it, never
// on the handle's address, which a later handle may reuse).
inline uint64_t next_handle_serial() {
    static std::atomic<uint64_t> n{0};
    return ++n;
}
}  // namespace spmvlib

struct spmv_matrix {
    spmvlib::DevMatrix M;
    uint64_t serial = spmvlib::next_handle_serial();
    spmv_info info{};
    int device = 0;
    int64_t bytes = 0;
    std::vector<void *> allocs;
    int32_t n_win_tiles = 0;       // ring-window tiles (all blocks)
    int32_t max_tile_entries = 0;  // stored entries of the largest row tile
};

namespace spmvlib {
// Maps a HIP error to SPMV_ENOMEM / SPMV_EDEVICE with a message.
int hip_fail(hipError_t e, const char *what);

// True when the one-reduction CG (CG_FP64_ONE_REDUCTION) accepts the handle.
bool cg1_eligible(const DevMatrix &M);

// A caller's cache of one solve's device workspace and captured iteration
// graph (FP64 and one-reduction modes), reused by the next solve on the same
// matrix handle and mode, on any stream (every solve ends synchronised): a
// repeat solve then only replays.  Used by one thread at a time; freed with
// cg_cache_free; cg_cache_bytes is the device memory it holds.
struct CgCache;
void cg_cache_free(CgCache *c);
size_t cg_cache_bytes(const CgCache *c);

// cg_solve on an explicit stream; pinned_state (optional) is a caller-owned
// pinned host buffer of at least 256 bytes for the solver's scalar mirror;
// cache (optional) as above.
int cg_run(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter, int32_t mode,
           cg_info *info, hipStream_t s, void *pinned_state, CgCache **cache = nullptr);
}  // namespace spmvlib
