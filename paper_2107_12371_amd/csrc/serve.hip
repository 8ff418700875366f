// Request server with continuous batching over resident mesh matrices.
//
// Requests (k SpMVs, or a CG solve) arrive at any time through srv_submit.
// A scheduler thread admits them as device memory and solver slots free up
// (BudgetLRU: resident matrices + request buffers within an HBM budget,
// least-recently-used idle matrices evicted) and hands out work:
//  * matrices are uploaded by an upload thread, on first request or ahead of
//    time (preloading), so a large upload never stalls the scheduler;
//  * admitted SpMV requests whose matrix is resident form rounds, and a free
//    SpMV lane (a worker thread with its own stream) runs each round: the
//    vectors in, one launch of the multi-matrix kernel k_multi over the
//    tiles of all of the round's vectors, whatever matrix each belongs to (a
//    workgroup finds its item by binary search over the round's tile
//    offsets), the results out.  Requests that move many vector words over
//    the host link get rounds of their own, so small ones keep batching;
//  * each admitted CG request runs on a solver slot: a worker thread with
//    its own stream drives the graph-captured CG iterations, overlapping
//    with the rounds and with the other slots.
// Every row of every result is summed in the order fixed by its matrix's
// plan, and CG reductions have a fixed partition, so a request's result is
// bitwise the same alone and in any mix.  Latency is measured from
// srv_submit to the moment the result is in the caller's host buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "device.h"
#include "internal.h"
#include "launch.h"
#include "matrix.h"
#include "serve_policy.h"
#include "tile.h"

namespace spmvlib {

struct MultiItem {
    const TileDesc *desc;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
    const double *x;
    double *y;
    int32_t tile_begin;  // first workgroup of this item in the launch
    int32_t n_tiles;
};

constexpr int kServeTile = 1024;  // tile capacity of server matrices

// y rows of one stream tile d of item it (a plain FP64 product, rows summed
// in the matrix's plan order).  Ends with prod still being read by the row
// sums: a caller that reuses prod synchronises first.
template <int NT>
__device__ __forceinline__ void multi_tile(const MultiItem &it, const TileDesc &d, double *prod, double *sh) {
    const double *__restrict__ x = it.x;
    TileRegs<double, NT> t;
    t.load(it.col, it.val, d.s, d.e);
    RowPre<double, EPI_PLAIN> pre;
    pre.load(it.row_ptr, x, static_cast<const double *>(nullptr), d.r0, d.r1, d.s & ~3);
    double xv[TileRegs<double, NT>::kMaxPass][4];
    t.gather([x](int c) { return x[c]; }, xv);
    t.products(xv, prod);
    __syncthreads();
    tile_rows<double, double, EPI_PLAIN>(pre, d.r0, d.r1, prod, it.y, nullptr, 0, sh);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void k_multi(const MultiItem *__restrict__ items, int n_items, int total) {
    __shared__ double prod[TileRegs<double, NT>::kProd];
    __shared__ double sh[kBlock / kWave];
    const int b = blockIdx.x;
    if (b >= total) return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const MultiItem it = items[lo];
    multi_tile<NT>(it, it.desc[b - it.tile_begin], prod, sh);
}

// ---------------------------------------------------------------------------
// Persistent multi-matrix kernel.  Instead of one launch per round, a lane
// publishes its round (the MultiItem table already on the device) to a queue
// and one long-lived launch works the tiles of every published round, from
// whichever lane, as they come:
//  * the host half of the queue is coherent pinned host memory: the host
//    writes the rounds and their count, the kernel writes each round's
//    completion;
//  * workgroup 0 is the doorbell: it alone polls host memory (so the host
//    link carries one poller, not hundreds), copies each new round into the
//    device half of the queue and readies the round's ring slot (claim and
//    finish counters);
//  * every other workgroup takes chunks of consecutive tiles, oldest round
//    first, with one fetch-and-add on the round's claim word, works them and
//    counts them finished; the workgroup that finishes a round's last tile
//    publishes the round's completion to the host.  A claim word carries its
//    round's tag, so a workgroup whose add lands after the slot has passed to
//    a later round knows which round's chunk it got, and works that one;
//  * every wave ends by itself: when the host asks it to stop, or when no
//    work has come for the idle time.  The host launches again whenever it
//    publishes work and finds the last launch ended.
// Memory ordering: the host makes a round's buffers complete on the device
// before publishing it; the doorbell's system-scope acquire, its
// device-scope release of the slot, and the workers' acquire of the slot
// order those buffers before the tiles' reads.  Each wave's system-scope
// release after its rows, and the finishing counter's acquire-release, order
// every y row before the completion store the host reads.

constexpr int kRing = 64;        // ring slots; round r may reuse slot r % kRing once round r - kRing is complete
constexpr int kStageTiles = 8;   // tile descriptors staged in LDS at once

struct PersistEntry {
    uint64_t tag;      // round + 1
    uint64_t items;    // device address of the round's MultiItem table
    uint64_t n_items;
    uint64_t shape;    // tiles << 32 | tiles per claim
};

// Host half (coherent pinned host memory).
struct PersistQueue {
    alignas(128) uint64_t published;  // host: rounds published so far
    alignas(128) uint64_t stop;       // host: 1 asks the kernel to end
    alignas(128) PersistEntry ring[kRing];
    alignas(128) uint64_t done[kRing];  // kernel: round + 1 once the round's tiles are all finished
    alignas(128) uint64_t span[kRing];  // kernel: clock ticks from the round's first claim to its last tile
};

// Device half (device memory, zeroed when the server is created).
struct PersistState {
    alignas(128) uint64_t published;  // the doorbell's copy
    alignas(128) uint64_t stop;
    alignas(128) uint64_t activity;   // clock of the latest publication or claim
    alignas(128) PersistEntry ring[kRing];
    alignas(128) uint64_t claim[kRing];     // claim words (claim_word)
    alignas(128) uint32_t finished[kRing];  // tiles finished of the slot's round
    alignas(128) uint64_t t_first[kRing];   // clock of the round's first claim
};

// A slot's claim word: the round's tag (round + 1 mod 2^24), its chunk
// count m (< 2^20) and the chunks claimed so far (an add past m takes
// nothing; the field has room for more such adds than there are workgroups).
// Each field is read from the add's own result, so a late add that lands on
// the slot's next round still knows whether it got a chunk, and of which
// round, without reading the entry of a round that may be complete.
constexpr uint64_t kChunkBits = 20;
constexpr uint64_t kMaxChunks = (uint64_t(1) << kChunkBits) - (uint64_t(1) << 16);
__host__ __device__ constexpr uint64_t claim_word(uint64_t round, uint64_t chunks) {
    return ((round + 1) & 0xFFFFFFull) << 40 | chunks << kChunkBits;
}

__device__ __forceinline__ uint64_t ld_acq_sys(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_acq_dev(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx_dev(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx_dev(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// True once neither this wave nor any other has seen work for idle_ticks.
__device__ __forceinline__ bool persist_idle(const PersistState *st, uint64_t last, uint64_t idle_ticks) {
    const uint64_t t = now_ticks(), a = ld_rlx_dev(&st->activity);
    return t - (a > last ? a : last) > idle_ticks && t > a;
}

// Workgroup 0, lane 0: copies the host's newly published rounds into device
// memory until stopped or idle.  A slot's round is complete before the host
// publishes the next round of that slot, so its counters are free to reset.
__device__ void persist_doorbell(PersistQueue *q, PersistState *st, uint64_t idle_ticks, uint64_t max_polls) {
    if (threadIdx.x != 0) return;
    uint64_t seen = ld_rlx_dev(&st->published);
    uint64_t last = now_ticks(), polls = 0;
    for (;;) {
        // relaxed polls (an acquire would invalidate this XCD's caches on
        // every poll); the acquire fence follows only a change
        const uint64_t stop = __hip_atomic_load(&q->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t p = __hip_atomic_load(&q->published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (p > seen) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            for (uint64_t r = seen; r < p; ++r) {
                const int s = int(r % kRing);
                const PersistEntry *h = &q->ring[s];
                PersistEntry *d = &st->ring[s];
                const uint64_t shape = ld_acq_sys(&h->shape);
                st_rlx_dev(&d->items, ld_acq_sys(&h->items));
                st_rlx_dev(&d->n_items, ld_acq_sys(&h->n_items));
                st_rlx_dev(&d->shape, shape);
                __hip_atomic_store(&st->finished[s], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // the claim word now counts round r's chunks; a worker whose
                // add reads it also sees the entry written above
                const uint64_t n = shape >> 32, g = shape & 0xFFFFFFFFull;
                __hip_atomic_store(&st->claim[s], claim_word(r, (n + g - 1) / g), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&d->tag, r + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            last = now_ticks();
            st_rlx_dev(&st->activity, last);
            __hip_atomic_store(&st->published, p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            seen = p;
            polls = 0;
        }
        if (stop) {
            __hip_atomic_store(&st->stop, uint64_t(1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        // the poll count bounds the wait even if the clock were to stand still
        if (persist_idle(st, last, idle_ticks) || ++polls > 8 * max_polls) return;
        __builtin_amdgcn_s_sleep(8);
    }
}

struct Chunk {
    uint64_t round;   // the round the tiles belong to (-1: end)
    uint32_t first;   // first tile
    uint32_t count;   // tiles
    uint32_t n;       // tiles of the round
};

// Lane 0: the next chunk this workgroup works.  r is the oldest round the
// workgroup may still find work in.
__device__ Chunk persist_claim(PersistState *st, uint64_t &r, uint64_t &pub, uint64_t &last, uint64_t idle_ticks,
                               uint64_t max_polls) {
    uint64_t polls = 0;
    for (;;) {
        if (r >= pub) {
            pub = ld_rlx_dev(&st->published);
            if (r >= pub) {
                if (ld_rlx_dev(&st->stop) || persist_idle(st, last, idle_ticks) || ++polls > max_polls)
                    return Chunk{~uint64_t(0), 0, 0, 0};
                // ~2 us between polls at first, ~14 us once idle for a while:
                // a thousand workgroups polling one word load one memory
                // channel that every other kernel also uses
                __builtin_amdgcn_s_sleep(64);
                if (polls > 32) {
                    __builtin_amdgcn_s_sleep(127);
                    __builtin_amdgcn_s_sleep(127);
                    __builtin_amdgcn_s_sleep(127);
                }
                continue;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the entries of the rounds below pub
        }
        const int s = int(r % kRing);
        PersistEntry *en = &st->ring[s];
        const uint64_t tag = ld_acq_dev(&en->tag);
        if (tag > r + 1) {  // the slot holds a later round: r is complete
            ++r;
            continue;
        }
        if (tag < r + 1) {  // not visible yet (cannot persist: published was read after it)
            if (++polls > max_polls) return Chunk{~uint64_t(0), 0, 0, 0};
            continue;
        }
        const uint64_t mask = (uint64_t(1) << kChunkBits) - 1;
        {  // a load first: a taken-out round costs no add
            const uint64_t w = ld_rlx_dev(&st->claim[s]);
            if ((w & mask) >= ((w >> kChunkBits) & mask)) {
                ++r;
                continue;
            }
        }
        const uint64_t v = __hip_atomic_fetch_add(&st->claim[s], uint64_t(1), __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t j = v & mask, m = (v >> kChunkBits) & mask;
        if (j >= m) {  // every chunk of the slot's round is taken; that round is r or later, so r is done
            ++r;
            continue;
        }
        // chunk j of round x (r, or a later round of the slot, unfinished
        // while this chunk is: its entry is still in the slot)
        const uint64_t x = r + (((v >> 40) - (r + 1)) & 0xFFFFFFull);
        const uint64_t shape = ld_rlx_dev(&en->shape);
        const uint32_t n = uint32_t(shape >> 32), g = uint32_t(shape);
        const uint64_t first = j * g;
        last = now_ticks();
        st_rlx_dev(&st->activity, last);
        if (j == 0) st_rlx_dev(&st->t_first[s], last);
        return Chunk{x, uint32_t(first), uint32_t(n - first < g ? n - first : g), n};
    }
}

// s_waitcnt immediate of gfx9: vmcnt 0 (bits 3:0 and 15:14), expcnt and
// lgkmcnt left at their maxima (7 in bits 6:4, 15 in bits 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

constexpr int kItemWords = (int)(sizeof(MultiItem) / 8);
static_assert(sizeof(MultiItem) % 8 == 0 && kItemWords <= kWave, "MultiItem staged as 8-byte words");
static_assert(offsetof(MultiItem, desc) == 0 && offsetof(MultiItem, tile_begin) % 8 == 0 &&
                  offsetof(MultiItem, n_tiles) == offsetof(MultiItem, tile_begin) + 4,
              "MultiItem layout");
static_assert(sizeof(TileDesc) == 32 && kStageTiles * 8 <= kWave, "descriptors staged one word per lane");

// max_polls bounds each wave's run of empty polls (a backstop of the idle
// clock: far more polls than the idle time holds).
template <int NT>
__global__ __launch_bounds__(kBlock) void k_persist(PersistQueue *q, PersistState *st, uint64_t r_start,
                                                    uint64_t idle_ticks, uint64_t max_polls) {
    if (blockIdx.x == 0) {
        persist_doorbell(q, st, idle_ticks, max_polls);
        return;
    }
    __shared__ double prod[TileRegs<double, NT>::kProd];
    __shared__ double sh[kBlock / kWave];
    __shared__ uint64_t w_it[kItemWords];          // the current item
    __shared__ int32_t w_d[kStageTiles * 8];       // descriptors of the staged tiles
    __shared__ uint64_t w_round;
    __shared__ uint32_t w_first, w_count, w_stage;
    const int lane = threadIdx.x;
    // wave 0's state (lane 0's copy is the one used)
    uint64_t r = r_start, pub = 0, last = now_ticks();
    uint64_t it_round = ~uint64_t(0);  // the round and tile range of the item in w_it
    int32_t it_begin = 0, it_tiles = 0;
    uint32_t n = 0;
    for (;;) {
        if (threadIdx.x < kWave) {
            Chunk c{};
            if (lane == 0) c = persist_claim(st, r, pub, last, idle_ticks, max_polls);
            if (lane == 0) {
                w_round = c.round;
                w_first = c.first;
                w_count = c.count;
                n = c.n;
            }
        }
        __syncthreads();
        const uint64_t x = w_round;
        if (x == ~uint64_t(0)) return;
        const uint32_t end = w_first + w_count;
        for (uint32_t t = w_first; t < end;) {
            if (threadIdx.x < kWave) {
                // the item holding tile t: a 64-way search over the round's
                // item table (sorted by first tile, every item at least one
                // tile), one load per lane a step
                const PersistEntry *en = &st->ring[x % kRing];
                if (x != it_round || (int32_t)t < it_begin || (int32_t)t >= it_begin + it_tiles) {
                    const MultiItem *tab = reinterpret_cast<const MultiItem *>(ld_rlx_dev(&en->items));
                    int hi = (int)ld_rlx_dev(&en->n_items), lo = 0;
                    while (hi - lo > 1) {
                        const int step = (hi - lo + kWave - 1) / kWave;
                        const int idx = lo + lane * step;
                        bool le = false;
                        if (idx < hi)
                            le = __hip_atomic_load(&tab[idx].tile_begin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
                                 (int32_t)t;
                        const unsigned long long m = __ballot(le);  // a prefix of lanes; lane 0 always set
                        lo += (63 - __builtin_clzll(m)) * step;
                        hi = min(lo + step, hi);
                    }
                    const uint64_t *src = reinterpret_cast<const uint64_t *>(tab + lo);
                    const uint64_t wv = lane < kItemWords ? ld_rlx_dev(src + lane) : 0;
                    if (lane < kItemWords) w_it[lane] = wv;
                    const uint64_t range =
                        __shfl((unsigned long long)wv, (int)(offsetof(MultiItem, tile_begin) / 8), kWave);
                    it_begin = (int32_t)(uint32_t)range;
                    it_tiles = (int32_t)(uint32_t)(range >> 32);
                    it_round = x;
                }
                // descriptors of up to kStageTiles tiles of this item, one
                // word per lane
                const uint32_t item_end = (uint32_t)(it_begin + it_tiles);
                const uint32_t stage_end = min(min(end, item_end), t + (uint32_t)kStageTiles);
                const uint64_t dp = __shfl((unsigned long long)w_it[0], 0, kWave);
                const int32_t *dsrc = reinterpret_cast<const int32_t *>(reinterpret_cast<const TileDesc *>(dp) +
                                                                        ((int32_t)t - it_begin));
                if (lane < (int)(stage_end - t) * 8)
                    w_d[lane] = __hip_atomic_load(dsrc + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lane == 0) w_stage = stage_end - t;
            }
            __syncthreads();
            const uint32_t ns = w_stage;
            // the staged tiles in a two-deep pipeline: the next tile's
            // stream loads go out right after this tile's gathers, so their
            // latency hides behind this tile's products and row sums
            const MultiItem &it = *reinterpret_cast<const MultiItem *>(w_it);
            const TileDesc *dd = reinterpret_cast<const TileDesc *>(w_d);
            const double *__restrict__ xx = it.x;
            TileRegs<double, NT> ta, tb;
            RowPre<double, EPI_PLAIN> pa, pb;
            auto load = [&](TileRegs<double, NT> &tr, RowPre<double, EPI_PLAIN> &pr, uint32_t u) {
                const TileDesc d = dd[u];
                tr.load(it.col, it.val, d.s, d.e);
                pr.load(it.row_ptr, xx, static_cast<const double *>(nullptr), d.r0, d.r1, d.s & ~3);
            };
            auto step = [&](TileRegs<double, NT> &cur, RowPre<double, EPI_PLAIN> &pcur, TileRegs<double, NT> &nxt,
                            RowPre<double, EPI_PLAIN> &pnxt, uint32_t u) {
                double xv[TileRegs<double, NT>::kMaxPass][4];
                cur.gather([xx](int c) { return xx[c]; }, xv);
                if (u + 1 < ns) load(nxt, pnxt, u + 1);
                cur.products(xv, prod);
                __syncthreads();
                const TileDesc d = dd[u];
                tile_rows<double, double, EPI_PLAIN>(pcur, d.r0, d.r1, prod, it.y, nullptr, 0, sh);
                __syncthreads();  // prod, and after the last tile w_it and w_d, free for reuse
            };
            load(ta, pa, 0);
            for (uint32_t u = 0; u < ns; u += 2) {
                step(ta, pa, tb, pb, u);
                if (u + 1 < ns) step(tb, pb, ta, pa, u + 1);
            }
            t += ns;
        }
        // every wave's rows reach the L2 (its stores complete) before the
        // barrier; thread 0's system-scope release then writes that L2 back
        // once for the workgroup (one writeback per chunk: each one is a
        // device-wide serialised step, so one per wave would cost five times
        // as much)
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int s = int(x % kRing);
            const uint32_t cnt = w_count;
            const uint32_t old =
                __hip_atomic_fetch_add(&st->finished[s], cnt, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
            if (old + cnt == n) {  // the round's last tiles: tell the host
                __hip_atomic_store(&q->span[s], now_ticks() - ld_rlx_dev(&st->t_first[s]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&q->done[s], x + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int32_t mid = 0, op = 0, k = 1, max_iter = 0;
    const spmv_matrix *A = nullptr;  // resident handle, set at dispatch (pinned from admission until done)
    uint32_t gen = 0;                // upload attempt of its matrix that it waits for
    const double *in = nullptr;
    double *out = nullptr;
    double tol = 0.0;
    uint64_t extra = 0;
    Clock::time_point t_submit, t_start, t_done;
    Clock::time_point t_run{};  // a lane or slot began its work
    // from HIP events on the lane's or slot's stream: host -> device copies
    // (with the buffers' stream-ordered allocation), the device work, the
    // copies back; the device work's interval on the server's device clock
    double copy_in_s = -1.0, compute_s = -1.0, copy_out_s = -1.0;
    double dev_begin_s = -1.0, dev_end_s = -1.0;
    double graph_s = 0.0;       // CG: graph capture and instantiation inside the solve
    double kernel_s = -1.0;     // SpMV on the persistent kernel: the round's first claim to its last tile
    bool done = false;
    int status = SPMV_OK;
    char message[160] = {0};
    int iterations = 0;
    double rel_residual = 0.0;
};

struct MatrixEntry {
    int32_t n_rows = 0, n_cols = 0;
    std::vector<int32_t> row_ptr, col_idx;  // host copy, immutable once added
    std::vector<double> values;
    // device state, under the server's mutex: a matrix is ready when dev is
    // set and no upload is running; an upload attempt that fails records its
    // generation and message for the requests that waited on it
    spmv_matrix *dev = nullptr;
    bool uploading = false;
    uint32_t gen = 0, failed_gen = 0;
    char error[160] = {0};
};

// Four events on a worker's stream: before the copies in, before the device
// work, after it, after the copies out.
struct PhaseEvents {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ok = false;
    hipError_t create() {
        for (auto &e : ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        ok = true;
        return hipSuccess;
    }
    void destroy() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i, hipStream_t s) const {
        if (ok) (void)hipEventRecord(ev[i], s);
    }
    // after the stream has synchronised: phase times, and the device-work
    // interval relative to the reference event `ref`
    void fill(Request *r, hipEvent_t ref) const {
        if (!ok) return;
        float a = 0, b = 0, c = 0;
        if (hipEventElapsedTime(&a, ev[0], ev[1]) == hipSuccess) r->copy_in_s = 1e-3 * a;
        if (hipEventElapsedTime(&b, ev[1], ev[2]) == hipSuccess) r->compute_s = 1e-3 * b;
        if (hipEventElapsedTime(&c, ev[2], ev[3]) == hipSuccess) r->copy_out_s = 1e-3 * c;
        float t0 = 0, t1 = 0;
        if (ref && hipEventElapsedTime(&t0, ref, ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t1, ref, ev[2]) == hipSuccess) {
            r->dev_begin_s = 1e-3 * t0;
            r->dev_end_s = 1e-3 * t1;
        }
    }
};

struct Slot {
    std::thread th;
    hipStream_t stream = nullptr;
    void *pinned = nullptr;
    PhaseEvents pe;
    Request *job = nullptr;
    CgCache *cache = nullptr;  // the solver checked out for the running solve
};

// An SpMV lane: a worker thread with its own stream that runs one round at a
// time (copies in, one k_multi launch, copies out), so that a round moving a
// large request's vectors over the host link does not hold up the others.
// Host copies of large request buffers go through pinned memory.  Measured
// on the part with 512 MB: the runtime's path for pageable memory moves
// 10 GB/s device to host into freshly allocated pages (17 GB/s into pages
// already touched) and 28 GB/s host to device, against 57 GB/s between the
// device and pinned memory.  A buffer of at least kStageMin bytes moves in
// chunks of kStageChunk through two pinned buffers of its lane: the DMA of
// one chunk overlaps the host copy of the next, and each host copy is split
// over the server's copy threads (which also take the first-touch page
// faults of a fresh output buffer in parallel).
constexpr size_t kStageChunk = size_t(16) << 20;
constexpr size_t kStageMin = size_t(4) << 20;

// A fixed pool of threads for splitting large memcpy calls.  Any number of
// threads may call copy() at once; each waits for its own parts only.
class CopyPool {
  public:
    explicit CopyPool(int n) {
        for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    CopyPool(const CopyPool &) = delete;
    CopyPool &operator=(const CopyPool &) = delete;

    void copy(void *dst, const void *src, size_t bytes) {
        const size_t parts = th_.size() + 1;  // the caller copies one part itself
        if (bytes < (size_t(1) << 20) || parts == 1) {
            std::memcpy(dst, src, bytes);
            return;
        }
        const size_t per = ((bytes + parts - 1) / parts + 4095) & ~size_t(4095);
        Job job;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (size_t off = per; off < bytes; off += per) {
                q_.push_back({&job, static_cast<char *>(dst) + off, static_cast<const char *>(src) + off,
                              std::min(per, bytes - off)});
                ++job.left;
            }
        }
        cv_.notify_all();
        std::memcpy(dst, src, std::min(per, bytes));
        std::unique_lock<std::mutex> lk(job.m);
        job.cv.wait(lk, [&] { return job.left == 0; });
    }

  private:
    struct Job {
        std::mutex m;
        std::condition_variable cv;
        size_t left = 0;
    };
    struct Part {
        Job *job;
        char *dst;
        const char *src;
        size_t n;
    };
    void loop() {
        for (;;) {
            Part t;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
                if (q_.empty()) return;  // stop_ and nothing left
                t = q_.front();
                q_.pop_front();
            }
            std::memcpy(t.dst, t.src, t.n);
            std::lock_guard<std::mutex> lk(t.job->m);
            if (--t.job->left == 0) t.job->cv.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Part> q_;
    std::vector<std::thread> th_;
    bool stop_ = false;
};

struct Lane {
    std::thread th;
    hipStream_t stream = nullptr;
    MultiItem *items_host = nullptr;  // pinned staging of the round's item table
    size_t items_cap = 0;
    PhaseEvents pe;
    std::vector<Request *> job;
    bool busy = false;
    // pinned staging of large request buffers (allocated on first use)
    void *stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};  // last DMA that used each buffer
    bool stage_pending[2] = {false, false};
    uint64_t stage_next = 0;  // the buffer of the next chunk: stage_next & 1
};

// The persistent kernel's host side (cfg.persistent_wgs > 0).
struct Persist {
    PersistQueue *q = nullptr;   // coherent pinned host memory
    PersistQueue *qd = nullptr;  // its device address
    PersistState *st = nullptr;  // device memory
    hipStream_t stream = nullptr;
    hipEvent_t end = nullptr;  // recorded after each launch
    bool launched = false;
    std::mutex mu;
    std::condition_variable cv;  // a ring slot freed
    uint64_t next = 0;           // rounds published
    std::set<uint64_t> open;     // published rounds not yet seen complete
    int wgs = 0;                 // workgroups per launch (doorbell included)
    uint64_t idle_ticks = 0;     // wall-clock ticks of idle time before a launch ends
    uint64_t max_polls = 0;      // empty polls a worker wave makes at most in a row (8x for the doorbell)
    double tick_s = 0.0;         // seconds per tick
    int64_t launches = 0;
};

// A request that has waited this long for device memory holds back every
// younger one (none is admitted before it), so a request that fits only in
// a nearly empty budget is not starved by a stream of small ones.
constexpr auto kStarveAfter = std::chrono::milliseconds(50);

// Requests moving at least this many vector words between host and device
// get rounds of their own.
constexpr int64_t kLargeRequestWords = int64_t(1) << 22;

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

}  // namespace

struct Server {
    srv_config cfg{};
    int device = 0;
    CopyPool copier{(int)std::max(1u, std::min(6u, std::thread::hardware_concurrency() / 2))};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_slot, cv_upload, cv_ready, cv_lane;
    std::deque<Request *> incoming, pending;
    std::vector<Request *> waiting_spmv;  // admitted SpMV requests not yet in a round
    std::deque<int> upload_queue;         // matrices for the upload thread
    int uploads_in_flight = 0;
    bool wake = false;                    // something the scheduler waits for changed
    std::unordered_map<uint64_t, Request *> all;
    std::deque<MatrixEntry> mats;  // stable element addresses; indexed under `mu` only
    BudgetLRU policy;
    std::vector<Slot> slots;
    std::vector<Lane> lanes;
    std::thread scheduler, uploader;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, failed = 0, rounds = 0;
    int in_flight_spmv = 0;
    bool stop = false;
    std::vector<double> latencies;
    Clock::time_point t_first{}, t_last{};
    bool any_submit = false;
    hipEvent_t ref_event = nullptr;  // zero of the device clock the requests' intervals are read on
    Persist P;
    // Solvers (device workspace + captured iteration graph of an FP64 solve)
    // kept per matrix handle, by its serial, for the next solve on it from
    // any slot: checked out while a solve runs, least recently used dropped
    // beyond solver_cap bytes, dropped with their matrix.  Under `mu`.
    struct SolverEntry {
        CgCache *c;
        uint64_t bytes;
        std::list<uint64_t>::iterator lru;
    };
    std::unordered_map<uint64_t, SolverEntry> solvers;
    std::list<uint64_t> solver_lru;  // front: most recently checked in
    uint64_t solver_bytes = 0, solver_cap = 0;
    int64_t solver_hits = 0, solver_solves = 0;

    CgCache *checkout_solver_locked(uint64_t serial) {
        auto it = solvers.find(serial);
        if (it == solvers.end()) return nullptr;
        CgCache *c = it->second.c;
        solver_bytes -= it->second.bytes;
        solver_lru.erase(it->second.lru);
        solvers.erase(it);
        ++solver_hits;
        return c;
    }

    // Returns the solvers to free (outside the lock: freeing takes the
    // capture gate).
    std::vector<CgCache *> checkin_solver_locked(uint64_t serial, CgCache *c) {
        std::vector<CgCache *> out;
        if (!c) return out;
        const uint64_t b = cg_cache_bytes(c);
        if (b == 0 || b > solver_cap || solvers.count(serial)) {
            out.push_back(c);  // empty, too large, or another slot's solver is already kept
            return out;
        }
        solver_lru.push_front(serial);
        solvers[serial] = SolverEntry{c, b, solver_lru.begin()};
        solver_bytes += b;
        while (solver_bytes > solver_cap && !solver_lru.empty()) {
            const uint64_t victim = solver_lru.back();
            auto it = solvers.find(victim);
            solver_bytes -= it->second.bytes;
            out.push_back(it->second.c);
            solver_lru.pop_back();
            solvers.erase(it);
        }
        return out;
    }

    void drop_solver_locked(uint64_t serial, std::vector<CgCache *> &out) {
        auto it = solvers.find(serial);
        if (it == solvers.end()) return;
        solver_bytes -= it->second.bytes;
        solver_lru.erase(it->second.lru);
        out.push_back(it->second.c);
        solvers.erase(it);
    }

    explicit Server(const srv_config &c) : cfg(c), policy(c.hbm_budget_bytes) {}

    uint64_t matrix_bytes(const MatrixEntry &m) const {
        const uint64_t nz = m.col_idx.size(), pad = ((nz + 3) & ~(uint64_t)3) + kPad;
        uint64_t b = 4ull * (m.n_rows + 1) + 12ull * pad + 64ull * (nz / 512 + 16);
        if (cfg.cg_mode == CG_MIXED_FP32) b += 4ull * pad;
        return b;
    }

    uint64_t request_bytes(const Request &r) const {
        const MatrixEntry &m = mats[r.mid];
        if (r.op == SRV_SPMV) return 8ull * (uint64_t)r.k * (uint64_t)(m.n_rows + m.n_cols);
        // b, x and the solver workspace (4 vectors + partials), FP32 copies for MIXED
        uint64_t b = 8ull * m.n_rows * 7 + 8ull * (m.col_idx.size() / 1000 + 4096);
        if (cfg.cg_mode == CG_MIXED_FP32) b += 4ull * m.n_rows * 5;
        return b;
    }

    // Marks r done.  A failed request keeps `msg`, else the message of the
    // error the calling thread has just recorded.
    void finish_locked(Request *r, int status, const char *msg = nullptr) {
        r->status = status;
        if (status != SPMV_OK) std::snprintf(r->message, sizeof r->message, "%s", msg ? msg : last_error());
        r->t_done = Clock::now();
        r->done = true;
        if (status == SPMV_OK) {
            ++completed;
            latencies.push_back(seconds(r->t_submit, r->t_done));
        } else {
            ++failed;
        }
        t_last = r->t_done;
        wake = true;
        cv_done.notify_all();
    }

    // The device handle of a server matrix (FP32 copy for mixed-precision
    // solves).  Reads only the entry's immutable host arrays.
    int create_handle(const MatrixEntry &m, spmv_matrix **out) const {
        spmv_params p{};
        p.tile_nnz = kServeTile;
        p.window_mode = SPMV_WINDOW_OFF;
        p.kernel = KV_ONE_TILE;
        const uint32_t flags = cfg.cg_mode == CG_MIXED_FP32 ? SPMV_VALUES_FP32 : 0u;
        return spmv_create(m.n_rows, m.n_cols, (int64_t)m.col_idx.size(), m.row_ptr.data(),
                           m.col_idx.empty() ? nullptr : m.col_idx.data(),
                           m.values.empty() ? nullptr : m.values.data(), flags, &p, out);
    }

    // Queues matrix mid for the upload thread; the policy already counts it
    // resident.  The upload holds its own pin until it ends.
    void start_upload_locked(int mid) {
        MatrixEntry &m = mats[mid];
        m.uploading = true;
        ++m.gen;
        policy.pin(mid);
        ++uploads_in_flight;
        upload_queue.push_back(mid);
        cv_upload.notify_one();
    }

    // Uploads run here, off the scheduler, so that rounds and admissions go
    // on while a large matrix is copied.
    void uploader_loop() {
        const hipError_t dev_err = hipSetDevice(device);
        for (;;) {
            int mid;
            MatrixEntry *m;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_upload.wait(lk, [&] { return stop || !upload_queue.empty(); });
                if (upload_queue.empty()) return;
                mid = upload_queue.front();
                upload_queue.pop_front();
                // the element's address is taken under the lock (indexing
                // reads the deque's block map, which srv_add_matrix may
                // reallocate); the element itself never moves
                m = &mats[mid];
            }
            clear_error();
            (void)hipGetLastError();
            spmv_matrix *h = nullptr;
            const int rc = dev_err != hipSuccess ? hip_fail(dev_err, "server upload thread: hipSetDevice")
                                                 : create_handle(*m, &h);
            std::lock_guard<std::mutex> lk(mu);
            MatrixEntry &e = *m;
            e.uploading = false;
            if (rc == SPMV_OK) {
                e.dev = h;
                policy.resize(mid, (uint64_t)h->bytes);
            } else {
                e.failed_gen = e.gen;
                std::snprintf(e.error, sizeof e.error, "%s", last_error());
                policy.unload(mid);  // waiting requests fail; a later request uploads again
            }
            policy.release(mid, 0);
            --uploads_in_flight;
            wake = true;
            cv_ready.notify_all();
            cv_sched.notify_all();
            cv_done.notify_all();
        }
    }

    // Launches the persistent kernel unless a launch is still running.
    // Caller holds P.mu.
    int persist_ensure_locked() {
        if (P.launched) {
            const hipError_t q = hipEventQuery(P.end);
            if (q == hipErrorNotReady) return SPMV_OK;
            if (q != hipSuccess) return hip_fail(q, "persistent kernel");
        }
        const uint64_t r0 = P.open.empty() ? P.next : *P.open.begin();
        hipLaunchKernelGGL((k_persist<kServeTile>), dim3(P.wgs), dim3(kBlock), 0, P.stream, P.qd, P.st, r0,
                           P.idle_ticks, P.max_polls);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(P.end, P.stream);
        if (e != hipSuccess) return hip_fail(e, "persistent kernel launch");
        P.launched = true;
        ++P.launches;
        return SPMV_OK;
    }

    // Publishes a round whose item table and vectors are complete on the
    // device, and waits until the persistent kernel has finished it.
    int persist_round(const MultiItem *ditems, int n_items, int total, double *kernel_s) {
        uint64_t seq;
        int rc;
        {
            std::unique_lock<std::mutex> lk(P.mu);
            // the slot's previous round (P.next - kRing) must be complete; a
            // round that never completed (its lane reported the error) keeps
            // its slot, so the wait is bounded
            if (!P.cv.wait_for(lk, std::chrono::seconds(120),
                               [&] { return P.open.empty() || *P.open.begin() + kRing > P.next; }))
                return fail(SPMV_EDEVICE, "persistent kernel: queue slot not free in 120 s");
            seq = P.next;
            PersistEntry &en = P.q->ring[seq % kRing];
            // about two claims per worker on a large round (each chunk ends
            // with an L2 writeback), one tile each on a small one
            const int64_t workers = std::max(1, P.wgs - 1);
            int64_t g = std::min<int64_t>(512, std::max<int64_t>(1, (total + 2 * workers - 1) / (2 * workers)));
            g = std::max<int64_t>(g, ((int64_t)total + (int64_t)kMaxChunks - 1) / (int64_t)kMaxChunks);
            en.items = reinterpret_cast<uint64_t>(ditems);
            en.n_items = (uint64_t)n_items;
            en.shape = ((uint64_t)(uint32_t)total << 32) | (uint64_t)g;
            __atomic_store_n(&en.tag, seq + 1, __ATOMIC_RELEASE);
            __atomic_store_n(&P.q->published, seq + 1, __ATOMIC_RELEASE);
            ++P.next;
            P.open.insert(seq);
            rc = persist_ensure_locked();
        }
        // the kernel finishes the round, or, if the launch ended first (its
        // idle time ran out as the round came), a new launch does; a launch
        // fault ends the wait with its error
        const uint64_t *done = &P.q->done[seq % kRing];
        const Clock::time_point t0 = Clock::now();
        Clock::time_point t_check = t0;
        while (rc == SPMV_OK && __atomic_load_n(done, __ATOMIC_ACQUIRE) != seq + 1) {
            const Clock::time_point t = Clock::now();
            // yield while the round is young, then sleep in short steps
            if (t - t0 < std::chrono::microseconds(500)) std::this_thread::yield();
            else std::this_thread::sleep_for(std::chrono::microseconds(20));
            if (t - t_check > std::chrono::microseconds(50)) {
                t_check = t;
                std::lock_guard<std::mutex> lk(P.mu);
                if (__atomic_load_n(done, __ATOMIC_ACQUIRE) != seq + 1) rc = persist_ensure_locked();
            }
            if (t - t0 > std::chrono::seconds(120)) rc = fail(SPMV_EDEVICE, "persistent kernel: round not finished in 120 s");
        }
        if (rc != SPMV_OK) return rc;  // the round stays open: its buffers are never freed
        *kernel_s = (double)__atomic_load_n(&P.q->span[seq % kRing], __ATOMIC_RELAXED) * P.tick_s;
        std::lock_guard<std::mutex> lk(P.mu);
        P.open.erase(seq);
        P.cv.notify_all();
        return SPMV_OK;
    }

    // One round on lane ln: every SpMV vector of the round's requests in one
    // launch.  Frees the lane when done.
    // The lane's pinned staging (allocated on first use); false when it
    // cannot be had, and the caller keeps the runtime's pageable copy.
    bool stage_ready(Lane &ln) {
        if (ln.stage[0]) return true;
        std::lock_guard<std::mutex> gate(capture_gate());
        void *a = nullptr, *b = nullptr;
        hipEvent_t ea = nullptr, eb = nullptr;
        if (hipHostMalloc(&a, kStageChunk, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b, kStageChunk, hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&ea, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&eb, hipEventDisableTiming) == hipSuccess) {
            ln.stage[0] = a;
            ln.stage[1] = b;
            ln.stage_ev[0] = ea;
            ln.stage_ev[1] = eb;
            return true;
        }
        (void)hipGetLastError();
        if (a) (void)hipHostFree(a);
        if (b) (void)hipHostFree(b);
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        return false;
    }

    // Waits for the last DMA that used staging buffer b.
    static hipError_t stage_wait(Lane &ln, int b) {
        if (!ln.stage_pending[b]) return hipSuccess;
        ln.stage_pending[b] = false;
        return hipEventSynchronize(ln.stage_ev[b]);
    }

    // Host to device on the lane's stream: large buffers through the staging
    // (the host returns once the last chunk is handed to the DMA).
    hipError_t copy_in(Lane &ln, void *dst, const void *src, size_t bytes) {
        if (bytes < kStageMin || !stage_ready(ln))
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ln.stream);
        for (size_t off = 0; off < bytes; off += kStageChunk) {
            const int b = (int)(ln.stage_next++ & 1);
            const size_t len = std::min(kStageChunk, bytes - off);
            hipError_t e = stage_wait(ln, b);
            if (e != hipSuccess) return e;
            copier.copy(ln.stage[b], static_cast<const char *>(src) + off, len);
            e = hipMemcpyAsync(static_cast<char *>(dst) + off, ln.stage[b], len, hipMemcpyHostToDevice, ln.stream);
            if (e == hipSuccess) e = hipEventRecord(ln.stage_ev[b], ln.stream);
            if (e != hipSuccess) return e;
            ln.stage_pending[b] = true;
        }
        return hipSuccess;
    }

    // Device to host: large buffers through the staging, and then the data
    // is in dst when the call returns (*staged = true, *tail_s = host time
    // after the last chunk's DMA); smaller ones are enqueued on the stream.
    hipError_t copy_out(Lane &ln, void *dst, const void *src, size_t bytes, bool *staged, double *tail_s) {
        *staged = false;
        if (bytes < kStageMin || !stage_ready(ln))
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ln.stream);
        *staged = true;
        const size_t n = (bytes + kStageChunk - 1) / kStageChunk;
        const uint64_t first = ln.stage_next;
        ln.stage_next += n;
        auto enqueue = [&](size_t i) {
            const int b = (int)((first + i) & 1);
            const size_t off = i * kStageChunk;
            hipError_t e = stage_wait(ln, b);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ln.stage[b], static_cast<const char *>(src) + off, std::min(kStageChunk, bytes - off),
                                   hipMemcpyDeviceToHost, ln.stream);
            if (e == hipSuccess) e = hipEventRecord(ln.stage_ev[b], ln.stream);
            if (e == hipSuccess) ln.stage_pending[b] = true;
            return e;
        };
        hipError_t e = enqueue(0);
        for (size_t i = 0; i < n && e == hipSuccess; ++i) {
            // the next chunk's DMA runs while this one is copied out
            if (i + 1 < n) e = enqueue(i + 1);
            const int b = (int)((first + i) & 1);
            if (e == hipSuccess) e = stage_wait(ln, b);
            if (e != hipSuccess) break;
            const Clock::time_point t0 = Clock::now();
            const size_t off = i * kStageChunk;
            copier.copy(static_cast<char *>(dst) + off, ln.stage[b], std::min(kStageChunk, bytes - off));
            *tail_s = std::chrono::duration<double>(Clock::now() - t0).count();
        }
        return e;
    }

    void run_round(std::vector<Request *> &round, Lane &ln) {
        const hipStream_t batch = ln.stream;
        clear_error();
        (void)hipGetLastError();  // drop an error an earlier call of this thread left behind
        const Clock::time_point t_run = Clock::now();
        ln.pe.mark(0, batch);
        std::vector<MultiItem> items;
        std::vector<std::pair<Request *, std::pair<double *, double *>>> bufs;
        // piece sums of long rows (products run one after another on the
        // lane's stream, so one workspace serves the round)
        double *lws = nullptr;
        size_t lws_n = 0;
        int total = 0;
        int err = SPMV_OK;
        bool abandoned = false;
        double kernel_s = -1.0;  // persistent kernel: its busy time on the round
        for (Request *r : round) {
            const DevMatrix &M = r->A->M;
            double *din = nullptr, *dout = nullptr;
            const size_t nin = (size_t)r->k * M.n_cols, nout = (size_t)r->k * M.n_rows;
            hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&din), 8 * std::max<size_t>(nin, 1), batch);
            if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void **>(&dout), 8 * std::max<size_t>(nout, 1), batch);
            if (e == hipSuccess && nin) e = copy_in(ln, din, r->in, 8 * nin);
            if (e != hipSuccess) err = hip_fail(e, "server round buffers");
            bufs.push_back({r, {din, dout}});
            for (int j = 0; j < r->k && e == hipSuccess; ++j) {
                const double *x = din + (size_t)j * M.n_cols;
                double *y = dout + (size_t)j * M.n_rows;
                if (M.n_long > 0) {
                    // rows longer than a tile: the matrix's own launch
                    // sequence, their pieces on a workgroup each
                    if (M.piece_long && (size_t)M.n_long_pieces > lws_n) {
                        if (lws) (void)hipFreeAsync(lws, batch);
                        lws = nullptr;
                        lws_n = 0;
                        e = hipMallocAsync(reinterpret_cast<void **>(&lws), 8 * (size_t)M.n_long_pieces, batch);
                        if (e != hipSuccess) {
                            err = hip_fail(e, "server long-row workspace");
                            lws = nullptr;
                            continue;
                        }
                        lws_n = (size_t)M.n_long_pieces;
                    }
                    e = launch_spmv<double, double, double, double>(M, M.val64, x, y, EPI_PLAIN, nullptr, nullptr,
                                                                    nullptr, batch, M.piece_long ? lws : nullptr);
                    if (e != hipSuccess) err = hip_fail(e, "server spmv");
                    continue;
                }
                if (M.n_stream == 0) continue;
                MultiItem it{M.stream_desc, M.row_ptr, M.col, M.val64, x, y, total, M.n_stream};
                items.push_back(it);
                total += M.n_stream;
            }
        }
        ln.pe.mark(1, batch);
        if (err == SPMV_OK && !items.empty()) {
            if (items.size() > ln.items_cap) {
                std::lock_guard<std::mutex> gate(capture_gate());
                if (ln.items_host) (void)hipHostFree(ln.items_host);
                ln.items_cap = std::max<size_t>(items.size(), 2 * ln.items_cap);
                hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&ln.items_host),
                                             ln.items_cap * sizeof(MultiItem), hipHostMallocDefault);
                if (e != hipSuccess) {
                    ln.items_host = nullptr;
                    ln.items_cap = 0;
                    err = hip_fail(e, "server item staging");
                }
            }
            if (err == SPMV_OK) {
                std::memcpy(ln.items_host, items.data(), items.size() * sizeof(MultiItem));
                MultiItem *ditems = nullptr;
                hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&ditems), items.size() * sizeof(MultiItem), batch);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(ditems, ln.items_host, items.size() * sizeof(MultiItem), hipMemcpyHostToDevice,
                                       batch);
                bool keep = false;  // buffers a round that never finished may still be read from
                if (e == hipSuccess && P.wgs > 0) {
                    e = hipStreamSynchronize(batch);
                    if (e == hipSuccess) {
                        err = persist_round(ditems, (int)items.size(), total, &kernel_s);
                        keep = err != SPMV_OK;
                    }
                } else if (e == hipSuccess) {
                    hipLaunchKernelGGL((k_multi<kServeTile>), dim3(total), dim3(kBlock), 0, batch, ditems,
                                       (int)items.size(), total);
                    e = hipGetLastError();
                }
                if (ditems && !keep) (void)hipFreeAsync(ditems, batch);
                if (keep) abandoned = true;
                if (e != hipSuccess) err = hip_fail(e, "server round launch");
            }
        }
        ln.pe.mark(2, batch);
        // host time after the last event of the round when the last copy
        // out was staged (its final chunk is copied after its DMA)
        double copy_tail_s = 0.0;
        for (auto &b : bufs) {
            Request *r = b.first;
            const size_t nout = (size_t)r->k * r->A->M.n_rows;
            if (err == SPMV_OK && nout) {
                bool staged = false;
                double tail = 0.0;
                hipError_t e = copy_out(ln, r->out, b.second.second, 8 * nout, &staged, &tail);
                copy_tail_s = staged ? tail : 0.0;
                if (e != hipSuccess) err = hip_fail(e, "server result copy");
            }
        }
        ln.pe.mark(3, batch);
        hipError_t e = hipStreamSynchronize(batch);
        if (e != hipSuccess && err == SPMV_OK) err = hip_fail(e, "server round");
        ln.stage_pending[0] = ln.stage_pending[1] = false;  // the stream has drained
        for (auto &b : bufs) {
            if (abandoned) break;
            if (b.second.first) (void)hipFreeAsync(b.second.first, batch);
            if (b.second.second) (void)hipFreeAsync(b.second.second, batch);
        }
        if (lws && !abandoned) (void)hipFreeAsync(lws, batch);
        std::lock_guard<std::mutex> lk(mu);
        ++rounds;
        for (Request *r : round) {
            r->t_run = t_run;
            r->kernel_s = kernel_s;
            if (e == hipSuccess) {
                ln.pe.fill(r, ref_event);
                r->copy_out_s += copy_tail_s;
            }
            policy.release(r->mid, r->extra);
            --in_flight_spmv;
            finish_locked(r, err);
        }
        round.clear();
        ln.busy = false;
    }

    void lane_loop(int li) {
        const hipError_t dev_err = hipSetDevice(device);
        Lane &ln = lanes[li];
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_lane.wait(lk, [&] { return stop || ln.busy; });
                if (!ln.busy) return;
                if (dev_err != hipSuccess) {
                    for (Request *r : ln.job) {
                        policy.release(r->mid, r->extra);
                        --in_flight_spmv;
                        finish_locked(r, hip_fail(dev_err, "server lane thread: hipSetDevice"));
                    }
                    ln.job.clear();
                    ln.busy = false;
                    continue;
                }
            }
            run_round(ln.job, ln);
        }
    }

    int free_lane_locked() const {
        for (size_t i = 0; i < lanes.size(); ++i)
            if (!lanes[i].busy) return (int)i;
        return -1;
    }

    void solver_loop(int si) {
        const hipError_t dev_err = hipSetDevice(device);
        Slot &sl = slots[si];
        for (;;) {
            Request *r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_slot.wait(lk, [&] { return stop || sl.job != nullptr; });
                if (sl.job == nullptr) return;
                r = sl.job;
                MatrixEntry &m = mats[r->mid];
                cv_ready.wait(lk, [&] { return !m.uploading && (m.dev || m.failed_gen >= r->gen); });
                if (!m.dev) {  // the upload this request waited for failed
                    policy.release(r->mid, r->extra);
                    sl.job = nullptr;
                    finish_locked(r, SPMV_EDEVICE, m.error);
                    cv_sched.notify_all();
                    continue;
                }
                r->A = m.dev;
            }
            clear_error();
            (void)hipGetLastError();  // drop an error an earlier call of this thread left behind
            const spmv_matrix *A = r->A;
            const int n = A ? A->M.n_rows : 0;
            double *db = nullptr, *dx = nullptr;
            int rc = SPMV_OK;
            const Clock::time_point t_run = Clock::now();
            sl.pe.mark(0, sl.stream);
            hipError_t e = dev_err != hipSuccess ? dev_err : hipMallocAsync(reinterpret_cast<void **>(&db), 8 * (size_t)std::max(n, 1), sl.stream);
            if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void **>(&dx), 8 * (size_t)std::max(n, 1), sl.stream);
            if (e == hipSuccess) e = hipMemcpyAsync(db, r->in, 8 * (size_t)n, hipMemcpyHostToDevice, sl.stream);
            if (e == hipSuccess) e = hipMemsetAsync(dx, 0, 8 * (size_t)n, sl.stream);
            cg_info info{};
            if (!A) {
                rc = fail(SPMV_EDEVICE, "server: matrix %d is not resident", r->mid);
            } else if (dev_err != hipSuccess) {
                rc = hip_fail(dev_err, "server solver thread: hipSetDevice");
            } else if (e != hipSuccess) {
                rc = hip_fail(e, "server solve buffers");
            } else {
                sl.pe.mark(1, sl.stream);
                // FP64 solves of small matrices take one reduction per iteration
                const int mode = cfg.cg_mode == CG_FP64 && n <= cfg.cg1_max_rows && cg1_eligible(A->M)
                                     ? CG_FP64_ONE_REDUCTION
                                     : cfg.cg_mode;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    sl.cache = checkout_solver_locked(A->serial);
                    ++solver_solves;
                }
                rc = cg_run(A, db, dx, r->tol, r->max_iter, mode, &info, sl.stream, sl.pinned, &sl.cache);
                sl.pe.mark(2, sl.stream);
                if (rc == SPMV_OK || rc == SPMV_ENOTCONV) {
                    e = hipMemcpyAsync(r->out, dx, 8 * (size_t)n, hipMemcpyDeviceToHost, sl.stream);
                    sl.pe.mark(3, sl.stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
                    if (e != hipSuccess) rc = hip_fail(e, "server solve result");
                    else sl.pe.fill(r, ref_event);
                }
            }
            if (db) (void)hipFreeAsync(db, sl.stream);
            if (dx) (void)hipFreeAsync(dx, sl.stream);
            (void)hipStreamSynchronize(sl.stream);
            std::vector<CgCache *> to_free;
            {
                std::lock_guard<std::mutex> lk(mu);
                // the solver goes back before the matrix's pin is released,
                // so an eviction of the matrix finds it
                if (A) to_free = checkin_solver_locked(A->serial, sl.cache);
                else if (sl.cache) to_free.push_back(sl.cache);
                sl.cache = nullptr;
                r->t_run = t_run;
                r->graph_s = info.graph_seconds;
                r->iterations = info.iterations;
                r->rel_residual = info.rel_residual;
                policy.release(r->mid, r->extra);
                sl.job = nullptr;
                finish_locked(r, rc);
                cv_sched.notify_all();
            }
            for (CgCache *c : to_free) cg_cache_free(c);
        }
    }

    int free_slot_locked() const {
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i].job) return (int)i;
        return -1;
    }

    void scheduler_loop() {
        const hipError_t dev_err = hipSetDevice(device);
        std::vector<int> evict;
        for (;;) {
            std::vector<spmv_matrix *> evicted;
            std::vector<CgCache *> dropped;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_sched.wait_for(lk, std::chrono::microseconds(500), [&] { return stop || wake; });
                wake = false;
                if (stop && incoming.empty() && pending.empty() && waiting_spmv.empty()) return;
                while (!incoming.empty()) {
                    pending.push_back(incoming.front());
                    incoming.pop_front();
                }
                // admission: reserve memory (evicting idle matrices), start
                // uploads, give each CG request a slot; in arrival order,
                // younger requests passing one that waits for memory until it
                // has waited kStarveAfter
                const Clock::time_point now = Clock::now();
                bool held = false;
                for (auto it = pending.begin(); it != pending.end();) {
                    Request *r = *it;
                    if (dev_err != hipSuccess) {  // this thread cannot reach the device
                        it = pending.erase(it);
                        finish_locked(r, hip_fail(dev_err, "server scheduler thread: hipSetDevice"));
                        continue;
                    }
                    if (held) {
                        if (policy.never(r->mid, r->extra)) {
                            it = pending.erase(it);
                            finish_locked(r, fail(SPMV_EBUDGET, "request needs more than the device budget"));
                        } else {
                            ++it;
                        }
                        continue;
                    }
                    int slot = -1;
                    if (r->op == SRV_CG) {
                        slot = free_slot_locked();
                        if (slot < 0) { ++it; continue; }
                    }
                    bool upload = false;
                    clear_error();
                    const auto v = policy.admit(r->mid, r->extra, evict, upload);
                    if (v == BudgetLRU::NEVER) {
                        it = pending.erase(it);
                        finish_locked(r, fail(SPMV_EBUDGET, "request needs more than the device budget"));
                        continue;
                    }
                    if (v == BudgetLRU::WAIT) {
                        held = now - r->t_submit > kStarveAfter;
                        ++it;
                        continue;
                    }
                    for (int m : evict) {  // idle and resident: never uploading
                        if (mats[m].dev) {
                            drop_solver_locked(mats[m].dev->serial, dropped);
                            evicted.push_back(mats[m].dev);
                        }
                        mats[m].dev = nullptr;
                    }
                    MatrixEntry &m = mats[r->mid];
                    if (upload || (!m.dev && !m.uploading)) start_upload_locked(r->mid);
                    r->gen = m.gen;
                    it = pending.erase(it);
                    r->t_start = Clock::now();
                    if (r->op == SRV_CG) {
                        slots[slot].job = r;
                        cv_slot.notify_all();
                    } else {
                        waiting_spmv.push_back(r);
                        ++in_flight_spmv;
                    }
                }
                // dispatch: each free lane takes a round of admitted SpMV
                // requests whose matrix is ready, up to the round's workgroup
                // cap; a large request goes alone
                for (int li = free_lane_locked(); li >= 0; li = free_lane_locked()) {
                    std::vector<Request *> &round = lanes[li].job;
                    int64_t round_tiles = 0;
                    bool alone = false;
                    for (auto it = waiting_spmv.begin(); it != waiting_spmv.end() && !alone;) {
                        Request *r = *it;
                        MatrixEntry &m = mats[r->mid];
                        if (m.uploading || (!m.dev && m.failed_gen < r->gen)) { ++it; continue; }
                        if (!m.dev) {  // the upload this request waited for failed
                            it = waiting_spmv.erase(it);
                            policy.release(r->mid, r->extra);
                            --in_flight_spmv;
                            finish_locked(r, SPMV_EDEVICE, m.error);
                            continue;
                        }
                        const bool large = (int64_t)r->k * (m.n_rows + m.n_cols) >= kLargeRequestWords;
                        const int64_t est = (int64_t)r->k * m.dev->M.n_stream;
                        if (!round.empty() && (large || round_tiles + est > cfg.max_round_tiles)) { ++it; continue; }
                        r->A = m.dev;
                        round.push_back(r);
                        round_tiles += est;
                        alone = large;
                        it = waiting_spmv.erase(it);
                    }
                    if (round.empty()) break;
                    lanes[li].busy = true;
                    cv_lane.notify_all();
                }
            }
            for (CgCache *c : dropped) cg_cache_free(c);
            for (spmv_matrix *d : evicted) (void)spmv_destroy(d);
        }
    }
};

}  // namespace spmvlib

using namespace spmvlib;

// The persistent kernel's queue, stream and launch size: one workgroup more
// than asked (the doorbell), capped by how many fit on the device at once.
static hipError_t persist_create(Server &S) {
    Persist &P = S.P;
    int cus = 0, per_cu = 0, khz = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S.device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S.device);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_persist<kServeTile>),
                                                         kBlock, 0);
    if (e != hipSuccess) return e;
    if (cus <= 0 || per_cu <= 0 || khz <= 0) return hipErrorInvalidDevice;
    P.wgs = (int)std::min<int64_t>((int64_t)S.cfg.persistent_wgs + 1, (int64_t)cus * per_cu);
    P.idle_ticks = (uint64_t)S.cfg.persist_idle_us * (uint64_t)khz / 1000u;
    // a worker's empty poll sleeps at least 4,096 cycles (>= 1.6 us at the
    // top clock), the doorbell's 512: 16 polls (128 for the doorbell) per
    // microsecond of idle time outlast the idle clock many times over
    P.max_polls = 16ull * (uint64_t)S.cfg.persist_idle_us + 1024;
    P.tick_s = 1e-3 / (double)khz;
    e = hipHostMalloc(reinterpret_cast<void **>(&P.q), sizeof(PersistQueue), hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) {
        P.q = nullptr;
        return e;
    }
    std::memset(P.q, 0, sizeof(PersistQueue));
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&P.qd), P.q, 0);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&P.st), sizeof(PersistState));
    if (e == hipSuccess) e = hipMemset(P.st, 0, sizeof(PersistState));
    // a stream of its own hardware queue (a CU-masked stream never shares
    // one), so that no other stream's work waits behind a running launch
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    for (int i = 0; i < cus; ++i) mask[(size_t)i / 32] |= 1u << (i % 32);
    if (e == hipSuccess) e = hipExtStreamCreateWithCUMask(&P.stream, (uint32_t)mask.size(), mask.data());
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P.end, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

// Stops a running launch (every wave sees the stop flag within its poll
// period), waits for it, frees the queue.
static void persist_destroy(Server &S) {
    Persist &P = S.P;
    if (P.q) __atomic_store_n(&P.q->stop, uint64_t(1), __ATOMIC_RELEASE);
    if (P.stream) {
        (void)hipStreamSynchronize(P.stream);
        (void)hipStreamDestroy(P.stream);
        P.stream = nullptr;
    }
    if (P.end) (void)hipEventDestroy(P.end);
    P.end = nullptr;
    if (P.st) (void)hipFree(P.st);
    P.st = nullptr;
    if (P.q) (void)hipHostFree(P.q);
    P.q = nullptr;
    P.wgs = 0;
}

struct spmv_server {
    Server *s;
};

extern "C" int srv_create(const srv_config *cfg_in, spmv_server **out) {
    clear_error();
    if (!out) return fail(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    srv_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.hbm_budget_bytes == 0) cfg.hbm_budget_bytes = 200ull << 30;
    if (cfg.n_slots <= 0) cfg.n_slots = 8;
    if (cfg.n_slots > 64) return fail(SPMV_EINVAL, "n_slots = %d exceeds 64", cfg.n_slots);
    if (cfg.max_round_tiles <= 0) cfg.max_round_tiles = 1 << 20;
    if (cfg.n_lanes <= 0) cfg.n_lanes = 4;
    if (cfg.n_lanes > 16) return fail(SPMV_EINVAL, "n_lanes = %d exceeds 16", cfg.n_lanes);
    if (cfg.cg_mode != CG_FP64 && cfg.cg_mode != CG_MIXED_FP32) return fail(SPMV_EINVAL, "unknown cg_mode");
    if (cfg.cg1_max_rows < 0) return fail(SPMV_EINVAL, "cg1_max_rows must be >= 0");
    if (cfg.persistent_wgs < 0 || cfg.persist_idle_us < 0)
        return fail(SPMV_EINVAL, "persistent_wgs and persist_idle_us must be >= 0");
    if (cfg.persist_idle_us == 0) cfg.persist_idle_us = 20000;
    if (cfg.persist_idle_us > 10000000) return fail(SPMV_EINVAL, "persist_idle_us = %d exceeds 10 s", cfg.persist_idle_us);
    auto *S = new (std::nothrow) Server(cfg);
    if (!S) return fail(SPMV_ENOMEM, "host allocation failed");
    S->solver_cap = cfg.hbm_budget_bytes / 16;
    hipError_t e = hipGetDevice(&S->device);
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "hipGetDevice");
    }
    S->slots.resize(cfg.n_slots);
    S->lanes.resize(cfg.n_lanes);
    std::unique_lock<std::mutex> gate(capture_gate());
    for (auto &sl : S->slots) {
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipHostMalloc(&sl.pinned, 256, hipHostMallocDefault);
        if (e == hipSuccess) e = sl.pe.create();
        if (e != hipSuccess) break;
    }
    for (size_t i = 0; i < S->lanes.size() && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&S->lanes[i].stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = S->lanes[i].pe.create();
    }
    if (e == hipSuccess) e = hipEventCreate(&S->ref_event);
    if (e == hipSuccess) e = hipEventRecord(S->ref_event, S->lanes[0].stream);
    if (e == hipSuccess) e = hipEventSynchronize(S->ref_event);
    if (e == hipSuccess && cfg.persistent_wgs > 0) e = persist_create(*S);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "server streams");
        persist_destroy(*S);
        for (auto &t : S->slots) {
            if (t.stream) (void)hipStreamDestroy(t.stream);
            if (t.pinned) (void)hipHostFree(t.pinned);
            t.pe.destroy();
        }
        for (auto &ln : S->lanes) {
            if (ln.stream) (void)hipStreamDestroy(ln.stream);
            ln.pe.destroy();
        }
        if (S->ref_event) (void)hipEventDestroy(S->ref_event);
        delete S;
        return rc;
    }
    gate.unlock();
    for (int i = 0; i < cfg.n_slots; ++i) S->slots[i].th = std::thread([S, i] { S->solver_loop(i); });
    for (int i = 0; i < cfg.n_lanes; ++i) S->lanes[i].th = std::thread([S, i] { S->lane_loop(i); });
    S->scheduler = std::thread([S] { S->scheduler_loop(); });
    S->uploader = std::thread([S] { S->uploader_loop(); });
    *out = new spmv_server{S};
    return SPMV_OK;
}

extern "C" int srv_add_matrix(spmv_server *srv, int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const double *values, int32_t *matrix_id) {
    clear_error();
    if (!srv || !matrix_id) return fail(SPMV_EINVAL, "NULL argument");
    int rc = validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    if (rc) return rc;
    if (nnz > 0 && !values) return fail(SPMV_EINVAL, "values is NULL with nnz > 0");
    Server *S = srv->s;
    MatrixEntry m;
    m.n_rows = n_rows;
    m.n_cols = n_cols;
    m.row_ptr.assign(row_ptr, row_ptr + n_rows + 1);
    m.col_idx.assign(col_idx, col_idx + nnz);
    m.values.assign(values, values + nnz);
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t bytes = S->matrix_bytes(m);
    S->mats.push_back(std::move(m));
    *matrix_id = S->policy.add_matrix(bytes);
    if (S->cfg.preload && S->policy.preload(*matrix_id)) S->start_upload_locked(*matrix_id);
    return SPMV_OK;
}

extern "C" int srv_submit(spmv_server *srv, int32_t matrix_id, int32_t op, int32_t k, const double *in, double *out,
                          double tol, int32_t max_iter, uint64_t *ticket) {
    clear_error();
    if (!srv || !ticket) return fail(SPMV_EINVAL, "NULL argument");
    Server *S = srv->s;
    auto *r = new (std::nothrow) Request();
    if (!r) return fail(SPMV_ENOMEM, "host allocation failed");
    std::lock_guard<std::mutex> lk(S->mu);
    if (matrix_id < 0 || matrix_id >= (int32_t)S->mats.size()) {
        delete r;
        return fail(SPMV_EINVAL, "unknown matrix id %d", matrix_id);
    }
    const MatrixEntry &m = S->mats[matrix_id];
    if (op != SRV_SPMV && op != SRV_CG) {
        delete r;
        return fail(SPMV_EINVAL, "unknown op %d", op);
    }
    if (op == SRV_SPMV && k < 1) {
        delete r;
        return fail(SPMV_EINVAL, "k = %d must be >= 1", k);
    }
    if (op == SRV_CG && (m.n_rows != m.n_cols || !(tol >= 0.0) || max_iter < 0)) {
        delete r;
        return fail(SPMV_EINVAL, "CG needs a square matrix, tol >= 0, max_iter >= 0");
    }
    if ((m.n_cols && !in) || (m.n_rows && !out)) {
        delete r;
        return fail(SPMV_EINVAL, "in or out is NULL");
    }
    r->ticket = S->next_ticket++;
    r->mid = matrix_id;
    r->op = op;
    r->k = op == SRV_CG ? 1 : k;
    r->in = in;
    r->out = out;
    r->tol = tol;
    r->max_iter = max_iter;
    r->t_submit = Clock::now();
    r->extra = S->request_bytes(*r);
    if (!S->any_submit) {
        S->t_first = r->t_submit;
        S->any_submit = true;
    }
    ++S->submitted;
    S->all[r->ticket] = r;
    S->incoming.push_back(r);
    *ticket = r->ticket;
    S->wake = true;
    S->cv_sched.notify_all();
    return SPMV_OK;
}

static void fill_result(const Request *r, srv_result *res) {
    std::memset(res, 0, sizeof *res);
    res->done = r->done ? 1 : 0;
    res->status = r->status;
    res->iterations = r->iterations;
    res->op = r->op;
    res->rel_residual = r->rel_residual;
    std::memcpy(res->message, r->message, sizeof res->message);
    if (r->done) {
        res->latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        res->queue_s = std::chrono::duration<double>(r->t_start - r->t_submit).count();
        if (res->queue_s < 0) res->queue_s = 0;
        if (r->t_run != Clock::time_point{}) {
            res->wait_s = std::chrono::duration<double>(r->t_run - r->t_start).count();
            if (res->wait_s < 0) res->wait_s = 0;
        }
        res->copy_in_s = r->copy_in_s;
        res->compute_s = r->compute_s;
        res->copy_out_s = r->copy_out_s;
        res->graph_s = r->graph_s;
        res->kernel_s = r->kernel_s;
        res->dev_begin_s = r->dev_begin_s;
        res->dev_end_s = r->dev_end_s;
    }
}

extern "C" int srv_poll(spmv_server *srv, uint64_t ticket, srv_result *res) {
    clear_error();
    if (!srv || !res) return fail(SPMV_EINVAL, "NULL argument");
    Server *S = srv->s;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SPMV_EINVAL, "unknown ticket");
    fill_result(it->second, res);
    return SPMV_OK;
}

extern "C" int srv_wait(spmv_server *srv, uint64_t ticket, srv_result *res) {
    clear_error();
    if (!srv) return fail(SPMV_EINVAL, "NULL argument");
    Server *S = srv->s;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SPMV_EINVAL, "unknown ticket");
    Request *r = it->second;
    S->cv_done.wait(lk, [&] { return r->done; });
    if (res) fill_result(r, res);
    return SPMV_OK;
}

extern "C" int srv_drain(spmv_server *srv) {
    clear_error();
    if (!srv) return fail(SPMV_EINVAL, "NULL argument");
    Server *S = srv->s;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->completed + S->failed == S->submitted && S->uploads_in_flight == 0; });
    return SPMV_OK;
}

extern "C" int srv_get_stats(spmv_server *srv, srv_stats *st) {
    clear_error();
    if (!srv || !st) return fail(SPMV_EINVAL, "NULL argument");
    Server *S = srv->s;
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->failed = S->failed;
    st->rounds = S->rounds;
    st->uploads = S->policy.uploads();
    st->persist_launches = S->P.launches;
    st->solver_reuses = S->solver_hits;
    st->solver_cached_bytes = (int64_t)S->solver_bytes;
    st->evictions = S->policy.evictions();
    st->used_bytes = (int64_t)S->policy.used();
    st->peak_bytes = (int64_t)S->policy.peak();
    std::vector<double> l = S->latencies;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)(f * (double)(l.size() - 1) + 0.5))]; };
        st->p50_s = q(0.50);
        st->p99_s = q(0.99);
        st->max_s = l.back();
        double sum = 0;
        for (double v : l) sum += v;
        st->mean_s = sum / (double)l.size();
        st->wall_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
        st->throughput_rps = st->wall_s > 0 ? (double)S->completed / st->wall_s : 0.0;
    }
    return SPMV_OK;
}

extern "C" int srv_destroy(spmv_server *srv) {
    clear_error();
    if (!srv) return SPMV_OK;
    Server *S = srv->s;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->completed + S->failed == S->submitted && S->uploads_in_flight == 0; });
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->cv_slot.notify_all();
    S->cv_upload.notify_all();
    S->cv_lane.notify_all();
    if (S->scheduler.joinable()) S->scheduler.join();
    if (S->uploader.joinable()) S->uploader.join();
    for (auto &sl : S->slots)
        if (sl.th.joinable()) sl.th.join();
    for (auto &ln : S->lanes)
        if (ln.th.joinable()) ln.th.join();
    for (auto &kv : S->solvers) cg_cache_free(kv.second.c);  // before the gate: freeing a graph takes it
    S->solvers.clear();
    S->solver_lru.clear();
    for (auto &sl : S->slots) {
        cg_cache_free(sl.cache);
        sl.cache = nullptr;
    }
    for (auto &m : S->mats)
        if (m.dev) (void)spmv_destroy(m.dev);
    std::lock_guard<std::mutex> gate(capture_gate());
    persist_destroy(*S);
    for (auto &sl : S->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pe.destroy();
    }
    for (auto &ln : S->lanes) {
        if (ln.items_host) (void)hipHostFree(ln.items_host);
        for (int i = 0; i < 2; ++i) {
            if (ln.stage[i]) (void)hipHostFree(ln.stage[i]);
            if (ln.stage_ev[i]) (void)hipEventDestroy(ln.stage_ev[i]);
        }
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        ln.pe.destroy();
    }
    if (S->ref_event) (void)hipEventDestroy(S->ref_event);
    for (auto &kv : S->all) delete kv.second;
    delete S;
    delete srv;
    return SPMV_OK;
}

extern "C" int srv_policy_simulate(uint64_t budget, int32_t n_mats, const uint64_t *mat_bytes, int32_t n_ops,
                                   const int32_t *op_kind, const int32_t *op_mat, const uint64_t *op_extra,
                                   int32_t *verdict, int32_t *n_evicted, int32_t *uploaded, uint64_t *used) {
    clear_error();
    if (n_mats < 0 || n_ops < 0 || (n_mats && !mat_bytes) || (n_ops && (!op_kind || !op_mat || !op_extra)))
        return fail(SPMV_EINVAL, "bad arguments");
    BudgetLRU P(budget);
    for (int i = 0; i < n_mats; ++i) P.add_matrix(mat_bytes[i]);
    std::vector<int> ev;
    for (int t = 0; t < n_ops; ++t) {
        if (op_mat[t] < 0 || op_mat[t] >= n_mats) return fail(SPMV_EINVAL, "op %d: bad matrix", t);
        int v = -1, ne = 0, up = 0;
        if (op_kind[t] == 0) {
            bool u = false;
            v = P.admit(op_mat[t], op_extra[t], ev, u);
            ne = (int)ev.size();
            up = u ? 1 : 0;
        } else if (op_kind[t] == 1) {
            if (P.pins(op_mat[t]) <= 0) return fail(SPMV_EINVAL, "op %d: release without admission", t);
            P.release(op_mat[t], op_extra[t]);
        } else if (op_kind[t] == 2) {  // the matrix's upload failed
            if (!P.resident(op_mat[t])) return fail(SPMV_EINVAL, "op %d: failed upload of a matrix not resident", t);
            P.unload(op_mat[t]);
        } else if (op_kind[t] == 3) {  // preload
            const bool made = P.preload(op_mat[t]);
            v = made ? 0 : 1;
            up = made ? 1 : 0;
        } else {
            return fail(SPMV_EINVAL, "op %d: kind %d unknown", t, op_kind[t]);
        }
        if (verdict) verdict[t] = v;
        if (n_evicted) n_evicted[t] = ne;
        if (uploaded) uploaded[t] = up;
        if (used) used[t] = P.used();
    }
    return SPMV_OK;
}
