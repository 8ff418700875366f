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
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
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
    const TileDesc d = it.desc[b - it.tile_begin];
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
};

// An SpMV lane: a worker thread with its own stream that runs one round at a
// time (copies in, one k_multi launch, copies out), so that a round moving a
// large request's vectors over the host link does not hold up the others.
struct Lane {
    std::thread th;
    hipStream_t stream = nullptr;
    MultiItem *items_host = nullptr;  // pinned staging of the round's item table
    size_t items_cap = 0;
    PhaseEvents pe;
    std::vector<Request *> job;
    bool busy = false;
};

// Requests moving at least this many vector words between host and device
// get rounds of their own.
constexpr int64_t kLargeRequestWords = int64_t(1) << 22;

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

}  // namespace

struct Server {
    srv_config cfg{};
    int device = 0;
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

    // One round on lane ln: every SpMV vector of the round's requests in one
    // launch.  Frees the lane when done.
    void run_round(std::vector<Request *> &round, Lane &ln) {
        const hipStream_t batch = ln.stream;
        clear_error();
        (void)hipGetLastError();  // drop an error an earlier call of this thread left behind
        const Clock::time_point t_run = Clock::now();
        ln.pe.mark(0, batch);
        std::vector<MultiItem> items;
        std::vector<std::pair<Request *, std::pair<double *, double *>>> bufs;
        int total = 0;
        int err = SPMV_OK;
        for (Request *r : round) {
            const DevMatrix &M = r->A->M;
            double *din = nullptr, *dout = nullptr;
            const size_t nin = (size_t)r->k * M.n_cols, nout = (size_t)r->k * M.n_rows;
            hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&din), 8 * std::max<size_t>(nin, 1), batch);
            if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void **>(&dout), 8 * std::max<size_t>(nout, 1), batch);
            if (e == hipSuccess && nin) e = hipMemcpyAsync(din, r->in, 8 * nin, hipMemcpyHostToDevice, batch);
            if (e != hipSuccess) err = hip_fail(e, "server round buffers");
            bufs.push_back({r, {din, dout}});
            for (int j = 0; j < r->k && e == hipSuccess; ++j) {
                const double *x = din + (size_t)j * M.n_cols;
                double *y = dout + (size_t)j * M.n_rows;
                if (M.n_long > 0) {
                    // rows longer than a tile: the matrix's own launch sequence
                    e = launch_spmv<double, double, double, double>(M, M.val64, x, y, EPI_PLAIN, nullptr, nullptr,
                                                                    nullptr, batch);
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
                if (e == hipSuccess) {
                    hipLaunchKernelGGL((k_multi<kServeTile>), dim3(total), dim3(kBlock), 0, batch, ditems,
                                       (int)items.size(), total);
                    e = hipGetLastError();
                }
                if (ditems) (void)hipFreeAsync(ditems, batch);
                if (e != hipSuccess) err = hip_fail(e, "server round launch");
            }
        }
        ln.pe.mark(2, batch);
        for (auto &b : bufs) {
            Request *r = b.first;
            const size_t nout = (size_t)r->k * r->A->M.n_rows;
            if (err == SPMV_OK && nout) {
                hipError_t e = hipMemcpyAsync(r->out, b.second.second, 8 * nout, hipMemcpyDeviceToHost, batch);
                if (e != hipSuccess) err = hip_fail(e, "server result copy");
            }
        }
        ln.pe.mark(3, batch);
        hipError_t e = hipStreamSynchronize(batch);
        if (e != hipSuccess && err == SPMV_OK) err = hip_fail(e, "server round");
        for (auto &b : bufs) {
            if (b.second.first) (void)hipFreeAsync(b.second.first, batch);
            if (b.second.second) (void)hipFreeAsync(b.second.second, batch);
        }
        std::lock_guard<std::mutex> lk(mu);
        ++rounds;
        for (Request *r : round) {
            r->t_run = t_run;
            if (e == hipSuccess) ln.pe.fill(r, ref_event);
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
                rc = cg_run(A, db, dx, r->tol, r->max_iter, cfg.cg_mode, &info, sl.stream, sl.pinned);
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
            std::lock_guard<std::mutex> lk(mu);
            r->t_run = t_run;
            r->graph_s = info.graph_seconds;
            r->iterations = info.iterations;
            r->rel_residual = info.rel_residual;
            policy.release(r->mid, r->extra);
            sl.job = nullptr;
            finish_locked(r, rc);
            cv_sched.notify_all();
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
                // uploads, give each CG request a slot
                for (auto it = pending.begin(); it != pending.end();) {
                    Request *r = *it;
                    if (dev_err != hipSuccess) {  // this thread cannot reach the device
                        it = pending.erase(it);
                        finish_locked(r, hip_fail(dev_err, "server scheduler thread: hipSetDevice"));
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
                    if (v == BudgetLRU::WAIT) { ++it; continue; }
                    for (int m : evict) {  // idle and resident: never uploading
                        if (mats[m].dev) evicted.push_back(mats[m].dev);
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
            for (spmv_matrix *d : evicted) (void)spmv_destroy(d);
        }
    }
};

}  // namespace spmvlib

using namespace spmvlib;

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
    auto *S = new (std::nothrow) Server(cfg);
    if (!S) return fail(SPMV_ENOMEM, "host allocation failed");
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
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "server streams");
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
    for (auto &m : S->mats)
        if (m.dev) (void)spmv_destroy(m.dev);
    std::lock_guard<std::mutex> gate(capture_gate());
    for (auto &sl : S->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pe.destroy();
    }
    for (auto &ln : S->lanes) {
        if (ln.items_host) (void)hipHostFree(ln.items_host);
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
