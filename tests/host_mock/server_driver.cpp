// Drives the request server (srv_*) over six banded matrices with mixes of
// SpMV and CG requests (several slot counts, both CG modes, uploads on first
// request or preloaded, and a small device budget that forces evictions and
// rejections), then checks the
// outcome of every request: it is reported done, and a failed one carries a
// message.  Prints one summary line; exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "spmv.h"

namespace {
constexpr int kCopies = 8;

struct Banded {
    int n = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<double> val;
};

Banded banded(int n) {
    Banded m;
    m.n = n;
    m.row_ptr.push_back(0);
    for (int i = 0; i < n; ++i) {
        for (int d = -2; d <= 2; ++d) {
            const int c = i + d;
            if (c < 0 || c >= n) continue;
            m.col.push_back(c);
            m.val.push_back(d == 0 ? 5.0 : -1.0);
        }
        m.row_ptr.push_back((int32_t)m.col.size());
    }
    return m;
}
}  // namespace

int main(int argc, char **argv) {
    const int reps = argc > 1 ? std::atoi(argv[1]) : 8;
    std::mt19937_64 rng(7);
    std::vector<Banded> pool;
    for (int n : {1000, 4000, 9000, 30000, 70000, 150000}) pool.push_back(banded(n));
    long completed = 0, failed = 0, without_message = 0, not_done = 0, bad_stats = 0, upload_failed = 0;
    for (int rep = 0; rep < reps; ++rep) {
        srv_config cfg{};
        cfg.n_slots = 2 + rep % 5;
        cfg.cg_mode = rep % 3 == 2 ? CG_MIXED_FP32 : CG_FP64;
        if (rep % 4 == 3) cfg.hbm_budget_bytes = 6000000;
        cfg.preload = rep % 2;
        spmv_server *S = nullptr;
        if (srv_create(&cfg, &S) != SPMV_OK) {
            std::printf("srv_create failed: %s\n", spmv_last_error());
            return 2;
        }
        // each matrix is registered kCopies times (matrix id = copy * 6 + i),
        // so registration goes on while preloads of earlier ids run
        for (int copy = 0; copy < kCopies; ++copy) {
            for (const Banded &m : pool) {
                int32_t id = -1;
                if (srv_add_matrix(S, m.n, m.n, (int64_t)m.col.size(), m.row_ptr.data(), m.col.data(), m.val.data(),
                                   &id) != SPMV_OK) {
                    std::printf("srv_add_matrix failed: %s\n", spmv_last_error());
                    return 2;
                }
            }
        }
        if (rep % 3 == 1) (void)srv_drain(S);  // preloads (if any) finish first
        const int n_req = 24 + rep % 13;
        std::vector<std::vector<double>> in(n_req), out(n_req);
        std::vector<uint64_t> ticket(n_req);
        for (int t = 0; t < n_req; ++t) {
            const int mid = (int)(rng() % (rep % 4 == 3 ? 4 : kCopies * pool.size()));
            const int n = pool[mid % pool.size()].n;
            int rc;
            if (t % 12 == 5) {
                // a large request: 16 vectors on the 150,000-row matrix
                const int k = 16, nb = pool[5].n;
                in[t].assign((size_t)k * nb, 1.0);
                out[t].assign((size_t)k * nb, 0.0);
                rc = srv_submit(S, 5, SRV_SPMV, k, in[t].data(), out[t].data(), 0.0, 0, &ticket[t]);
            } else if (rng() % 2) {
                const int k = 1 + (int)(rng() % 8);
                in[t].assign((size_t)k * n, 1.0);
                out[t].assign((size_t)k * n, 0.0);
                rc = srv_submit(S, mid, SRV_SPMV, k, in[t].data(), out[t].data(), 0.0, 0, &ticket[t]);
            } else {
                in[t].assign(n, 1.0);
                out[t].assign(n, 0.0);
                rc = srv_submit(S, mid, SRV_CG, 1, in[t].data(), out[t].data(), 1e-8, 1000, &ticket[t]);
            }
            if (rc != SPMV_OK) {
                std::printf("srv_submit failed: %s\n", spmv_last_error());
                return 2;
            }
            if (rng() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        }
        for (int t = 0; t < n_req; ++t) {
            srv_result r;
            if (t % 2) (void)srv_poll(S, ticket[t], &r);
            (void)srv_wait(S, ticket[t], &r);
            if (!r.done) ++not_done;
            if (r.status == SPMV_OK) {
                ++completed;
            } else {
                ++failed;
                if (!r.message[0]) ++without_message;
                if (std::strncmp(r.message, "hipMemcpyAsync", 14) == 0) ++upload_failed;  // a matrix upload
            }
        }
        srv_stats st;
        (void)srv_get_stats(S, &st);
        if (st.completed + st.failed != st.submitted || st.submitted != n_req) ++bad_stats;
        (void)srv_destroy(S);
    }
    std::printf("summary completed=%ld failed=%ld upload_failed=%ld without_message=%ld not_done=%ld bad_stats=%ld\n",
                completed, failed, upload_failed, without_message, not_done, bad_stats);
    return (without_message || not_done || bad_stats) ? 3 : 0;
}
