"""GPU tests of the continuous-batching server: results against the oracle,
the same result alone and in the mix (bitwise), and the device-memory
budget (eviction and rejection)."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

# A failed matrix upload inside the server used to leave the matrix marked
# resident with no device handle, and the next request on it dereferenced a
# null handle in a server thread (one of eight runs of these tests ended in
# that host segmentation fault).  The failure path is covered on the CPU by
# test_serve_host_cpu.py; here every failed request names its error.
pytestmark = pytest.mark.gpu


def _ok(res):
    assert res.done == 1 and res.status == 0, f"status {res.status}: {res.message}"


@pytest.fixture(scope="module")
def pool():
    sizes = [1000, 4000, 9000, 30000, 70000, 150000]
    return [mg.serving_matrix(n, seed=mg.seed_for(4) ^ (i + 1)) for i, n in enumerate(sizes)]


def _requests(pool, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(n):
        mid = int(rng.integers(len(pool)))
        A = pool[mid]
        if rng.random() < 0.5:
            k = int(rng.integers(1, 9))
            reqs.append(("spmv", mid, mg.uniform(k * A.n_cols, seed + t, 3).reshape(k, A.n_cols)))
        else:
            reqs.append(("cg", mid, mg.uniform(A.n_rows, seed + t, 4)))
    return reqs


def _submit(srv, r, tol=1e-8):
    kind, mid, data = r
    return srv.submit_spmv(mid, data) if kind == "spmv" else srv.submit_cg(mid, data, tol=tol)


def test_results_match_the_oracle(pool):
    reqs = _requests(pool, 24, 100)
    with spmv.Server(n_slots=4) as srv:
        ids = [srv.add_matrix(A) for A in pool]
        assert ids == list(range(len(pool)))
        tickets = [_submit(srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            out, res = srv.wait(t)
            _ok(res)
            kind, mid, data = r
            A = pool[mid]
            if kind == "spmv":
                for j in range(data.shape[0]):
                    y_ref, bound = oracle.spmv(A, data[j])
                    assert oracle.spmv_accept(out[j], y_ref, bound).all()
            else:
                Ax, _ = oracle.spmv(A, out)
                assert np.linalg.norm(data - Ax) / np.linalg.norm(data) <= 1.05e-8
                assert res.iterations > 0
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["p99_s"] >= st["p50_s"] > 0


def test_alone_equals_mix_bitwise(pool):
    reqs = _requests(pool, 30, 200)
    with spmv.Server(n_slots=6) as srv:
        for A in pool:
            srv.add_matrix(A)
        alone = []
        for r in reqs:                      # one request at a time on an idle server
            out, res = srv.wait(_submit(srv, r))
            _ok(res)
            alone.append(out.copy())
        tickets = [_submit(srv, r) for r in reqs]   # everything at once
        mixed = []
        for t in tickets:
            out, res = srv.wait(t)
            _ok(res)
            mixed.append(out)
        st = srv.stats()
    for a, m in zip(alone, mixed):
        assert np.array_equal(a, m)
    assert st["rounds"] < sum(1 for r in reqs if r[0] == "spmv") * 2   # SpMVs were batched


def test_server_spmv_equals_direct_apply(pool):
    A = pool[3]
    X = mg.uniform(3 * A.n_cols, 7, 3).reshape(3, A.n_cols)
    with spmv.Server() as srv:
        srv.add_matrix(A)
        out, res = srv.wait(srv.submit_spmv(0, X))
        _ok(res)
    with spmv.Matrix.from_csr(A, params={"tile_nnz": 1024, "kernel": 1, "window_mode": spmv.WINDOW_OFF}) as M:
        for j in range(3):
            y = M.apply(torch.as_tensor(X[j], device="cuda")).cpu().numpy()
            assert np.array_equal(y, out[j])


def test_staged_copies_at_chunk_boundaries():
    # a 131,072-row matrix: k vectors move k MB each way, so k = 3 goes
    # through the runtime's copy, k = 4 is the smallest staged buffer (4 MB),
    # 16 and 32 fill one and two 16 MB chunks exactly, 33 leaves a 1 MB
    # tail chunk; every result bitwise equal to the handle's own product,
    # several requests in flight at once so lanes stage concurrently
    n = 131_072
    A = mg.random_csr(n, n, seed=21, mean_len=6.0, empty_frac=0.05, duplicates=True)
    ks = [3, 4, 16, 32, 33, 4, 17]
    Xs = [mg.uniform(k * n, 300 + i, 3).reshape(k, n) for i, k in enumerate(ks)]
    with spmv.Server(n_lanes=3) as srv:
        srv.add_matrix(A)
        tickets = [srv.submit_spmv(0, X) for X in Xs]
        outs = []
        for t in tickets:
            out, res = srv.wait(t)
            _ok(res)
            outs.append(out)
    with spmv.Matrix.from_csr(A) as M:
        for X, out in zip(Xs, outs):
            Y = M.spmm(torch.as_tensor(np.ascontiguousarray(X.T), device="cuda")).cpu().numpy()
            assert np.array_equal(Y.T, out), X.shape


def test_budget_eviction_and_rejection(pool):
    small = pool[:4]
    est = lambda A: 12 * (A.nnz + 20) + 4 * (A.n_rows + 1) + 64 * (A.nnz // 512 + 16)
    # the largest matrix plus a tenth, plus two request buffers: the four
    # matrices together do not fit, so cycling over them must evict
    budget = int(1.1 * est(small[3]) + 2 * 16 * small[3].n_rows)
    assert sum(est(A) for A in small) > budget
    reqs = [("spmv", i % 4, mg.uniform(small[i % 4].n_cols, i, 5)[None, :]) for i in range(12)]
    with spmv.Server(hbm_budget_bytes=budget, n_slots=2) as srv:
        for A in small:
            srv.add_matrix(A)
        outs = [srv.wait(_submit(srv, r)) for r in reqs]
        st = srv.stats()
        assert st["evictions"] > 0 and st["peak_bytes"] <= budget
        for (kind, mid, X), (out, res) in zip(reqs, outs):
            _ok(res)
            y_ref, bound = oracle.spmv(small[mid], X[0])
            assert oracle.spmv_accept(out[0], y_ref, bound).all()
        big = pool[-1]
        bid = srv.add_matrix(big)
        _, res = srv.wait(srv.submit_spmv(bid, np.ones((1, big.n_cols))))
        assert res.status == spmv.SPMV_EBUDGET and "budget" in res.message


def _check(pool, r, out, res):
    _ok(res)
    kind, mid, data = r
    A = pool[mid]
    if kind == "spmv":
        for j in range(data.shape[0]):
            y_ref, bound = oracle.spmv(A, data[j])
            assert oracle.spmv_accept(out[j], y_ref, bound).all()
    else:
        Ax, _ = oracle.spmv(A, out)
        assert np.linalg.norm(data - Ax) / np.linalg.norm(data) <= 1.05e-8


def test_preload_uploads_at_registration(pool):
    reqs = _requests(pool, 16, 300)
    with spmv.Server(n_slots=4, preload=True) as srv:
        for A in pool:
            srv.add_matrix(A)
        srv.drain()                                   # waits for the background uploads
        assert srv.stats()["uploads"] == len(pool)
        tickets = [_submit(srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            out, res = srv.wait(t)
            _check(pool, r, out, res)
        assert srv.stats()["uploads"] == len(pool)   # no upload on the request path


def test_preload_within_budget_then_on_demand(pool):
    small = pool[:4]
    est = lambda A: 12 * (A.nnz + 20) + 4 * (A.n_rows + 1) + 64 * (A.nnz // 512 + 16)
    # room for matrices 0-2 preloaded in order but not for matrix 3 as well;
    # requests on matrix 3 then evict idle preloaded ones
    budget = int(est(small[0]) + est(small[1]) + est(small[3]) + 32 * small[3].n_rows)
    assert sum(est(A) for A in small) > budget
    reqs = [("spmv", i % 4, mg.uniform(small[i % 4].n_cols, 40 + i, 5)[None, :]) for i in range(8)]
    with spmv.Server(hbm_budget_bytes=budget, n_slots=2, preload=True) as srv:
        for A in small:
            srv.add_matrix(A)
        srv.drain()
        st = srv.stats()
        assert st["uploads"] == 3 and st["peak_bytes"] <= budget
        for r in reqs:
            out, res = srv.wait(_submit(srv, r))
            _check(small, r, out, res)
        st = srv.stats()
        assert st["evictions"] > 0 and st["peak_bytes"] <= budget


def test_mixed_precision_cg_requests(pool):
    A = pool[2]
    b = mg.uniform(A.n_rows, 9, 4)
    with spmv.Server(cg_mode=spmv.CG_MIXED_FP32) as srv:
        srv.add_matrix(A)
        x, res = srv.wait(srv.submit_cg(0, b, tol=1e-8))
    _ok(res)
    Ax, _ = oracle.spmv(A, x)
    assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 1.05e-8


def test_bad_requests_are_rejected(pool):
    with spmv.Server() as srv:
        srv.add_matrix(pool[0])
        with pytest.raises(spmv.SpmvError) as e:
            srv.submit_spmv(5, np.ones((1, 3)))
        assert e.value.code == spmv.SPMV_EINVAL
        with pytest.raises(ValueError):
            srv.submit_spmv(0, np.ones((1, pool[0].n_cols + 1)))
    for bad in ({"n_lanes": 17}, {"n_slots": 65}, {"cg_mode": 7}):
        with pytest.raises(spmv.SpmvError) as e:
            spmv.Server(**bad)
        assert e.value.code == spmv.SPMV_EINVAL


def test_one_lane_and_small_rounds(pool):
    # a single SpMV lane and a tiny round cap: rounds serialize and split, and
    # results are still the oracle's
    reqs = [r for r in _requests(pool, 12, 500) if r[0] == "spmv"]
    with spmv.Server(n_lanes=1, max_round_tiles=8) as srv:
        for A in pool:
            srv.add_matrix(A)
        tickets = [_submit(srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            out, res = srv.wait(t)
            _check(pool, r, out, res)
        assert srv.stats()["rounds"] >= len(reqs)


def test_large_request_takes_a_round_of_its_own(pool):
    # k = 32 vectors on the 150K-row matrix move 9.6 M words (>= 2^22): the
    # request gets a round of its own while small requests keep batching;
    # every column is checked against the oracle
    A = pool[-1]
    big = mg.uniform(32 * A.n_cols, 61, 3).reshape(32, A.n_cols)
    assert 32 * (A.n_rows + A.n_cols) >= 1 << 22
    small = [("spmv", i % 4, mg.uniform(pool[i % 4].n_cols * 2, 70 + i, 3).reshape(2, pool[i % 4].n_cols))
             for i in range(8)]
    with spmv.Server(n_slots=2) as srv:
        for M in pool:
            srv.add_matrix(M)
        srv.wait(srv.submit_spmv(len(pool) - 1, big[:1]))        # upload the matrix first
        t_big = srv.submit_spmv(len(pool) - 1, big)
        t_small = [_submit(srv, r) for r in small]
        out, res = srv.wait(t_big)
        _ok(res)
        for j in range(32):
            y_ref, bound = oracle.spmv(A, big[j])
            assert oracle.spmv_accept(out[j], y_ref, bound).all(), j
        others = []
        for r, t in zip(small, t_small):
            o, rs = srv.wait(t)
            _check(pool, r, o, rs)
            others.append(rs)
    # the large request's device interval is shared with no other request's
    assert res.compute_s > 0 and res.dev_end_s > res.dev_begin_s >= 0
    assert all((o.dev_begin_s, o.dev_end_s) != (res.dev_begin_s, res.dev_end_s) for o in others)


def test_cg_solves_and_spmv_rounds_overlap_on_the_device(pool):
    # solver slots and SpMV lanes work on their own streams: in a mix, at
    # least one CG solve's device interval overlaps an SpMV round's, and
    # every request's phase times are consistent with its latency
    reqs = [("cg", 4 + (i % 2), mg.uniform(pool[4 + (i % 2)].n_rows, 80 + i, 4)) for i in range(4)]
    reqs += [("spmv", i % 6, mg.uniform(pool[i % 6].n_cols * 4, 90 + i, 3).reshape(4, pool[i % 6].n_cols))
             for i in range(40)]
    with spmv.Server(n_slots=4, preload=True) as srv:
        for M in pool:
            srv.add_matrix(M)
        srv.drain()
        tickets = [_submit(srv, r) for r in reqs]
        done = [srv.wait(t) for t in tickets]
    spans = {"cg": [], "spmv": []}
    for r, (out, res) in zip(reqs, done):
        _check(pool, r, out, res)
        assert res.compute_s > 0 and res.copy_in_s >= 0 and res.copy_out_s >= 0
        assert res.compute_s <= res.latency_s and res.queue_s + res.wait_s <= res.latency_s
        assert res.dev_end_s > res.dev_begin_s >= 0
        spans[r[0]].append((res.dev_begin_s, res.dev_end_s))
    overlap = any(c0 < s1 and s0 < c1 for c0, c1 in spans["cg"] for s0, s1 in spans["spmv"])
    assert overlap, (spans["cg"], spans["spmv"][:8])


def test_solvers_are_kept_per_matrix_and_small_matrices_take_one_reduction(pool):
    # the server keeps each matrix's FP64 solver (workspace and captured
    # graph): a later solve on the same matrix captures nothing and gives the
    # same bits as a direct cg_solve; with cg1_max_rows covering the matrix
    # it solves with one reduction per iteration, bitwise as the direct
    # CG_FP64_ONE_REDUCTION solve on a handle with the server's plan
    A = pool[2]
    b = mg.uniform(A.n_rows, 21, 4)
    params = {"tile_nnz": 1024, "kernel": 1, "window_mode": spmv.WINDOW_OFF}
    with spmv.Matrix.from_csr(A, params=params) as M:
        bd = torch.as_tensor(b, device="cuda")
        x_hs, _ = M.cg(bd, tol=1e-8)
        x_1r, _ = M.cg(bd, tol=1e-8, mode=spmv.CG_FP64_ONE_REDUCTION)
    x_hs, x_1r = x_hs.cpu().numpy(), x_1r.cpu().numpy()
    assert not np.array_equal(x_hs, x_1r)   # the two methods round differently
    other = mg.uniform(pool[1].n_rows, 22, 4)
    for cg1_rows, want in ((0, x_hs), (A.n_rows, x_1r)):
        with spmv.Server(n_slots=1, cg1_max_rows=cg1_rows, preload=True) as srv:
            for M_ in pool[:4]:
                srv.add_matrix(M_)
            srv.drain()
            outs = []
            for mid in (2, 2, 1, 2):
                rhs = b if mid == 2 else other
                out, res = srv.wait(srv.submit_cg(mid, rhs, tol=1e-8))
                _check(pool, ("cg", mid, rhs), out, res)
                outs.append((mid, out.copy(), res.graph_s))
            st = srv.stats()
        assert outs[0][2] > 0 and outs[1][2] == 0 and outs[2][2] > 0 and outs[3][2] == 0
        assert st["solver_reuses"] == 2 and st["solver_cached_bytes"] > 0
        for mid, out, _ in outs:
            if mid == 2:
                assert np.array_equal(out, want)


def test_kept_solvers_follow_their_matrices_out(pool):
    # under a budget that forces evictions, CG requests cycling over four
    # matrices: a kept solver is dropped with its evicted matrix and never
    # used for the matrix uploaded again later (results stay the oracle's)
    small = pool[:4]
    est = lambda A: 12 * (A.nnz + 20) + 4 * (A.n_rows + 1) + 64 * (A.nnz // 512 + 16)
    cg_bytes = lambda A: 56 * A.n_rows + 8 * (A.nnz // 1000 + 4096)  # b, x and the workspace
    # room for the largest matrix and one solve on it, not for all four
    budget = int(1.1 * est(small[3]) + cg_bytes(small[3]) + (200 << 10))
    assert sum(est(A) for A in small) + cg_bytes(small[3]) > budget
    reqs = [("cg", i % 4, mg.uniform(small[i % 4].n_rows, 300 + i, 4)) for i in range(12)]
    with spmv.Server(hbm_budget_bytes=budget, n_slots=1, cg1_max_rows=20000) as srv:
        for A in small:
            srv.add_matrix(A)
        for r in reqs:
            out, res = srv.wait(_submit(srv, r))
            _check(small, r, out, res)
        st = srv.stats()
    assert st["evictions"] > 0 and st["failed"] == 0
    assert st["solver_cached_bytes"] <= budget // 16


def test_a_large_request_is_not_starved_by_small_ones(pool):
    # the budget holds the 150K-row matrix and a 16-vector request on it only
    # when the 30K-row matrix is not pinned by a request in flight.  CG solves
    # on the 30K-row matrix arrive every 0.5 ms for 1 s on four slots, so
    # their lifetimes overlap and the matrix stays pinned; a large request
    # that arrived among them is admitted only because, after 50 ms of
    # waiting, younger requests are no longer admitted before it (without
    # that rule it waits for the whole stream)
    import time
    big, small = pool[-1], pool[3]
    est = lambda A: 12 * (A.nnz + 20) + 4 * (A.n_rows + 1) + 64 * (A.nnz // 512 + 16)
    k = 16
    big_extra = 8 * k * (big.n_rows + big.n_cols)
    small_need = est(small) + 56 * small.n_rows
    budget = int(1.05 * est(big) + big_extra + (1 << 20))
    assert est(big) + big_extra + small_need > budget   # not both at once
    X = mg.uniform(k * big.n_cols, 77, 3).reshape(k, big.n_cols)
    b = mg.uniform(small.n_rows, 78, 4)
    with spmv.Server(hbm_budget_bytes=budget, n_slots=4) as srv:
        for M in pool:
            srv.add_matrix(M)
        tickets = [srv.submit_cg(3, b, tol=1e-8) for _ in range(8)]
        t_big = srv.submit_spmv(len(pool) - 1, X)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 1.0:
            tickets.append(srv.submit_cg(3, b, tol=1e-8))
            time.sleep(0.0005)
        out, res = srv.wait(t_big)
        _ok(res)
        outs = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert res.latency_s < 0.4, res.latency_s   # admitted while the stream still ran
    assert st["evictions"] > 0 and st["peak_bytes"] <= budget
    for j in range(0, k, 5):
        y_ref, bound = oracle.spmv(big, X[j])
        assert oracle.spmv_accept(out[j], y_ref, bound).all()
    for x, rs in outs[::100]:
        _check(pool, ("cg", 3, b), x, rs)
