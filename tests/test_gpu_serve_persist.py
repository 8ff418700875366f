"""GPU tests of the server's persistent multi-matrix kernel: SpMV rounds fed
through the queue in host memory give bitwise the results of rounds launched
one by one (and the oracle's), across more rounds than the queue has slots;
the kernel ends when idle and is launched again when work comes; CG solves
on their own streams run beside it; a request's result is the same alone and
in the mix."""
import time

import numpy as np
import pytest

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu

RING = 64  # queue slots of the persistent kernel


def _ok(res):
    assert res.done == 1 and res.status == 0, f"status {res.status}: {res.message}"


@pytest.fixture(scope="module")
def pool():
    sizes = [1000, 4000, 9000, 30000, 70000, 150000]
    return [mg.serving_matrix(n, seed=mg.seed_for(4) ^ (i + 11)) for i, n in enumerate(sizes)]


def _spmv_requests(pool, n, seed, kmax=8):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n):
        mid = int(rng.integers(len(pool)))
        k = int(rng.integers(1, kmax + 1))
        out.append((mid, mg.uniform(k * pool[mid].n_cols, seed + t, 3).reshape(k, pool[mid].n_cols)))
    return out


def _run(srv, pool, reqs, batch):
    """Submits reqs in groups of `batch`, waiting for each group."""
    outs = []
    for i in range(0, len(reqs), batch):
        tickets = [srv.submit_spmv(mid, X) for mid, X in reqs[i:i + batch]]
        for t in tickets:
            out, res = srv.wait(t)
            _ok(res)
            outs.append(out.copy())
    return outs


def test_persistent_rounds_equal_launched_rounds_bitwise(pool):
    # groups of 6, then one request at a time: well over RING rounds, so
    # every queue slot and its claim word are reused, and request buffers
    # come back from the memory pool at addresses used before
    reqs = _spmv_requests(pool, 40, 1000) + _spmv_requests(pool[:4], 90, 2000, kmax=2)
    with spmv.Server(persistent_wgs=96) as srv:
        for A in pool:
            srv.add_matrix(A)
        got = _run(srv, pool, reqs[:40], 6) + _run(srv, pool, reqs[40:], 1)
        st = srv.stats()
    assert st["rounds"] > RING and st["persist_launches"] >= 1 and st["failed"] == 0
    with spmv.Server() as srv:
        for A in pool:
            srv.add_matrix(A)
        ref = _run(srv, pool, reqs, 8)
        assert srv.stats()["persist_launches"] == 0
    for (mid, X), a, b in zip(reqs, got, ref):
        assert np.array_equal(a, b), mid
    for (mid, X), a in list(zip(reqs, got))[::7]:
        for j in range(X.shape[0]):
            y_ref, bound = oracle.spmv(pool[mid], X[j])
            assert oracle.spmv_accept(a[j], y_ref, bound).all()


def test_persistent_kernel_ends_when_idle_and_is_launched_again(pool):
    reqs = _spmv_requests(pool[:3], 6, 3000)
    with spmv.Server(persistent_wgs=32, persist_idle_us=300) as srv:
        for A in pool[:3]:
            srv.add_matrix(A)
        outs = []
        for mid, X in reqs:
            out, res = srv.wait(srv.submit_spmv(mid, X))
            _ok(res)
            outs.append(out)
            time.sleep(0.05)   # far longer than the idle time: the launch ends
        st = srv.stats()
    assert st["persist_launches"] >= len(reqs) - 1
    for (mid, X), out in zip(reqs, outs):
        for j in range(X.shape[0]):
            y_ref, bound = oracle.spmv(pool[mid], X[j])
            assert oracle.spmv_accept(out[j], y_ref, bound).all()


def test_persistent_large_round_and_cg_beside_it(pool):
    # a 32-vector request on the 150K-row matrix (a round of its own, about
    # 4,700 tiles claimed by all workgroups) while CG solves run on the
    # solver slots' streams
    A = pool[-1]
    big = mg.uniform(32 * A.n_cols, 61, 3).reshape(32, A.n_cols)
    cg = [(4 + (i % 2), mg.uniform(pool[4 + (i % 2)].n_rows, 80 + i, 4)) for i in range(3)]
    with spmv.Server(n_slots=3, persistent_wgs=512, preload=True) as srv:
        for M in pool:
            srv.add_matrix(M)
        srv.drain()
        t_cg = [srv.submit_cg(mid, b, tol=1e-8) for mid, b in cg]
        t_big = srv.submit_spmv(len(pool) - 1, big)
        out, res = srv.wait(t_big)
        _ok(res)
        sols = [srv.wait(t) for t in t_cg]
    for j in range(32):
        y_ref, bound = oracle.spmv(A, big[j])
        assert oracle.spmv_accept(out[j], y_ref, bound).all(), j
    for (mid, b), (x, r) in zip(cg, sols):
        _ok(r)
        Ax, _ = oracle.spmv(pool[mid], x)
        assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 1.05e-8


def test_persistent_alone_equals_mix_bitwise(pool):
    rng = np.random.default_rng(4000)
    reqs = []
    for t in range(30):
        mid = int(rng.integers(len(pool)))
        if rng.random() < 0.6:
            k = int(rng.integers(1, 9))
            reqs.append(("spmv", mid, mg.uniform(k * pool[mid].n_cols, 4000 + t, 3).reshape(k, pool[mid].n_cols)))
        else:
            reqs.append(("cg", mid, mg.uniform(pool[mid].n_rows, 4000 + t, 4)))
    sub = lambda srv, r: srv.submit_spmv(r[1], r[2]) if r[0] == "spmv" else srv.submit_cg(r[1], r[2], tol=1e-8)
    with spmv.Server(n_slots=4, persistent_wgs=128) as srv:
        for A in pool:
            srv.add_matrix(A)
        alone = []
        for r in reqs:
            out, res = srv.wait(sub(srv, r))
            _ok(res)
            alone.append(out.copy())
        tickets = [sub(srv, r) for r in reqs]
        mixed = []
        for t in tickets:
            out, res = srv.wait(t)
            _ok(res)
            assert res.compute_s > 0 and res.compute_s <= res.latency_s
            mixed.append(out)
    for a, m in zip(alone, mixed):
        assert np.array_equal(a, m)


def test_persistent_configuration_is_checked():
    for bad in ({"persistent_wgs": -1}, {"persist_idle_us": -5}, {"persist_idle_us": 10_000_001}):
        with pytest.raises(spmv.SpmvError) as e:
            spmv.Server(**bad)
        assert e.value.code == spmv.SPMV_EINVAL
