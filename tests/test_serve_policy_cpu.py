"""The server's admission policy (device-memory budget + LRU eviction),
replayed on the host through the library's test hook (no GPU)."""
import paper_2107_12371_amd as spmv

ADMIT, WAIT, NEVER = 0, 1, 2


def test_admit_upload_reuse_and_release():
    r = spmv.policy_simulate(100, [40, 30], [(0, 0, 10), (0, 0, 10), (1, 0, 10), (1, 0, 10)])
    assert r[0] == (ADMIT, 0, 1, 50)      # upload 40 + 10 buffers
    assert r[1] == (ADMIT, 0, 0, 60)      # resident already: only buffers
    assert r[2][3] == 50 and r[3][3] == 40  # releases keep the matrix resident


def test_lru_eviction_of_idle_matrices_only():
    ops = [(0, 0, 0), (1, 0, 0),           # matrix 0 resident, idle (t=1)
           (0, 1, 0), (1, 1, 0),           # matrix 1 resident, idle (t=2)
           (0, 2, 0)]                      # needs 50: must evict the LRU idle one (matrix 0)
    r = spmv.policy_simulate(100, [40, 40, 50], ops)
    assert r[4] == (ADMIT, 1, 1, 90)
    # pinned matrices are never evicted: with 0 and 1 in flight, 2 must wait
    ops = [(0, 0, 0), (0, 1, 0), (0, 2, 0), (1, 0, 0), (0, 2, 0)]
    r = spmv.policy_simulate(100, [40, 40, 50], ops)
    assert r[2][0] == WAIT
    assert r[4] == (ADMIT, 1, 1, 90)       # after 0 is released it is evicted


def test_never_fits_and_buffers_count():
    r = spmv.policy_simulate(100, [60], [(0, 0, 50)])
    assert r[0][0] == NEVER
    r = spmv.policy_simulate(100, [60], [(0, 0, 20), (0, 0, 20), (0, 0, 1)])
    assert [v[0] for v in r] == [ADMIT, ADMIT, WAIT]


def test_many_matrices_stay_within_budget():
    import numpy as np
    rng = np.random.default_rng(0)
    sizes = rng.integers(1, 30, 40).tolist()
    budget = 120
    live, done_ops = [], []
    for _ in range(300):
        if live and rng.random() < 0.5:
            m, e = live.pop(int(rng.integers(len(live))))
            op = (1, m, e)
        else:
            op = (0, int(rng.integers(40)), int(rng.integers(0, 10)))
        trial = spmv.policy_simulate(budget, sizes, done_ops + [op])
        if op[0] == 0:
            if trial[-1][0] != ADMIT:
                continue
            live.append(op[1:])
        done_ops.append(op)
        assert trial[-1][3] <= budget
    # every in-flight request's matrix is resident: its bytes are counted
    final = spmv.policy_simulate(budget, sizes, done_ops)
    assert final[-1][3] >= sum(e for _, e in live) + sum(sizes[m] for m in {m for m, _ in live})


def test_failed_upload_leaves_matrix_not_resident():
    # admission asks for the upload of matrix 0; the upload fails (kind 2) and
    # the request is released: nothing stays reserved, and the next request
    # on matrix 0 uploads it again
    r = spmv.policy_simulate(100, [40, 30], [(0, 0, 10), (2, 0, 0), (1, 0, 10), (0, 0, 10), (1, 0, 10)])
    assert r[0] == (ADMIT, 0, 1, 50)
    assert r[1][3] == 10 and r[2][3] == 0
    assert r[3] == (ADMIT, 0, 1, 50)
    assert r[4][3] == 40
    # a failed upload frees room for others: matrix 1 fits without evicting
    r = spmv.policy_simulate(60, [40, 50], [(0, 0, 0), (2, 0, 0), (1, 0, 0), (0, 1, 5)])
    assert r[3] == (ADMIT, 0, 1, 55)


def test_preload_only_into_free_budget():
    r = spmv.policy_simulate(100, [40, 30, 50], [(3, 0, 0), (3, 1, 0), (3, 2, 0), (3, 0, 0)])
    assert [x[0] for x in r] == [ADMIT, ADMIT, WAIT, WAIT]     # 2 does not fit; 0 is already resident
    assert [x[2] for x in r] == [1, 1, 0, 0] and r[-1][3] == 70
    # a preloaded matrix serves requests without another upload and, idle,
    # can be evicted like any other
    r = spmv.policy_simulate(80, [40, 30, 50], [(3, 0, 0), (0, 0, 10), (1, 0, 10), (0, 2, 0)])
    assert r[1] == (ADMIT, 0, 0, 50)
    assert r[3] == (ADMIT, 1, 1, 50)


def test_simulator_rejects_bad_ops():
    import pytest
    with pytest.raises(spmv.SpmvError):
        spmv.policy_simulate(100, [40], [(5, 0, 0)])
    with pytest.raises(spmv.SpmvError):
        spmv.policy_simulate(100, [40], [(2, 0, 0)])        # not resident: no upload to fail
