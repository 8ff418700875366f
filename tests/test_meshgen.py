"""Invariants of the seeded input generators (no SpMV arithmetic here)."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import meshgen as mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _S(A):
    return sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))


SYM = [
    ("cfg0", lambda: mg.config0()),
    ("knn", lambda: mg.knn(14, seed=5)),
    ("stencil27", lambda: mg.lattice(12, 11, 10, "stencil27", seed=6)),
    ("cfg1-random", lambda: mg.config1("random", m=12)),
]


@pytest.mark.parametrize("name,make", SYM, ids=[s[0] for s in SYM])
def test_symmetric_dominant_sorted(name, make):
    A = make()
    S = _S(A)
    assert abs(S - S.T).max() == 0.0
    assert (A.nnz - A.n_rows) % 2 == 0          # symmetric pattern with full diagonal
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - d
    assert np.all(d > off)
    assert np.allclose(d - off, 1e-3, rtol=0, atol=1e-12)
    for i in range(0, A.n_rows, max(1, A.n_rows // 200)):
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


def test_row_length_ranges():
    A = mg.config0()
    L = A.row_lengths()
    assert A.n_rows == 32768 and L.min() >= 4 and L.max() <= 1 + 6 + 118
    assert 10.0 < L.mean() < 11.5
    B = mg.lattice(20, 20, 20, "stencil27", seed=7)
    L = B.row_lengths().reshape(20, 20, 20)[1:-1, 1:-1, 1:-1]
    assert L.min() >= 7 and L.max() <= 27 and 16 < L.mean() < 18
    C = mg.knn(20, seed=8)
    L = C.row_lengths()
    assert L.min() >= 5 and 6.3 < L.mean() < 7.5


def test_table1_shape_invariants():
    """The paper's tetrahedral matrices: symmetric pattern with a full diagonal
    (nnz - rows even) and at most five non-zeros per row."""
    with open(os.path.join(GOLDEN, "table1_matrices.csv")) as f:
        rows = [r for r in csv.DictReader(line for line in f if not line.startswith("#"))]
    assert len(rows) == 5
    for r in rows:
        n, nnz = int(r["rows"]), int(r["nnz"])
        assert (nnz - n) % 2 == 0
        assert 4.9 < nnz / n <= 5.0


def test_deterministic_and_thread_independent():
    A = mg.lattice(9, 8, 7, "extras", seed=3)
    B = mg.lattice(9, 8, 7, "extras", seed=3)
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.values, B.values)
    code = ("import meshgen as mg, hashlib;"
            "A=mg.reorder(mg.knn(16, seed=4),'rcm',4);"
            "print(hashlib.sha256(A.col_idx.tobytes()+A.values.tobytes()).hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=root)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   text=True, check=True).stdout.strip())
    assert outs[0] == outs[1]


def test_rcm_is_permutation_and_reduces_band():
    A = mg.knn(16, seed=9)
    p = mg.rcm_perm(A)
    assert np.array_equal(np.sort(p), np.arange(A.n_rows))
    B = mg.permute(A, p)
    ref = reverse_cuthill_mckee(_S(A), symmetric_mode=True)
    C = mg.permute(A, ref.astype(np.int32))
    bw_ours = mg.bandwidth(B)[1]
    bw_scipy = mg.bandwidth(C)[1]
    assert bw_ours <= 1.2 * bw_scipy and bw_scipy <= 1.2 * bw_ours
    rnd = mg.permute(A, mg.random_perm(A.n_rows, 1))
    assert bw_ours < mg.bandwidth(rnd)[1] / 4


def test_rcm_path_graph_bandwidth_one():
    n = 50
    perm = mg.random_perm(n, 2)
    # path graph in natural order, then scrambled
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    S = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    A = mg.CSR(n, n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    A = mg.permute(A, perm)
    assert mg.bandwidth(A)[1] > 1
    B = mg.permute(A, mg.rcm_perm(A))
    assert mg.bandwidth(B)[1] == 1


def test_rcm_disconnected_and_isolated():
    n = 30
    d = np.ones(n)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    p = mg.rcm_perm(A)
    assert np.array_equal(np.sort(p), np.arange(n))


def test_permute_roundtrip():
    A = mg.lattice(7, 6, 5, "extras", seed=12)
    p = mg.random_perm(A.n_rows, 3)
    inv = np.empty_like(p)
    inv[p] = np.arange(A.n_rows, dtype=np.int32)
    B = mg.permute(mg.permute(A, p), inv)
    assert np.array_equal(A.row_ptr, B.row_ptr)
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.values, B.values)


def test_dyadic_values():
    A = mg.lattice(6, 6, 6, "extras", seed=1, dyadic=True)
    assert np.all(A.values * 1024 == np.round(A.values * 1024))
    x = mg.dyadic_x(1000, 2)
    assert len(np.unique(x)) == 1000 and np.all(x * 2 ** 20 == np.round(x * 2 ** 20))


def test_tet_like_stand_in_matches_table1_shape():
    """The tetrahedral stand-in at the paper's C50K size: at most four
    neighbours per cell (five non-zeros per row, Sec. 2), symmetric pattern
    and values, full diagonal, strictly dominant, nnz/rows as in Table 1,
    deterministic."""
    with open(os.path.join(GOLDEN, "table1_matrices.csv")) as f:
        rows = {r["name"]: r for r in csv.DictReader(line for line in f if not line.startswith("#"))}
    assert mg.TABLE1_ROWS == {k: int(v["rows"]) for k, v in rows.items()}
    A = mg.tet_like(mg.TABLE1_ROWS["C50K"])
    n = A.n_rows
    L = np.diff(A.row_ptr)
    assert n == 49336 and L.max() <= 5 and L.min() >= 1
    assert (A.nnz - n) % 2 == 0
    paper = int(rows["C50K"]["nnz"]) / n
    assert abs(A.nnz / n - paper) < 0.02
    S = sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(n, n))
    assert abs(S - S.T).max() == 0
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d > 0) and np.all(d - off > 0.9e-3)
    B = mg.tet_like(mg.TABLE1_ROWS["C50K"])
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.values, B.values)


def test_with_long_rows_replaces_only_the_chosen_rows():
    """with_long_rows: n_long rows spread over the matrix get `length`
    sorted distinct columns; every other row keeps its entries; seeded."""
    A = mg.lattice(12, 12, 12, "extras", seed=3)
    B = mg.with_long_rows(A, 5, 1500, seed=9)
    la, lb = np.diff(A.row_ptr), np.diff(B.row_ptr)
    long_rows = np.nonzero(lb == 1500)[0]
    assert len(long_rows) == 5 and long_rows.min() > 0 and long_rows.max() < A.n_rows - 1
    keep = np.setdiff1d(np.arange(A.n_rows), long_rows)
    assert np.array_equal(la[keep], lb[keep])
    for r in keep[::37]:
        assert np.array_equal(A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]], B.col_idx[B.row_ptr[r]:B.row_ptr[r + 1]])
        assert np.array_equal(A.values[A.row_ptr[r]:A.row_ptr[r + 1]], B.values[B.row_ptr[r]:B.row_ptr[r + 1]])
    for r in long_rows:
        c = B.col_idx[B.row_ptr[r]:B.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0) and c[0] >= 0 and c[-1] < A.n_cols
    C = mg.with_long_rows(A, 5, 1500, seed=9)
    assert np.array_equal(B.col_idx, C.col_idx) and np.array_equal(B.values, C.values)
    with pytest.raises(ValueError):
        mg.with_long_rows(A, 1, A.n_cols + 1, seed=9)
