"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times: the 16,003,008-row hex mesh matrix (RCM, default plan =
compact windows on 2048-entry tiles) and the 4,000,000-block-row 3x3 block
operator.  The oracle checks sampled rows one by one (a fixed random sample,
the first and last rows, and every row of a few whole tiles); properties
that hold at any size check the rest (kernel variants agree bit for bit,
the CG answer's true residual is recomputed by the oracle on all rows)."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mesh16m():
    A = mg.config2()
    assert A.n_rows == 252 ** 3 and A.nnz == 270_148_760
    return A


def _sample_rows(A, info, seed):
    rng = np.random.default_rng(seed)
    rows = set(rng.integers(0, A.n_rows, 20000).tolist())
    rows |= {0, 1, A.n_rows - 2, A.n_rows - 1}
    # every row of three whole tiles (first, middle, last 512 rows)
    for r0 in (0, A.n_rows // 2, A.n_rows - 512):
        rows |= set(range(r0, r0 + 512))
    return np.array(sorted(rows), np.int32)


def test_mesh16m_default_plan_sampled_rows(mesh16m):
    A = mesh16m
    x = mg.uniform(A.n_cols, 101, 0)
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        info = M.info
        assert info["tile_nnz"] == 2048 and info["n_window_tiles"] > info["n_tiles"] // 2
        xd = torch.as_tensor(x, device=DEV)
        y = M.apply(xd).cpu().numpy()
        y32 = M.apply_f32(xd.float()).cpu().numpy().astype(np.float64)
    rows = _sample_rows(A, info, 7)
    y_ref, bound = oracle.spmv_rows(A, x, rows)
    ok = oracle.spmv_accept(y[rows], y_ref, bound)
    assert ok.all(), f"{(~ok).sum()} sampled rows fail"
    m = np.diff(A.row_ptr)[rows].astype(np.float64)
    assert np.all(np.abs(y32[rows] - y_ref) <= 1.01 * (m + 2) * 2.0 ** -24 * bound)
    assert np.isfinite(y).all()


def test_mesh16m_spmm_k8_sampled_rows(mesh16m):
    # the k = 8 product the bench times: sampled rows of every column against
    # the oracle, two whole columns bitwise against the single-vector product
    A = mesh16m
    k = 8
    X = mg.uniform(A.n_cols * k, 104, 5).reshape(A.n_cols, k)
    with spmv.Matrix.from_csr(A) as M:
        info = M.info
        Xd = torch.as_tensor(X, device=DEV)
        Y = M.spmm(Xd)
        for j in (0, k - 1):
            y = M.apply(Xd[:, j].contiguous())
            assert torch.equal(Y[:, j], y), j
        Y = Y.cpu().numpy()
    rows = _sample_rows(A, info, 8)
    for j in range(k):
        y_ref, bound = oracle.spmv_rows(A, np.ascontiguousarray(X[:, j]), rows)
        assert oracle.spmv_accept(Y[rows, j], y_ref, bound).all(), j


def test_mesh16m_kernels_and_plans_bitwise(mesh16m):
    # compact windows (one workgroup per tile and persistent), direct
    # gathers and sliced ELLPACK give the same bits on every row
    A = mesh16m
    x = torch.as_tensor(mg.uniform(A.n_cols, 102, 0), device=DEV)
    ys = []
    for params in ({}, {"kernel": 2}, {"window_mode": spmv.WINDOW_OFF, "tile_nnz": 2048},
                   {"format": spmv.FORMAT_SELL}):
        with spmv.Matrix.from_csr(A, params=params) as M:
            ys.append(M.apply(x).cpu())
    assert all(torch.equal(ys[0], y) for y in ys[1:])


@pytest.mark.parametrize("mode", [spmv.CG_FP64, spmv.CG_MIXED_FP32, spmv.CG_PCG_BF16, spmv.CG_MIXED_FP32V,
                                  spmv.CG_PCG_JACOBI])
def test_mesh16m_cg_to_1e10(mesh16m, mode):
    A = mesh16m
    b = mg.uniform(A.n_rows, 103, 4)
    fp32 = mode in (spmv.CG_MIXED_FP32, spmv.CG_MIXED_FP32V)
    with spmv.Matrix.from_csr(A, fp32=fp32, bf16=(mode == spmv.CG_PCG_BF16)) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=1e-10, max_iter=5000, mode=mode)
        x = x.cpu().numpy()
    assert info.iterations > 0
    Ax, _ = oracle.spmv(A, x)
    rel = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    assert rel <= 1.05e-10, rel
    assert abs(rel - info.rel_residual) <= 0.05 * rel + 1e-14


def test_bsr3_4m_block_rows_sampled():
    A = mg.config3()
    assert A.n_rows == 4_000_000
    rng = np.random.default_rng(9)
    brs = np.unique(np.concatenate([rng.integers(0, A.n_rows, 4000), [0, A.n_rows - 1],
                                    np.arange(A.n_rows // 2, A.n_rows // 2 + 200)]))
    # the sampled block rows as a block matrix of their own (same columns)
    lens = np.diff(A.row_ptr)[brs]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in brs])
    S = mg.CSR(len(brs), A.n_cols, rp, A.col_idx[idx], A.values.reshape(-1, 3, 3)[idx], 3)
    srows = (3 * brs[:, None] + np.arange(3)).reshape(-1)
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        for k in (1, 4, 8):
            X = mg.uniform(3 * A.n_cols * k, 110 + k, 0).reshape(3 * A.n_cols, k)
            Xd = torch.as_tensor(X, device=DEV)
            Y = M.spmm(Xd).cpu().numpy()
            Y32 = M.spmm_f32(Xd.float()).cpu().numpy().astype(np.float64)
            Yr, Bd = oracle.bsr3_spmm(S, X)
            assert oracle.spmv_accept(Y[srows], Yr, Bd).all()
            m = 3 * np.repeat(lens, 3)[:, None].astype(np.float64)
            assert np.all(np.abs(Y32[srows] - Yr) <= 1.01 * (m + 2) * 2.0 ** -24 * Bd)
            if k > 1:
                y1 = M.spmm(Xd[:, k - 1:].contiguous()).cpu().numpy()
                assert np.array_equal(y1[:, 0], Y[:, k - 1])
            if k == 8:
                # a 2.7 GB matrix is dealt to the XCDs in chunks of tiles; one
                # contiguous range per XCD gives the same bits
                with spmv.Matrix.from_csr(A, xcd_contiguous=True) as Mc:
                    assert np.array_equal(Mc.spmm(Xd).cpu().numpy(), Y)
