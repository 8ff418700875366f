"""GPU parity of rows longer than a tile, summed in pieces of 16,384 stored
entries.  Each piece runs on a workgroup of its own and a second launch adds
the pieces' sums, kept in scratch: the output vector's own rows (the longest
run without a long row, written by the same call afterwards; spmv_apply and
every product), or the caller's workspace (spmv_apply_ws).  Without scratch,
or with spmv_params.long_rows = 1, one workgroup walks a row's pieces.  All
must give the same bits, meet the oracle's per-row bound (equal it bit for
bit on dyadic inputs), and so must the products and solvers built on them:
k-vector products, SELL handles, FP32 and BF16 products, CG in every mode
and the allocation-free solve, graph-captured products.

Acceptance as in the other SpMV parity tests: binary64 within
1e-12 * sum_k |a_ik||x_k| per row; FP32 within (m + 2) * 2^-24 of that bound
with m the row length; BF16 values within (2^-8 + (m + 1) * 2^-24).
"""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PIECE = 16384
# around every boundary that matters: one piece below and above a tile
# (2048-entry tiles hold 2045), exactly one and two pieces, one past them,
# and rows of many pieces
LENS = [2046, 4093, 4094, 16384, 16385, 32768, 32769, 40000, 100_000, 1_000_003]


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def long_row_matrix(n_rows, n_cols, lens, seed, dyadic=False):
    """Short Poisson(6) rows with rows of the given lengths spread over the
    matrix (the first and last rows among them); long rows take random,
    unsorted columns with repeats.  Dyadic values are k / 2^10, |k| <= 2^10,
    so with dyadic x every product and partial sum is exact."""
    rng = np.random.default_rng(seed)
    rl = np.minimum(rng.poisson(6.0, n_rows), n_cols).astype(np.int64)
    where = np.linspace(0, n_rows - 1, len(lens)).astype(np.int64)
    rl[where] = lens
    rp = np.zeros(n_rows + 1, np.int64)
    rp[1:] = np.cumsum(rl)
    ci = rng.integers(0, n_cols, int(rp[-1])).astype(np.int32)
    if dyadic:
        va = rng.integers(-1024, 1025, int(rp[-1])).astype(np.float64) / 1024.0
    else:
        va = rng.uniform(-1.0, 1.0, int(rp[-1]))
    return mg.CSR(n_rows, n_cols, rp.astype(np.int32), ci, va, 1), where


@pytest.fixture(scope="module")
def mats():
    A, where = long_row_matrix(50_000, 1 << 20, LENS, seed=71)
    Ad, _ = long_row_matrix(50_000, 1 << 20, LENS, seed=72, dyadic=True)
    return A, Ad, where


def _pieces(lens, cap):
    return sum(-(-L // PIECE) for L in lens if L > cap)


def assert_parity(y, A, x, rtol=oracle.SPMV_RTOL):
    y_ref, bound = oracle.spmv(A, x)
    ok = oracle.spmv_accept(y, y_ref, bound, rtol)
    assert ok.all(), f"{int((~ok).sum())} rows fail, first {int(np.nonzero(~ok)[0][0])}"


@pytest.mark.parametrize("tile_nnz", [1024, 2048, 4096])
def test_pieces_on_their_own_workgroups_equal_one_workgroup_per_row(mats, tile_nnz):
    A, _, where = mats
    x = mg.uniform(A.n_cols, 5, 1)
    xd = to_dev(x)
    with spmv.Matrix.from_csr(A, params={"tile_nnz": tile_nnz}) as M:
        inf = M.info
        cap = tile_nnz - 3
        assert inf["n_long_rows"] == sum(1 for L in LENS if L > cap)
        assert inf["n_long_pieces"] == _pieces(LENS, cap)
        assert M.workspace_bytes == inf["workspace_bytes"] == 8 * inf["n_long_pieces"]
        assert inf["y_scratch_ok"] == 1
        y_out = M.apply(xd).cpu().numpy()        # scratch in the output's rows
        y_ws = M.apply_ws(xd).cpu().numpy()      # scratch from the caller
    with spmv.Matrix.from_csr(A, params={"tile_nnz": tile_nnz, "long_rows": 1}) as M1:
        assert M1.info["y_scratch_ok"] == 0
        y_one = M1.apply(xd).cpu().numpy()       # one workgroup per row
        y_one_ws = M1.apply_ws(xd).cpu().numpy()  # long_rows = 1 holds with a workspace too
    assert np.array_equal(y_out, y_ws)
    assert np.array_equal(y_out, y_one)
    assert np.array_equal(y_out, y_one_ws)
    assert_parity(y_out, A, x)


def test_no_room_in_the_output_falls_back_to_one_workgroup_per_row():
    # long rows (3 pieces each) alternate with single short rows: no run of
    # short rows holds the 96 pieces' sums, so spmv_apply walks each long
    # row on one workgroup; spmv_apply_ws still splits; same bits
    rl = np.full(64, 5)
    rl[::2] = 40_000
    rng = np.random.default_rng(75)
    rp = np.concatenate([[0], np.cumsum(rl)]).astype(np.int32)
    A = mg.CSR(64, 50_000, rp, rng.integers(0, 50_000, int(rp[-1])).astype(np.int32),
               rng.uniform(-1.0, 1.0, int(rp[-1])), 1)
    x = mg.uniform(A.n_cols, 17, 1)
    with spmv.Matrix.from_csr(A, fp32=True, params={"tile_nnz": 1024}) as M:
        assert M.info["n_long_pieces"] == 96 and M.info["y_scratch_ok"] == 0
        xd = to_dev(x)
        y1 = M.apply(xd).cpu().numpy()
        y2 = M.apply_ws(xd).cpu().numpy()
        y32 = M.apply_f32(xd.float()).cpu().numpy()
    assert np.array_equal(y1, y2)
    assert_parity(y1, A, x)
    y_ref, bound = oracle.spmv(A, x)
    m = np.maximum(np.diff(A.row_ptr), 1).astype(np.float64)
    assert (np.abs(y32.astype(np.float64) - y_ref) <= 1.01 * (m + 2) * 2.0 ** -24 * bound).all()


def test_dyadic_long_rows_equal_the_oracle_bitwise(mats):
    _, Ad, where = mats
    x = mg.dyadic_x(Ad.n_cols, seed=9)
    y_ref, _ = oracle.spmv(Ad, x)
    with spmv.Matrix.from_csr(Ad) as M:
        xd = to_dev(x)
        y1 = M.apply(xd).cpu().numpy()
        y2 = M.apply_ws(xd).cpu().numpy()
    assert np.array_equal(y1, y_ref)
    assert np.array_equal(y2, y_ref)


def test_non_finite_values_in_one_piece(mats):
    A, _, where = mats
    B = mg.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.values.copy(), 1)
    r = int(where[-1])  # the 1,000,003-entry row: NaN in its 40th piece only
    B.values[B.row_ptr[r] + 39 * PIECE + 5] = np.nan
    r2 = int(where[-2])  # the 100,000-entry row: +Inf in its last piece
    B.values[B.row_ptr[r2 + 1] - 1] = np.inf
    x = mg.uniform(B.n_cols, 6, 1) + 2.0  # positive, so the Inf row is +Inf
    with spmv.Matrix.from_csr(B) as M:
        xd = to_dev(x)
        y1 = M.apply(xd).cpu().numpy()
        y2 = M.apply_ws(xd).cpu().numpy()
    assert np.isnan(y1[r]) and np.isnan(y2[r])
    assert y1[r2] == np.inf and y2[r2] == np.inf
    assert np.array_equal(y1, y2, equal_nan=True)
    assert_parity(y2, B, x)


def test_workspace_is_checked(mats):
    A, _, _ = mats
    x = to_dev(mg.uniform(A.n_cols, 7, 1))
    with spmv.Matrix.from_csr(A) as M:
        need = M.workspace_bytes
        assert need > 0
        ws = torch.empty(need // 8 + 2, dtype=torch.float64, device=DEV)
        y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        for bad in (ws[: need // 8 - 1], None):
            with pytest.raises(spmv.SpmvError) as e:
                M.apply_ws(x, y, ws=bad if bad is not None else torch.empty(0, device=DEV))
            assert e.value.code == spmv.SPMV_EINVAL
        # misaligned by 4 bytes
        raw = torch.empty(need + 16, dtype=torch.uint8, device=DEV)
        with pytest.raises(spmv.SpmvError) as e:
            M.apply_ws(x, y, ws=raw[4:4 + need])
        assert e.value.code == spmv.SPMV_EINVAL
        # overlapping y
        big = torch.empty(A.n_rows + need // 8, dtype=torch.float64, device=DEV)
        with pytest.raises(spmv.SpmvError) as e:
            M.apply_ws(x, big[:A.n_rows], ws=big[A.n_rows - 1:])
        assert e.value.code == spmv.SPMV_EINVAL
        # a larger workspace is fine
        ref = M.apply(x).cpu().numpy()
        assert np.array_equal(M.apply_ws(x, y, ws=ws).cpu().numpy(), ref)


def test_no_split_without_rows_of_several_pieces():
    # long rows of one piece each, and a matrix without long rows: nothing
    # to split, no workspace, apply_ws is apply
    for lens in ([3000, 9000, 16384], []):
        A, _ = long_row_matrix(20_000, 50_000, lens or [5], seed=73)
        x = mg.uniform(A.n_cols, 8, 1)
        with spmv.Matrix.from_csr(A, params={"tile_nnz": 1024}) as M:
            assert M.workspace_bytes == 0 and M.info["n_long_pieces"] == len(lens)
            xd = to_dev(x)
            y1 = M.apply(xd).cpu().numpy()
            y2 = M.apply_ws(xd).cpu().numpy()
        assert np.array_equal(y1, y2)
        assert_parity(y2, A, x)


def test_k_vector_products_on_long_rows_equal_single_products(mats):
    # the pieces of the k columns on a workgroup each (their sums in Y's own
    # rows) and one workgroup per (row, column): both equal the single
    # products column by column
    A, _, _ = mats
    k = 3
    X = mg.uniform(A.n_cols * k, 10, 1).reshape(A.n_cols, k)
    with spmv.Matrix.from_csr(A) as M, spmv.Matrix.from_csr(A, params={"long_rows": 1}) as M1:
        Y = M.spmm(to_dev(X)).cpu().numpy()
        Y1 = M1.spmm(to_dev(X)).cpu().numpy()
        assert np.array_equal(Y, Y1)
        for j in range(k):
            yj = M.apply_ws(to_dev(X[:, j])).cpu().numpy()
            assert np.array_equal(Y[:, j], yj), j


def test_sell_handle_long_rows(mats):
    A, _, _ = mats
    x = mg.uniform(A.n_cols, 11, 1)
    xd = to_dev(x)
    with spmv.Matrix.from_csr(A, params={"format": spmv.FORMAT_SELL}) as M:
        assert M.info["n_long_pieces"] == _pieces(LENS, 255)
        assert M.workspace_bytes == 8 * M.info["n_long_pieces"] and M.info["y_scratch_ok"] == 1
        y1 = M.apply(xd).cpu().numpy()
        y2 = M.apply_ws(xd).cpu().numpy()
    with spmv.Matrix.from_csr(A, params={"format": spmv.FORMAT_SELL, "long_rows": 1}) as M1:
        y3 = M1.apply(xd).cpu().numpy()
    assert np.array_equal(y1, y2) and np.array_equal(y1, y3)
    assert_parity(y2, A, x)


def test_reduced_precision_long_rows(mats):
    # the FP32 and BF16 products split the long rows in their output's rows
    # (4 bytes each: two per piece sum); same bits as one workgroup per row
    A, _, _ = mats
    x = mg.uniform(A.n_cols, 12, 1)
    y_ref, bound = oracle.spmv(A, x)
    m = np.maximum(np.diff(A.row_ptr), 1).astype(np.float64)
    x32 = to_dev(x, torch.float32)
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True, params={"long_rows": 1}) as M1:
        one = [M1.apply_f32(x32).cpu().numpy(), M1.apply_bf16(x32).cpu().numpy(),
               M1.apply_f32v(to_dev(x)).cpu().numpy()]
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True) as M:
        split = [M.apply_f32(x32).cpu().numpy(), M.apply_bf16(x32).cpu().numpy(),
                 M.apply_f32v(to_dev(x)).cpu().numpy()]
        y32 = M.apply_f32(x32).cpu().numpy().astype(np.float64)
        y16 = M.apply_bf16(x32).cpu().numpy().astype(np.float64)
    for a, b in zip(one, split):
        assert np.array_equal(a, b)
    # x rounded to FP32 adds 2^-24 per product: inside the (m + 2) term
    assert (np.abs(y32 - y_ref) <= 1.01 * (m + 2) * 2.0 ** -24 * bound).all()
    assert (np.abs(y16 - y_ref) <= 1.01 * (2.0 ** -8 + (m + 1) * 2.0 ** -24) * bound).all()


def arrow_spd(base, hubs, seed, w=1e-2):
    """base + sum over hub h and neighbour c of w (e_c - e_h)(e_c - e_h)^T:
    SPD when base is, with row and column h holding len(C_h) + 1 entries."""
    import scipy.sparse as sp
    n = base.n_rows
    rng = np.random.default_rng(seed)
    B = sp.csr_matrix((base.values, base.col_idx, base.row_ptr), shape=(n, n))
    rows, cols, vals = [], [], []
    for h, L in hubs:
        C = rng.choice(np.setdiff1d(np.arange(n), [h]), size=L, replace=False)
        rows += [C, np.full(L, h), C, np.array([h])]
        cols += [np.full(L, h), C, C, np.array([h])]
        vals += [np.full(L, -w), np.full(L, -w), np.full(L, w), np.array([w * L])]
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    S = (B + D).tocsr()
    S.sort_indices()
    return mg.CSR(n, n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64), 1)


@pytest.fixture(scope="module")
def arrow():
    base = mg.lattice(40, 40, 40, "extras", seed=mg.seed_for(0))
    return arrow_spd(base, [(777, 40_000), (31_000, 20_000), (63_999, 33_000)], seed=74)


def test_cg_with_long_rows_split_equals_one_workgroup_per_row(arrow):
    A = arrow
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True) as M:
        assert M.info["n_long_rows"] == 3 and M.workspace_bytes > 0
        b = to_dev(mg.uniform(A.n_rows, 13, 4))
        x1, i1 = M.cg(b, tol=1e-10)            # pieces' sums in the solver's workspace
        x2, i2 = M.cg_noalloc(b, tol=1e-10)    # ... in the product's output rows
        assert i1.iterations == i2.iterations
        assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
        with spmv.Matrix.from_csr(A, params={"long_rows": 1}) as M1:
            x3, i3 = M1.cg(b, tol=1e-10)       # one workgroup per long row
        assert i3.iterations == i1.iterations
        assert np.array_equal(x1.cpu().numpy(), x3.cpu().numpy())
        # the FP32 and bfloat16 products of the other solvers split the long
        # rows the same way
        xm, im = M.cg(b, tol=1e-10, mode=spmv.CG_MIXED_FP32)
        xj, ij = M.cg(b, tol=1e-10, mode=spmv.CG_PCG_JACOBI)
        xp, ip = M.cg(b, tol=1e-10, mode=spmv.CG_PCG_BF16)
    bh = b.cpu().numpy()
    for xs in (x1, xm, xj, xp):
        Ax, _ = oracle.spmv(A, xs.cpu().numpy())
        assert np.linalg.norm(bh - Ax) / np.linalg.norm(bh) <= 1.05e-10


def test_split_products_replay_from_a_graph(mats):
    A, _, _ = mats
    with spmv.Matrix.from_csr(A, params={"long_rows": 1}) as M1, spmv.Matrix.from_csr(A) as M:
        x = torch.zeros(A.n_cols, dtype=torch.float64, device=DEV)
        y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        y2 = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        ws = torch.empty(M.workspace_bytes // 8, dtype=torch.float64, device=DEV)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            M.apply_ws(x, y, ws=ws)
            M.apply(x, y2)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            M.apply_ws(x, y, ws=ws)
            M.apply(x, y2)
        for rep in range(3):
            xr = mg.uniform(A.n_cols, 14, rep)
            x.copy_(to_dev(xr))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            ref = M1.apply(to_dev(xr)).cpu().numpy()   # one workgroup per row, eagerly
            assert np.array_equal(y.cpu().numpy(), ref), rep
            assert np.array_equal(y2.cpu().numpy(), ref), rep


def test_server_products_and_solves_on_long_rows(mats, arrow):
    # the server runs such matrices with their own launch sequence, pieces
    # on a workgroup each: bitwise the handle's own product; CG solves to
    # the requested tolerance
    A = mats[0]
    X = mg.uniform(3 * A.n_cols, 15, 1).reshape(3, A.n_cols)
    b = mg.uniform(arrow.n_rows, 16, 4)
    with spmv.Server(n_slots=2) as srv:
        ia, ib = srv.add_matrix(A), srv.add_matrix(arrow)
        t1, t2 = srv.submit_spmv(ia, X), srv.submit_cg(ib, b, tol=1e-9)
        out, res = srv.wait(t1)
        assert res.done == 1 and res.status == 0, res.message
        xs, res2 = srv.wait(t2)
        assert res2.done == 1 and res2.status == 0, res2.message
    with spmv.Matrix.from_csr(A) as M:
        for j in range(3):
            assert np.array_equal(out[j], M.apply(to_dev(X[j])).cpu().numpy()), j
    Ax, _ = oracle.spmv(arrow, xs)
    assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 1.05e-9


def _run_layout(lead_long, run, n_long, L=20_000, n_cols=60_000, seed=76):
    """Rows: an optional long row, a run of `run` short rows, then n_long
    long rows (two pieces each) alternating with single short rows."""
    rl = ([L] if lead_long else []) + [4] * run
    for _ in range(n_long):
        rl += [L, 3]
    rl = np.array(rl, np.int64)
    rng = np.random.default_rng(seed)
    rp = np.concatenate([[0], np.cumsum(rl)]).astype(np.int32)
    return mg.CSR(len(rl), n_cols, rp, rng.integers(0, n_cols, int(rp[-1])).astype(np.int32),
                  rng.uniform(-1.0, 1.0, int(rp[-1])), 1)


def test_output_scratch_at_its_size_limits():
    # binary64: a run of exactly as many rows as pieces holds the sums; FP32
    # (4-byte rows) needs two rows per sum, and one more when the run starts
    # at an odd row (the sums are 8-byte aligned)
    # (binary64 fits exactly / one row short; FP32 fits exactly after the
    # 4-byte alignment shift / one row short)
    cases = [(False, 24, 12), (False, 23, 12), (True, 57, 13), (True, 56, 13)]
    for lead, run, n_long in cases:
        A = _run_layout(lead, run, n_long)
        pieces = 2 * (n_long + (1 if lead else 0))
        x = mg.uniform(A.n_cols, 18, 1)
        xd = to_dev(x)
        with spmv.Matrix.from_csr(A, fp32=True, params={"tile_nnz": 1024}) as M, \
                spmv.Matrix.from_csr(A, fp32=True, params={"tile_nnz": 1024, "long_rows": 1}) as M1:
            assert M.info["n_long_pieces"] == pieces
            assert M.info["y_scratch_ok"] == (1 if run >= pieces else 0)
            y, y1 = M.apply(xd).cpu().numpy(), M1.apply(xd).cpu().numpy()
            f, f1 = M.apply_f32(xd.float()).cpu().numpy(), M1.apply_f32(xd.float()).cpu().numpy()
        assert np.array_equal(y, y1), (lead, run)
        assert np.array_equal(f, f1), (lead, run)
        assert_parity(y, A, x)
