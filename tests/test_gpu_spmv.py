"""GPU parity of the SpMV paths against the CPU oracle, element by element.

Acceptance (binary64): |y_gpu - y_ref| <= 1e-12 * sum_k |a_ik||x_k| per row
(rows with a zero bound must be exactly zero; NaN/Inf compared by class).
Dyadic inputs make every partial sum exact, so there the GPU must equal the
oracle bit for bit.  Reduced-precision paths are held to first-order bounds
derived from their arithmetic:
  FP32 values, x, accumulation:  (m + 2) * 2^-24 * bound
  FP32 values, binary64 x/acc:   (2^-24 + m * 2^-53) * bound
  BF16 values, FP32 x/acc:       (2^-8 + (m + 1) * 2^-24) * bound
with m the row length and a 1% slack for the second-order terms.
"""
import ctypes

import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def run64(A, x, **kw):
    with spmv.Matrix.from_csr(A, **kw) as M:
        y = M.apply(to_dev(x))
        torch.cuda.synchronize()
        return y.cpu().numpy(), M.info


def assert_parity(y, A, x, rtol=oracle.SPMV_RTOL):
    y_ref, bound = oracle.spmv(A, x)
    ok = oracle.spmv_accept(y, y_ref, bound, rtol)
    if not ok.all():
        i = int(np.nonzero(~ok)[0][0])
        raise AssertionError(f"{(~ok).sum()} rows fail; first row {i}: gpu={y[i]!r} ref={y_ref[i]!r} "
                             f"bound={bound[i]!r}")


EDGE = {
    "empty_rows": dict(n_rows=5000, n_cols=5000, seed=1, mean_len=4.0, empty_frac=0.4),
    "dense_rows_long_path": dict(n_rows=3000, n_cols=20000, seed=2, mean_len=6.0, dense_rows=3),
    "duplicates_unsorted": dict(n_rows=4099, n_cols=777, seed=3, mean_len=9.0, duplicates=True,
                                unsorted=True),
    "rectangular_wide": dict(n_rows=1025, n_cols=70000, seed=4, mean_len=30.0),
    "rectangular_tall": dict(n_rows=70001, n_cols=33, seed=5, mean_len=3.0),
    "single_row": dict(n_rows=1, n_cols=10, seed=6, empty_frac=0.0),
    "all_empty": dict(n_rows=3000, n_cols=3000, seed=7, empty_frac=1.0),
}


@pytest.mark.parametrize("name", list(EDGE))
@pytest.mark.parametrize("tile", [1024, 4096])
def test_edge_cases_fp64(name, tile):
    A = mg.random_csr(**EDGE[name])
    x = mg.uniform(A.n_cols, 11, 0)
    y, info = run64(A, x, params={"tile_nnz": tile})
    assert_parity(y, A, x)
    if name == "dense_rows_long_path":
        assert info["n_long_rows"] == 3


def test_zero_nnz_and_zero_rows():
    A = mg.CSR(4, 3, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0))
    y, _ = run64(A, np.ones(3))
    assert np.all(y == 0.0)
    # without stored entries every product only zero-fills its output (a y
    # full of NaN comes back zero), with a real x and with no column at all
    for n_cols in (3, 0):
        Z = mg.CSR(4, n_cols, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0))
        with spmv.Matrix.from_csr(Z, fp32=True, bf16=True) as M:
            x64 = torch.ones(n_cols, dtype=torch.float64, device=DEV)
            x32 = torch.ones(n_cols, dtype=torch.float32, device=DEV)
            for fn, x, dt in ((M.apply, x64, torch.float64), (M.apply_f32, x32, torch.float32),
                              (M.apply_f32v, x64, torch.float64), (M.apply_bf16, x32, torch.float32)):
                y = torch.full((4,), float("nan"), dtype=dt, device=DEV)
                fn(x, y)
                assert bool(torch.all(y == 0))
            Y = torch.full((4, 3), float("nan"), dtype=torch.float64, device=DEV)
            M.spmm(torch.ones((n_cols, 3), dtype=torch.float64, device=DEV), Y)
            assert bool(torch.all(Y == 0))
    B = mg.CSR(2, 2, np.zeros(3, np.int32), np.zeros(0, np.int32), np.zeros((0, 3, 3)))
    with spmv.Matrix.from_bsr3(2, 2, B.row_ptr, B.col_idx, B.values) as M:
        Y = torch.full((6, 2), float("nan"), dtype=torch.float64, device=DEV)
        M.spmm(torch.ones((6, 2), dtype=torch.float64, device=DEV), Y)
        assert bool(torch.all(Y == 0))
    A = mg.CSR(0, 3, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    with spmv.Matrix.from_csr(A) as M:
        y = M.apply(to_dev(np.ones(3)))
        assert y.numel() == 0


def test_long_row_of_100k_entries():
    n = 300
    rows = [np.arange(3) for _ in range(n)]
    rows[17] = np.arange(100_000)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    A = mg.CSR(n, 100_000, rp, np.concatenate(rows).astype(np.int32),
               mg.uniform(int(rp[-1]), 5, 2))
    x = mg.uniform(A.n_cols, 6, 0)
    y, info = run64(A, x)
    assert info["n_long_rows"] == 1
    assert_parity(y, A, x)


def test_nan_inf_propagate_like_the_oracle():
    A = mg.random_csr(500, 500, seed=8, mean_len=5.0, empty_frac=0.0)
    x = mg.uniform(A.n_cols, 9, 0)
    x[[3, 77]] = np.nan
    x[[10]] = np.inf
    y, _ = run64(A, x)
    assert_parity(y, A, x)


@pytest.mark.parametrize("mode", [spmv.WINDOW_OFF, spmv.WINDOW_RING, spmv.WINDOW_AUTO])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
@pytest.mark.parametrize("kernel,remap", [(1, True), (1, False), (2, True), (3, True)])
def test_mesh_config0_paths(mode, tile, kernel, remap):
    A = mg.config0()
    x = mg.uniform(A.n_cols, 12, 0)
    y, info = run64(A, x, xcd_remap=remap,
                    params={"tile_nnz": 1024 if kernel == 3 else tile, "window_mode": mode, "window_block": 8,
                            "ring_words": 8192, "kernel": kernel})
    if mode != spmv.WINDOW_OFF:
        assert info["n_window_tiles"] > 0
    assert_parity(y, A, x)


@pytest.mark.parametrize("mode", [spmv.WINDOW_OFF, spmv.WINDOW_RING, spmv.WINDOW_AUTO])
def test_dyadic_bitwise(mode):
    for A in (mg.config0(dyadic=True), mg.config1("rcm", m=40, dyadic=True),
              mg.lattice(30, 30, 30, "stencil27", seed=5, dyadic=True)):
        x = mg.dyadic_x(A.n_cols, seed=4)
        y, _ = run64(A, x, params={"window_mode": mode, "window_block": 4, "ring_words": 8192,
                                   "tile_nnz": 1024})
        y_ref, _ = oracle.spmv(A, x)
        assert np.array_equal(y, y_ref)


def test_ring_window_sizes_and_restarts():
    # 7-point lattice: band nx*ny = 1024, so a tile of ~150 rows spans ~2200
    # columns: rings of 1024/2048 words cannot hold a tile (direct path), 4096
    # and 8192 can.
    A = mg.lattice(32, 32, 40, "faces", seed=9)
    x = mg.uniform(A.n_cols, 13, 0)
    for ring in (1024, 2048, 4096, 8192):
        y, info = run64(A, x, params={"window_mode": spmv.WINDOW_RING, "ring_words": ring,
                                      "window_block": 32, "tile_nnz": 1024})
        assert (info["n_window_tiles"] > 0) == (ring >= 4096)
        assert_parity(y, A, x)
    # reversing 2048-row chunks makes consecutive tiles jump across the matrix,
    # forcing ring restarts inside a block
    n = A.n_rows
    perm = np.concatenate([np.arange(min(n, s + 2048) - 1, s - 1, -1) for s in range(0, n, 2048)])
    B = mg.permute(A, perm.astype(np.int32))
    P = spmv.plan_inspect(B.n_rows, B.n_cols, B.row_ptr, B.col_idx,
                          {"window_mode": spmv.WINDOW_RING, "ring_words": 8192, "window_block": 32,
                           "tile_nnz": 1024})
    win = P["seg_kind"] == 2
    spans = np.array([B.col_idx[B.row_ptr[a]:B.row_ptr[b]].max() - B.col_idx[B.row_ptr[a]:B.row_ptr[b]].min() + 1
                      for a, b in zip(P["seg_bound"][:-1], P["seg_bound"][1:])])
    restarts = np.sum(win & (P["win_cnt"] == spans))
    blocks = len(np.unique(P["win_block"][win]))
    assert restarts > blocks          # more full reloads than one per block
    xb = x[perm]
    y, info = run64(B, xb, params={"window_mode": spmv.WINDOW_RING, "ring_words": 8192,
                                   "window_block": 32, "tile_nnz": 1024})
    assert info["n_window_tiles"] > 0
    assert_parity(y, B, xb)


def test_reproducible_and_independent_of_concurrent_work():
    A = mg.config0()
    B = mg.config1("random", m=48)
    x = to_dev(mg.uniform(A.n_cols, 14, 0))
    xb = to_dev(mg.uniform(B.n_cols, 15, 0))
    with spmv.Matrix.from_csr(A) as M, spmv.Matrix.from_csr(B) as N:
        y1 = M.apply(x)
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        outs = []
        for _ in range(5):
            with torch.cuda.stream(s1):
                ya = M.apply(x, stream=s1)
            with torch.cuda.stream(s2):
                N.apply(xb, stream=s2)
            outs.append(ya)
        torch.cuda.synchronize()
        for ya in outs:
            assert torch.equal(ya, y1)


@pytest.fixture(scope="module")
def cfg1():
    return {o: mg.config1(o) for o in ("rcm", "random")}


@pytest.mark.parametrize("ordering", ["rcm", "random"])
@pytest.mark.parametrize("kernel", [1, 2, 3])
def test_config1_full_size_and_permutation_equivariance(cfg1, ordering, kernel):
    A = cfg1[ordering]
    assert A.n_rows == 126 ** 3
    x = mg.uniform(A.n_cols, 16, 0)
    y, _ = run64(A, x, params={"kernel": kernel})
    assert_parity(y, A, x)


@pytest.mark.parametrize("gap", [0, 16, 64])
def test_compact_windows_equal_direct_bitwise(cfg1, gap):
    # staging x in LDS changes where x comes from, not the per-row sums
    A = cfg1["rcm"]
    x = mg.uniform(A.n_cols, 21, 0)
    y_dir, _ = run64(A, x, params={"window_mode": spmv.WINDOW_OFF, "tile_nnz": 2048})
    y_win, info = run64(A, x, params={"window_mode": spmv.WINDOW_AUTO, "window_gap": gap, "tile_nnz": 2048})
    assert info["n_window_tiles"] > 0
    assert np.array_equal(y_dir, y_win)
    y_pipe, _ = run64(A, x, params={"window_mode": spmv.WINDOW_AUTO, "window_gap": gap, "tile_nnz": 2048,
                                    "kernel": 2})
    assert np.array_equal(y_dir, y_pipe)
    assert_parity(y_win, A, x)


def test_compact_windows_nonfinite_empty_and_long_rows():
    # 2048-entry compact tiles (packed positions) next to direct tiles inside
    # the window launch, empty rows, rows longer than a tile, NaN/Inf in x
    A = mg.config1("rcm", m=48)
    n = A.n_rows
    lens = np.diff(A.row_ptr).copy()
    rows = [A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]] for i in range(n)]
    vals = [A.values[A.row_ptr[i]:A.row_ptr[i + 1]] for i in range(n)]
    rng = np.random.default_rng(5)
    for i in rng.choice(n, 300, replace=False):
        rows[i], vals[i] = rows[i][:0], vals[i][:0]          # empty rows
    for i in (17, n // 2):
        rows[i] = np.arange(0, n, 7, dtype=np.int32)[:5000]  # long rows
        vals[i] = rng.uniform(-1, 1, rows[i].size)
    rp = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int32)
    B = mg.CSR(n, n, rp, np.concatenate(rows).astype(np.int32), np.concatenate(vals))
    x = mg.uniform(n, 23, 0)
    x[[5, 999]] = np.nan
    x[[77]] = np.inf
    y_win, info = run64(B, x, params={"tile_nnz": 2048})
    assert info["n_window_tiles"] > 0 and info["n_long_rows"] == 2
    assert_parity(y_win, B, x)
    y_dir, _ = run64(B, x, params={"tile_nnz": 2048, "window_mode": spmv.WINDOW_OFF})
    assert np.array_equal(np.isnan(y_win), np.isnan(y_dir))
    fin = ~np.isnan(y_dir)
    assert np.array_equal(y_win[fin], y_dir[fin])


def test_kernel_variants_bitwise_identical(cfg1):
    # the variants differ only in scheduling: every row's sum has the same order
    A = cfg1["rcm"]
    x = mg.uniform(A.n_cols, 19, 0)
    ys = [run64(A, x, params={"kernel": k, "tile_nnz": 1024 if k == 3 else 2048})[0] for k in (1, 2, 3)]
    assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2])


@pytest.mark.parametrize("window", [spmv.WINDOW_OFF, spmv.WINDOW_AUTO])
def test_xcd_assignments_bitwise_identical(cfg1, window):
    # which workgroup takes which tile changes nothing in any row's sum:
    # chunks of 1, 16 (the default) and 4096 tiles, one contiguous range per
    # XCD and no grouping all give the same bits, FP64 and FP32, and SELL too
    A = cfg1["rcm"]
    x = mg.uniform(A.n_cols, 31, 0)
    ys = []
    for c in (0, 1, 16, 4096, -2, -1):
        params = {"tile_nnz": 2048, "window_mode": window, "xcd_chunk": c}
        with spmv.Matrix.from_csr(A, fp32=True, params=params) as M:
            ys.append((M.apply(to_dev(x)).cpu().numpy(), M.apply_f32(to_dev(x, torch.float32)).cpu().numpy()))
    for y64, y32 in ys[1:]:
        assert np.array_equal(y64, ys[0][0]) and np.array_equal(y32, ys[0][1])
    assert_parity(ys[0][0], A, x)
    sel = [run64(A, x, params={"format": spmv.FORMAT_SELL, "xcd_chunk": c})[0] for c in (0, -2, 2)]
    assert np.array_equal(sel[0], sel[1]) and np.array_equal(sel[0], sel[2]) and np.array_equal(sel[0], ys[0][0])


def test_config1_orderings_agree(cfg1):
    # the same operator in two orderings: both are the RCM / random
    # renumbering of one natural-order matrix, so y must agree after mapping
    nat = mg.knn(126, seed=mg.seed_for(1))
    p_rcm = mg.rcm_perm(nat)
    x = mg.uniform(nat.n_cols, 17, 0)
    y_rcm, _ = run64(cfg1["rcm"], x[p_rcm])
    y_nat, _ = oracle.spmv(nat, x)
    _, bound = oracle.spmv(nat, x)
    assert np.all(np.abs(y_rcm - y_nat[p_rcm]) <= 1e-12 * bound[p_rcm])


def _bounds(A, x):
    y_ref, bound = oracle.spmv(A, x)
    m = np.diff(A.row_ptr).astype(np.float64)
    return y_ref, bound, m


def test_fp32_paths_within_derived_bounds():
    A = mg.config0()
    x = mg.uniform(A.n_cols, 18, 0)
    y_ref, bound, m = _bounds(A, x)
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True) as M:
        y32 = M.apply_f32(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
        yv = M.apply_f32v(to_dev(x)).cpu().numpy()
        y16 = M.apply_bf16(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    u32, u16 = 2.0 ** -24, 2.0 ** -8
    assert np.all(np.abs(y32 - y_ref) <= 1.01 * (m + 2) * u32 * bound)
    assert np.all(np.abs(yv - y_ref) <= 1.01 * (u32 + m * 2.0 ** -53) * bound)
    assert np.all(np.abs(y16 - y_ref) <= 1.01 * (u16 + (m + 1) * u32) * bound)
    # the reduced-precision results are not just the binary64 result rounded
    assert np.max(np.abs(y32 - y_ref) / np.maximum(bound, 1e-300)) > 1e-9


def test_reduced_precision_on_a_compact_window_handle(cfg1):
    # on a handle planned with compact windows, FP32 values (with FP32 or
    # FP64 x) and BF16 values go through the windows too; every precision
    # equals the direct-gather handle bit for bit
    A = cfg1["rcm"]
    x = mg.uniform(A.n_cols, 22, 0)
    y_ref, bound, m = _bounds(A, x)
    with spmv.Matrix.from_csr(A) as M:
        assert M.info["n_window_tiles"] == 0          # 165 MB matrix: served from cache, no windows
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True, params={"tile_nnz": 2048, "window_mode": 0}) as M:
        assert M.info["n_window_tiles"] > 0
        y64 = M.apply(to_dev(x)).cpu().numpy()
        y32 = M.apply_f32(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
        yv = M.apply_f32v(to_dev(x)).cpu().numpy()
        y16 = M.apply_bf16(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True, params={"tile_nnz": 2048, "window_mode": spmv.WINDOW_OFF}) as D:
        assert D.info["n_window_tiles"] == 0
        assert np.array_equal(D.apply(to_dev(x)).cpu().numpy(), y64)
        assert np.array_equal(D.apply_f32(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64), y32)
        assert np.array_equal(D.apply_f32v(to_dev(x)).cpu().numpy(), yv)
        assert np.array_equal(D.apply_bf16(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64), y16)
    u32, u16 = 2.0 ** -24, 2.0 ** -8
    assert oracle.spmv_accept(y64, y_ref, bound).all()
    assert np.all(np.abs(y32 - y_ref) <= 1.01 * (m + 2) * u32 * bound)
    assert np.all(np.abs(yv - y_ref) <= 1.01 * (u32 + m * 2.0 ** -53) * bound)
    assert np.all(np.abs(y16 - y_ref) <= 1.01 * (u16 + (m + 1) * u32) * bound)


def test_fp32_dyadic_bitwise():
    A = mg.config0(dyadic=True)
    x = mg.dyadic_x32(A.n_cols, seed=3)
    y_ref, _ = oracle.spmv(A, x)
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        y32 = M.apply_f32(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.array_equal(y32, y_ref)


def _bf16_bits(a):
    """bfloat16 rounding of float32(a) by the bit recipe (add 0x7fff plus the
    lowest kept bit, truncate): nearest, ties to even."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("window", [spmv.WINDOW_OFF, spmv.WINDOW_AUTO])
def test_bf16_dyadic_bitwise(window):
    # Values m/1024 (11 significant bits) are not bfloat16 numbers; their
    # bfloat16 roundings have 8 bits and x = k/64 (|k| <= 64) has 7, so every
    # product is a multiple of 2^-14 and every partial sum of a row stays
    # below 2^6: exact in FP32 in any order.  The bfloat16 product must
    # therefore equal the oracle run on the rounded values bit for bit, and
    # a path that read the FP32 or binary64 values would give the oracle's
    # result on the unrounded ones, which differs on most rows.
    A = mg.config0(dyadic=True)
    x = mg.dyadic_x32(A.n_cols, seed=5)
    At = mg.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, _bf16_bits(A.values))
    assert np.count_nonzero(At.values != A.values) > A.nnz // 2
    y16_ref, _ = oracle.spmv(At, x)
    y_unrounded, _ = oracle.spmv(A, x)
    params = {"tile_nnz": 2048, "window_mode": window}
    with spmv.Matrix.from_csr(A, bf16=True, params=params) as M:
        assert (M.info["n_window_tiles"] > 0) == (window == spmv.WINDOW_AUTO)
        y16 = M.apply_bf16(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.array_equal(y16, y16_ref)
    assert np.count_nonzero(y16 != y_unrounded) > A.n_rows // 2


def test_bf16_rounding_is_visible():
    # on non-dyadic values the bfloat16 product's error against the binary64
    # oracle is of the order of 2^-9 of the row scale; an FP32-value product
    # stays below (m + 2) 2^-24, four orders smaller
    A = mg.config0()
    x = mg.uniform(A.n_cols, 19, 0)
    y_ref, bound, m = _bounds(A, x)
    with spmv.Matrix.from_csr(A, bf16=True) as M:
        y16 = M.apply_bf16(to_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    ratio = np.abs(y16 - y_ref) / np.maximum(bound, 1e-300)
    assert np.all(ratio <= 1.01 * (2.0 ** -8 + (m + 1) * 2.0 ** -24))
    assert np.max(ratio) > 2.0 ** -12
    assert np.max(ratio) > 100 * np.max((m + 2) * 2.0 ** -24)


def test_missing_copies_and_bad_arguments():
    A = mg.config0()
    with spmv.Matrix.from_csr(A) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.apply_f32(torch.zeros(A.n_cols, dtype=torch.float32, device=DEV))
        assert e.value.code == spmv.SPMV_ENOTSUP
        buf = torch.zeros(A.n_rows + A.n_cols, dtype=torch.float64, device=DEV)
        with pytest.raises(spmv.SpmvError) as e:
            M.apply(buf[:A.n_cols], buf[A.n_cols - 5:A.n_cols - 5 + A.n_rows])
        assert e.value.code == spmv.SPMV_EINVAL
        with pytest.raises(TypeError):
            M.apply(torch.zeros(A.n_cols, dtype=torch.float32, device=DEV))
        with pytest.raises(ValueError):
            M.apply(torch.zeros(A.n_cols + 1, dtype=torch.float64, device=DEV))


# ------------------------------------------------------------ 3x3 block CSR

def _bsr_bound_check(Y, A, X, rel):
    Yr, Bd = oracle.bsr3_spmm(A, X)
    assert np.all(np.abs(Y - Yr) <= rel * Bd), float(np.max(np.abs(Y - Yr) / np.maximum(Bd, 1e-300)))
    return Yr


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 13])
def test_bsr3_multi_rhs_fp64(k):
    A = mg.bsr3(23, 17, 11, seed=5)
    X = mg.uniform(3 * A.n_cols * k, 20 + k, 0).reshape(3 * A.n_cols, k)
    with spmv.Matrix.from_csr(A) as M:
        Y = M.spmm(to_dev(X)).cpu().numpy()
        if k == 1:
            y1 = M.apply(to_dev(X[:, 0])).cpu().numpy()
            assert np.array_equal(y1, Y[:, 0])
        # each column equals the one-column product of that column
        for j in (0, k - 1):
            yj = M.spmm(to_dev(X[:, j:j + 1].copy())).cpu().numpy()
            assert np.array_equal(yj[:, 0], Y[:, j])
    _bsr_bound_check(Y, A, X, 1e-12)


def test_bsr3_fp32_storage_and_long_block_rows():
    A = mg.bsr3(20, 20, 10, seed=6)
    X = mg.uniform(3 * A.n_cols * 4, 30, 0).reshape(3 * A.n_cols, 4)
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        Y = M.spmm_f32(to_dev(X, torch.float32)).cpu().numpy().astype(np.float64)
    m = 3 * np.repeat(np.diff(A.row_ptr), 3)[:, None].astype(np.float64)
    _bsr_bound_check(Y, A, X, 1.01 * (m + 2) * 2.0 ** -24)
    # a block row with 700 blocks (more than one tile can stage)
    nbr, nbc = 40, 800
    lens = np.full(nbr, 3)
    lens[7] = 700
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    rng = np.random.default_rng(1)
    ci = np.concatenate([np.sort(rng.choice(nbc, size=L, replace=False)) for L in lens]).astype(np.int32)
    va = rng.uniform(-1, 1, (ci.shape[0], 3, 3))
    B = mg.CSR(nbr, nbc, rp, ci, va, 3)
    Xb = mg.uniform(3 * nbc * 8, 31, 0).reshape(3 * nbc, 8)
    with spmv.Matrix.from_csr(B) as M:
        Yb = M.spmm(to_dev(Xb)).cpu().numpy()
    _bsr_bound_check(Yb, B, Xb, 1e-12)


@pytest.mark.parametrize("k", [1, 2, 4, 8, 11])
def test_bsr3_empty_rows_and_nonfinite_x(k):
    # 300 block rows: a run of 120 empty rows (a whole tile without blocks),
    # odd row lengths 0..13 so tiles start at odd block offsets, and one
    # column of X holding NaN and another holding Inf
    nbr, nbc = 300, 260
    rng = np.random.default_rng(11)
    lens = rng.integers(0, 14, nbr)
    lens[100:220] = 0
    lens[0] = 1
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(nbc, size=L, replace=False)) for L in lens]).astype(np.int32)
    va = rng.uniform(-1, 1, (ci.shape[0], 3, 3))
    B = mg.CSR(nbr, nbc, rp, ci, va, 3)
    X = mg.uniform(3 * nbc * k, 40 + k, 0).reshape(3 * nbc, k)
    X[3 * int(ci[0]) + 1, 0] = np.nan
    X[3 * int(ci[-1]) + 2, k - 1] = np.inf
    with spmv.Matrix.from_csr(B, fp32=True) as M:
        assert M.info["n_tiles"] >= 3
        Y = M.spmm(to_dev(X)).cpu().numpy()
        Y32 = M.spmm_f32(to_dev(X, torch.float32)).cpu().numpy().astype(np.float64)
    Yr, Bd = oracle.bsr3_spmm(B, X)
    assert np.isnan(Yr).any() and np.isinf(Yr).any()
    assert oracle.spmv_accept(Y, Yr, Bd).all()
    assert np.all(Y[3 * 100:3 * 220] == 0)
    rt = np.broadcast_to(1.01 * (3 * np.repeat(lens, 3)[:, None] + 2) * 2.0 ** -24, Yr.shape)
    fin = np.isfinite(Yr)
    assert np.all(np.abs(Y32 - Yr)[fin] <= (rt * Bd)[fin])
    assert np.array_equal(np.isnan(Y32), np.isnan(Yr))
    assert np.array_equal(Y32[np.isinf(Yr)], Yr[np.isinf(Yr)])


@pytest.mark.parametrize("fp32", [False, True])
def test_bsr3_one_column_rows_of_every_length(fp32):
    # block rows of 0..40 blocks (the one-column kernel gathers a row's first
    # 12 blocks with the value stream, the rest in rounds afterwards), a
    # 700-block row (values read from global memory), tiles starting at odd
    # block offsets: the one-column product equals column 0 of the
    # two-column product bit for bit, and the oracle within its bound
    nbr, nbc = 500, 900
    rng = np.random.default_rng(21)
    lens = rng.integers(0, 41, nbr)
    lens[250] = 700
    lens[300:330] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(nbc, size=L, replace=False)) for L in lens]).astype(np.int32)
    va = rng.uniform(-1, 1, (ci.shape[0], 3, 3))
    B = mg.CSR(nbr, nbc, rp, ci, va, 3)
    X = mg.uniform(3 * nbc * 2, 50, 0).reshape(3 * nbc, 2)
    dt = torch.float32 if fp32 else torch.float64
    with spmv.Matrix.from_csr(B, fp32=fp32) as M:
        assert M.info["n_tiles"] >= 8
        mm = M.spmm_f32 if fp32 else M.spmm
        Y2 = mm(to_dev(X, dt)).cpu().numpy()
        Y1 = mm(to_dev(X[:, :1].copy(), dt)).cpu().numpy()
    assert np.array_equal(Y1[:, 0], Y2[:, 0])
    assert np.all(Y1[3 * 300:3 * 330] == 0)
    if fp32:
        Yr, Bd = oracle.bsr3_spmm(B, X[:, :1].astype(np.float32).astype(np.float64))
        m = 3 * np.repeat(lens, 3)[:, None].astype(np.float64)
        assert np.all(np.abs(Y1 - Yr) <= 1.01 * (m + 2) * 2.0 ** -24 * Bd)
    else:
        _bsr_bound_check(Y1, B, X[:, :1].copy(), 1e-12)


def test_bsr3_config3_shape_bitwise_dyadic():
    A = mg.bsr3(40, 40, 20, seed=7)
    # dyadic copy of the values: multiples of 2^-10 in [-2, 2]
    A.values = np.round(A.values * 1024) / 1024
    X = (np.floor(mg.uniform(3 * A.n_cols * 8, 32, 0, 0.0, 1.0) * 2049) - 1024).reshape(3 * A.n_cols, 8) / 1024
    with spmv.Matrix.from_csr(A) as M:
        Y = M.spmm(to_dev(X)).cpu().numpy()
    Yr, _ = oracle.bsr3_spmm(A, X)
    assert np.array_equal(Y, Yr)


@pytest.mark.parametrize("k", [1, 8])
def test_bsr3_xcd_assignments_bitwise_identical(k):
    A = mg.bsr3(40, 30, 20, seed=64)
    X = mg.uniform(3 * A.n_cols * k, 12, 0).reshape(3 * A.n_cols, k)
    outs = []
    for kw in ({}, {"xcd_contiguous": True}, {"xcd_remap": False}):
        with spmv.Matrix.from_csr(A, **kw) as M:
            outs.append(M.spmm(to_dev(X)).cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    Yr, Bd = oracle.bsr3_spmm(A, X)
    assert np.all(np.abs(outs[0] - Yr) <= 1e-12 * Bd)


def test_bsr3_rejects_misuse():
    A = mg.bsr3(5, 5, 5, seed=8)
    with spmv.Matrix.from_csr(A) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.ones(3 * A.n_rows, dtype=torch.float64, device=DEV))
        assert e.value.code == spmv.SPMV_ENOTSUP
    C = mg.config0()
    X = torch.ones((C.n_cols, 1), dtype=torch.float64, device=DEV)
    Y = torch.empty((C.n_rows, 1), dtype=torch.float64, device=DEV)
    with spmv.Matrix.from_csr(C) as M:   # the block product on a scalar handle
        assert spmv.lib().bsr3_spmm(M.handle, 1, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                    None) == spmv.SPMV_ENOTSUP


SPMM_PLANS = {
    "auto": {},
    "direct1024": {"window_mode": spmv.WINDOW_OFF, "tile_nnz": 1024},
    "ring1024": {"window_mode": spmv.WINDOW_RING, "tile_nnz": 1024},
    "tiles4096": {"tile_nnz": 4096},
}


@pytest.mark.parametrize("k", [1, 3, 8, 13])
@pytest.mark.parametrize("plan", list(SPMM_PLANS))
def test_spmm_columns_equal_spmv_bitwise(plan, k):
    # irregular CSR with empty rows, rows longer than any tile, duplicates,
    # unsorted columns and NaN/Inf in X: every column of the k-column product
    # equals the single-vector product bit for bit and meets the oracle bound
    A = mg.random_csr(3000, 2500, seed=61, mean_len=9.0, empty_frac=0.1, dense_rows=3, duplicates=True,
                      unsorted=True)
    X = mg.uniform(A.n_cols * k, 62 + k, 0).reshape(A.n_cols, k)
    X[5, 0] = np.nan
    X[77, k - 1] = np.inf
    with spmv.Matrix.from_csr(A, params=SPMM_PLANS[plan]) as M:
        Xd = torch.as_tensor(X, device=DEV)
        Y = M.spmm(Xd).cpu().numpy()
        for j in range(k):
            y = M.apply(torch.as_tensor(np.ascontiguousarray(X[:, j]), device=DEV)).cpu().numpy()
            assert np.array_equal(Y[:, j], y, equal_nan=True), (plan, k, j)
            y_ref, bound = oracle.spmv(A, X[:, j])
            assert oracle.spmv_accept(Y[:, j], y_ref, bound).all()


def test_spmm_mesh_compact_windows_and_ring():
    A = mg.config0()
    k = 8
    X = mg.uniform(A.n_cols * k, 63, 0).reshape(A.n_cols, k)
    for params in ({"tile_nnz": 2048}, {"window_mode": spmv.WINDOW_RING, "tile_nnz": 1024}):
        with spmv.Matrix.from_csr(A, params=params) as M:
            assert M.info["n_window_tiles"] > 0
            Y = M.spmm(torch.as_tensor(X, device=DEV)).cpu().numpy()
            for j in range(k):
                y = M.apply(torch.as_tensor(np.ascontiguousarray(X[:, j]), device=DEV)).cpu().numpy()
                assert np.array_equal(Y[:, j], y)
    Ad = mg.config0(dyadic=True)
    Xd = np.stack([mg.dyadic_x(Ad.n_cols, seed=70 + j) for j in range(4)], axis=1)
    with spmv.Matrix.from_csr(Ad) as M:
        Y = M.spmm(torch.as_tensor(Xd, device=DEV)).cpu().numpy()
    for j in range(4):
        assert np.array_equal(Y[:, j], oracle.spmv(Ad, Xd[:, j])[0])


def test_spmm_rejects_misuse():
    A = mg.config0()
    L = spmv.lib()
    X = torch.ones((A.n_cols, 2), dtype=torch.float64, device=DEV)
    Y = torch.empty((A.n_rows, 2), dtype=torch.float64, device=DEV)
    with spmv.Matrix.from_csr(A) as M:
        assert L.spmv_spmm(M.handle, 0, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), None) == \
            spmv.SPMV_EINVAL
        assert L.spmv_spmm(M.handle, 2, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()), None) == \
            spmv.SPMV_EINVAL
    with spmv.Matrix.from_csr(A, params={"format": spmv.FORMAT_SELL}) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.spmm(X)
        assert e.value.code == spmv.SPMV_ENOTSUP
    B = mg.config3(nx=6, ny=5, nz=4)
    with spmv.Matrix.from_csr(B) as M:
        assert L.spmv_spmm(M.handle, 2, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), None) == \
            spmv.SPMV_ENOTSUP


def test_create_from_device_arrays():
    # a handle made from device arrays (SPMV_DEVICE_PTRS) is the handle made
    # from the same host arrays: bitwise equal products and the same plan
    A = mg.random_csr(4000, 3500, seed=81, mean_len=8.0, empty_frac=0.1, dense_rows=2, duplicates=True,
                      unsorted=True)
    x = torch.as_tensor(mg.uniform(A.n_cols, 82, 0), device=DEV)
    rp = torch.as_tensor(A.row_ptr, device=DEV)
    ci = torch.as_tensor(A.col_idx, device=DEV)
    va = torch.as_tensor(A.values, device=DEV)
    with spmv.Matrix.from_csr(A, fp32=True) as H, \
            spmv.Matrix.from_device_csr(A.n_rows, A.n_cols, rp, ci, va, fp32=True) as D:
        assert np.array_equal(H.apply(x).cpu().numpy(), D.apply(x).cpu().numpy())
        assert np.array_equal(H.apply_f32(x.float()).cpu().numpy(), D.apply_f32(x.float()).cpu().numpy())
        assert {k: v for k, v in H.info.items() if k != "device_bytes"} == \
            {k: v for k, v in D.info.items() if k != "device_bytes"}
    B = mg.config3(nx=6, ny=5, nz=4)
    Xb = torch.as_tensor(mg.uniform(B.n_cols * 3 * 2, 83, 0), device=DEV).view(3 * B.n_cols, 2)
    L = spmv.lib()
    h = ctypes.c_void_p()
    brp, bci = torch.as_tensor(B.row_ptr, device=DEV), torch.as_tensor(B.col_idx, device=DEV)
    bva = torch.as_tensor(np.ascontiguousarray(B.values).reshape(-1), device=DEV)
    assert L.spmv_create_bsr3(B.n_rows, B.n_cols, B.nnz, ctypes.c_void_p(brp.data_ptr()),
                              ctypes.c_void_p(bci.data_ptr()), ctypes.c_void_p(bva.data_ptr()),
                              spmv.SPMV_DEVICE_PTRS, ctypes.byref(h)) == spmv.SPMV_OK
    try:
        Yd = torch.empty((3 * B.n_rows, 2), dtype=torch.float64, device=DEV)
        assert L.bsr3_spmm(h, 2, ctypes.c_void_p(Xb.data_ptr()), ctypes.c_void_p(Yd.data_ptr()), None) == 0
        with spmv.Matrix.from_csr(B) as M:
            assert np.array_equal(M.spmm(Xb).cpu().numpy(), Yd.cpu().numpy())
    finally:
        L.spmv_destroy(h)


def test_create_from_device_arrays_rejects_host_pointers():
    A = mg.config0()
    L = spmv.lib()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(A.row_ptr)
    ci = torch.as_tensor(A.col_idx, device=DEV)
    va = torch.as_tensor(A.values, device=DEV)
    rc = L.spmv_create(A.n_rows, A.n_cols, A.nnz, rp.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ci.data_ptr()),
                       ctypes.c_void_p(va.data_ptr()), spmv.SPMV_DEVICE_PTRS, None, ctypes.byref(h))
    assert rc == spmv.SPMV_EINVAL and not h.value
    assert b"not device memory" in L.spmv_last_error()
    # the device arrays are validated like host ones
    bad = torch.as_tensor(A.col_idx, device=DEV).clone()
    bad[7] = A.n_cols
    rc = L.spmv_create(A.n_rows, A.n_cols, A.nnz, ctypes.c_void_p(torch.as_tensor(A.row_ptr, device=DEV).data_ptr()),
                       ctypes.c_void_p(bad.data_ptr()), ctypes.c_void_p(va.data_ptr()), spmv.SPMV_DEVICE_PTRS, None,
                       ctypes.byref(h))
    assert rc == spmv.SPMV_EINVAL


def test_read_calibration_sums_and_rejects_misuse():
    buf = torch.as_tensor(mg.uniform(1 << 20, 91, 0), device=DEV)
    part = torch.empty(64, dtype=torch.float64, device=DEV)
    spmv.calibrate_read(buf, part)
    assert abs(part.sum().item() - buf.sum().item()) <= 1e-9 * buf.abs().sum().item()
    L = spmv.lib()
    odd = torch.ones(5, dtype=torch.float64, device=DEV)
    assert L.spmv_calibrate_read(ctypes.c_void_p(odd.data_ptr()), 5, ctypes.c_void_p(part.data_ptr()), 64,
                                 None) == spmv.SPMV_EINVAL
    assert L.spmv_calibrate_read(ctypes.c_void_p(buf.data_ptr() + 8), 2, ctypes.c_void_p(part.data_ptr()), 64,
                                 None) == spmv.SPMV_EINVAL
    assert L.spmv_calibrate_read(ctypes.c_void_p(buf.data_ptr()), 2, ctypes.c_void_p(part.data_ptr()), 0,
                                 None) == spmv.SPMV_EINVAL


@pytest.mark.parametrize("name", ["C50K", "C800K"])
def test_table1_sized_tet_stand_ins(name):
    # the paper's matrix sizes (Table 1), tet-like stand-ins: every row against
    # the oracle on the default plan and on the ring window (the paper's cache)
    A = mg.table1_matrix(name)
    x = mg.uniform(A.n_cols, 93, 0)
    for params in ({}, {"window_mode": spmv.WINDOW_RING, "tile_nnz": 1024, "ring_words": 8192,
                        "window_block": 8}):
        y, info = run64(A, x, params=params)
        assert_parity(y, A, x)


@pytest.mark.parametrize("params", [{}, {"tile_nnz": 2048}, {"window_mode": spmv.WINDOW_RING, "tile_nnz": 1024}])
def test_apply_and_spmm_replay_from_a_hip_graph(params):
    # the apply calls only enqueue kernels, so a caller may record them into a
    # HIP graph: three chained products y1 = A x, y2 = A y1, y3 = A y2 and one
    # three-column product, captured once, replayed with a new x each time
    # (eager copies and synchronisations between replays), every replay equal
    # bit for bit to the same calls made eagerly
    A = mg.config0()
    k = 3
    with spmv.Matrix.from_csr(A, params=params) as M:
        if params:
            assert M.info["n_window_tiles"] > 0
        x = torch.zeros(A.n_cols, dtype=torch.float64, device=DEV)
        X = torch.zeros((A.n_cols, k), dtype=torch.float64, device=DEV)
        ys = [torch.empty(A.n_rows, dtype=torch.float64, device=DEV) for _ in range(3)]
        Y = torch.empty((A.n_rows, k), dtype=torch.float64, device=DEV)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            M.apply(x, ys[0])
            M.spmm(X, Y)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            M.apply(x, ys[0])
            M.apply(ys[0], ys[1])
            M.apply(ys[1], ys[2])
            M.spmm(X, Y)
        for rep in range(4):
            xr = mg.uniform(A.n_cols, 94, rep)
            Xr = mg.uniform(A.n_cols * k, 95, rep).reshape(A.n_cols, k)
            x.copy_(to_dev(xr))
            X.copy_(to_dev(Xr))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = [y.cpu().numpy() for y in ys]
            got_Y = Y.cpu().numpy()
            e = [M.apply(to_dev(xr))]
            e.append(M.apply(e[0]))
            e.append(M.apply(e[1]))
            eY = M.spmm(to_dev(Xr), torch.empty_like(Y))
            torch.cuda.synchronize()
            for a, b in zip(got, e):
                assert np.array_equal(a, b.cpu().numpy()), f"replay {rep}"
            assert np.array_equal(got_Y, eY.cpu().numpy()), f"replay {rep}"
            assert_parity(got[0], A, xr)
        del g
