"""Host-side tests of the C-ABI library: it loads, exports every declared
symbol, validates its inputs, and builds a correct analysis plan.  None of
these touch a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import meshgen as mg
import paper_2107_12371_amd as spmv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\([^;{]*\)\s*;", text, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "spmv_create" in names and "cg_solve" in names and "spmv_apply" in names
    L = ctypes.CDLL(spmv.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(spmv.EXPORTED) <= set(names)


def _bad(n_rows, n_cols, rp, ci, params=None):
    with pytest.raises(spmv.SpmvError) as e:
        spmv.plan_inspect(n_rows, n_cols, rp, ci, params)
    return e.value


def test_validation_errors():
    assert _bad(2, 2, [1, 1, 2], [0, 1]).code == spmv.SPMV_EINVAL           # row_ptr[0] != 0
    assert _bad(2, 2, [0, 2, 1], [0, 1]).code == spmv.SPMV_EINVAL           # decreasing
    assert _bad(2, 2, [0, 1, 3], [0, 1]).code == spmv.SPMV_EINVAL           # row_ptr[n] != nnz
    assert _bad(2, 2, [0, 1, 2], [0, 2]).code == spmv.SPMV_EINVAL           # column out of range
    assert _bad(2, 2, [0, 1, 2], [-1, 0]).code == spmv.SPMV_EINVAL          # negative column
    assert _bad(-1, 2, [0], []).code == spmv.SPMV_EINVAL                    # negative dimension
    assert _bad(2, 2, [0, 1, 2], [0, 1], {"tile_nnz": 1000}).code == spmv.SPMV_EINVAL
    assert _bad(2, 2, [0, 1, 2], [0, 1], {"ring_words": 3000}).code == spmv.SPMV_EINVAL
    assert _bad(2, 2, [0, 1, 2], [0, 1], {"window_mode": 7}).code == spmv.SPMV_EINVAL
    assert "row_ptr" in str(_bad(2, 2, [0, 2, 1], [0, 1]))


def test_nnz_limit_leaves_headroom_for_tile_offsets():
    # the kernels form 32-bit entry offsets up to a tile past the last entry,
    # so the largest accepted nnz is 2^31 - 2^16; one more is rejected before
    # any array is read (row_ptr here is too short to be read at all)
    L = spmv.lib()
    n_tiles = ctypes.c_int32()
    lim = (1 << 31) - (1 << 16)
    for nnz, code in ((lim + 1, spmv.SPMV_EINVAL), ((1 << 31) - 64, spmv.SPMV_EINVAL)):
        rc = L.spmv_plan_inspect(1, 1, nnz, np.zeros(2, np.int32).ctypes.data, None, None,
                                 ctypes.byref(n_tiles), None, None, None, None, None, None, None, None, None)
        assert rc == code
        assert "2^31 - 2^16" in spmv.lib().spmv_last_error().decode()
    h = ctypes.c_void_p()
    rc = L.spmv_create_bsr3(1, 1, lim // 9 + 1, np.zeros(2, np.int32).ctypes.data, None, None, 0,
                            ctypes.byref(h))
    assert rc == spmv.SPMV_EINVAL and not h.value


def test_create_rejects_malformed_input_before_touching_the_device():
    L = spmv.lib()
    h = ctypes.c_void_p()
    rp = np.array([0, 1, 3], np.int32)
    ci = np.array([0, 5, 1], np.int32)
    va = np.ones(3)
    rc = L.spmv_create(2, 2, 3, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, 0, None, ctypes.byref(h))
    assert rc == spmv.SPMV_EINVAL and not h.value
    rc = L.spmv_create(2, 2, 3, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, 0x80, None, ctypes.byref(h))
    assert rc == spmv.SPMV_EINVAL
    assert L.spmv_apply(None, None, None, None) == spmv.SPMV_EINVAL
    assert L.cg_solve(None, None, None, 1e-8, 10, 0, None, None) == spmv.SPMV_EINVAL
    assert L.spmv_destroy(None) == spmv.SPMV_OK
    assert L.spmv_get_info(None, None) == spmv.SPMV_EINVAL


def test_server_configuration_is_checked_before_touching_the_device():
    L = spmv.lib()
    for bad in ({"persistent_wgs": -1}, {"persist_idle_us": -5}, {"persist_idle_us": 10_000_001},
                {"n_lanes": 17}, {"n_slots": 65}, {"cg_mode": 7}):
        cfg = spmv.srv_config(**bad)
        h = ctypes.c_void_p()
        assert L.srv_create(ctypes.byref(cfg), ctypes.byref(h)) == spmv.SPMV_EINVAL and not h.value
        assert list(bad)[0].split("_")[-1] in spmv.lib().spmv_last_error().decode()


def check_plan(A, params=None):
    P = spmv.plan_inspect(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, params)
    info = P["info"]
    sb, kind = P["seg_bound"], P["seg_kind"]
    tnz, trows = info["tile_nnz"], info["tile_rows"]
    rp = A.row_ptr.astype(np.int64)
    # every row in exactly one segment
    assert sb[0] == 0 and sb[-1] == A.n_rows
    assert np.all(np.diff(sb) > 0)
    seg_nnz = rp[sb[1:]] - rp[sb[:-1]]
    seg_rows = np.diff(sb)
    lng = kind == 1
    cap = tnz - 3                     # a tile's 4-aligned span must fit tnz
    assert np.all(seg_rows[lng] == 1) and np.all(seg_nnz[lng] > cap)
    assert np.all(seg_nnz[~lng] <= cap) and np.all(seg_rows[~lng] <= trows)
    s4 = rp[sb[:-1]] & ~3
    assert np.all(rp[sb[1:]][~lng] - s4[~lng] <= tnz)
    # every row longer than a tile is a long-row segment
    long_rows = np.nonzero(np.diff(rp) > cap)[0]
    assert set(long_rows) == set(sb[:-1][lng])
    # window tiles: replay the staging of each block and check every column
    # a tile reads is resident, with the paper's count_i = colend_i - colend_{i-1}
    R = info["ring_words"]
    win = np.nonzero(kind == 2)[0]
    staged = 0
    for blk in np.unique(P["win_block"][win]):
        segs = win[P["win_block"][win] == blk]
        assert np.all(np.diff(segs) == 1)          # adjacent tiles, walked in order
        ring = {}
        hi_prev = None
        for s in segs:
            off, cnt = int(P["win_off"][s]), int(P["win_cnt"][s])
            for w in range(off, off + cnt):
                ring[w % R] = w
            staged += cnt
            cols = A.col_idx[rp[sb[s]]:rp[sb[s + 1]]]
            if cols.size == 0:
                continue
            for c in np.unique(cols):
                assert ring.get(int(c) % R) == int(c)
            if hi_prev is not None and cnt and off == hi_prev + 1:
                assert off + cnt - 1 == cols.max()   # loads exactly up to colend_i
            hi_prev = max(hi_prev if hi_prev is not None else -1, int(cols.max()))
    # compact windows: every entry's 16-bit position maps back to its column
    # through its tile's runs; windows fit the tile capacity, runs are ordered
    cw = np.nonzero(kind == 3)[0]
    runs = P["runs"]
    for s in cw:
        r0, nr = int(P["win_off"][s]), int(P["win_cnt"][s])
        assert 0 <= nr <= 64
        if nr == 0:
            continue                  # direct-gather tile inside the window launch
        rx, rpos = runs[r0:r0 + nr, 0].astype(np.int64), runs[r0:r0 + nr, 1].astype(np.int64)
        assert rpos[0] == 0 and np.all(np.diff(rpos) > 0) and np.all(np.diff(rx) > 0)
        a, b = rp[sb[s]], rp[sb[s + 1]]
        pos = P["lidx"][a:b].astype(np.int64)
        r = np.searchsorted(rpos, pos, side="right") - 1
        assert np.array_equal(rx[r] + (pos - rpos[r]), A.col_idx[a:b])
        cols = A.col_idx[a:b]
        width = int(rpos[-1] + (cols[cols >= rx[-1]].max() - rx[-1] + 1))
        assert width <= tnz
        staged += width
    assert staged == info["window_words"]
    assert info["n_window_tiles"] == win.size + int(np.sum(P["win_cnt"][cw] > 0))
    # 2048-entry tiles: the packed 12-bit positions, decoded the way the
    # kernel's lanes read them, are the 16-bit positions (0 outside the tile)
    if tnz == 2048 and cw.size and P["runs"].size:
        w = P["lidx12"].reshape(cw.size, 256, 3).astype(np.uint64)
        lo = w[:, :, 0] | (w[:, :, 1] << np.uint64(32))
        hi = w[:, :, 1] | (w[:, :, 2] << np.uint64(32))
        lane = np.arange(256)
        for t, sg in enumerate(cw):
            a, b = rp[sb[sg]], rp[sb[sg + 1]]
            for m in range(8):
                k = (a & ~3) + (m // 4) * 1024 + 4 * lane + (m % 4)
                got = ((lo[t] >> np.uint64(12 * m)) if m < 5 else (hi[t] >> np.uint64(12 * m - 32))) & np.uint64(0xfff)
                inside = (k >= a) & (k < b)
                want = np.zeros(256, np.uint64)
                if P["win_cnt"][sg] > 0:
                    want[inside] = P["lidx"][k[inside]]
                assert np.array_equal(got, want), (t, m)
    return P


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_plan_invariants_mesh(tile):
    A = mg.config0()
    check_plan(A, {"tile_nnz": tile})


def test_plan_invariants_hex_mesh_packed_positions():
    # the headline matrix family (hex 27-subset lattice, RCM) at 40^3
    A = mg.config2(m=40)
    P = check_plan(A, {"tile_nnz": 2048})
    assert P["lidx12"].size == 768 * int(np.sum(P["seg_kind"] == 3)) > 0


def test_plan_invariants_edge_cases():
    A = mg.random_csr(3000, 3000, seed=1, mean_len=3.0, empty_frac=0.3, dense_rows=2)
    P = check_plan(A, {"tile_nnz": 1024})
    assert P["info"]["n_long_rows"] == 2
    # all rows empty
    n = 700
    P = spmv.plan_inspect(n, 5, np.zeros(n + 1, np.int32), np.zeros(0, np.int32))
    assert P["seg_bound"][-1] == n and np.all(P["seg_kind"] == 0)
    # no rows at all
    P = spmv.plan_inspect(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert P["info"]["n_tiles"] == 0


def test_plan_long_row_pieces_and_workspace():
    # rows longer than a tile are summed in pieces of 16,384 entries; the
    # workspace of spmv_apply_ws holds one double per piece, and is needed
    # only when some row has more than one piece
    lens = [1021, 1022, 5000, 16384, 16385, 50_000, 0, 3]   # 1024-entry tiles hold 1021
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = (np.arange(rp[-1]) % 60_000).astype(np.int32)
    P = check_plan(mg.CSR(len(lens), 60_000, rp, ci, np.ones(rp[-1]), 1), {"tile_nnz": 1024})
    pieces = 1 + 1 + 1 + 2 + 4  # the rows of 1022, 5000, 16384, 16385 and 50000 entries
    assert P["info"]["n_long_rows"] == 5 and P["info"]["n_long_pieces"] == pieces
    assert P["info"]["workspace_bytes"] == 8 * pieces
    # long rows of one piece each: nothing to split
    rp1 = np.array([0, 5000, 5003, 21_387], np.int32)
    P = check_plan(mg.CSR(3, 60_000, rp1, (np.arange(rp1[-1]) % 60_000).astype(np.int32), np.ones(rp1[-1]), 1),
                   {"tile_nnz": 1024})
    assert P["info"]["n_long_pieces"] == 2 and P["info"]["workspace_bytes"] == 0
    # spmv_params.long_rows is 0 (split where scratch exists) or 1
    for bad in (-1, 2):
        with pytest.raises(spmv.SpmvError) as e:
            spmv.plan_inspect(3, 60_000, rp1, (np.arange(rp1[-1]) % 60_000).astype(np.int32),
                              {"tile_nnz": 1024, "long_rows": bad})
        assert e.value.code == spmv.SPMV_EINVAL


@pytest.mark.parametrize("ring", [256, 1024, 4096])
def test_plan_window_forced_ring_sizes(ring):
    A = mg.lattice(16, 16, 16, "faces", seed=3)         # bandwidth 256: many tiles fit
    P = check_plan(A, {"tile_nnz": 1024, "window_mode": spmv.WINDOW_RING, "ring_words": ring,
                       "window_block": 8})
    if ring >= 1024:
        assert P["info"]["n_window_tiles"] > 0
        # walking blocks of 8 adjacent tiles stages far fewer words than the tiles' spans
        assert P["info"]["window_words"] < A.nnz


def test_plan_window_off_and_auto():
    A = mg.lattice(16, 16, 16, "faces", seed=3)
    P = check_plan(A, {"window_mode": spmv.WINDOW_OFF})
    assert P["info"]["n_window_tiles"] == 0
    P = check_plan(A, {"window_mode": spmv.WINDOW_AUTO, "tile_nnz": 1024})
    assert P["info"]["n_window_tiles"] == P["info"]["n_tiles"]          # every tile fits
    assert P["info"]["window_words"] < A.nnz


@pytest.mark.parametrize("gap", [1, 16, 256])
def test_plan_compact_windows_mesh_and_scattered(gap):
    A = mg.config0()
    P = check_plan(A, {"tile_nnz": 4096, "window_gap": gap})
    assert P["info"]["n_window_tiles"] > 0
    # random order: columns scatter over the whole vector, windows do not fit
    B = mg.config1("random", m=40)
    P = check_plan(B, {"tile_nnz": 4096, "window_gap": gap})
    assert P["info"]["n_window_tiles"] < P["info"]["n_tiles"]
    C = mg.random_csr(5000, 5000, seed=9, mean_len=6.0, empty_frac=0.2, dense_rows=2, duplicates=True,
                      unsorted=True)
    check_plan(C, {"tile_nnz": 2048, "window_gap": gap})


def check_sell(A, sigma):
    """Invariants of the SELL-C-sigma layout against the CSR it came from."""
    S = spmv.sell_inspect(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, sigma)
    rp = A.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    short = np.nonzero(lens <= 255)[0]
    longr = np.nonzero(lens > 255)[0]
    sig = sigma or 4096
    perm, ln, sp, col = S["perm"], S["len"].astype(np.int64), S["slice_ptr"].astype(np.int64), S["col"]
    ns = S["n_slices"]
    assert ns == (short.size + 63) // 64 and perm.size == 64 * ns
    # slots: the short rows, each once, sorted by length (descending, ties by
    # row) inside each window of sigma short rows; empty slots only at the end
    filled = perm[perm >= 0]
    assert filled.size == short.size and np.all(perm[filled.size:] == -1)
    for w0 in range(0, short.size, sig):
        win = short[w0:w0 + sig]
        want = sorted(win.tolist(), key=lambda r: (-lens[r], r))
        assert filled[w0:w0 + sig].tolist() == want
    assert np.array_equal(ln[perm >= 0], lens[filled]) and np.all(ln[perm < 0] == 0)
    # slices: width = longest row, column-major entries, padding repeats the
    # row's last column (0 for an empty row)
    widths = np.diff(sp) // 64
    assert np.all(np.diff(sp) % 64 == 0) and sp[0] == 0 and sp[-1] == S["n_entries"]
    assert np.array_equal(widths, ln.reshape(ns, 64).max(axis=1) if ns else widths)
    for sl in range(ns):
        for lane in range(64):
            r, L = perm[64 * sl + lane], ln[64 * sl + lane]
            got = col[sp[sl] + 64 * np.arange(widths[sl]) + lane]
            if r < 0:
                assert np.all(got == 0)
                continue
            row = A.col_idx[rp[r]:rp[r + 1]]
            pad = row[-1] if L else 0
            assert np.array_equal(got[:L], row) and np.all(got[L:] == pad)
    # long rows after the slices, in CSR order
    assert np.array_equal(S["long_rows"], longr)
    tail = np.concatenate([A.col_idx[rp[r]:rp[r + 1]] for r in longr]) if longr.size else np.zeros(0, np.int32)
    assert np.array_equal(col[S["n_entries"]:], tail)
    return S


@pytest.mark.parametrize("sigma", [64, 512, 0])
def test_sell_layout_mesh(sigma):
    A = mg.config0()
    S = check_sell(A, sigma)
    # sorting inside windows cuts padding: the mesh rows vary from 7 to 23 entries
    if sigma != 64:
        assert S["n_entries"] <= 1.10 * A.nnz


def test_sell_layout_edge_cases():
    check_sell(mg.random_csr(1000, 700, seed=3, mean_len=4.0, empty_frac=0.3, dense_rows=2), 128)
    check_sell(mg.random_csr(130, 130, seed=4, mean_len=0.0, empty_frac=1.0), 0)
    n = 70
    rows = [np.arange(300) if i in (5, 66) else np.arange(i % 7) for i in range(n)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    A = mg.CSR(n, 300, rp, np.concatenate(rows).astype(np.int32), np.ones(int(rp[-1])))
    S = check_sell(A, 64)
    assert S["long_rows"].tolist() == [5, 66]


def test_sell_rejects_bad_sigma():
    A = mg.config0()
    for bad in (32, 100, -64):
        with pytest.raises(spmv.SpmvError) as e:
            spmv.sell_inspect(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, bad)
        assert e.value.code == spmv.SPMV_EINVAL
    with pytest.raises(spmv.SpmvError):
        spmv.plan_inspect(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, {"format": spmv.FORMAT_SELL})
    with pytest.raises(ValueError):
        spmv.plan_inspect(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, {"tile_nzz": 1024})


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = __import__("os").path.dirname(__import__("os").path.dirname(__file__))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
