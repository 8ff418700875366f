"""Seeded synthetic mesh matrices and vectors (input generation only).

The generators build the workloads the SpMV and CG paths run on: sparsity
patterns of 3-D finite-volume meshes (row i = cell i, columns = neighbouring
cells, paper Sec. 2), Laplacian-like symmetric coefficients, reorderings
(reverse Cuthill-McKee, paper Sec. 4.1, or a random permutation) and input
vectors.  Nothing here multiplies a matrix by a vector or solves a system: the
CPU oracle (``oracle/``) and the GPU library both take these arrays as inputs
and share no arithmetic.

The heavy lifting is in ``meshgen.c`` (OpenMP), loaded through ctypes.  Every
draw is a pure function of (seed, stream, index), so results do not depend on
the thread count.

Workload recipes (the paper's own matrices are not available; these stand in
for them):

* ``config0``  32^3 lattice, 6 face neighbours plus 0-4 random extra
  neighbours per cell within Chebyshev distance 2, union-symmetrised, RCM.
* ``config1``  m^3 jittered lattice (m = 126 -> 2,000,376 rows), each cell
  keeps 4-6 nearest neighbours, union-symmetrised; RCM or random order.
* ``config2``  m^3 lattice (m = 252 -> 16,003,008 rows), faces plus each
  edge/vertex neighbour pair kept with probability 1/2 (7-27 nnz per row), RCM.
* ``config3``  200x200x100 lattice, 3x3 block-CSR, 7-11 blocks per block row.
* ``serving_matrix``  config0-style lattices of any size for request streams.
* ``tet_like`` / ``table1_matrix``  stand-ins for the paper's tetrahedral
  matrices (Table 1 row counts, at most four neighbours per cell), RCM.

Off-diagonals are -w with one w ~ U[0.5, 1.5) per undirected edge, and the
diagonal is sum(w) + shift (shift = 1e-3), so A is symmetric, strictly
diagonally dominant and A*(c*1) = shift*c*1 in exact arithmetic.  With
``dyadic=True`` the weights are m/1024 (integer m in [512, 1536]) and the
shift is 2**-10, so every product and partial sum with dyadic x is exact.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "meshgen.c")
_LIB_PATH = os.path.join(_HERE, "libmeshgen.so")

SEED_BASE = 0x21071237


def seed_for(config: int) -> int:
    """Seed of workload configuration ``config`` (0..4)."""
    return SEED_BASE + int(config)


def build(force: bool = True) -> str:
    """Compile ``libmeshgen.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
        lib.mg_lattice.restype = vp
        lib.mg_lattice.argtypes = [i32, i32, i32, i32, u64, dbl, i32]
        lib.mg_knn.restype = vp
        lib.mg_knn.argtypes = [i32, u64, dbl, i32]
        lib.mg_bsr3.restype = vp
        lib.mg_bsr3.argtypes = [i32, i32, i32, u64, dbl]
        lib.mg_permute.restype = vp
        lib.mg_permute.argtypes = [vp, vp]
        lib.mg_from_arrays.restype = vp
        lib.mg_from_arrays.argtypes = [i32, i32, i64, i32, vp, vp, vp]
        lib.mg_rcm.restype = ctypes.c_int
        lib.mg_rcm.argtypes = [vp, vp]
        lib.mg_random_perm.restype = None
        lib.mg_random_perm.argtypes = [i32, u64, vp]
        lib.mg_degree_capped.restype = i64
        lib.mg_degree_capped.argtypes = [i64, vp, vp, i64, i32, vp]
        lib.mg_uniform.restype = None
        lib.mg_uniform.argtypes = [i64, u64, u64, dbl, dbl, vp]
        for f in ("mg_n_rows", "mg_n_cols", "mg_block"):
            getattr(lib, f).restype = i32
            getattr(lib, f).argtypes = [vp]
        lib.mg_nnz.restype = i64
        lib.mg_nnz.argtypes = [vp]
        lib.mg_fetch.restype = None
        lib.mg_fetch.argtypes = [vp, vp, vp, vp]
        lib.mg_free.restype = None
        lib.mg_free.argtypes = [vp]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Host CSR (``block == 1``) or 3x3 block CSR (``block == 3``, 9 row-major
    values per stored block).  int32 row_ptr/col_idx, float64 values."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    block: int = 1

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(h) -> CSR:
    lib = _L()
    if not h:
        raise MemoryError("meshgen: generation failed (size limits or out of memory)")
    try:
        n, nc, nnz, b = lib.mg_n_rows(h), lib.mg_n_cols(h), lib.mg_nnz(h), lib.mg_block(h)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        va = np.empty(nnz * b * b, np.float64)
        lib.mg_fetch(h, rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    finally:
        lib.mg_free(h)
    if b == 3:
        va = va.reshape(nnz, 3, 3)
    return CSR(n, nc, rp, ci, va, b)


def _handle(A: CSR):
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    ci = np.ascontiguousarray(A.col_idx, np.int32)
    va = np.ascontiguousarray(A.values, np.float64)
    h = _L().mg_from_arrays(A.n_rows, A.n_cols, A.nnz, A.block,
                            rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    if not h:
        raise MemoryError("meshgen: copy failed")
    return h


_KIND = {"extras": 0, "faces": 1, "stencil27": 2}


def lattice(nx: int, ny: int, nz: int, kind: str = "extras", seed: int = SEED_BASE,
            shift: float | None = None, dyadic: bool = False) -> CSR:
    """Laplacian-like matrix on an nx*ny*nz lattice in natural order.

    kind: "extras" (faces + 0-4 extras within Chebyshev 2, union), "faces"
    (7-point), "stencil27" (faces + each edge/vertex pair with prob. 1/2).
    shift defaults to 1e-3 (2**-10 when dyadic); 0 gives the pure-Neumann
    Laplacian whose rows sum to zero.
    """
    if shift is None:
        shift = 2.0 ** -10 if dyadic else 1e-3
    return _take(_L().mg_lattice(nx, ny, nz, _KIND[kind], seed, shift, int(dyadic)))


def knn(m: int, seed: int = SEED_BASE + 1, shift: float | None = None,
        dyadic: bool = False) -> CSR:
    """Jittered m^3 lattice, 4-6 nearest neighbours per cell, union-symmetrised."""
    if shift is None:
        shift = 2.0 ** -10 if dyadic else 1e-3
    return _take(_L().mg_knn(m, seed, shift, int(dyadic)))


def bsr3(nx: int, ny: int, nz: int, seed: int = SEED_BASE + 3, sigma: float = 0.1) -> CSR:
    """3x3 block-CSR coupled operator (nonsymmetric, diagonally dominant)."""
    return _take(_L().mg_bsr3(nx, ny, nz, seed, sigma))


def rcm_perm(A: CSR) -> np.ndarray:
    """Reverse Cuthill-McKee permutation, ``perm[new] = old``."""
    h = _handle(A)
    perm = np.empty(A.n_rows, np.int32)
    try:
        if _L().mg_rcm(h, perm.ctypes.data) != 0:
            raise MemoryError("meshgen: rcm failed")
    finally:
        _L().mg_free(h)
    return perm


def random_perm(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, np.int32)
    _L().mg_random_perm(n, seed, perm.ctypes.data)
    return perm


def permute(A: CSR, perm: np.ndarray) -> CSR:
    """P A P^T with ``perm[new] = old`` (columns re-sorted per row)."""
    perm = np.ascontiguousarray(perm, np.int32)
    h = _handle(A)
    try:
        out = _L().mg_permute(h, perm.ctypes.data)
    finally:
        _L().mg_free(h)
    return _take(out)


def uniform(count: int, seed: int, stream: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """``count`` draws of U[lo, hi) from stream ``stream`` (float64)."""
    out = np.empty(int(count), np.float64)
    _L().mg_uniform(int(count), seed, stream, lo, hi, out.ctypes.data)
    return out


def dyadic_x(n: int, seed: int) -> np.ndarray:
    """x_i = k_i / 2**20 with distinct integers |k_i| <= 2**20 (n <= 2**21), so a
    wrong column shows up in the product and every product with a dyadic
    matrix value is exact."""
    if n > 2 ** 21:
        raise ValueError("dyadic_x needs n <= 2**21")
    k = random_perm(n, seed).astype(np.int64) - n // 2
    return k.astype(np.float64) / 2.0 ** 20


def dyadic_x32(n: int, seed: int) -> np.ndarray:
    """x_i = k_i / 64 with integer |k_i| <= 64: exact for float32 products and
    sums of up to 33 terms with the dyadic weights."""
    u = uniform(n, seed, stream=7, lo=0.0, hi=1.0)
    k = np.floor(u * 129.0).astype(np.int64) - 64
    return k.astype(np.float64) / 64.0


def bandwidth(A: CSR) -> tuple[int, int]:
    """(max over rows of max col - min col, max |i - j|) -- the two readings of
    'width of the band'."""
    if A.nnz == 0:
        return 0, 0
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    nonempty = np.diff(A.row_ptr) > 0
    mx = np.maximum.reduceat(cols, A.row_ptr[:-1][nonempty])
    mn = np.minimum.reduceat(cols, A.row_ptr[:-1][nonempty])
    return int((mx - mn).max()), int(np.abs(rows - cols).max())


# ----------------------------------------------------------- workloads

def _cached(name: str, build_fn) -> CSR:
    """Build a workload, or load it from ``$SPMV_CACHE_DIR/<name>.npz`` when
    that directory is set (lets several processes of one run share a large
    generated matrix).  Plain arrays only; no pickles."""
    d = os.environ.get("SPMV_CACHE_DIR")
    if not d:
        return build_fn()
    path = os.path.join(d, name + ".npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return CSR(int(z["n_rows"]), int(z["n_cols"]), z["row_ptr"], z["col_idx"], z["values"],
                       int(z["block"]))
    A = build_fn()
    os.makedirs(d, exist_ok=True)
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, n_rows=A.n_rows, n_cols=A.n_cols, row_ptr=A.row_ptr, col_idx=A.col_idx,
             values=A.values, block=A.block)
    os.replace(tmp, path)
    return A


def config0(seed: int | None = None, dyadic: bool = False, ordering: str = "rcm") -> CSR:
    """32^3 lattice with 0-4 extras (32768 rows), RCM-ordered."""
    s = seed_for(0) if seed is None else seed
    A = lattice(32, 32, 32, "extras", s, dyadic=dyadic)
    return reorder(A, ordering, s)


def config1(ordering: str = "rcm", m: int = 126, seed: int | None = None,
            dyadic: bool = False) -> CSR:
    """Jittered-lattice kNN matrix (m=126: 2,000,376 rows) in RCM or random order."""
    s = seed_for(1) if seed is None else seed
    return _cached(f"cfg1_m{m}_{ordering}_s{s}_d{int(dyadic)}",
                   lambda: reorder(knn(m, s, dyadic=dyadic), ordering, s))


def config2(m: int = 252, ordering: str = "rcm", seed: int | None = None,
            dyadic: bool = False) -> CSR:
    """27-point-subset lattice (m=252: 16,003,008 rows, 7-27 nnz/row), RCM."""
    s = seed_for(2) if seed is None else seed
    return _cached(f"cfg2_m{m}_{ordering}_s{s}_d{int(dyadic)}",
                   lambda: reorder(lattice(m, m, m, "stencil27", s, dyadic=dyadic), ordering, s))


def config3(nx: int = 200, ny: int = 200, nz: int = 100, seed: int | None = None) -> CSR:
    """3x3 block CSR on 200x200x100 cells (4,000,000 block rows), natural order."""
    s = seed_for(3) if seed is None else seed
    return bsr3(nx, ny, nz, s)


# the paper's Table 1 matrices (rows); nnz/rows is 4.93-4.97 there
TABLE1_ROWS = {"C50K": 49336, "C100K": 97521, "C200K": 187078, "C400K": 398000, "C800K": 775058}


def tet_like(n: int, seed: int | None = None, shift: float = 1e-3) -> CSR:
    """Stand-in for the paper's tetrahedral-mesh matrices (Table 1, Sec. 2: a
    cell of a tetrahedral mesh has at most four face neighbours, so a row has
    at most five non-zeros).  n cells on a jittered lattice (+-0.35 per
    axis); candidate pairs are each cell's 16 nearest cells, taken by
    increasing distance (ties by index) and kept while both cells have fewer
    than four neighbours.  Weights, diagonal and RCM order as in the other
    meshes; row lengths 1-5."""
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    s = seed_for(5) if seed is None else seed
    m = int(np.ceil(n ** (1.0 / 3.0)))
    idx = np.arange(n, dtype=np.int64)
    pts = np.stack([idx % m, (idx // m) % m, idx // (m * m)], axis=1).astype(np.float64)
    pts += 0.35 * uniform(3 * n, s, 11).reshape(n, 3)
    dist, nb = cKDTree(pts).query(pts, k=17)
    i = np.repeat(idx, 16)
    j = nb[:, 1:].reshape(-1).astype(np.int64)
    d = dist[:, 1:].reshape(-1)
    key = np.minimum(i, j) * n + np.maximum(i, j)
    ukey, first = np.unique(key, return_index=True)          # each pair once (same distance both ways)
    ukey = ukey[np.lexsort((ukey, d[first]))]                 # by distance, ties by index
    pa, pb = ukey // n, ukey % n
    keep = np.empty(len(ukey), np.uint8)
    if _L().mg_degree_capped(len(ukey), pa.ctypes.data, pb.ctypes.data, n, 4, keep.ctypes.data) < 0:
        raise MemoryError("meshgen: degree-capped fill failed")
    ea, eb = pa[keep == 1], pb[keep == 1]
    w = 1.0 + 0.5 * uniform(len(ea), s, 12)                     # U[0.5, 1.5) per undirected edge
    diag = np.bincount(ea, w, n) + np.bincount(eb, w, n) + shift
    S = sp.coo_matrix((np.concatenate([-w, -w, diag]),
                       (np.concatenate([ea, eb, idx]), np.concatenate([eb, ea, idx]))), shape=(n, n)).tocsr()
    S.sort_indices()
    A = CSR(n, n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    return reorder(A, "rcm", s)


def table1_matrix(name: str) -> CSR:
    """The tet-like stand-in with the row count of the paper's matrix ``name``."""
    n = TABLE1_ROWS[name]
    return _cached(f"table1_{name}", lambda: tet_like(n))


def serving_matrix(n_target: int, seed: int) -> CSR:
    """A config0-style lattice of about ``n_target`` rows, RCM-ordered."""
    nx = max(2, int(round(n_target ** (1.0 / 3.0))))
    nz = max(1, int(round(n_target / (nx * nx))))
    A = lattice(nx, nx, nz, "extras", seed)
    return reorder(A, "rcm", seed)


def reorder(A: CSR, ordering: str, seed: int) -> CSR:
    if ordering == "natural":
        return A
    if ordering == "rcm":
        return permute(A, rcm_perm(A))
    if ordering == "random":
        return permute(A, random_perm(A.n_rows, seed ^ 0x5EED))
    raise ValueError(f"unknown ordering {ordering!r}")


def random_csr(n_rows: int, n_cols: int, seed: int, mean_len: float = 4.0,
               empty_frac: float = 0.1, dense_rows: int = 0, duplicates: bool = False,
               unsorted: bool = False) -> CSR:
    """Small irregular CSR for edge cases: empty rows, dense rows, duplicate
    entries and unsorted columns.  Values U[-1, 1)."""
    rng = np.random.default_rng(seed)
    lens = rng.poisson(mean_len, n_rows)
    lens[rng.random(n_rows) < empty_frac] = 0
    if dense_rows:
        lens[rng.choice(n_rows, size=min(dense_rows, n_rows), replace=False)] = n_cols
    lens = np.minimum(lens, n_cols if not duplicates else 4 * n_cols)
    rp = np.zeros(n_rows + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    cols = []
    for i in range(n_rows):
        L = int(lens[i])
        if L == 0:
            continue
        if duplicates:
            c = rng.integers(0, n_cols, L)
        elif L == n_cols:
            c = np.arange(n_cols)
        else:
            c = rng.choice(n_cols, size=L, replace=False)
        if not unsorted:
            c = np.sort(c)
        cols.append(c)
    ci = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    va = rng.uniform(-1.0, 1.0, ci.shape[0])
    return CSR(n_rows, n_cols, rp.astype(np.int32), ci, va, 1)


def with_long_rows(A: CSR, n_long: int, length: int, seed: int) -> CSR:
    """A copy of A in which n_long rows, spread evenly over the matrix, are
    replaced by rows of `length` entries over sorted distinct random columns
    (a coupling row over a subset of the cells, such as a global constraint),
    values U[-1, 1)."""
    if length > A.n_cols:
        raise ValueError("length exceeds n_cols")
    rng = np.random.default_rng(seed)
    where = np.linspace(0, A.n_rows - 1, n_long + 2)[1:-1].astype(np.int64)
    lens = np.diff(A.row_ptr).astype(np.int64)
    new_lens = lens.copy()
    new_lens[where] = length
    rp = np.zeros(A.n_rows + 1, np.int64)
    rp[1:] = np.cumsum(new_lens)
    if rp[-1] > (1 << 31) - (1 << 16):
        raise ValueError("too many stored entries")
    keep = np.ones(A.n_rows, bool)
    keep[where] = False
    old_row = np.repeat(np.arange(A.n_rows), lens)
    m = keep[old_row]
    pos = rp[old_row[m]] + (np.arange(A.nnz)[m] - A.row_ptr[old_row[m]].astype(np.int64))
    ci = np.empty(int(rp[-1]), np.int32)
    va = np.empty(int(rp[-1]), np.float64)
    ci[pos] = A.col_idx[m]
    va[pos] = A.values[m]
    for r in where:
        ci[rp[r]:rp[r + 1]] = np.sort(rng.choice(A.n_cols, size=length, replace=False))
        va[rp[r]:rp[r + 1]] = rng.uniform(-1.0, 1.0, length)
    return CSR(A.n_rows, A.n_cols, rp.astype(np.int32), ci, va, 1)
