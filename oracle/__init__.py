"""CPU oracle for the sparse matrix-vector product and conjugate gradients.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or runs anything here, and this package imports nothing from the library.

``oracle.c`` holds the arithmetic (binary64, no FMA contraction, ascending
index order, single thread); this module marshals numpy arrays through
ctypes.  See the header of ``oracle.c`` for the passages each routine follows.

Acceptance rule for a GPU SpMV result (per row, binary64):
``|y_gpu[i] - y_ref[i]| <= 1e-12 * bound[i]`` with
``bound[i] = sum_k |a_ik| |x_k|``; rows with ``bound[i] == 0`` must give 0.
Any correct summation order satisfies it: the forward error of an m-term dot
product is at most gamma_m * bound with gamma_m = m u / (1 - m u), u = 2**-53
(Higham, Sec. 3.1), about 3.7e-15 * bound for m = 33.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

U64 = 2.0 ** -53
SPMV_RTOL = 1e-12


def gamma(m) -> np.ndarray:
    """gamma_m = m u / (1 - m u) for binary64 (u = 2**-53)."""
    m = np.asarray(m, dtype=np.float64)
    return m * U64 / (1.0 - m * U64)


def _compile(path: str, extra: list[str]) -> None:
    tmp = path + ".tmp"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-Wall", *extra, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` (plain C, -O2, no FP contraction, no OpenMP:
    the checker) and ``liboracle_omp.so`` (the same source with OpenMP, used
    only to time the product on all host cores)."""
    if force or not os.path.exists(_LIB_PATH):
        _compile(_LIB_PATH, [])
    if force or not os.path.exists(_OMP_PATH):
        _compile(_OMP_PATH, ["-fopenmp"])
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        lib.oracle_spmv.restype = None
        lib.oracle_spmv.argtypes = [i32, vp, vp, vp, vp, vp, vp]
        lib.oracle_spmv_rows.restype = None
        lib.oracle_spmv_rows.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_bsr3_spmm.restype = None
        lib.oracle_bsr3_spmm.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp]
        lib.oracle_dot.restype = dbl
        lib.oracle_dot.argtypes = [i32, vp, vp]
        lib.oracle_cg.restype = ctypes.c_int
        lib.oracle_cg.argtypes = [i32, vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_pcg_bf16.restype = ctypes.c_int
        lib.oracle_pcg_bf16.argtypes = [i32, vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_cg1.restype = ctypes.c_int
        lib.oracle_cg1.argtypes = [i32, vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_pcg_jacobi.restype = ctypes.c_int
        lib.oracle_pcg_jacobi.argtypes = [i32, vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


_omp_lib = None


def spmv_all_cores(A, x) -> np.ndarray:
    """y = A x with the OpenMP timing build of ``oracle_spmv``: rows split
    statically over OMP_NUM_THREADS threads, each row summed as in the
    single-threaded checker (so the result is the same bits).  For timing
    the oracle on all host cores; the tests check against ``spmv``."""
    global _omp_lib
    if _omp_lib is None:
        if not os.path.exists(_OMP_PATH):
            build(force=False)
        lib = ctypes.CDLL(_OMP_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.oracle_spmv.restype = None
        lib.oracle_spmv.argtypes = [i32, vp, vp, vp, vp, vp, vp]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _omp_lib = lib
    rp, ci, va = _csr(A)
    x = _c(x, np.float64)
    if x.shape[0] < A.n_cols:
        raise ValueError("x too short")
    y = np.empty(A.n_rows, np.float64)
    _omp_lib.oracle_spmv(A.n_rows, _ptr(rp), _ptr(ci), _ptr(va), _ptr(x), _ptr(y), None)
    return y


def all_cores_threads() -> int:
    """Threads the OpenMP timing build runs the product on."""
    if _omp_lib is None:
        spmv_all_cores(_Empty(), np.zeros(0))
    return int(_omp_lib.oracle_threads())


class _Empty:
    n_rows = n_cols = 0
    row_ptr = np.zeros(1, np.int32)
    col_idx = np.zeros(0, np.int32)
    values = np.zeros(0)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _csr(A):
    rp = _c(A.row_ptr, np.int32)
    ci = _c(A.col_idx, np.int32)
    va = _c(A.values, np.float64)
    return rp, ci, va


def spmv(A, x) -> tuple[np.ndarray, np.ndarray]:
    """(y, bound) with y = A x and bound_i = sum |a_ik||x_k| (binary64)."""
    rp, ci, va = _csr(A)
    x = _c(x, np.float64)
    if x.shape[0] < A.n_cols:
        raise ValueError("x too short")
    y = np.empty(A.n_rows, np.float64)
    b = np.empty(A.n_rows, np.float64)
    _L().oracle_spmv(A.n_rows, _ptr(rp), _ptr(ci), _ptr(va), _ptr(x), _ptr(y), _ptr(b))
    return y, b


def spmv_rows(A, x, rows) -> tuple[np.ndarray, np.ndarray]:
    """(y, bound) for the listed rows only."""
    rp, ci, va = _csr(A)
    x = _c(x, np.float64)
    rows = _c(rows, np.int32)
    y = np.empty(rows.shape[0], np.float64)
    b = np.empty(rows.shape[0], np.float64)
    _L().oracle_spmv_rows(rows.shape[0], _ptr(rows), _ptr(rp), _ptr(ci), _ptr(va), _ptr(x),
                          _ptr(y), _ptr(b))
    return y, b


def bsr3_spmm(A, X) -> tuple[np.ndarray, np.ndarray]:
    """(Y, bound) for a 3x3 block-CSR A and X of shape (3*n_cols, k), row-major."""
    rp = _c(A.row_ptr, np.int32)
    ci = _c(A.col_idx, np.int32)
    va = _c(A.values, np.float64).reshape(-1)
    X = _c(X, np.float64)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    k = X.shape[1]
    Y = np.empty((3 * A.n_rows, k), np.float64)
    B = np.empty((3 * A.n_rows, k), np.float64)
    _L().oracle_bsr3_spmm(A.n_rows, _ptr(rp), _ptr(ci), _ptr(va), k, _ptr(X), _ptr(Y), _ptr(B))
    return Y, B


def dot(a, b) -> float:
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    return float(_L().oracle_dot(a.shape[0], _ptr(a), _ptr(b)))


@dataclass
class CGResult:
    x: np.ndarray
    status: int          # 0 converged, 1 max_iter reached, 2 breakdown
    iterations: int
    rel_residual: float  # true ||b - A x|| / ||b||, recomputed in binary64
    alphas: np.ndarray
    betas: np.ndarray


def cg(A, b, tol: float = 1e-10, max_iter: int = 10000, x0=None) -> CGResult:
    """Textbook conjugate gradients in binary64 (see oracle.c)."""
    rp, ci, va = _csr(A)
    n = A.n_rows
    b = _c(b, np.float64)
    x = np.zeros(n, np.float64) if x0 is None else _c(x0, np.float64).copy()
    r = np.empty(n, np.float64)
    p = np.empty(n, np.float64)
    q = np.empty(n, np.float64)
    al = np.zeros(max(max_iter, 1), np.float64)
    be = np.zeros(max(max_iter, 1), np.float64)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    st = _L().oracle_cg(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(b), _ptr(x), tol, max_iter,
                        _ptr(r), _ptr(p), _ptr(q), ctypes.byref(it), ctypes.byref(rr),
                        _ptr(al), _ptr(be))
    k = it.value
    return CGResult(x, int(st), k, rr.value, al[:k].copy(), be[:k].copy())


def cg1(A, b, tol: float = 1e-10, max_iter: int = 10000, x0=None) -> CGResult:
    """CG with one reduction phase per iteration (Chronopoulos-Gear, see
    oracle.c); the result carries no coefficients, `alphas` holds the number
    of restarts from the true residual as its only element."""
    rp, ci, va = _csr(A)
    n = A.n_rows
    b = _c(b, np.float64)
    x = np.zeros(n, np.float64) if x0 is None else _c(x0, np.float64).copy()
    work = [np.empty(n, np.float64) for _ in range(4)]
    it = ctypes.c_int32(0)
    rs = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    st = _L().oracle_cg1(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(b), _ptr(x), tol, max_iter,
                         *[_ptr(a) for a in work], ctypes.byref(it), ctypes.byref(rs), ctypes.byref(rr))
    return CGResult(x, int(st), it.value, rr.value, np.array([rs.value]), np.zeros(0))


def pcg_bf16(A, b, tol: float = 1e-10, max_iter: int = 10000, x0=None):
    """CG preconditioned with the bfloat16 damped Neumann polynomial (see
    oracle.c).  Returns (CGResult without coefficients, weight w)."""
    rp, ci, va = _csr(A)
    n = A.n_rows
    b = _c(b, np.float64)
    x = np.zeros(n, np.float64) if x0 is None else _c(x0, np.float64).copy()
    work = [np.empty(n, np.float64) for _ in range(5)]
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    w = ctypes.c_double(0.0)
    st = _L().oracle_pcg_bf16(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(b), _ptr(x), tol, max_iter,
                              *[_ptr(a) for a in work], ctypes.byref(it), ctypes.byref(rr), ctypes.byref(w))
    return CGResult(x, int(st), it.value, rr.value, np.zeros(0), np.zeros(0)), w.value


def pcg_jacobi(A, b, tol: float = 1e-10, max_iter: int = 10000, x0=None) -> CGResult:
    """CG preconditioned with M = diag(A) (see oracle.c); the result carries
    no coefficients."""
    rp, ci, va = _csr(A)
    n = A.n_rows
    b = _c(b, np.float64)
    x = np.zeros(n, np.float64) if x0 is None else _c(x0, np.float64).copy()
    work = [np.empty(n, np.float64) for _ in range(4)]
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    st = _L().oracle_pcg_jacobi(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(b), _ptr(x), tol, max_iter,
                                *[_ptr(a) for a in work], ctypes.byref(it), ctypes.byref(rr))
    return CGResult(x, int(st), it.value, rr.value, np.zeros(0), np.zeros(0))


def spmv_accept(y_gpu, y_ref, bound, rtol: float = SPMV_RTOL) -> np.ndarray:
    """Boolean mask of rows meeting the acceptance rule (NaN/Inf by class)."""
    y_gpu = np.asarray(y_gpu, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    bound = np.asarray(bound, np.float64)
    fin = np.isfinite(y_ref) & np.isfinite(bound)
    ok = np.zeros(y_ref.shape, bool)
    with np.errstate(invalid="ignore"):
        ok[fin] = np.abs(y_gpu[fin] - y_ref[fin]) <= rtol * bound[fin]
    nan = np.isnan(y_ref)
    ok[nan] = np.isnan(y_gpu[nan])
    inf = np.isinf(y_ref)
    ok[inf] = y_gpu[inf] == y_ref[inf]
    # finite y_ref with non-finite bound (overflow of the bound only)
    odd = np.isfinite(y_ref) & ~np.isfinite(bound)
    ok[odd] = np.isfinite(y_gpu[odd])
    return ok
