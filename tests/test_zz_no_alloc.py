"""cg_solve_noalloc (the FP64 CG on the library's per-device scratch array)
against cg_solve, through the C ABI: two solves in a row, the second on a
smaller system, each bitwise equal to cg_solve in CG_FP64 mode (the same
kernels in the same order) and within the CG acceptance rule of the
oracle; the size limit and the mode restriction are reported as errors."""
import ctypes

import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _noalloc(M, b, tol, max_iter=20000, mode=spmv.CG_FP64):
    x = torch.zeros(M.n_rows, dtype=torch.float64, device=DEV)
    inf = spmv.cg_info()
    rc = spmv.lib().cg_solve_noalloc(M.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     tol, max_iter, mode, ctypes.byref(inf), None)
    return rc, x, inf


def _check_against_cg_solve(A, seed, tol=1e-10):
    b_h = mg.uniform(A.n_rows, seed, 1)
    b = torch.as_tensor(b_h, device=DEV)
    with spmv.Matrix.from_csr(A) as M:
        x_ref, info_ref = M.cg(b, tol=tol)
        rc, x, inf = _noalloc(M, b, tol)
        torch.cuda.synchronize()
    assert rc == spmv.SPMV_OK, spmv.lib().spmv_last_error()
    assert inf.iterations == info_ref.iterations and inf.refinements == info_ref.refinements
    assert torch.equal(x, x_ref)
    assert inf.rel_residual == info_ref.rel_residual
    # the acceptance rule of the CG tests: true residual by the oracle's product
    Ax, _ = oracle.spmv(A, x.cpu().numpy())
    assert np.linalg.norm(b_h - Ax) / np.linalg.norm(b_h) <= 1.05 * tol
    return inf.iterations


def test_noalloc_cg_equals_cg_solve_twice_second_smaller():
    big = mg.table1_matrix("C100K")          # 97,521 rows
    small = mg.config0()                      # 32,768 rows
    it1 = _check_against_cg_solve(big, 71)
    it2 = _check_against_cg_solve(small, 72)
    assert it1 > 0 and it2 > 0


def test_noalloc_cg_limits_and_modes():
    n = (1 << 19) + 1
    D = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    with spmv.Matrix.from_csr(D) as M:
        b = torch.ones(n, dtype=torch.float64, device=DEV)
        rc, _, _ = _noalloc(M, b, 1e-10)
        assert rc == spmv.SPMV_EINVAL
        assert b"524288" in spmv.lib().spmv_last_error()
    A = mg.config0()
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        b = torch.as_tensor(mg.uniform(A.n_rows, 73, 1), device=DEV)
        rc, _, _ = _noalloc(M, b, 1e-10, mode=spmv.CG_MIXED_FP32)
        assert rc == spmv.SPMV_ENOTSUP
        # b = 0 gives x = 0 and no iteration; the iteration cap is reported
        rc, x, inf = _noalloc(M, torch.zeros_like(b), 1e-10)
        assert rc == spmv.SPMV_OK and inf.iterations == 0 and bool(torch.all(x == 0))
        rc, x, inf = _noalloc(M, b, 1e-14, max_iter=5)
        assert rc == spmv.SPMV_ENOTCONV and inf.iterations == 5
        x_ref, info_ref = M.cg(b, tol=1e-14, max_iter=5, raise_on_error=False)
        assert torch.equal(x, x_ref)
