"""GPU CG against the CPU oracle's CG.

Several answers are correct (iterates depend on rounding order), so the rule
compares what is fixed:
  1. the true relative residual ||b - A x_gpu|| / ||b||, recomputed with the
     oracle's SpMV, is within tol (5% slack for the residual's own rounding,
     at most u * kappa relative to tol);
  2. ||x_gpu - x_ref|| / ||x_ref|| <= 2 * kappa * tol, with kappa bounded by
     Gershgorin: (max_i (a_ii + sum_j |a_ij|)) / shift for these
     diagonally dominant Laplacians (smallest eigenvalue = shift);
  3. FP64 iteration counts within 10% of the oracle's.
"""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gershgorin_kappa(A, shift):
    v = np.abs(A.values)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    return np.bincount(rows, weights=v, minlength=A.n_rows).max() / shift


def true_rel_residual(A, x, b):
    Ax, _ = oracle.spmv(A, x)
    return np.linalg.norm(b - Ax) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg0():
    A = mg.config0()
    b = mg.uniform(A.n_rows, mg.seed_for(0), 3)
    ref = oracle.cg(A, b, tol=1e-10, max_iter=20000)
    assert ref.status == 0
    return A, b, ref


@pytest.mark.parametrize("mode", [spmv.CG_FP64, spmv.CG_MIXED_FP32, spmv.CG_MIXED_FP32V])
def test_cg_config0_against_oracle(cfg0, mode):
    A, b, ref = cfg0
    tol = 1e-10
    with spmv.Matrix.from_csr(A, fp32=True) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=tol, mode=mode)
    x = x.cpu().numpy()
    assert info.status == 0
    rr = true_rel_residual(A, x, b)
    assert rr <= 1.05 * tol
    assert abs(info.rel_residual - rr) <= 0.05 * tol
    kappa = gershgorin_kappa(A, 1e-3)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 2 * kappa * tol
    if mode == spmv.CG_FP64:
        assert abs(info.iterations - ref.iterations) <= 0.1 * ref.iterations
    else:
        assert info.refinements >= 1


def test_cg_closed_form_one_iteration():
    A = mg.config0()
    with spmv.Matrix.from_csr(A) as M:
        x, info = M.cg(torch.ones(A.n_rows, dtype=torch.float64, device=DEV), tol=1e-10)
    assert info.iterations == 1
    assert np.allclose(x.cpu().numpy(), 1000.0, rtol=1e-9)
    Ad = mg.config0(dyadic=True)
    with spmv.Matrix.from_csr(Ad) as M:
        x, info = M.cg(torch.ones(Ad.n_rows, dtype=torch.float64, device=DEV), tol=1e-12)
    assert info.iterations == 1 and bool(torch.all(x == 1024.0))


def test_cg_reproducible_bitwise(cfg0):
    A, b, _ = cfg0
    with spmv.Matrix.from_csr(A) as M:
        bt = torch.as_tensor(b, device=DEV)
        x1, i1 = M.cg(bt, tol=1e-8)
        x2, i2 = M.cg(bt, tol=1e-8)
    assert i1.iterations == i2.iterations and torch.equal(x1, x2)


def test_cg_warm_start_zero_rhs_and_max_iter(cfg0):
    A, b, ref = cfg0
    with spmv.Matrix.from_csr(A) as M:
        bt = torch.as_tensor(b, device=DEV)
        x, info = M.cg(torch.zeros_like(bt), x=torch.ones_like(bt))
        assert info.iterations == 0 and bool(torch.all(x == 0))
        x, info = M.cg(bt, tol=1e-12, max_iter=5, raise_on_error=False)
        assert info.status == spmv.SPMV_ENOTCONV and info.iterations == 5
        # resume from the last iterate (warm start)
        x2, info2 = M.cg(bt, x=x, tol=1e-10)
        assert info2.status == 0
        assert true_rel_residual(A, x2.cpu().numpy(), b) <= 1.05e-10


def test_cg_rejects_bad_input():
    A = mg.random_csr(50, 40, seed=1)
    with spmv.Matrix.from_csr(A) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.zeros(50, dtype=torch.float64, device=DEV))
        assert e.value.code == spmv.SPMV_EINVAL
    B = mg.config0()
    with spmv.Matrix.from_csr(B) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.ones(B.n_rows, dtype=torch.float64, device=DEV), mode=spmv.CG_MIXED_FP32)
        assert e.value.code == spmv.SPMV_ENOTSUP
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.ones(B.n_rows, dtype=torch.float64, device=DEV), mode=spmv.CG_MIXED_FP32V)
        assert e.value.code == spmv.SPMV_ENOTSUP
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.ones(B.n_rows, dtype=torch.float64, device=DEV), mode=6)
        assert e.value.code == spmv.SPMV_EINVAL


def test_cg_breakdown_on_indefinite_matrix():
    n = 64
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.zeros(n)
    b[0], b[1] = 1.0, 1.0   # p.q = 1 - 1 = 0 at the first step
    with spmv.Matrix.from_csr(A) as M:
        _, info = M.cg(torch.as_tensor(b, device=DEV), raise_on_error=False)
    assert info.status == spmv.SPMV_EBREAK


@pytest.mark.parametrize("n,neg,first", [(200, 3, False), (2_000_000, 0, True)])
def test_cg_breakdown_step_matches_oracle(n, neg, first):
    # a p.q breakdown is reported at the oracle's step: after two iterations on
    # a small indefinite diagonal system (few SpMV partials: alpha is formed
    # inside the x/r update), and at once on a 2M-row one (many partials:
    # alpha from a reduction launch)
    if first:
        d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        b = np.zeros(n)
        b[0], b[1] = 1.0, 1.0
    else:
        d = np.linspace(1.0, 10.0, n)
        d[-neg:] = -np.linspace(0.5, 5.0, neg)
        b = np.ones(n)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    ref = oracle.cg(A, b, tol=1e-10, max_iter=1000)
    assert ref.status == 2 and ref.iterations == (0 if first else 2)
    with spmv.Matrix.from_csr(A) as M:
        assert (M.info["n_tiles"] > 1024) == first
        _, info = M.cg(torch.as_tensor(b, device=DEV), tol=1e-10, max_iter=1000, raise_on_error=False)
    assert info.status == spmv.SPMV_EBREAK and info.iterations == ref.iterations


# ------------------------------------ preconditioned CG (bfloat16 copy)

@pytest.fixture(scope="module")
def pcg_ref(cfg0):
    A, b, ref = cfg0
    pref, w = oracle.pcg_bf16(A, b, tol=1e-10, max_iter=20000)
    assert pref.status == 0
    return pref


def test_pcg_config0_against_oracle(cfg0, pcg_ref):
    A, b, ref = cfg0
    tol = 1e-10
    with spmv.Matrix.from_csr(A, bf16=True) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=tol, mode=spmv.CG_PCG_BF16)
    x = x.cpu().numpy()
    assert info.status == 0
    rr = true_rel_residual(A, x, b)
    assert rr <= 1.05 * tol and abs(info.rel_residual - rr) <= 0.05 * tol
    kappa = gershgorin_kappa(A, 1e-3)
    assert np.linalg.norm(x - pcg_ref.x) / np.linalg.norm(pcg_ref.x) <= 2 * kappa * tol
    # the GPU applies A~ to an FP32 vector with FP32 sums, the oracle in
    # binary64, so the preconditioners differ in rounding: counts agree to 10%
    assert abs(info.iterations - pcg_ref.iterations) <= 0.1 * pcg_ref.iterations
    assert info.iterations < 0.8 * ref.iterations


@pytest.mark.parametrize("k", [1, 3, 6])
def test_pcg_bf16_first_iterates_match_the_oracle(cfg0, k):
    # k steps from zero (tol = 0, so the cap ends the solve) against the
    # oracle's k-step iterate, whose preconditioner is pinned to a dense
    # M^-1 built from the bfloat16 copy.  The GPU applies that copy to an
    # FP32 vector with FP32 sums, which moves the iterate by about 5e-8
    # relative (emulated on the CPU); the same steps with the FP32 or
    # binary64 values in the preconditioner move it by about 1e-3, so the
    # 1e-6 bound tells the two apart.
    A, b, _ = cfg0
    ref, _ = oracle.pcg_bf16(A, b, tol=0.0, max_iter=k)
    assert ref.status == 1 and ref.iterations == k
    with spmv.Matrix.from_csr(A, bf16=True) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=0.0, max_iter=k, mode=spmv.CG_PCG_BF16,
                       raise_on_error=False)
    assert info.status == spmv.SPMV_ENOTCONV and info.iterations == k
    x = x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_pcg_diagonal_one_iteration_and_reproducible():
    n = 4000
    d = np.tile([1.0, 2.5, 4.0, 7.0, 0.375], n // 5)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 4, 0)
    # M^-1 A is a multiple of I up to the FP32 rounding of the preconditioner's
    # vectors (the oracle, all binary64, takes exactly one step): one step
    # reaches 1e-6, a few reach 1e-12
    with spmv.Matrix.from_csr(A, bf16=True) as M:
        bt = torch.as_tensor(b, device=DEV)
        kappa = d.max() / d.min()
        rel = lambda v: np.linalg.norm(v.cpu().numpy() - b / d) / np.linalg.norm(b / d)
        x, info = M.cg(bt, tol=1e-6, mode=spmv.CG_PCG_BF16)
        assert info.iterations == 1 and rel(x) <= 2 * kappa * 1e-6
        x, info = M.cg(bt, tol=1e-12, mode=spmv.CG_PCG_BF16)
        x2, info2 = M.cg(bt, tol=1e-12, mode=spmv.CG_PCG_BF16)
    assert info.iterations <= 3 and rel(x) <= 2 * kappa * 1e-12
    assert torch.equal(x, x2) and info2.iterations == info.iterations


def test_pcg_rejects_missing_copy_sell_and_bad_diagonal():
    A = mg.config0()
    b = torch.ones(A.n_rows, dtype=torch.float64, device=DEV)
    with spmv.Matrix.from_csr(A) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(b, mode=spmv.CG_PCG_BF16)
        assert e.value.code == spmv.SPMV_ENOTSUP
    with spmv.Matrix.from_csr(A, bf16=True, params={"format": spmv.FORMAT_SELL}) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(b, mode=spmv.CG_PCG_BF16)
        assert e.value.code == spmv.SPMV_ENOTSUP
    n = 64
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    B = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    with spmv.Matrix.from_csr(B, bf16=True) as M:
        _, info = M.cg(torch.ones(n, dtype=torch.float64, device=DEV), mode=spmv.CG_PCG_BF16,
                       raise_on_error=False)
    assert info.status == spmv.SPMV_EBREAK


def _badly_scaled(nx, seed):
    # S A S for an SPD mesh matrix A, S = diag(s) with s log-uniform in
    # [1, 100]: SPD with a diagonal spread over four decades
    import scipy.sparse as sp
    A = mg.lattice(nx, nx, nx, "stencil27", seed=seed)
    s = np.exp(np.random.default_rng(seed).uniform(0.0, np.log(100.0), A.n_rows))
    S = (sp.diags(s) @ sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
         @ sp.diags(s)).tocsr()
    S.sort_indices()
    return mg.CSR(A.n_rows, A.n_cols, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


def _check_jacobi(A, b, tol, kappa):
    ref = oracle.pcg_jacobi(A, b, tol=tol, max_iter=20000)
    assert ref.status == 0
    with spmv.Matrix.from_csr(A) as M:
        bt = torch.as_tensor(b, device=DEV)
        x, info = M.cg(bt, tol=tol, mode=spmv.CG_PCG_JACOBI)
        x2, info2 = M.cg(bt, tol=tol, mode=spmv.CG_PCG_JACOBI)
    assert torch.equal(x, x2) and info2.iterations == info.iterations
    x = x.cpu().numpy()
    assert info.status == 0
    rr = true_rel_residual(A, x, b)
    assert rr <= 1.05 * tol and abs(info.rel_residual - rr) <= 0.05 * tol
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 2 * kappa * tol
    # both sides in binary64: the counts differ only by rounding order
    assert abs(info.iterations - ref.iterations) <= 0.1 * ref.iterations
    return info


def test_pcg_jacobi_badly_scaled_against_oracle():
    A = _badly_scaled(12, 71)
    b = mg.uniform(A.n_rows, 71, 1)
    tol = 1e-10
    D = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    np.add.at(D, (rows, A.col_idx), A.values)
    info = _check_jacobi(A, b, tol, np.linalg.cond(D))
    with spmv.Matrix.from_csr(A) as M:
        _, plain = M.cg(torch.as_tensor(b, device=DEV), tol=tol, mode=spmv.CG_FP64)
    assert info.iterations < 0.5 * plain.iterations


@pytest.mark.parametrize("name", ["config0", "C400K"])
def test_pcg_jacobi_mesh_against_oracle(name):
    # config0: the SpMV leaves few partials (alpha formed inside the update);
    # the Table 1 sized C400K stand-in: a separate reduction forms alpha
    A = mg.config0() if name == "config0" else mg.table1_matrix(name)
    b = mg.uniform(A.n_rows, 72, 1)
    with spmv.Matrix.from_csr(A) as M:
        n_seg = M.info["n_tiles"]
    assert (n_seg <= 1024) == (name == "config0")
    _check_jacobi(A, b, 1e-10, gershgorin_kappa(A, 1e-3))


def test_pcg_jacobi_diagonal_one_iteration():
    n = 4000
    d = np.random.default_rng(5).uniform(0.5, 50.0, n)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 4, 1)
    with spmv.Matrix.from_csr(A) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=1e-12, mode=spmv.CG_PCG_JACOBI)
    assert info.status == 0 and info.iterations == 1
    assert np.allclose(x.cpu().numpy(), b / d, rtol=1e-14)


def test_pcg_jacobi_rejects_sell_and_bad_diagonal():
    A = mg.config0()
    b = torch.ones(A.n_rows, dtype=torch.float64, device=DEV)
    with spmv.Matrix.from_csr(A, params={"format": spmv.FORMAT_SELL}) as M:
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(b, mode=spmv.CG_PCG_JACOBI)
        assert e.value.code == spmv.SPMV_ENOTSUP
    n = 64
    for bad in (-1.0, 0.0, float("nan")):
        d = np.ones(n)
        d[n // 2] = bad
        B = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
        with spmv.Matrix.from_csr(B) as M:
            _, info = M.cg(torch.ones(n, dtype=torch.float64, device=DEV), mode=spmv.CG_PCG_JACOBI,
                           raise_on_error=False)
        assert info.status == spmv.SPMV_EBREAK
        with spmv.Matrix.from_csr(B) as M:
            with pytest.raises(spmv.SpmvError, match="positive finite diagonal"):
                M.cg(torch.ones(n, dtype=torch.float64, device=DEV), mode=spmv.CG_PCG_JACOBI)


@pytest.mark.parametrize("mode", [spmv.CG_FP64, spmv.CG_PCG_BF16])
def test_table1_c400k_against_oracle(mode):
    # 398,000 rows: the SpMV leaves more than 1,024 p.q partials (alpha from a
    # reduction launch) and the x/r update at most 1,024 r.r partials (the
    # convergence test and beta formed inside the p update)
    A = mg.table1_matrix("C400K")
    b = mg.uniform(A.n_rows, 73, 1)
    tol = 1e-10
    if mode == spmv.CG_FP64:
        ref = oracle.cg(A, b, tol=tol, max_iter=20000)
    else:
        ref, _ = oracle.pcg_bf16(A, b, tol=tol, max_iter=20000)
    assert ref.status == 0
    with spmv.Matrix.from_csr(A, bf16=(mode == spmv.CG_PCG_BF16)) as M:
        assert M.info["n_tiles"] > 1024 and (A.n_rows + 1023) // 1024 <= 1024
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=tol, mode=mode)
    x = x.cpu().numpy()
    assert info.status == 0
    rr = true_rel_residual(A, x, b)
    assert rr <= 1.05 * tol and abs(info.rel_residual - rr) <= 0.05 * tol
    kappa = gershgorin_kappa(A, 1e-3)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 2 * kappa * tol
    assert abs(info.iterations - ref.iterations) <= 0.1 * ref.iterations


# -------------- one reduction per iteration (Chronopoulos-Gear, one launch)

def _cg1_params(tile=1024):
    return {"window_mode": spmv.WINDOW_OFF, "tile_nnz": tile}


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_cg1_first_iterates_match_the_oracle(cfg0, tile, k):
    # k steps from zero (tol = 0: the cap ends the solve) against the
    # oracle's k-step iterate (pinned to textbook CG): the two differ only in
    # summation order and fused multiply-adds, about 1e-16 relative a step;
    # a dropped term or a sign moves the iterate by O(1) from the second step
    A, b, _ = cfg0
    ref = oracle.cg1(A, b, tol=0.0, max_iter=k)
    assert ref.status == 1 and ref.iterations == k
    with spmv.Matrix.from_csr(A, params=_cg1_params(tile)) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=0.0, max_iter=k, mode=spmv.CG_FP64_ONE_REDUCTION,
                       raise_on_error=False)
    assert info.status == spmv.SPMV_ENOTCONV and info.iterations == k
    x = x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("name", ["config0", "C50K"])
def test_cg1_converges_like_the_oracle_and_textbook_cg(name):
    A = mg.config0() if name == "config0" else mg.table1_matrix(name)
    b = mg.uniform(A.n_rows, 17, 3)
    tol = 1e-10
    ref = oracle.cg1(A, b, tol=tol, max_iter=20000)
    assert ref.status == 0
    with spmv.Matrix.from_csr(A, params=_cg1_params()) as M:
        bd = torch.as_tensor(b, device=DEV)
        x, info = M.cg(bd, tol=tol, mode=spmv.CG_FP64_ONE_REDUCTION)
        x2, _ = M.cg(bd, tol=tol, mode=spmv.CG_FP64_ONE_REDUCTION)
        _, info_hs = M.cg(bd, tol=tol, mode=spmv.CG_FP64)
    assert torch.equal(x, x2)  # bitwise reproducible
    x = x.cpu().numpy()
    rr = true_rel_residual(A, x, b)
    assert info.status == 0 and rr <= 1.05 * tol and abs(info.rel_residual - rr) <= 0.05 * tol
    assert abs(info.iterations - ref.iterations) <= 0.1 * ref.iterations
    assert abs(info.iterations - info_hs.iterations) <= 0.1 * info_hs.iterations
    kappa = gershgorin_kappa(A, 1e-3) if name == "config0" else None
    if kappa:
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 2 * kappa * tol


def test_cg1_on_the_largest_table1_system():
    # C800K: 3,753 tiles, close to the 4,096 every workgroup sums itself
    A = mg.table1_matrix("C800K")
    b = mg.uniform(A.n_rows, 18, 3)
    tol = 1e-10
    with spmv.Matrix.from_csr(A, params=_cg1_params()) as M:
        assert M.info["n_tiles"] == 3753
        bd = torch.as_tensor(b, device=DEV)
        x, info = M.cg(bd, tol=tol, mode=spmv.CG_FP64_ONE_REDUCTION)
        _, info_hs = M.cg(bd, tol=tol, mode=spmv.CG_FP64)
    rr = true_rel_residual(A, x.cpu().numpy(), b)
    assert info.status == 0 and rr <= 1.05 * tol
    assert abs(info.iterations - info_hs.iterations) <= 0.1 * info_hs.iterations


def test_cg1_restarts_from_the_true_residual():
    # at tol = 1e-15 the recursive r.r meets the tolerance before the true
    # residual does (the oracle restarts too); the solve restarts from
    # r = b - A x and ends near the binary64 floor
    A = mg.lattice(6, 5, 5, "stencil27", seed=94, shift=0.1)
    b = mg.uniform(A.n_rows, 94, 1)
    ref = oracle.cg1(A, b, tol=1e-15, max_iter=600)
    assert ref.status == 0 and ref.alphas[0] >= 1
    with spmv.Matrix.from_csr(A, params=_cg1_params()) as M:
        x, info = M.cg(torch.as_tensor(b, device=DEV), tol=1e-15, max_iter=600,
                       mode=spmv.CG_FP64_ONE_REDUCTION, raise_on_error=False)
    assert info.status in (spmv.SPMV_OK, spmv.SPMV_ENOTCONV) and info.refinements >= 1
    assert true_rel_residual(A, x.cpu().numpy(), b) <= 1e-14


def test_cg1_breakdown_zero_rhs_and_rejections(cfg0):
    # w.r = 0 at the start on an indefinite diagonal system (the oracle
    # breaks down before its first step too)
    n = 64
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.zeros(n)
    b[0], b[1] = 1.0, 1.0
    ref = oracle.cg1(A, b, tol=1e-10, max_iter=100)
    assert ref.status == 2 and ref.iterations == 0
    with spmv.Matrix.from_csr(A, params=_cg1_params()) as M:
        _, info = M.cg(torch.as_tensor(b, device=DEV), mode=spmv.CG_FP64_ONE_REDUCTION, raise_on_error=False)
        assert info.status == spmv.SPMV_EBREAK and info.iterations == 0
    # a later breakdown at the oracle's step
    n = 200
    d = np.linspace(1.0, 10.0, n)
    d[-3:] = -np.linspace(0.5, 5.0, 3)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.ones(n)
    ref = oracle.cg1(A, b, tol=1e-10, max_iter=1000)
    assert ref.status == 2
    with spmv.Matrix.from_csr(A, params=_cg1_params()) as M:
        _, info = M.cg(torch.as_tensor(b, device=DEV), tol=1e-10, max_iter=1000,
                       mode=spmv.CG_FP64_ONE_REDUCTION, raise_on_error=False)
    assert info.status == spmv.SPMV_EBREAK and info.iterations == ref.iterations
    A0, b0, _ = cfg0
    with spmv.Matrix.from_csr(A0, params=_cg1_params()) as M:
        x, info = M.cg(torch.zeros(A0.n_rows, dtype=torch.float64, device=DEV), mode=spmv.CG_FP64_ONE_REDUCTION)
        assert info.status == 0 and info.iterations == 0 and not x.any()
    with spmv.Matrix.from_csr(A0, params={"window_mode": spmv.WINDOW_RING}) as M:  # not plain row tiles
        with pytest.raises(spmv.SpmvError) as e:
            M.cg(torch.as_tensor(b0, device=DEV), mode=spmv.CG_FP64_ONE_REDUCTION)
        assert e.value.code == spmv.SPMV_ENOTSUP and "one-reduction" in str(e.value)
