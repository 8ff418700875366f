"""Pins for the CPU oracle: each check is fixed by mathematics or by an
independent implementation, never by re-running the oracle's own formula.

* exact rational brute force (fractions.Fraction) on irregular CSR with empty
  rows, a dense row, duplicate entries and unsorted columns;
* dyadic inputs whose every product and partial sum is exact in binary64, so
  the oracle must equal the rational result bit for bit;
* the pure-Neumann Laplacian (shift 0) annihilates constants, and with shift
  s, A(c 1) = s c 1;
* symmetry x.(Ay) = y.(Ax) of the mesh matrices;
* permutation equivariance (P A P^T)(P x) = P (A x) (reordering keeps the
  coefficients, paper Sec. 4.1);
* linearity; scipy's CSR product and numpy's dense product (independent code);
* CG: one-step closed form on A 1 = s 1, termination in d steps for d
  distinct eigenvalues, rational-arithmetic CG that ends with the exact
  solution within n steps, a dense LAPACK solve, Ritz values from the
  alpha/beta recurrences;
* planted mistakes (dropped term, wrong sign, transposed operand, shifted
  column) are caught by the pins above.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
import oracle


def exact_rows(A, x):
    """Exact y_i (Fraction) and exact bound_i for every row."""
    ys, bs = [], []
    xf = [Fraction(float(v)) for v in x]
    for i in range(A.n_rows):
        s = Fraction(0)
        b = Fraction(0)
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            a = Fraction(float(A.values[k]))
            xv = xf[int(A.col_idx[k])]
            s += a * xv
            b += abs(a) * abs(xv)
        ys.append(s)
        bs.append(b)
    return ys, bs


def bruteforce_ok(A, x, y) -> bool:
    """|y_i - exact_i| <= gamma_m * exact_bound_i for every row (m = row length)."""
    ys, bs = exact_rows(A, x)
    lens = np.diff(A.row_ptr)
    for i in range(A.n_rows):
        g = Fraction(float(oracle.gamma(max(int(lens[i]), 1)))) * Fraction(1000001, 1000000)
        if abs(Fraction(float(y[i])) - ys[i]) > g * bs[i]:
            return False
    return True


CASES = [
    dict(n_rows=40, n_cols=37, seed=1, dense_rows=1),
    dict(n_rows=64, n_cols=64, seed=2, duplicates=True),
    dict(n_rows=50, n_cols=30, seed=3, unsorted=True, empty_frac=0.3),
    dict(n_rows=33, n_cols=60, seed=4, duplicates=True, unsorted=True, dense_rows=2),
    dict(n_rows=1, n_cols=1, seed=5, empty_frac=0.0),
    dict(n_rows=20, n_cols=20, seed=6, empty_frac=1.0),
]


@pytest.mark.parametrize("case", CASES)
def test_spmv_bruteforce_exact(case):
    A = mg.random_csr(**case)
    x = np.random.default_rng(case["seed"] + 100).uniform(-1, 1, A.n_cols)
    y, bound = oracle.spmv(A, x)
    assert bruteforce_ok(A, x, y)
    _, bs = exact_rows(A, x)
    lens = np.maximum(np.diff(A.row_ptr), 1)
    for i in range(A.n_rows):
        assert abs(Fraction(float(bound[i])) - bs[i]) <= Fraction(float(oracle.gamma(lens[i]))) * bs[i]
    # empty rows give exactly zero
    empty = np.diff(A.row_ptr) == 0
    assert np.all(y[empty] == 0.0) and np.all(bound[empty] == 0.0)


def _dyadic_mats():
    return [
        mg.lattice(6, 5, 4, "extras", seed=11, dyadic=True),
        mg.lattice(5, 5, 5, "stencil27", seed=12, dyadic=True),
        mg.knn(5, seed=13, dyadic=True),
        mg.reorder(mg.lattice(6, 6, 3, "extras", seed=14, dyadic=True), "rcm", 14),
    ]


@pytest.mark.parametrize("idx", range(4))
def test_spmv_dyadic_bitwise(idx):
    A = _dyadic_mats()[idx]
    x = mg.dyadic_x(A.n_cols, seed=idx)
    y, _ = oracle.spmv(A, x)
    ys, _ = exact_rows(A, x)
    assert all(Fraction(float(y[i])) == ys[i] for i in range(A.n_rows))


def test_neumann_rows_sum_to_zero():
    A = mg.lattice(7, 6, 5, "extras", seed=21, shift=0.0, dyadic=True)
    y, _ = oracle.spmv(A, np.full(A.n_cols, 0.375))
    assert np.all(y == 0.0)
    B = mg.knn(8, seed=22, shift=0.0)
    y, b = oracle.spmv(B, np.full(B.n_cols, -1.25))
    assert np.all(np.abs(y) <= 1e-12 * b)


def test_shifted_constant_closed_form():
    A = mg.lattice(7, 6, 5, "stencil27", seed=23, dyadic=True)
    y, _ = oracle.spmv(A, np.full(A.n_cols, 3.0))
    assert np.all(y == 3.0 * 2.0 ** -10)
    B = mg.config0()
    y, b = oracle.spmv(B, np.full(B.n_cols, 2.0))
    assert np.all(np.abs(y - 2e-3) <= 1e-12 * b)


def test_symmetry_xAy_equals_yAx():
    for A in (mg.config0(), mg.knn(12, seed=31), mg.lattice(10, 9, 8, "stencil27", seed=32)):
        x = mg.uniform(A.n_cols, 1, 0)
        z = mg.uniform(A.n_cols, 2, 0)
        Az, bz = oracle.spmv(A, z)
        Ax, _ = oracle.spmv(A, x)
        lhs = float(np.dot(x, Az))
        rhs = float(np.dot(z, Ax))
        scale = float(np.dot(np.abs(x), bz))
        assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("ordering", ["rcm", "random"])
def test_permutation_equivariance(ordering):
    A = mg.lattice(8, 7, 6, "extras", seed=41, dyadic=True)
    perm = mg.rcm_perm(A) if ordering == "rcm" else mg.random_perm(A.n_rows, 41)
    B = mg.permute(A, perm)
    x = mg.dyadic_x(A.n_cols, seed=3)
    yA, _ = oracle.spmv(A, x)
    yB, _ = oracle.spmv(B, x[perm])
    assert np.array_equal(yB, yA[perm])
    # non-dyadic: within the bound
    A2 = mg.knn(10, seed=42)
    perm2 = mg.random_perm(A2.n_rows, 5)
    B2 = mg.permute(A2, perm2)
    x2 = mg.uniform(A2.n_cols, 7, 0)
    y2, b2 = oracle.spmv(A2, x2)
    yp, _ = oracle.spmv(B2, x2[perm2])
    assert np.all(np.abs(yp - y2[perm2]) <= 1e-12 * b2[perm2])


def test_linearity():
    A = mg.knn(10, seed=51)
    x = mg.uniform(A.n_cols, 8, 0)
    z = mg.uniform(A.n_cols, 9, 0)
    a = -0.7
    y1, b1 = oracle.spmv(A, a * x + z)
    yx, bx = oracle.spmv(A, x)
    yz, bz = oracle.spmv(A, z)
    assert np.all(np.abs(y1 - (a * yx + yz)) <= 1e-12 * (abs(a) * bx + bz))


@pytest.mark.parametrize("case", CASES[:4])
def test_against_scipy_csr(case):
    A = mg.random_csr(**case)
    x = np.random.default_rng(7).uniform(-1, 1, A.n_cols)
    S = sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
    y, b = oracle.spmv(A, x)
    m = np.maximum(np.diff(A.row_ptr), 1)
    assert np.all(np.abs(y - S @ x) <= 2 * oracle.gamma(m) * b + 0.0)


def test_all_cores_timing_build_gives_the_same_bits():
    # the OpenMP build only splits rows between threads; each row is the
    # checker's sum, so the results are identical
    A = mg.knn(24, seed=33)
    x = mg.uniform(A.n_cols, 4, 1)
    y, _ = oracle.spmv(A, x)
    assert np.array_equal(oracle.spmv_all_cores(A, x), y)
    assert oracle.all_cores_threads() >= 1


def test_spmv_rows_matches_full():
    A = mg.config0()
    x = mg.uniform(A.n_cols, 4, 0)
    y, b = oracle.spmv(A, x)
    rows = np.array([0, 5, A.n_rows - 1, 1234, 1234], np.int32)
    ys, bs = oracle.spmv_rows(A, x, rows)
    assert np.array_equal(ys, y[rows]) and np.array_equal(bs, b[rows])


def _dense_bsr(A):
    n = A.n_rows
    D = np.zeros((3 * n, 3 * A.n_cols))
    for br in range(n):
        for q in range(A.row_ptr[br], A.row_ptr[br + 1]):
            bc = A.col_idx[q]
            D[3 * br:3 * br + 3, 3 * bc:3 * bc + 3] += A.values[q]
    return D


@pytest.mark.parametrize("k", [1, 4, 8])
def test_bsr3_against_dense(k):
    A = mg.bsr3(6, 5, 4, seed=61)
    X = mg.uniform(3 * A.n_cols * k, 10, 0).reshape(3 * A.n_cols, k)
    Y, B = oracle.bsr3_spmm(A, X)
    D = _dense_bsr(A)
    lens = 3 * np.repeat(np.diff(A.row_ptr), 3)[:, None]
    assert np.all(np.abs(Y - D @ X) <= 2 * oracle.gamma(lens) * B)
    # each right-hand side equals the one-column product of that column
    for j in range(k):
        yj, _ = oracle.bsr3_spmm(A, X[:, j:j + 1].copy())
        assert np.array_equal(yj[:, 0], Y[:, j])


def test_bsr3_generator_diagonal_dominance():
    A = mg.bsr3(5, 4, 3, seed=62)
    D = _dense_bsr(A)
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.allclose(np.diag(D), 1.0 + off, rtol=1e-13)


# --------------------------------------------------------------- CG pins

def test_cg_closed_form_one_step_dyadic():
    A = mg.lattice(6, 6, 5, "extras", seed=71, dyadic=True)
    b = np.ones(A.n_rows)
    r = oracle.cg(A, b, tol=1e-12, max_iter=50)
    assert r.status == 0 and r.iterations == 1
    assert np.all(r.x == 2.0 ** 10)
    assert r.rel_residual == 0.0


def test_cg_closed_form_one_step():
    A = mg.config0()
    r = oracle.cg(A, np.ones(A.n_rows), tol=1e-10, max_iter=50)
    assert r.status == 0 and r.iterations == 1
    assert np.allclose(r.x, 1000.0, rtol=1e-9)


def test_cg_terminates_in_d_steps_for_d_eigenvalues():
    n, evals = 60, np.array([1.0, 2.5, 4.0, 7.0])
    d = np.repeat(evals, n // len(evals))
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 3, 0)
    r = oracle.cg(A, b, tol=1e-12, max_iter=100)
    assert r.status == 0 and r.iterations <= len(evals)
    assert np.allclose(r.x, b / d, rtol=1e-11)


def _dense(A):
    S = sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
    return S.toarray()


def _exact_cg(D, b):
    """Conjugate gradients in rational arithmetic; returns (x, steps)."""
    n = len(b)
    A = [[Fraction(v) for v in row] for row in D]
    mv = lambda v: [sum(A[i][j] * v[j] for j in range(n)) for i in range(n)]
    dt = lambda u, v: sum(a * c for a, c in zip(u, v))
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    p = list(r)
    rho = dt(r, r)
    steps = 0
    while rho != 0:
        q = mv(p)
        alpha = rho / dt(p, q)
        x = [xi + alpha * pi for xi, pi in zip(x, p)]
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        steps += 1
        rho_new = dt(r, r)
        if rho_new == 0:
            break
        p = [ri + (rho_new / rho) * pi for ri, pi in zip(r, p)]
        rho = rho_new
        assert steps <= n, "exact CG must end within n steps"
    return x, steps


@pytest.mark.parametrize("n", [3, 5, 8])
def test_cg_exact_arithmetic_finite_termination(n):
    # a small SPD mesh-style matrix with dyadic entries: exact CG reaches A x = b
    # exactly in at most n steps; the oracle's binary64 CG lands within
    # kappa * tol of that exact solution
    rng = np.random.default_rng(100 + n)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if j == i + 1 or rng.random() < 0.3:
                D[i, j] = D[j, i] = -float(rng.integers(4, 13)) / 8.0
    np.fill_diagonal(D, -D.sum(axis=1) + 0.25)
    b = rng.integers(-8, 9, n).astype(float) / 4.0
    b[0] = 1.0
    x_exact, steps = _exact_cg(D, b)
    assert steps <= n
    A_f = [[Fraction(v) for v in row] for row in D]
    assert [sum(A_f[i][j] * x_exact[j] for j in range(n)) for i in range(n)] == [Fraction(v) for v in b]
    S = sp.csr_matrix(D)
    A = mg.CSR(n, n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    tol = 1e-12
    r = oracle.cg(A, b, tol=tol, max_iter=10 * n)
    xe = np.array([float(v) for v in x_exact])
    assert r.status == 0
    assert np.linalg.norm(r.x - xe) / np.linalg.norm(xe) <= 2 * np.linalg.cond(D) * tol


def test_cg_against_dense_lapack_solve():
    A = mg.lattice(5, 4, 4, "extras", seed=81, shift=0.05)
    D = _dense(A)
    b = mg.uniform(A.n_rows, 81, 1)
    tol = 1e-10
    r = oracle.cg(A, b, tol=tol, max_iter=1000)
    xs = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert r.status == 0
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 2 * kappa * tol
    # self-certification with an independent (dense) residual
    assert np.linalg.norm(b - D @ r.x) / np.linalg.norm(b) <= tol * 1.01
    assert abs(r.rel_residual - np.linalg.norm(b - D @ r.x) / np.linalg.norm(b)) <= 1e-3 * tol


def test_cg_ritz_values_match_extreme_eigenvalues():
    A = mg.lattice(6, 5, 5, "stencil27", seed=91, shift=0.1)
    D = _dense(A)
    b = mg.uniform(A.n_rows, 91, 1)
    r = oracle.cg(A, b, tol=1e-14, max_iter=400)
    k = r.iterations
    al, be = r.alphas, r.betas
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / al[j] + (be[j - 1] / al[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(be[j]) / al[j]
    ritz = np.linalg.eigvalsh(T)
    ev = np.linalg.eigvalsh(D)
    assert abs(ritz[-1] - ev[-1]) <= 1e-8 * ev[-1]
    assert abs(ritz[0] - ev[0]) <= 1e-6 * ev[-1]


def test_cg_zero_rhs_and_max_iter():
    A = mg.config0()
    r = oracle.cg(A, np.zeros(A.n_rows), tol=1e-10)
    assert r.status == 0 and r.iterations == 0 and np.all(r.x == 0)
    b = mg.uniform(A.n_rows, 5, 1)
    r = oracle.cg(A, b, tol=1e-12, max_iter=3)
    assert r.status == 1 and r.iterations == 3 and r.rel_residual > 1e-12


# ---------------- CG with one reduction phase per iteration (Chronopoulos-Gear)

def test_cg1_first_iterate_closed_form():
    # x0 = 0: x1 = alpha0 r0 = (b.b / b.Ab) b
    A = mg.lattice(6, 5, 5, "stencil27", seed=93, shift=0.1)
    b = mg.uniform(A.n_rows, 93, 1)
    D = _dense(A)
    r = oracle.cg1(A, b, tol=0.0, max_iter=1)
    assert r.status == 1 and r.iterations == 1
    alpha0 = (b @ b) / (b @ (D @ b))
    assert np.allclose(r.x, alpha0 * b, rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("k", [2, 5, 12])
def test_cg1_iterates_match_textbook_cg(k):
    # the same Krylov iterates as Hestenes-Stiefel CG (pinned above) in exact
    # arithmetic; in binary64 they agree to rounding over the first steps
    # (a dropped beta s term, a wrong sign or alpha = gamma / delta alone
    # moves them by O(1) from the second step on)
    A = mg.lattice(6, 5, 5, "stencil27", seed=94, shift=0.1)
    b = mg.uniform(A.n_rows, 94, 1)
    r1 = oracle.cg1(A, b, tol=0.0, max_iter=k)
    r0 = oracle.cg(A, b, tol=0.0, max_iter=k)
    assert r1.iterations == r0.iterations == k
    assert np.linalg.norm(r1.x - r0.x) <= 1e-13 * np.linalg.norm(r0.x)


def test_cg1_terminates_in_d_steps_for_d_eigenvalues():
    n, evals = 60, np.array([1.0, 2.5, 4.0, 7.0])
    d = np.repeat(evals, n // len(evals))
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 3, 0)
    r = oracle.cg1(A, b, tol=1e-12, max_iter=100)
    assert r.status == 0 and r.iterations <= len(evals)
    assert np.allclose(r.x, b / d, rtol=1e-11)


def test_cg1_against_dense_lapack_solve():
    A = mg.lattice(5, 4, 4, "extras", seed=81, shift=0.05)
    D = _dense(A)
    b = mg.uniform(A.n_rows, 81, 1)
    tol = 1e-10
    r = oracle.cg1(A, b, tol=tol, max_iter=1000)
    xs = np.linalg.solve(D, b)
    assert r.status == 0
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 2 * np.linalg.cond(D) * tol
    assert np.linalg.norm(b - D @ r.x) / np.linalg.norm(b) <= tol * 1.01
    assert abs(r.rel_residual - np.linalg.norm(b - D @ r.x) / np.linalg.norm(b)) <= 1e-3 * tol


def test_cg1_restarts_from_the_true_residual_when_the_recurrence_drifts():
    # at tol = 1e-15 the recursive r.r falls below tol^2 ||b||^2 before the
    # true residual does: the solve restarts from r = b - A x and still ends
    # below tol (the restart count is returned as the only element of alphas)
    A = mg.lattice(6, 5, 5, "stencil27", seed=94, shift=0.1)
    b = mg.uniform(A.n_rows, 94, 1)
    D = _dense(A)
    r = oracle.cg1(A, b, tol=1e-15, max_iter=600)
    assert r.status == 0 and r.alphas[0] >= 1
    assert np.linalg.norm(b - D @ r.x) / np.linalg.norm(b) <= 1e-15


def test_cg1_zero_rhs_and_max_iter():
    A = mg.config0()
    r = oracle.cg1(A, np.zeros(A.n_rows), tol=1e-10)
    assert r.status == 0 and r.iterations == 0 and np.all(r.x == 0)
    b = mg.uniform(A.n_rows, 5, 1)
    r = oracle.cg1(A, b, tol=1e-12, max_iter=3)
    assert r.status == 1 and r.iterations == 3 and r.rel_residual > 1e-12


# ------------------------------------- preconditioned CG (bfloat16 copy)

def _bf16_bits_round(a):
    """bfloat16 rounding of float32(a) by the usual bit recipe (add 0x7fff plus
    the lowest kept bit, truncate) -- a second, independent route to the
    nearest-even 8-bit significand."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_pcg_diagonal_matrix_one_iteration():
    # A = D with bfloat16-exact entries: the Gershgorin weight is 1.9 / 1 and
    # M^-1 A = 1.9 (2 - 1.9) I, so one step solves the system exactly
    n = 40
    d = np.tile([1.0, 2.5, 4.0, 7.0, 0.375], n // 5)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 4, 0)
    r, w = oracle.pcg_bf16(A, b, tol=1e-12, max_iter=20)
    assert w == 1.9
    assert r.status == 0 and r.iterations == 1
    assert np.allclose(r.x, b / d, rtol=1e-14)


def test_pcg_weight_uses_bfloat16_values():
    # one row [a]: g = |bf16(a)| / a, so w = 1.9 a / bf16(a); rounding checked
    # against the bit recipe on values that round down, up and to even
    for a in (1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, 3.14159, 0.1, 1234.5678, 1.0 + 2.0 ** -8):
        A = mg.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([a]))
        _, w = oracle.pcg_bf16(A, np.ones(1), tol=1e-12, max_iter=5)
        # a wrong rounding moves bf16(a) by 2^-8 relative; w is formed in a
        # different order here, so compare to a few ulps
        ref = 1.9 / (_bf16_bits_round(a) / a)
        assert abs(w - ref) <= 1e-14 * ref, a


def test_pcg_preconditioner_is_spd_and_helps():
    A = mg.lattice(6, 6, 5, "stencil27", seed=95)
    D = _dense(A)
    vt = np.zeros_like(D)
    vt[np.nonzero(D)] = _bf16_bits_round(D[np.nonzero(D)])
    dinv = 1.0 / np.diag(D)
    g = np.max(np.abs(vt).dot(np.sqrt(dinv)) * np.sqrt(dinv))
    w = 1.9 / g
    Minv = w * np.diag(dinv) @ (2 * np.eye(len(dinv)) - w * vt @ np.diag(dinv))
    assert np.allclose(Minv, Minv.T, atol=1e-14) and np.linalg.eigvalsh(Minv).min() > 0
    b = mg.uniform(A.n_rows, 95, 1)
    r_cg = oracle.cg(A, b, tol=1e-10, max_iter=5000)
    r_p, w_o = oracle.pcg_bf16(A, b, tol=1e-10, max_iter=5000)
    assert abs(w_o - w) <= 1e-12 * w
    assert r_p.status == 0 and r_p.iterations < 0.8 * r_cg.iterations


def test_pcg_against_dense_lapack_solve():
    A = mg.lattice(5, 4, 4, "extras", seed=83, shift=0.05)
    D = _dense(A)
    b = mg.uniform(A.n_rows, 83, 1)
    tol = 1e-10
    r, _ = oracle.pcg_bf16(A, b, tol=tol, max_iter=1000)
    xs = np.linalg.solve(D, b)
    assert r.status == 0
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 2 * np.linalg.cond(D) * tol
    assert np.linalg.norm(b - D @ r.x) / np.linalg.norm(b) <= tol * 1.01


def test_pcg_zero_rhs_and_bad_diagonal():
    A = mg.config0()
    r, _ = oracle.pcg_bf16(A, np.zeros(A.n_rows), tol=1e-10)
    assert r.status == 0 and r.iterations == 0 and np.all(r.x == 0)
    B = mg.CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    r, _ = oracle.pcg_bf16(B, np.ones(2), tol=1e-10)
    assert r.status == 3


def _dense_bf16_pcg(Ad, b, k, w=None, rounded=True):
    """k steps of textbook preconditioned CG (Saad, Alg. 9.1) from x0 = 0 in
    dense numpy, with the preconditioner formed here as a dense matrix:
    A~ = the bfloat16 rounding of A's entries by the bit recipe (or A itself
    when rounded is False), w = 1.9 / max_i sum_j |a~_ij| / sqrt(d_i d_j)
    unless given, M^-1 = w D^-1 (2 I - w A~ D^-1).  Returns (x_k, w)."""
    nz = np.nonzero(Ad)
    At = np.zeros_like(Ad)
    At[nz] = _bf16_bits_round(Ad[nz]) if rounded else Ad[nz]
    dinv = 1.0 / np.diag(Ad)
    if w is None:
        w = 1.9 / np.max(np.abs(At) @ np.sqrt(dinv) * np.sqrt(dinv))
    Dinv = np.diag(dinv)
    Minv = w * Dinv @ (2.0 * np.eye(len(b)) - w * At @ Dinv)
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv @ r
    p = z.copy()
    rho = r @ z
    for _ in range(k):
        q = Ad @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = Minv @ r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, w


@pytest.mark.parametrize("k", [1, 3, 6])
def test_pcg_bf16_iterates_match_a_dense_preconditioner(k):
    # The preconditioner's action is pinned through the iterates: after k
    # steps from zero the oracle's x must equal dense PCG with an explicitly
    # built M^-1 in the bfloat16 copy.  Values U[0.5, 1.5) are not bfloat16
    # numbers, so reading the binary64 values instead of the rounded copy
    # moves the iterate by about 2^-9 relative, and any change of the
    # polynomial's coefficients moves it by far more; the tolerance is the
    # rounding noise of two summation orders over six steps.
    A = mg.lattice(6, 5, 5, "stencil27", seed=97)
    Ad = _dense(A)
    assert np.count_nonzero(Ad) == A.nnz
    b = mg.uniform(A.n_rows, 97, 1)
    x_ref, w_ref = _dense_bf16_pcg(Ad, b, k)
    r, w = oracle.pcg_bf16(A, b, tol=0.0, max_iter=k)
    assert r.status == 1 and r.iterations == k
    assert abs(w - w_ref) <= 1e-14 * w_ref
    scale = np.max(np.abs(x_ref))
    assert np.max(np.abs(r.x - x_ref)) <= 1e-12 * scale
    # the pin can see the rounding: the same steps with the binary64 values
    # in the polynomial (same weight) land more than 1000x the tolerance away
    x64, _ = _dense_bf16_pcg(Ad, b, k, w=w_ref, rounded=False)
    assert np.max(np.abs(x64 - x_ref)) > 1e-9 * scale


# ------------------------------------- preconditioned CG (Jacobi)

def _badly_scaled(seed):
    """S A S for an SPD mesh matrix A and S = diag(s), s log-uniform in
    [1, 100]: still SPD, with a diagonal spread over four decades."""
    A = mg.lattice(6, 6, 5, "stencil27", seed=seed)
    s = np.exp(np.random.default_rng(seed).uniform(0.0, np.log(100.0), A.n_rows))
    S = sp.diags(s) @ sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols)) @ sp.diags(s)
    S = S.tocsr()
    S.sort_indices()
    return mg.CSR(A.n_rows, A.n_cols, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


def test_pcg_jacobi_diagonal_system_one_iteration():
    # A = D: z = D^-1 b is the solution and alpha = 1, so one step solves it
    n = 37
    d = np.random.default_rng(5).uniform(0.5, 50.0, n)
    A = mg.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = mg.uniform(n, 4, 1)
    r = oracle.pcg_jacobi(A, b, tol=1e-12, max_iter=20)
    assert r.status == 0 and r.iterations == 1
    assert np.allclose(r.x, b / d, rtol=1e-14)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_pcg_jacobi_is_cg_on_the_symmetrically_scaled_system(k):
    # with M = D, the PCG iterates are x_k = D^-1/2 y_k, y_k the CG iterates
    # for D^-1/2 A D^-1/2 y = D^-1/2 b (both from zero); the scaled system is
    # formed here with scipy and solved by the plain CG oracle
    A = _badly_scaled(61)
    Ad = _dense(A)
    dh = 1.0 / np.sqrt(np.diag(Ad))
    Sc = sp.csr_matrix(dh[:, None] * Ad * dh[None, :])
    As = mg.CSR(A.n_rows, A.n_cols, Sc.indptr.astype(np.int32), Sc.indices.astype(np.int32), Sc.data)
    b = mg.uniform(A.n_rows, 61, 1)
    y = oracle.cg(As, dh * b, tol=0.0, max_iter=k)
    x = oracle.pcg_jacobi(A, b, tol=0.0, max_iter=k)
    assert x.status == 1 and y.status == 1 and x.iterations == y.iterations == k
    assert np.linalg.norm(x.x - dh * y.x) <= 1e-11 * np.linalg.norm(x.x)


def test_pcg_jacobi_helps_on_a_badly_scaled_diagonal_and_matches_lapack():
    A = _badly_scaled(62)
    Ad = _dense(A)
    b = mg.uniform(A.n_rows, 62, 1)
    tol = 1e-10
    r_cg = oracle.cg(A, b, tol=tol, max_iter=20000)
    r = oracle.pcg_jacobi(A, b, tol=tol, max_iter=20000)
    assert r.status == 0 and r_cg.status == 0
    assert r.iterations < 0.5 * r_cg.iterations
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 2 * np.linalg.cond(Ad) * tol
    assert np.linalg.norm(b - Ad @ r.x) / np.linalg.norm(b) <= tol * 1.01


def test_pcg_jacobi_zero_rhs_bad_diagonal_and_max_iter():
    A = mg.config0()
    r = oracle.pcg_jacobi(A, np.zeros(A.n_rows), tol=1e-10)
    assert r.status == 0 and r.iterations == 0 and np.all(r.x == 0)
    B = mg.CSR(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    assert oracle.pcg_jacobi(B, np.ones(2), tol=1e-10).status == 3
    r = oracle.pcg_jacobi(A, mg.uniform(A.n_rows, 3, 0), tol=1e-14, max_iter=4)
    assert r.status == 1 and r.iterations == 4


# -------------------------------------------------- planted mistakes

def _mutant_dropped_term(A):
    keep = np.ones(A.nnz, bool)
    ends = A.row_ptr[1:][np.diff(A.row_ptr) > 0] - 1
    keep[ends] = False
    rp = np.concatenate([[0], np.cumsum(np.diff(A.row_ptr) - (np.diff(A.row_ptr) > 0))]).astype(np.int32)
    return mg.CSR(A.n_rows, A.n_cols, rp, A.col_idx[keep], A.values[keep])


def _mutant_sign(A):
    v = A.values.copy()
    v[A.nnz // 2] = -v[A.nnz // 2]
    return mg.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, v)


def _mutant_shifted_col(A):
    return mg.CSR(A.n_rows, A.n_cols, A.row_ptr, (A.col_idx + 1) % A.n_cols, A.values)


def _mutant_transpose(A):
    S = sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols)).T.tocsr()
    return mg.CSR(S.shape[0], S.shape[1], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


@pytest.mark.parametrize("mutant", [_mutant_dropped_term, _mutant_sign, _mutant_shifted_col,
                                    _mutant_transpose])
def test_pins_catch_planted_mistakes(mutant):
    A = mg.random_csr(48, 48, seed=99, mean_len=5.0, empty_frac=0.05)
    x = np.random.default_rng(3).uniform(-1, 1, A.n_cols)
    y_bad, _ = oracle.spmv(mutant(A), x)
    assert not bruteforce_ok(A, x, y_bad)
    y_good, _ = oracle.spmv(A, x)
    assert bruteforce_ok(A, x, y_good)
