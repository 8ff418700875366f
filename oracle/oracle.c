/*
 * oracle.c -- plain CPU reference for the sparse matrix-vector product and
 * for conjugate gradients.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the library's product path never does.  It
 * shares no code, header or helper with the GPU library.
 *
 * Precision: binary64 throughout, compiled with -ffp-contract=off so every
 * product and sum is rounded separately, in ascending index order, single
 * threaded.  Obviously correct beats fast here.  A second build of this same
 * file with OpenMP (liboracle_omp.so) exists only to time oracle_spmv on all
 * host cores; it splits rows between threads and changes no row's sum.
 *
 * What is computed and where it comes from:
 *
 *  oracle_spmv     y = A x for A in CSR (values, column indices, row
 *                  pointers; binary64 values and 4-byte column indices as in
 *                  the paper's storage format, Sec. 4.2).  The paper's naive
 *                  and cached kernels (Secs. 4.3, 5.1, 5.2) are
 *                  reorganisations of this same per-row sum: reordering
 *                  keeps the coefficients (Sec. 4.1), padding adds exact
 *                  zeros (Sec. 4.2, 5.2) and the cache-relative indices only
 *                  change addressing (Sec. 5.1).  So the oracle is the
 *                  definition: y_i = sum_k values[k] * x[col_idx[k]].
 *                  It also returns bound_i = sum_k |values[k]| * |x[col_idx[k]]|,
 *                  the scale of the dot-product forward error bound
 *                  (|fl(y_i) - y_i| <= gamma_m * bound_i, Higham, Accuracy and
 *                  Stability of Numerical Algorithms, Sec. 3.1).
 *  oracle_spmv_rows  the same for a list of sampled rows only.
 *  oracle_bsr3_spmm  Y = A X for a 3x3 block-CSR A and k right-hand sides
 *                  (X row-major, n_cols*3 by k); per scalar row the same sum
 *                  over the row's stored blocks and their three columns.
 *  oracle_cg       Hestenes-Stiefel conjugate gradients (Hestenes & Stiefel,
 *                  J. Res. NBS 49, 1952) for SPD A.  The paper names only "the
 *                  linear solver" (Sec. 2); this is the textbook method with
 *                  x0 given, stopping on the recursive residual and confirming
 *                  with the true residual b - A x before returning.
 *  oracle_pcg_bf16 conjugate gradients preconditioned with a polynomial in a
 *                  bfloat16 copy of A (the scope's "BF16 for the preconditioner
 *                  copy"): with D = diag(A), A~ = A's values rounded to
 *                  binary32 and then to bfloat16 (8 significant bits, nearest,
 *                  ties to even), the damped two-term Neumann series
 *                      M^-1 r = w D^-1 (2 r - w A~ D^-1 r),
 *                  i.e. w D^-1 sum_{k<2} (I - w A~ D^-1)^k, and the weight
 *                  w = 1.9 / g with g = max_i sum_j |a~_ij| / sqrt(d_i d_j), a
 *                  Gershgorin bound on the spectrum of D^-1/2 A~ D^-1/2, so M^-1
 *                  is symmetric positive definite (M^-1 = 2w D^-1 - w^2
 *                  D^-1 A~ D^-1, positive iff w * lambda_max < 2).  Standard
 *                  preconditioned CG (e.g. Saad, Iterative Methods for Sparse
 *                  Linear Systems, Alg. 9.1) on top, stopping and confirming as
 *                  oracle_cg does.
 *  oracle_cg1      conjugate gradients with one reduction phase per
 *                  iteration (Chronopoulos & Gear, J. Comput. Appl. Math. 25,
 *                  1989, with s = 1): besides x, r and p it carries w = A r
 *                  and s = A p, updated by recurrence (s = w + beta s), so the
 *                  two inner products an iteration needs, r.r and w.r, are
 *                  taken together after the one product w = A r, and alpha
 *                  follows from them as r.r / (w.r - beta r.r / alpha_prev).
 *                  In exact arithmetic its iterates are those of oracle_cg.
 *  oracle_pcg_jacobi the same preconditioned CG with the Jacobi
 *                  preconditioner M = D = diag(A) (duplicates summed), i.e.
 *                  z = D^-1 r: the first preconditioner of the scope's
 *                  preconditioned-CG step, in binary64.
 *
 * Pins (tests, independent of this code): exact rational brute force,
 * dyadic inputs whose results are exact in binary64, zero row sums of the
 * pure-Neumann Laplacian, symmetry x.(Ay) = y.(Ax), permutation
 * equivariance, linearity, a dense library product, CG closed forms and a
 * dense LAPACK solve.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads oracle_spmv runs on in this build (1 without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* y_i and bound_i for one row */
static void row_sum(const int32_t *row_ptr, const int32_t *col_idx, const double *values,
                    const double *x, int32_t i, double *yi, double *bi) {
    double s = 0.0, b = 0.0;
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        double a = values[k];
        double xv = x[col_idx[k]];
        double p = a * xv;
        s = s + p;
        b = b + fabs(a) * fabs(xv);
    }
    *yi = s;
    *bi = b;
}

/* The row loop is the only place OpenMP may split work: the timing build
 * (liboracle_omp.so, -fopenmp) runs rows on all host cores with a static
 * schedule, each row summed exactly as here; the checker build has no
 * OpenMP and runs single-threaded. */
void oracle_spmv(int32_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *values, const double *x, double *y, double *bound) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int32_t i = 0; i < n_rows; ++i) {
        double yi, bi;
        row_sum(row_ptr, col_idx, values, x, i, &yi, &bi);
        y[i] = yi;
        if (bound) bound[i] = bi;
    }
}

void oracle_spmv_rows(int32_t n_sample, const int32_t *rows, const int32_t *row_ptr,
                      const int32_t *col_idx, const double *values, const double *x,
                      double *y, double *bound) {
    for (int32_t t = 0; t < n_sample; ++t) {
        double yi, bi;
        row_sum(row_ptr, col_idx, values, x, rows[t], &yi, &bi);
        y[t] = yi;
        if (bound) bound[t] = bi;
    }
}

/* Block row br, block k holds the 3x3 block at (br, bcol[k]) stored row-major
 * in bval[9k .. 9k+9).  Scalar row 3*br + r of Y, column j:
 *   Y[3br+r][j] = sum_k sum_c bval[9k + 3r + c] * X[3*bcol[k] + c][j]. */
void oracle_bsr3_spmm(int32_t nb_rows, const int32_t *brow_ptr, const int32_t *bcol,
                      const double *bval, int32_t k, const double *X, double *Y,
                      double *bound) {
    for (int32_t br = 0; br < nb_rows; ++br)
        for (int32_t r = 0; r < 3; ++r)
            for (int32_t j = 0; j < k; ++j) {
                double s = 0.0, b = 0.0;
                for (int32_t q = brow_ptr[br]; q < brow_ptr[br + 1]; ++q)
                    for (int32_t c = 0; c < 3; ++c) {
                        double a = bval[9 * (int64_t)q + 3 * r + c];
                        double xv = X[(3 * (int64_t)bcol[q] + c) * k + j];
                        s = s + a * xv;
                        b = b + fabs(a) * fabs(xv);
                    }
                Y[(3 * (int64_t)br + r) * k + j] = s;
                if (bound) bound[(3 * (int64_t)br + r) * k + j] = b;
            }
}

static double dot(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

double oracle_dot(int32_t n, const double *a, const double *b) { return dot(n, a, b); }

/* r = b - A x */
static void residual(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *values, const double *b, const double *x, double *r) {
    for (int32_t i = 0; i < n; ++i) {
        double yi, bi;
        row_sum(row_ptr, col_idx, values, x, i, &yi, &bi);
        r[i] = b[i] - yi;
    }
}

/*
 * Conjugate gradients.  Work arrays r, p, q (n each) are supplied by the
 * caller.  x holds x0 on entry and the last iterate on exit.
 *
 *   r = b - A x;  p = r;  rho = r.r
 *   repeat:  q = A p;  alpha = rho / (p.q)
 *            x = x + alpha p;  r = r - alpha q;  rho' = r.r
 *            if sqrt(rho') <= tol ||b||: confirm with the true residual;
 *               stop if it passes, otherwise continue from r = b - A x
 *            beta = rho' / rho;  p = r + beta p;  rho = rho'
 *
 * Returns 0 when converged, 1 when max_iter was reached, 2 on breakdown
 * (p.q <= 0 or not finite).  *iters is the number of iterations done and
 * *rel_res the true relative residual ||b - A x|| / ||b|| at exit.  When
 * alphas/betas are non-NULL they receive the coefficients of each iteration
 * (max_iter entries), from which the Lanczos tridiagonal follows.
 */
int oracle_cg(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
              const double *b, double *x, double tol, int32_t max_iter,
              double *r, double *p, double *q,
              int32_t *iters, double *rel_res, double *alphas, double *betas) {
    double nb = sqrt(dot(n, b, b));
    *iters = 0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        *rel_res = 0.0;
        return 0;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    for (int32_t i = 0; i < n; ++i) p[i] = r[i];
    double rho = dot(n, r, r);
    int status = 1;
    if (sqrt(rho) <= tol * nb) status = 0;
    for (int32_t it = 1; it <= max_iter && status != 0; ++it) {
        for (int32_t i = 0; i < n; ++i) {
            double yi, bi;
            row_sum(row_ptr, col_idx, values, p, i, &yi, &bi);
            q[i] = yi;
        }
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; *iters = it - 1; break; }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        double rho_new = dot(n, r, r);
        *iters = it;
        if (alphas) alphas[it - 1] = alpha;
        if (sqrt(rho_new) <= tol * nb) {
            residual(n, row_ptr, col_idx, values, b, x, r);
            rho_new = dot(n, r, r);
            if (sqrt(rho_new) <= tol * nb) { status = 0; if (betas) betas[it - 1] = 0.0; break; }
        }
        double beta = rho_new / rho;
        if (betas) betas[it - 1] = beta;
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    *rel_res = sqrt(dot(n, r, r)) / nb;
    return status;
}

/*
 * CG with one reduction phase per iteration (Chronopoulos-Gear).  Work
 * arrays r, p, w, s (n each) are supplied by the caller; x holds x0 on
 * entry and the last iterate on exit.
 *
 *   r = b - A x;  w = A r;  gamma = r.r;  delta = w.r
 *   alpha = gamma / delta;  beta = 0;  p = 0;  s = 0
 *   repeat:  p = r + beta p;  s = w + beta s
 *            x = x + alpha p;  r = r - alpha s;  w = A r
 *            gamma' = r.r;  delta' = w.r
 *            if sqrt(gamma') <= tol ||b||: confirm with the true residual;
 *               stop if it passes, otherwise start again from r = b - A x
 *            beta = gamma' / gamma
 *            alpha = gamma' / (delta' - beta gamma' / alpha);  gamma = gamma'
 *
 * Returns 0 when converged, 1 when max_iter was reached, 2 on breakdown
 * (a denominator of alpha not positive and finite).  *iters is the number
 * of iterations done, *restarts the restarts from the true residual and
 * *rel_res the true relative residual ||b - A x|| / ||b|| at exit.
 */
static int cg1_start(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
                     const double *b, const double *x, double *r, double *p, double *w, double *s,
                     double *gamma, double *alpha) {
    residual(n, row_ptr, col_idx, values, b, x, r);
    for (int32_t i = 0; i < n; ++i) {
        double yi, bi;
        row_sum(row_ptr, col_idx, values, r, i, &yi, &bi);
        w[i] = yi;
        p[i] = 0.0;
        s[i] = 0.0;
    }
    *gamma = dot(n, r, r);
    double delta = dot(n, w, r);
    if (!(delta > 0.0) || !isfinite(delta)) return 2;
    *alpha = *gamma / delta;
    return 0;
}

int oracle_cg1(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
               const double *b, double *x, double tol, int32_t max_iter,
               double *r, double *p, double *w, double *s,
               int32_t *iters, int32_t *restarts, double *rel_res) {
    double nb = sqrt(dot(n, b, b));
    *iters = 0;
    *restarts = 0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        *rel_res = 0.0;
        return 0;
    }
    double gamma, alpha, beta = 0.0;
    int status = 1;
    residual(n, row_ptr, col_idx, values, b, x, r);
    if (sqrt(dot(n, r, r)) <= tol * nb) status = 0;
    else if (cg1_start(n, row_ptr, col_idx, values, b, x, r, p, w, s, &gamma, &alpha)) status = 2;
    for (int32_t it = 1; it <= max_iter && status == 1; ++it) {
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        for (int32_t i = 0; i < n; ++i) s[i] = w[i] + beta * s[i];
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * s[i];
        for (int32_t i = 0; i < n; ++i) {
            double yi, bi;
            row_sum(row_ptr, col_idx, values, r, i, &yi, &bi);
            w[i] = yi;
        }
        double gamma_new = dot(n, r, r);
        double delta = dot(n, w, r);
        *iters = it;
        if (sqrt(gamma_new) <= tol * nb) {
            residual(n, row_ptr, col_idx, values, b, x, r);
            if (sqrt(dot(n, r, r)) <= tol * nb) { status = 0; break; }
            ++*restarts;
            if (cg1_start(n, row_ptr, col_idx, values, b, x, r, p, w, s, &gamma, &alpha)) { status = 2; break; }
            beta = 0.0;
            continue;
        }
        beta = gamma_new / gamma;
        double den = delta - beta * gamma_new / alpha;
        if (!(den > 0.0) || !isfinite(den)) { status = 2; break; }
        alpha = gamma_new / den;
        gamma = gamma_new;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    *rel_res = sqrt(dot(n, r, r)) / nb;
    return status;
}

/* Nearest bfloat16 value (8 significant bits, ties to even) of a binary32
 * value, from the definition: f = m 2^e with 1/2 <= |m| < 1, keep
 * rint(m 2^8) 2^(e-8) (rint rounds to nearest even).  Finite normal inputs
 * only, which is all the preconditioner sees. */
static double bf16_round(float f) {
    if (f == 0.0f || !isfinite(f)) return (double)f;
    int e;
    double m = frexp((double)f, &e);
    return ldexp(rint(ldexp(m, 8)), e - 8);
}

/* z = w D^-1 (2 r - w A~ (D^-1 r)) */
static void precond(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *vt,
                    const double *dinv, double w, const double *r, double *t, double *z) {
    for (int32_t i = 0; i < n; ++i) t[i] = dinv[i] * r[i];
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s = s + vt[k] * t[col_idx[k]];
        z[i] = w * dinv[i] * (2.0 * r[i] - w * s);
    }
}

/*
 * Preconditioned CG with the bfloat16 polynomial preconditioner above.  Work
 * arrays r, p, q, z, t (n each) are supplied by the caller; x holds x0 on
 * entry.
 *
 *   r = b - A x;  z = M^-1 r;  p = z;  rho = r.z
 *   repeat:  q = A p;  alpha = rho / (p.q)
 *            x = x + alpha p;  r = r - alpha q
 *            if ||r|| <= tol ||b||: confirm with the true residual; stop if
 *               it passes, otherwise restart from r = b - A x (p = M^-1 r)
 *            z = M^-1 r;  rho' = r.z;  beta = rho' / rho;  p = z + beta p
 *
 * Returns 0 when converged, 1 at max_iter, 2 on breakdown (p.q or r.z not
 * positive and finite), 3 when a diagonal entry is not positive.  *weight
 * receives w.
 */
int oracle_pcg_bf16(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
                    const double *b, double *x, double tol, int32_t max_iter,
                    double *r, double *p, double *q, double *z, double *t,
                    int32_t *iters, double *rel_res, double *weight) {
    *iters = 0;
    *rel_res = 0.0;
    int64_t nnz = row_ptr[n];
    double *vt = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!vt || !dinv) { free(vt); free(dinv); return 3; }
    for (int64_t k = 0; k < nnz; ++k) vt[k] = bf16_round((float)values[k]);
    int status = 0;
    for (int32_t i = 0; i < n && status == 0; ++i) {
        double d = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] == i) d = d + values[k];
        if (!(d > 0.0) || !isfinite(d)) status = 3;
        else dinv[i] = 1.0 / d;
    }
    if (status != 0) { free(vt); free(dinv); return status; }
    double g = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s = s + fabs(vt[k]) * sqrt(dinv[i] * dinv[col_idx[k]]);
        if (s > g) g = s;
    }
    double w = g > 0.0 ? 1.9 / g : 1.0;
    *weight = w;
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        free(vt); free(dinv);
        return 0;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    status = 1;
    if (sqrt(dot(n, r, r)) <= tol * nb) status = 0;
    precond(n, row_ptr, col_idx, vt, dinv, w, r, t, z);
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    for (int32_t it = 1; it <= max_iter && status != 0; ++it) {
        for (int32_t i = 0; i < n; ++i) {
            double yi, bi;
            row_sum(row_ptr, col_idx, values, p, i, &yi, &bi);
            q[i] = yi;
        }
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; *iters = it - 1; break; }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        *iters = it;
        int restart = 0;
        if (sqrt(dot(n, r, r)) <= tol * nb) {
            residual(n, row_ptr, col_idx, values, b, x, r);
            if (sqrt(dot(n, r, r)) <= tol * nb) { status = 0; break; }
            restart = 1;
        }
        precond(n, row_ptr, col_idx, vt, dinv, w, r, t, z);
        double rho_new = dot(n, r, z);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) { status = 2; break; }
        double beta = restart ? 0.0 : rho_new / rho;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    *rel_res = sqrt(dot(n, r, r)) / nb;
    free(vt);
    free(dinv);
    return status;
}

/*
 * Preconditioned CG with M = D = diag(A): the recurrences, stopping rule and
 * restarts of oracle_pcg_bf16 with z = D^-1 r.  Work arrays r, p, q, z (n
 * each) are supplied by the caller; x holds x0 on entry.  Returns 0 when
 * converged, 1 at max_iter, 2 on breakdown (p.q or r.z not positive and
 * finite), 3 when a diagonal entry is not positive and finite.
 */
int oracle_pcg_jacobi(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *values,
                      const double *b, double *x, double tol, int32_t max_iter,
                      double *r, double *p, double *q, double *z,
                      int32_t *iters, double *rel_res) {
    *iters = 0;
    *rel_res = 0.0;
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!dinv) return 3;
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] == i) d = d + values[k];
        if (!(d > 0.0) || !isfinite(d)) { free(dinv); return 3; }
        dinv[i] = 1.0 / d;
    }
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        free(dinv);
        return 0;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    int status = 1;
    if (sqrt(dot(n, r, r)) <= tol * nb) status = 0;
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    for (int32_t it = 1; it <= max_iter && status != 0; ++it) {
        for (int32_t i = 0; i < n; ++i) {
            double yi, bi;
            row_sum(row_ptr, col_idx, values, p, i, &yi, &bi);
            q[i] = yi;
        }
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; *iters = it - 1; break; }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        *iters = it;
        int restart = 0;
        if (sqrt(dot(n, r, r)) <= tol * nb) {
            residual(n, row_ptr, col_idx, values, b, x, r);
            if (sqrt(dot(n, r, r)) <= tol * nb) { status = 0; break; }
            restart = 1;
        }
        for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rho_new = dot(n, r, z);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) { status = 2; break; }
        double beta = restart ? 0.0 : rho_new / rho;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    residual(n, row_ptr, col_idx, values, b, x, r);
    *rel_res = sqrt(dot(n, r, r)) / nb;
    free(dinv);
    return status;
}
