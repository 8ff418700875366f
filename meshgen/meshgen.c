/*
 * meshgen.c -- seeded synthetic mesh matrices for the SpMV / CG workloads.
 *
 * This module only builds inputs: sparsity patterns of finite-volume meshes,
 * their coefficients, vectors and orderings.  It contains no part of the
 * sparse product or of the solver.  Both the CPU oracle and the GPU library
 * consume what it produces; neither of them is linked against it.
 *
 * Data model (paper, Sec. 2): row i of an operator is cell i, the non-zero
 * columns of the row are the cell's neighbours, and the matrix of a
 * Laplacian-like operator is symmetric.  Matrices are assembled here as
 *   a_ij = -w_ij   (i != j, one weight per undirected edge, so a_ij = a_ji)
 *   a_ii = sum_j w_ij + shift
 * which makes each row strictly diagonally dominant with a positive diagonal
 * (hence SPD when shift > 0) and gives A*(c*1) = shift*c*1 exactly in real
 * arithmetic.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a
 * counter-based generator, h = mix(mix(seed ^ stream*K) + counter), so every
 * draw is a pure function of (seed, stream, counter) and generation is
 * reproducible under any thread count.
 *
 * Reordering: reverse Cuthill-McKee (Cuthill & McKee 1969; George & Liu 1981)
 * with a George-Liu pseudo-peripheral start vertex, neighbours visited in
 * ascending (degree, index) order.  The paper (Sec. 4.1) applies
 * Cuthill-McKee once before the simulation; reordering permutes rows and
 * columns and leaves the coefficients unchanged.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ rng */

static inline uint64_t sm64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return sm64(sm64(seed ^ (stream * 0xD1B54A32D192ED03ull)) + ctr);
}
static inline double u01(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

enum {
    S_WEIGHT = 1, S_ECOUNT = 2, S_EPICK = 3, S_PAIR = 4, S_JITTER = 5,
    S_KCOUNT = 6, S_PERM = 7, S_VEC = 8, S_BVAL = 9, S_BECOUNT = 10,
    S_BEPICK = 11, S_DYX = 12
};

/* ------------------------------------------------------------------ csr */

typedef struct mg_csr {
    int32_t n_rows, n_cols;
    int64_t nnz;
    int32_t *row_ptr;   /* n_rows + 1 */
    int32_t *col_idx;   /* nnz */
    double *values;     /* nnz (or 9*nnz for block matrices) */
    int32_t block;      /* 1 for scalar CSR, 3 for 3x3 block CSR */
} mg_csr;

static mg_csr *csr_alloc(int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t block) {
    mg_csr *A = (mg_csr *)calloc(1, sizeof(mg_csr));
    if (!A) return NULL;
    A->n_rows = n_rows; A->n_cols = n_cols; A->nnz = nnz; A->block = block;
    A->row_ptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_rows + 1));
    A->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    A->values = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1) * (size_t)(block * block));
    if (!A->row_ptr || !A->col_idx || !A->values) {
        free(A->row_ptr); free(A->col_idx); free(A->values); free(A);
        return NULL;
    }
    return A;
}

void mg_free(mg_csr *A) {
    if (!A) return;
    free(A->row_ptr); free(A->col_idx); free(A->values); free(A);
}
int32_t mg_n_rows(const mg_csr *A) { return A->n_rows; }
int32_t mg_n_cols(const mg_csr *A) { return A->n_cols; }
int64_t mg_nnz(const mg_csr *A) { return A->nnz; }
int32_t mg_block(const mg_csr *A) { return A->block; }
void mg_fetch(const mg_csr *A, int32_t *row_ptr, int32_t *col_idx, double *values) {
    size_t bb = (size_t)A->block * (size_t)A->block;
    if (row_ptr) memcpy(row_ptr, A->row_ptr, sizeof(int32_t) * ((size_t)A->n_rows + 1));
    if (col_idx && A->nnz) memcpy(col_idx, A->col_idx, sizeof(int32_t) * (size_t)A->nnz);
    if (values && A->nnz) memcpy(values, A->values, sizeof(double) * (size_t)A->nnz * bb);
}

/* exclusive prefix sum of counts[0..n) into row_ptr[0..n]; returns total */
static int64_t prefix(const int32_t *counts, int32_t *row_ptr, int32_t n) {
    int64_t s = 0;
    for (int32_t i = 0; i < n; ++i) { row_ptr[i] = (int32_t)s; s += counts[i]; }
    row_ptr[n] = (int32_t)s;
    return s;
}

static void isort_i32(int32_t *a, int m) {
    for (int i = 1; i < m; ++i) {
        int32_t v = a[i]; int j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}
static int uniq_i32(int32_t *a, int m) {
    if (m == 0) return 0;
    int w = 1;
    for (int i = 1; i < m; ++i) if (a[i] != a[w - 1]) a[w++] = a[i];
    return w;
}

/* ------------------------------------------------------- edge weights */

/* weight of the undirected edge {i, j}; in [0.5, 1.5) (or m/1024 with
 * integer m in [512, 1536] when dyadic, so every product with a dyadic x is
 * exact in binary64) */
static inline double edge_w(uint64_t seed, int64_t n, int32_t i, int32_t j, int dyadic) {
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    uint64_t h = rnd(seed, S_WEIGHT, (uint64_t)(lo * n + hi));
    if (dyadic) return (double)(512 + (int)(h % 1025u)) / 1024.0;
    return 0.5 + u01(h);
}

/* Fill values for a symmetric pattern: off-diagonals -w_ij, diagonal sum w + shift.
 * Columns of each row are sorted; the diagonal is present in every row. */
static void fill_laplacian_values(mg_csr *A, uint64_t seed, double shift, int dyadic) {
    const int64_t n = A->n_rows;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < A->n_rows; ++i) {
        double diag = 0.0; int32_t dpos = -1;
        for (int32_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
            int32_t j = A->col_idx[k];
            if (j == i) { dpos = k; continue; }
            double w = edge_w(seed, n, i, j, dyadic);
            A->values[k] = -w;
            diag += w;
        }
        if (dpos >= 0) A->values[dpos] = diag + shift;
    }
}

/* --------------------------------------------------------- lattices */

static inline int32_t cell_id(int32_t x, int32_t y, int32_t z, int32_t nx, int32_t ny) {
    return (z * ny + y) * nx + x;
}

/* offsets with Chebyshev norm in [1, 2]; "faces" are the 6 unit-axis ones */
static int g_off_init = 0;
static int8_t g_face[6][3];
static int8_t g_nonface[118][3];   /* Chebyshev 1..2 minus faces */
static int8_t g_cheb2[124][3];     /* Chebyshev 1..2 */
static int8_t g_edgevert[20][3];   /* Chebyshev 1 with 2 or 3 non-zero components */

static void offsets_init(void) {
    if (g_off_init) return;
    int nf = 0, nn = 0, nc = 0, ne = 0;
    for (int dz = -2; dz <= 2; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                int ax = abs(dx), ay = abs(dy), az = abs(dz);
                int cheb = ax > ay ? ax : ay; cheb = cheb > az ? cheb : az;
                if (cheb == 0) continue;
                int nzc = (dx != 0) + (dy != 0) + (dz != 0);
                int8_t d[3] = {(int8_t)dx, (int8_t)dy, (int8_t)dz};
                memcpy(g_cheb2[nc++], d, 3);
                if (cheb == 1 && nzc == 1) memcpy(g_face[nf++], d, 3);
                else memcpy(g_nonface[nn++], d, 3);
                if (cheb == 1 && nzc >= 2) memcpy(g_edgevert[ne++], d, 3);
            }
    g_off_init = 1;
}

static inline int in_grid(int32_t x, int32_t y, int32_t z, int32_t nx, int32_t ny, int32_t nz) {
    return x >= 0 && y >= 0 && z >= 0 && x < nx && y < ny && z < nz;
}

/* extras[i*4 + t]: up to 4 distinct non-face neighbours within Chebyshev
 * distance 2, e ~ U{0..4} per cell, chosen by partial Fisher-Yates. */
static void pick_extras(int32_t nx, int32_t ny, int32_t nz, uint64_t seed,
                        uint64_t s_count, uint64_t s_pick, int32_t *extras) {
    const int32_t n = nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        int32_t cand[118]; int cnt = 0;
        for (int t = 0; t < 118; ++t) {
            int32_t xx = x + g_nonface[t][0], yy = y + g_nonface[t][1], zz = z + g_nonface[t][2];
            if (in_grid(xx, yy, zz, nx, ny, nz)) cand[cnt++] = cell_id(xx, yy, zz, nx, ny);
        }
        int e = (int)(rnd(seed, s_count, (uint64_t)i) % 5u);
        if (e > cnt) e = cnt;
        for (int t = 0; t < 4; ++t) extras[(int64_t)i * 4 + t] = -1;
        for (int t = 0; t < e; ++t) {
            int r = t + (int)(rnd(seed, s_pick, (uint64_t)i * 128u + (uint64_t)t) % (uint64_t)(cnt - t));
            int32_t tmp = cand[t]; cand[t] = cand[r]; cand[r] = tmp;
            extras[(int64_t)i * 4 + t] = cand[t];
        }
    }
}

/* Neighbour set of cell i (sorted, unique, including i itself) for lattice kinds:
 *   kind 0: faces + own extras + reverse extras (union symmetrisation)
 *   kind 1: faces only (7-point)
 *   kind 2: faces + each edge/vertex pair kept with probability 1/2
 * returns count written into buf (capacity >= 130). */
static int lattice_row(int kind, int32_t i, int32_t nx, int32_t ny, int32_t nz,
                       uint64_t seed, const int32_t *extras, int32_t *buf) {
    const int64_t n = (int64_t)nx * ny * nz;
    int32_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    int m = 0;
    buf[m++] = i;
    for (int t = 0; t < 6; ++t) {
        int32_t xx = x + g_face[t][0], yy = y + g_face[t][1], zz = z + g_face[t][2];
        if (in_grid(xx, yy, zz, nx, ny, nz)) buf[m++] = cell_id(xx, yy, zz, nx, ny);
    }
    if (kind == 0) {
        for (int t = 0; t < 4; ++t) {
            int32_t j = extras[(int64_t)i * 4 + t];
            if (j >= 0) buf[m++] = j;
        }
        for (int t = 0; t < 118; ++t) {
            int32_t xx = x + g_nonface[t][0], yy = y + g_nonface[t][1], zz = z + g_nonface[t][2];
            if (!in_grid(xx, yy, zz, nx, ny, nz)) continue;
            int32_t j = cell_id(xx, yy, zz, nx, ny);
            for (int u = 0; u < 4; ++u)
                if (extras[(int64_t)j * 4 + u] == i) { buf[m++] = j; break; }
        }
    } else if (kind == 2) {
        for (int t = 0; t < 20; ++t) {
            int32_t xx = x + g_edgevert[t][0], yy = y + g_edgevert[t][1], zz = z + g_edgevert[t][2];
            if (!in_grid(xx, yy, zz, nx, ny, nz)) continue;
            int32_t j = cell_id(xx, yy, zz, nx, ny);
            int64_t lo = i < j ? i : j, hi = i < j ? j : i;
            if (rnd(seed, S_PAIR, (uint64_t)(lo * n + hi)) & 1u) buf[m++] = j;
        }
    }
    isort_i32(buf, m);
    return uniq_i32(buf, m);
}

/* Laplacian-like matrix on an nx*ny*nz lattice (natural ordering). */
mg_csr *mg_lattice(int32_t nx, int32_t ny, int32_t nz, int32_t kind, uint64_t seed,
                   double shift, int32_t dyadic) {
    offsets_init();
    if (nx <= 0 || ny <= 0 || nz <= 0) return NULL;
    int64_t n64 = (int64_t)nx * ny * nz;
    if (n64 > 0x7fffffff / 32) return NULL;
    int32_t n = (int32_t)n64;
    int32_t *extras = NULL;
    if (kind == 0) {
        extras = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * 4);
        if (!extras) return NULL;
        pick_extras(nx, ny, nz, seed, S_ECOUNT, S_EPICK, extras);
    }
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t buf[160];
        counts[i] = lattice_row(kind, i, nx, ny, nz, seed, extras, buf);
    }
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) nnz += counts[i];
    mg_csr *A = csr_alloc(n, n, nnz, 1);
    if (!A) { free(counts); free(extras); return NULL; }
    prefix(counts, A->row_ptr, n);
    free(counts);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t buf[160];
        int m = lattice_row(kind, i, nx, ny, nz, seed, extras, buf);
        memcpy(A->col_idx + A->row_ptr[i], buf, sizeof(int32_t) * (size_t)m);
    }
    free(extras);
    fill_laplacian_values(A, seed, shift, dyadic);
    return A;
}

/* ------------------------------------------------ jittered-lattice kNN */

/* m^3 jittered lattice (jitter U[-0.35, 0.35] per axis, lattice spacing 1);
 * each cell keeps k ~ U{4,5,6} Euclidean nearest neighbours among the cells
 * within Chebyshev lattice distance 2 (ties by index), then the pattern is
 * symmetrised by union.  A mesh-like graph with ~5-6 neighbours per cell. */
mg_csr *mg_knn(int32_t m, uint64_t seed, double shift, int32_t dyadic) {
    offsets_init();
    if (m <= 2) return NULL;
    int64_t n64 = (int64_t)m * m * m;
    if (n64 > 0x7fffffff / 32) return NULL;
    int32_t n = (int32_t)n64;
    double *pos = (double *)malloc(sizeof(double) * (size_t)n * 3);
    int32_t *knn = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * 6);
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!pos || !knn || !counts) { free(pos); free(knn); free(counts); return NULL; }
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        int32_t x = i % m, y = (i / m) % m, z = i / (m * m);
        pos[3 * (int64_t)i + 0] = x + 0.7 * (u01(rnd(seed, S_JITTER, 3 * (uint64_t)i + 0)) - 0.5);
        pos[3 * (int64_t)i + 1] = y + 0.7 * (u01(rnd(seed, S_JITTER, 3 * (uint64_t)i + 1)) - 0.5);
        pos[3 * (int64_t)i + 2] = z + 0.7 * (u01(rnd(seed, S_JITTER, 3 * (uint64_t)i + 2)) - 0.5);
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t i = 0; i < n; ++i) {
        int32_t x = i % m, y = (i / m) % m, z = i / (m * m);
        double d2[124]; int32_t id[124]; int cnt = 0;
        for (int t = 0; t < 124; ++t) {
            int32_t xx = x + g_cheb2[t][0], yy = y + g_cheb2[t][1], zz = z + g_cheb2[t][2];
            if (!in_grid(xx, yy, zz, m, m, m)) continue;
            int32_t j = cell_id(xx, yy, zz, m, m);
            double dx = pos[3 * (int64_t)j] - pos[3 * (int64_t)i];
            double dy = pos[3 * (int64_t)j + 1] - pos[3 * (int64_t)i + 1];
            double dz = pos[3 * (int64_t)j + 2] - pos[3 * (int64_t)i + 2];
            d2[cnt] = dx * dx + dy * dy + dz * dz; id[cnt] = j; ++cnt;
        }
        int k = 4 + (int)(rnd(seed, S_KCOUNT, (uint64_t)i) % 3u);
        if (k > cnt) k = cnt;
        /* partial selection sort by (distance, index) */
        for (int a = 0; a < k; ++a) {
            int best = a;
            for (int b = a + 1; b < cnt; ++b)
                if (d2[b] < d2[best] || (d2[b] == d2[best] && id[b] < id[best])) best = b;
            double td = d2[a]; d2[a] = d2[best]; d2[best] = td;
            int32_t ti = id[a]; id[a] = id[best]; id[best] = ti;
        }
        for (int a = 0; a < 6; ++a) knn[(int64_t)i * 6 + a] = a < k ? id[a] : -1;
    }
    free(pos);
    /* union symmetrisation: row i = {i} + knn(i) + {j : i in knn(j)} */
#define KNN_ROW(i, buf, mm)                                                              \
    do {                                                                                  \
        int32_t x_ = (i) % m, y_ = ((i) / m) % m, z_ = (i) / (m * m);                    \
        mm = 0; buf[mm++] = (i);                                                          \
        for (int a_ = 0; a_ < 6; ++a_) { int32_t j_ = knn[(int64_t)(i) * 6 + a_]; if (j_ >= 0) buf[mm++] = j_; } \
        for (int t_ = 0; t_ < 124; ++t_) {                                                \
            int32_t xx_ = x_ + g_cheb2[t_][0], yy_ = y_ + g_cheb2[t_][1], zz_ = z_ + g_cheb2[t_][2]; \
            if (!in_grid(xx_, yy_, zz_, m, m, m)) continue;                               \
            int32_t j_ = cell_id(xx_, yy_, zz_, m, m);                                     \
            for (int u_ = 0; u_ < 6; ++u_) if (knn[(int64_t)j_ * 6 + u_] == (i)) { buf[mm++] = j_; break; } \
        }                                                                                 \
        isort_i32(buf, mm); mm = uniq_i32(buf, mm);                                       \
    } while (0)
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t buf[160]; int mm;
        KNN_ROW(i, buf, mm);
        counts[i] = mm;
    }
    int64_t nnz = 0;
    for (int32_t i = 0; i < n; ++i) nnz += counts[i];
    mg_csr *A = csr_alloc(n, n, nnz, 1);
    if (!A) { free(knn); free(counts); return NULL; }
    prefix(counts, A->row_ptr, n);
    free(counts);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t buf[160]; int mm;
        KNN_ROW(i, buf, mm);
        memcpy(A->col_idx + A->row_ptr[i], buf, sizeof(int32_t) * (size_t)mm);
    }
#undef KNN_ROW
    free(knn);
    fill_laplacian_values(A, seed, shift, dyadic);
    return A;
}

/* ------------------------------------------------------ block matrices */

static inline double gauss(uint64_t seed, uint64_t ctr) {
    /* Box-Muller on two counter-based uniforms; u1 in (0, 1] */
    double u1 = 1.0 - u01(rnd(seed, S_BVAL, 2 * ctr));
    double u2 = u01(rnd(seed, S_BVAL, 2 * ctr + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* 3x3 block-CSR coupled operator on an nx*ny*nz lattice: block row i holds
 * the diagonal block, the face neighbours and e ~ U{0..4} directed extras
 * within Chebyshev distance 2 (not symmetrised).  Off-diagonal scalar
 * entries ~ N(0, sigma^2); each scalar diagonal entry = 1 + sum of |other
 * entries| of its scalar row.  Blocks stored row-major, 9 values each. */
mg_csr *mg_bsr3(int32_t nx, int32_t ny, int32_t nz, uint64_t seed, double sigma) {
    offsets_init();
    int64_t n64 = (int64_t)nx * ny * nz;
    if (nx <= 0 || ny <= 0 || nz <= 0 || n64 > 0x7fffffff / 32) return NULL;
    int32_t n = (int32_t)n64;
    int32_t *extras = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * 4);
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!extras || !counts) { free(extras); free(counts); return NULL; }
    pick_extras(nx, ny, nz, seed, S_BECOUNT, S_BEPICK, extras);
#define BSR_ROW(i, buf, mm)                                                                \
    do {                                                                                    \
        int32_t x_ = (i) % nx, y_ = ((i) / nx) % ny, z_ = (i) / (nx * ny);                 \
        mm = 0; buf[mm++] = (i);                                                            \
        for (int t_ = 0; t_ < 6; ++t_) {                                                    \
            int32_t xx_ = x_ + g_face[t_][0], yy_ = y_ + g_face[t_][1], zz_ = z_ + g_face[t_][2]; \
            if (in_grid(xx_, yy_, zz_, nx, ny, nz)) buf[mm++] = cell_id(xx_, yy_, zz_, nx, ny); \
        }                                                                                   \
        for (int t_ = 0; t_ < 4; ++t_) { int32_t j_ = extras[(int64_t)(i) * 4 + t_]; if (j_ >= 0) buf[mm++] = j_; } \
        isort_i32(buf, mm); mm = uniq_i32(buf, mm);                                         \
    } while (0)
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) { int32_t buf[16]; int mm; BSR_ROW(i, buf, mm); counts[i] = mm; }
    int64_t nnzb = 0;
    for (int32_t i = 0; i < n; ++i) nnzb += counts[i];
    mg_csr *A = csr_alloc(n, n, nnzb, 3);
    if (!A) { free(extras); free(counts); return NULL; }
    prefix(counts, A->row_ptr, n);
    free(counts);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < n; ++i) {
        int32_t buf[16]; int mm; BSR_ROW(i, buf, mm);
        int32_t base = A->row_ptr[i];
        memcpy(A->col_idx + base, buf, sizeof(int32_t) * (size_t)mm);
        double rowsum[3] = {0.0, 0.0, 0.0};
        int32_t dblk = -1;
        for (int b = 0; b < mm; ++b) {
            int32_t j = buf[b];
            double *blk = A->values + 9 * (int64_t)(base + b);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    uint64_t ctr = (((uint64_t)i * (uint64_t)n + (uint64_t)j) * 9u) + (uint64_t)(3 * r + c);
                    if (j == i && r == c) { blk[3 * r + c] = 0.0; continue; }
                    double v = sigma * gauss(seed, ctr);
                    blk[3 * r + c] = v;
                    rowsum[r] += fabs(v);
                }
            if (j == i) dblk = b;
        }
        double *d = A->values + 9 * (int64_t)(base + dblk);
        for (int r = 0; r < 3; ++r) d[4 * r] = 1.0 + rowsum[r];
    }
#undef BSR_ROW
    free(extras);
    return A;
}

/* ------------------------------------------------------------ vectors */

/* out[i] = lo + (hi - lo) * U[0,1)  from stream `stream` */
void mg_uniform(int64_t count, uint64_t seed, uint64_t stream, double lo, double hi, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = lo + (hi - lo) * u01(rnd(seed, S_VEC + 16 * stream, (uint64_t)i));
}

/* ------------------------------------------------------- permutations */

typedef struct { uint64_t key; int32_t idx; } keyidx;
static int cmp_keyidx(const void *a, const void *b) {
    const keyidx *x = (const keyidx *)a, *y = (const keyidx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* perm[new] = old, a seeded uniformly random permutation (sort by random keys) */
void mg_random_perm(int32_t n, uint64_t seed, int32_t *perm) {
    keyidx *k = (keyidx *)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { k[i].key = rnd(seed, S_PERM, (uint64_t)i); k[i].idx = i; }
    qsort(k, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int32_t i = 0; i < n; ++i) perm[i] = k[i].idx;
    free(k);
}

/* B = P A P^T with perm[new] = old: new row r is old row perm[r], column c
 * becomes inv[c]; columns sorted within each row (values move with them). */
mg_csr *mg_permute(const mg_csr *A, const int32_t *perm) {
    const int32_t n = A->n_rows;
    const int bb = A->block * A->block;
    if (A->n_rows != A->n_cols) return NULL;
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!inv || !counts) { free(inv); free(counts); return NULL; }
    for (int32_t r = 0; r < n; ++r) inv[perm[r]] = r;
    for (int32_t r = 0; r < n; ++r) counts[r] = A->row_ptr[perm[r] + 1] - A->row_ptr[perm[r]];
    mg_csr *B = csr_alloc(n, n, A->nnz, A->block);
    if (!B) { free(inv); free(counts); return NULL; }
    prefix(counts, B->row_ptr, n);
    free(counts);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t r = 0; r < n; ++r) {
        int32_t o = perm[r];
        int32_t s = A->row_ptr[o], len = A->row_ptr[o + 1] - s, d = B->row_ptr[r];
        for (int32_t t = 0; t < len; ++t) {
            /* insertion by new column index; rows are short */
            int32_t c = inv[A->col_idx[s + t]];
            int32_t u = t - 1;
            while (u >= 0 && B->col_idx[d + u] > c) {
                B->col_idx[d + u + 1] = B->col_idx[d + u];
                memcpy(B->values + (int64_t)bb * (d + u + 1), B->values + (int64_t)bb * (d + u), sizeof(double) * bb);
                --u;
            }
            B->col_idx[d + u + 1] = c;
            memcpy(B->values + (int64_t)bb * (d + u + 1), A->values + (int64_t)bb * (s + t), sizeof(double) * bb);
        }
    }
    free(inv);
    return B;
}

/* ---------------------------------------------------------------- RCM */

/* BFS from `root` over unvisited-by-`mark` vertices of the adjacency in A;
 * writes the visit order into order[] and level of each vertex into level[]
 * (level must be -1 for unvisited).  Returns number visited, sets *ecc to the
 * last level index and *last_begin to the start of the last level in order[]. */
static int32_t bfs_levels(const mg_csr *A, int32_t root, int32_t *level, int32_t *order,
                          int32_t *ecc, int32_t *last_begin) {
    int32_t head = 0, tail = 0;
    order[tail++] = root; level[root] = 0;
    int32_t cur_level = 0, lb = 0;
    while (head < tail) {
        int32_t v = order[head++];
        if (level[v] != cur_level) { cur_level = level[v]; lb = head - 1; }
        for (int32_t k = A->row_ptr[v]; k < A->row_ptr[v + 1]; ++k) {
            int32_t w = A->col_idx[k];
            if (level[w] < 0) { level[w] = level[v] + 1; order[tail++] = w; }
        }
    }
    *ecc = cur_level; *last_begin = lb;
    return tail;
}

static inline int32_t degree_of(const mg_csr *A, int32_t v) {
    int32_t d = 0;
    for (int32_t k = A->row_ptr[v]; k < A->row_ptr[v + 1]; ++k) d += (A->col_idx[k] != v);
    return d;
}

/* perm[new] = old, reverse Cuthill-McKee over the symmetric pattern of A
 * (the pattern is symmetrised implicitly only if it already is; callers pass
 * structurally symmetric matrices). */
int mg_rcm(const mg_csr *A, int32_t *perm) {
    const int32_t n = A->n_rows;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    char *done = (char *)calloc((size_t)n, 1);
    if (!deg || !level || !order || !done) { free(deg); free(level); free(order); free(done); return -1; }
    int32_t maxdeg = 0;
    for (int32_t v = 0; v < n; ++v) {
        deg[v] = degree_of(A, v); level[v] = -1;
        int32_t len = A->row_ptr[v + 1] - A->row_ptr[v];
        if (len > maxdeg) maxdeg = len;
    }
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    if (!nb) { free(deg); free(level); free(order); free(done); return -1; }
    int32_t out = 0;       /* next position in perm (Cuthill-McKee order) */
    int32_t scan = 0;      /* lowest possibly-unvisited vertex */
    while (out < n) {
        while (done[scan]) ++scan;
        /* The component of `scan`; vertices of earlier components keep their
         * non-negative levels, so the BFS never enters them again. */
        int32_t ecc, lb;
        int32_t cnt = bfs_levels(A, scan, level, order, &ecc, &lb);
        int32_t root = scan;
        for (int32_t t = 0; t < cnt; ++t) {
            int32_t v = order[t];
            if (deg[v] < deg[root] || (deg[v] == deg[root] && v < root)) root = v;
        }
        /* George-Liu pseudo-peripheral iteration: move to a minimum-degree
         * vertex of the last level while that lengthens the level structure. */
        for (int32_t t = 0; t < cnt; ++t) level[order[t]] = -1;
        bfs_levels(A, root, level, order, &ecc, &lb);
        for (int it = 0; it < 8; ++it) {
            int32_t cand = order[lb];
            for (int32_t t = lb; t < cnt; ++t) {
                int32_t v = order[t];
                if (deg[v] < deg[cand] || (deg[v] == deg[cand] && v < cand)) cand = v;
            }
            if (cand == root) break;
            for (int32_t t = 0; t < cnt; ++t) level[order[t]] = -1;
            int32_t e2, lb2;
            bfs_levels(A, cand, level, order, &e2, &lb2);
            if (e2 <= ecc) break;
            root = cand; ecc = e2; lb = lb2;
        }
        /* Cuthill-McKee BFS from root, children in ascending (degree, index) */
        int32_t head = out;
        perm[out++] = root; done[root] = 1;
        while (head < out) {
            int32_t v = perm[head++];
            int32_t m = 0;
            for (int32_t k = A->row_ptr[v]; k < A->row_ptr[v + 1]; ++k) {
                int32_t w = A->col_idx[k];
                if (!done[w]) { done[w] = 1; nb[m++] = w; }
            }
            for (int32_t a = 1; a < m; ++a) {
                int32_t w = nb[a]; int32_t b = a - 1;
                while (b >= 0 && (deg[nb[b]] > deg[w] || (deg[nb[b]] == deg[w] && nb[b] > w))) { nb[b + 1] = nb[b]; --b; }
                nb[b + 1] = w;
            }
            for (int32_t a = 0; a < m; ++a) perm[out++] = nb[a];
        }
        for (int32_t t = 0; t < cnt; ++t) if (level[order[t]] < 0) level[order[t]] = 0;
    }
    /* reverse */
    for (int32_t a = 0, b = n - 1; a < b; ++a, --b) { int32_t t = perm[a]; perm[a] = perm[b]; perm[b] = t; }
    free(nb); free(deg); free(level); free(order); free(done);
    return 0;
}

/* CSR from caller arrays (copied), for permuting matrices built elsewhere */
mg_csr *mg_from_arrays(int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t block,
                       const int32_t *row_ptr, const int32_t *col_idx, const double *values) {
    mg_csr *A = csr_alloc(n_rows, n_cols, nnz, block);
    if (!A) return NULL;
    memcpy(A->row_ptr, row_ptr, sizeof(int32_t) * ((size_t)n_rows + 1));
    if (nnz) {
        memcpy(A->col_idx, col_idx, sizeof(int32_t) * (size_t)nnz);
        memcpy(A->values, values, sizeof(double) * (size_t)nnz * (size_t)(block * block));
    }
    return A;
}

/* Walks the pairs (a[p], b[p]) of vertices in [0, n) in the given order and
 * keeps a pair while both of its vertices have fewer than `cap` kept pairs
 * (the degree-capped greedy fill of the tetrahedral stand-in).  keep[p] is
 * set to 1 or 0.  Returns the number of pairs kept, or -1 if a vertex is out
 * of range or memory runs out. */
int64_t mg_degree_capped(int64_t n_pairs, const int64_t *a, const int64_t *b, int64_t n, int32_t cap,
                         uint8_t *keep) {
    int32_t *deg = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!deg) return -1;
    int64_t kept = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int64_t u = a[p], v = b[p];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            free(deg);
            return -1;
        }
        keep[p] = 0;
        if (deg[u] < cap && deg[v] < cap) {
            ++deg[u];
            ++deg[v];
            keep[p] = 1;
            ++kept;
        }
    }
    free(deg);
    return kept;
}
