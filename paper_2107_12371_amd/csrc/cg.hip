// Conjugate gradients on the GPU (the paper's "linear solver", Sec. 2),
// Hestenes & Stiefel (1952):
//
//   r = b - A x;  p = r;  rho = r.r
//   repeat:  q = A p;  alpha = rho / (p.q)
//            x += alpha p;  r -= alpha q;  rho' = r.r
//            if rho' <= tol^2 ||b||^2: confirm with the true residual b - A x;
//               stop if it passes, else continue from r = b - A x
//            beta = rho' / rho;  p = r + beta p;  rho = rho'
//
// On systems up to 1,048,576 rows whose product is plain row tiles, one
// iteration is two launches: the SpMV, whose workgroups first form beta
// (and workgroup 0 the convergence flag) from the r.r partials and then
// gather p_new = r + beta p for every column (the previous iteration's p
// update folded into this product's gathers), with the p.q partial in its
// epilogue; and the x/r update, which writes p_new for its own rows beside
// x and r, with the r.r partial, its workgroups each forming alpha from the
// SpMV's partials.  Otherwise the p update is a launch of its own (three
// launches), and with more than 4,096 SpMV partials or 1,024 r.r partials
// that scalar takes a reduction launch of its own (five launches on the
// largest systems).  All scalars live on the device;
// every kernel returns at once when the device flag `done` is set, so a
// captured graph of several iterations can be replayed blindly and the host
// synchronises once per replay.  Reductions are two-stage with a fixed
// partition and a fixed order, so a solve is bitwise reproducible.
//
// Preconditioned (CG_PCG_BF16): standard preconditioned CG with the damped
// Neumann polynomial M^-1 = w D^-1 (2I - w A~ D^-1) in the bfloat16 copy A~
// of A (described with its kernels below); restarts from the true residual
// when the recursive one drifts.
//
// Jacobi-preconditioned (CG_PCG_JACOBI): the same preconditioned CG with
// M = diag(A).
//
// Mixed precision (CG_MIXED_FP32): iterative refinement (Wilkinson; Moler
// 1967).  The residual r = b - A x is formed with binary64 values and
// vectors; the correction solve A d = r / ||r|| runs CG with the FP32 copy
// of A, FP32 vectors and FP32 SpMV accumulation, while its dot products and
// scalar recurrences stay in binary64; x += ||r|| d in binary64.
// CG_MIXED_FP32V is the same refinement whose correction solve keeps binary64
// vectors and accumulation and reads only the values in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "device.h"
#include "internal.h"
#include "launch.h"
#include "matrix.h"
#include "tile.h"

namespace spmvlib {

// rho_new is the rho the next alpha step divides by; that step also copies
// it to rho.  Every step that sets rho sets rho_new too, except the p update
// with beta formed in it (R_BETA_DEFER), whose workgroups all read rho.
struct CgState {
    double rho, rho_new, pq, alpha, beta, bb, tol2, rt2;
    double rr, omega;  // preconditioned CG: r.r of the iterate, polynomial weight
    int32_t iter, max_iter, done, flags;
};

// F_FRESH: the next fused product (k_spmv_pfused) takes beta from the state
// instead of forming it from r.r partials, and records no step: set at the
// start of a solve (beta = 0 with p = 0) and after a residual replacement
// (beta = rt2 / rho); cleared by workgroup 0 of the following x/r update.
// Within a launch only workgroup 0 of a reduction step changes other bits,
// and never this one, so every workgroup reads the same value.
enum : int32_t { F_CONVERGED = 1, F_BREAKDOWN = 2, F_MAXITER = 4, F_BADDIAG = 8, F_FRESH = 16 };
enum : int {
    R_BB = 0, R_RHO0 = 1, R_ALPHA = 2, R_BETA = 3, R_TRUE = 4, R_RR = 5, R_RZ = 6, R_RZ0 = 7, R_DIAG = 8,
    R_BETA_DEFER = 9, R_RZ_DEFER = 10
};

// Sum of part[0..n) in the one fixed order every reduction of the solver
// uses (lane l adds l, l + kBlock, ...; then block_sum); the result is in
// thread 0.  The loops over a workgroup's elements here and below are
// unrolled by 4 so that a lane's loads are in flight together (one memory
// round trip instead of four on small systems); the order of the additions
// is unchanged.
__device__ __forceinline__ double sum_partials(const double *part, int n, double *sh) {
    double s = 0.0;
#pragma unroll 4
    for (int i = (int)threadIdx.x; i < n; i += kBlock) s += part[i];
    return block_sum(s, sh);
}

// Applies the finished sum t of reduction `mode` to the solver state.
__device__ void apply_reduction(CgState *st, int mode, double t) {
    switch (mode) {
        case R_BB: st->bb = t; break;
        case R_RHO0:
            st->rho = t;
            st->rho_new = t;
            break;
        case R_TRUE: st->rt2 = t; break;
        case R_ALPHA:
            st->pq = t;
            if (!(t > 0.0) || !isfinite(t)) {
                st->flags |= F_BREAKDOWN;
                st->done = 1;
            } else {
                st->alpha = st->rho_new / t;
                st->rho = st->rho_new;
            }
            break;
        case R_RR:  // preconditioned CG, after the x/r update: convergence on r.r
            st->rr = t;
            st->iter += 1;
            if (!isfinite(t)) {
                st->flags |= F_BREAKDOWN;
                st->done = 1;
            } else if (t <= st->tol2) {
                st->flags |= F_CONVERGED;
                st->done = 1;
            }
            break;
        case R_RZ:  // preconditioned CG, after z = M^-1 r: beta from r.z
        case R_RZ_DEFER:  // as R_RZ; rho is left to the next alpha step
            if (!(t > 0.0) || !isfinite(t)) {
                st->flags |= F_BREAKDOWN;
                st->done = 1;
            } else {
                st->beta = t / st->rho;
                if (mode == R_RZ) st->rho = t;
                st->rho_new = t;
                if (st->iter >= st->max_iter) {
                    st->flags |= F_MAXITER;
                    st->done = 1;
                }
            }
            break;
        case R_RZ0:  // preconditioned CG, (re)start: rho = r.z, p = z follows
            st->rho = t;
            st->rho_new = t;
            st->beta = 0.0;
            st->flags = 0;
            st->done = st->iter >= st->max_iter ? 1 : 0;
            if (st->done) st->flags = F_MAXITER;
            if (!(t > 0.0) || !isfinite(t)) {
                st->flags |= F_BREAKDOWN;
                st->done = 1;
            }
            break;
        case R_DIAG:  // Jacobi preconditioner: t counts diagonals that are not positive and finite
            if (t != 0.0) {
                st->flags |= F_BADDIAG;
                st->done = 1;
            }
            break;
        case R_BETA:
        case R_BETA_DEFER:  // as R_BETA; rho is left to the next alpha step
            st->rho_new = t;
            st->iter += 1;
            if (!isfinite(t)) {
                st->flags |= F_BREAKDOWN;
                st->done = 1;
            } else if (t <= st->tol2) {
                st->flags |= F_CONVERGED;
                st->done = 1;
            } else {
                st->beta = t / st->rho;
                if (mode == R_BETA) st->rho = t;
                if (st->iter >= st->max_iter) {
                    st->flags |= F_MAXITER;
                    st->done = 1;
                }
            }
            break;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ part, int n, CgState *st, int mode) {
    __shared__ double sh[kBlock / kWave];
    if ((mode == R_ALPHA || mode == R_BETA || mode == R_RR || mode == R_RZ) && st->done) return;
    const double t = sum_partials(part, n, sh);
    if (threadIdx.x == 0) apply_reduction(st, mode, t);
}

// First stage of a reduction over many partials: workgroup b sums the fixed
// chunk [b*chunk, min(n, (b+1)*chunk)) in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_stage(const double *__restrict__ part, int n, int chunk,
                                                         double *__restrict__ out, const CgState *st, int mode) {
    __shared__ double sh[kBlock / kWave];
    if ((mode == R_ALPHA || mode == R_BETA || mode == R_RR || mode == R_RZ) && st->done) return;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// After a failed true-residual check: continue from r = b - A x.  With
// `fresh` the p update p = r + beta p is left to the fused product.
__global__ void k_replace(CgState *st, int fresh) {
    st->beta = st->rt2 / st->rho;
    st->rho = st->rt2;
    st->rho_new = st->rt2;
    st->flags = 0;
    st->done = st->iter >= st->max_iter ? 1 : 0;
    if (st->done) st->flags = F_MAXITER;
    if (fresh) st->flags |= F_FRESH;
}

// Start of a fused solve: p = 0 (set by the caller) and beta = 0, so the
// first fused product gathers p_new = r.
__global__ void k_set_fresh(CgState *st) {
    st->beta = 0.0;
    st->flags |= F_FRESH;
}

__global__ void k_init_state(CgState *st, double tol, int max_iter) {
    st->tol2 = tol * tol * st->bb;
    st->iter = 0;
    st->max_iter = max_iter;
    st->flags = 0;
    st->done = 0;
    st->alpha = st->beta = st->pq = st->rho_new = 0.0;
}

// alpha for the x/r update.  With n_pq >= 0 every workgroup forms p.q from
// the SpMV's n_pq partials itself (few partials: cheaper than a reduction
// launch) and alpha = rho / p.q from it; with n_pq < 0 alpha was formed by a
// reduction launch.  The sum is sum_partials over the same partials as that
// launch, so the iterates are bit for bit the same.  Returns false on a p.q
// breakdown, which every workgroup detects alike and workgroup 0 records;
// the state's done flag is read once at kernel entry, and within a launch
// only that record sets it.
__device__ __forceinline__ bool form_alpha(CgState *st, const double *__restrict__ part_pq, int n_pq, double *sh,
                                           double *pq_all, double &alpha) {
    if (n_pq < 0) {
        alpha = st->alpha;
        return true;
    }
    const double t = sum_partials(part_pq, n_pq, sh);
    if (threadIdx.x == 0) *pq_all = t;
    __syncthreads();
    const double pq = *pq_all;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) apply_reduction(st, R_ALPHA, pq);
        return false;
    }
    alpha = st->rho_new / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
        st->rho = st->rho_new;
    }
    return true;
}

// x += alpha p, r -= alpha q and the r.r partial of each workgroup
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_xr(int n, int chunk, T *__restrict__ x, T *__restrict__ r,
                                                      const T *__restrict__ p, const T *__restrict__ q,
                                                      CgState *st, const double *__restrict__ part_pq, int n_pq,
                                                      double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    __shared__ double pq_all;
    if (st->done) return;
    double alpha;
    if (!form_alpha(st, part_pq, n_pq, sh, &pq_all, alpha)) return;
    const T a = static_cast<T>(alpha);
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double d = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
        const T xi = x[i] + a * p[i];
        const T ri = r[i] - a * q[i];
        x[i] = xi;
        r[i] = ri;
        d += static_cast<double>(ri) * static_cast<double>(ri);
    }
    const double t = block_sum(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_p(int n, T *__restrict__ p, const T *__restrict__ r,
                                                     const CgState *st) {
    if (st->done) return;
    const T b = static_cast<T>(st->beta);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = r[i] + b * p[i];
}

// p = r + beta p with beta formed in the same launch: when the x/r update
// left few r.r partials, every workgroup sums them itself (sum_partials, the
// order of the reduction launch) and takes beta = r.r / rho from the rho of
// this iteration, which no workgroup writes here.  Workgroup 0 records the
// step (R_BETA_DEFER: iteration count, convergence, beta, rho_new); the next
// alpha step copies rho_new to rho.  The done flag is read at entry and set
// here only where no workgroup updates p (converged, breakdown) or where p
// is no longer read (the iteration cap).  Same beta, bit for bit, as the
// reduction launch followed by k_update_p.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_p_fold(int n, T *__restrict__ p, const T *__restrict__ r,
                                                          CgState *st, const double *__restrict__ part,
                                                          int n_part) {
    __shared__ double sh[kBlock / kWave];
    __shared__ double rr_all;
    if (st->done) return;
    const double t0 = sum_partials(part, n_part, sh);
    if (threadIdx.x == 0) rr_all = t0;
    __syncthreads();
    const double t = rr_all;
    const double rho = st->rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) apply_reduction(st, R_BETA_DEFER, t);
    if (!isfinite(t) || t <= st->tol2) return;
    const T b = static_cast<T>(t / rho);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = r[i] + b * p[i];
}

// Unconditional p = r + beta p (used after a residual replacement).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_p_force(int n, T *__restrict__ p, const T *__restrict__ r,
                                                           const CgState *st) {
    const T b = static_cast<T>(st->beta);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = r[i] + b * p[i];
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The SpMV of a fused iteration: q = A p_new with p_new = r + beta p formed
// for every gathered column and for the tile's own rows (the p.q partial of
// the epilogue), exactly as k_update_p_fold forms it (fma(beta, p, r), beta
// rounded to T).  beta comes from the r.r partials, summed as
// sum_partials sums them, and workgroup 0 records the step (R_BETA_DEFER),
// unless F_FRESH hands beta over in the state.  On these small systems the
// launch is a chain of memory round trips, so every load that does not
// depend on another is issued before any is waited for: the descriptor and
// the state together, then the tile's stream, the row data and the r.r
// partials, then the gathers of p and r, all before beta is formed.  Same
// q and p.q partials, bit for bit, as the p update followed by the plain
// SpMV on p_new.
template <typename T, typename V, int NT>
__global__ __launch_bounds__(kBlock) void k_spmv_pfused(const TileDesc *__restrict__ desc, int n_list, int per_xcd,
                                                        int chunk_log2, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, const V *__restrict__ val,
                                                        const T *__restrict__ p, const T *__restrict__ r,
                                                        T *__restrict__ q, double *__restrict__ part_pq, CgState *st,
                                                        const double *__restrict__ part_rr, int n_rr) {
    using Regs = TileRegs<V, NT>;
    __shared__ T prod[Regs::kProd];
    __shared__ double sh[kBlock / kWave];
    __shared__ double rr_all;
    const int li = xcd_tile(blockIdx.x, per_xcd, chunk_log2);
    if (li >= n_list) return;
    const TileDesc d = desc[li];
    const int done = st->done, flags = st->flags;
    const double rho = st->rho, tol2 = st->tol2, beta_state = st->beta;
    Regs t;
    t.load(col, val, d.s, d.e);
    RowPre<T, EPI_DOT> pre;
    pre.load(row_ptr, p, static_cast<const T *>(nullptr), d.r0, d.r1, d.s & ~3);  // op = p of the tile's rows
    T r_row[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) r_row[i] = r[min(d.r0 + (int)threadIdx.x + i * kBlock, d.r1 - 1)];
    const bool fresh = (flags & F_FRESH) != 0;
    double part = 0.0;  // this lane's share of the r.r sum, in sum_partials' order
    if (!fresh) {
#pragma unroll 4
        for (int i = (int)threadIdx.x; i < n_rr; i += kBlock) part += part_rr[i];
    }
    T pv[Regs::kMaxPass][4], rv[Regs::kMaxPass][4];
    t.gather([p](int c) { return p[c]; }, pv);
    t.gather([r](int c) { return r[c]; }, rv);
    if (done) return;
    double beta = beta_state;
    if (!fresh) {
        const double t0 = block_sum(part, sh);
        if (threadIdx.x == 0) rr_all = t0;
        __syncthreads();
        const double tt = rr_all;
        if (blockIdx.x == 0 && threadIdx.x == 0) apply_reduction(st, R_BETA_DEFER, tt);
        if (!isfinite(tt) || tt <= tol2) return;
        beta = tt / rho;
    }
    const T b = static_cast<T>(beta);
    T xv[Regs::kMaxPass][4];
#pragma unroll
    for (int ps = 0; ps < Regs::kMaxPass; ++ps)
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[ps][j] = fma_t(b, pv[ps][j], rv[ps][j]);
#pragma unroll
    for (int i = 0; i < 2; ++i) pre.op[i] = fma_t(b, pre.op[i], r_row[i]);
    t.products(xv, prod);
    __syncthreads();
    tile_rows<T, T, EPI_DOT>(pre, d.r0, d.r1, prod, q, part_pq, d.seg, sh);
}

// ------------------------------------------------ one reduction per iteration
//
// CG with one reduction phase per iteration (Chronopoulos and Gear, J.
// Comput. Appl. Math. 25, 1989): besides x, r and p it carries w = A r and
// s = A p (by the recurrence s = w + beta s), so that r.r and w.r are taken
// together after the single product and
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
// with gamma = r.r and delta = w.r.  One launch is one iteration: each
// workgroup (one row tile) sums the previous launch's gamma and delta
// partials, forms alpha and beta, and then forms, for every column it
// gathers and every row it owns,
//   s_new = w + beta s,  r_new = r - alpha s_new       (gathered: the product's input)
//   p_new = r + beta p,  x_new = x + alpha p_new       (own rows only)
// and w_new = A r_new with the gamma and delta partials of its rows.  r, w
// and s are read at other workgroups' rows, so they alternate between two
// copies by launch parity, as do the partials and the scalar slots: no
// workgroup reads anything another workgroup of the same launch writes.

struct Cg1Scalars {
    double gamma;   // r.r of the step the slot's launch finished checking
    double alpha;   // the alpha and beta that launch used
    double beta;
    int32_t fresh;  // 1: the reading launch takes alpha and beta from here (a start)
    int32_t iter;   // iterations completed
};

// Start or restart: r (the true residual), w = A r with its w.r partials and
// st->rt2 = r.r are in place, p = s = 0.  Sets the slot the first launch
// reads: alpha0 = r.r / w.r, beta = 0.
__global__ __launch_bounds__(kBlock) void k_cg1_start(CgState *st, Cg1Scalars *slot,
                                                      const double *__restrict__ part_wr, int n) {
    __shared__ double sh[kBlock / kWave];
    const double delta = sum_partials(part_wr, n, sh);
    if (threadIdx.x != 0) return;
    const double gamma = st->rt2;
    st->rho = gamma;
    st->rho_new = gamma;
    st->flags = 0;
    st->done = st->iter >= st->max_iter ? 1 : 0;
    if (st->done) st->flags = F_MAXITER;
    if (!(delta > 0.0) || !isfinite(delta)) {
        st->flags |= F_BREAKDOWN;
        st->done = 1;
    }
    slot->gamma = gamma;
    slot->alpha = gamma / delta;
    slot->beta = 0.0;
    slot->fresh = 1;
    slot->iter = st->iter;
}

template <typename T, typename V, int NT>
__global__ __launch_bounds__(kBlock) void k_cg1(const TileDesc *__restrict__ desc, int n_list, int per_xcd,
                                                int chunk_log2, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, const V *__restrict__ val,
                                                T *__restrict__ x, T *__restrict__ p,
                                                const T *__restrict__ r_in, const T *__restrict__ w_in,
                                                const T *__restrict__ s_in, T *__restrict__ r_out,
                                                T *__restrict__ w_out, T *__restrict__ s_out,
                                                const double *__restrict__ gam_in, const double *__restrict__ del_in,
                                                double *__restrict__ gam_out, double *__restrict__ del_out,
                                                int n_part, const Cg1Scalars *__restrict__ sc_in,
                                                Cg1Scalars *__restrict__ sc_out, CgState *st) {
    using Regs = TileRegs<V, NT>;
    __shared__ T prod[Regs::kProd];
    __shared__ double sh[kBlock / kWave], sh2[kBlock / kWave];
    __shared__ double sums[2];
    const int li = xcd_tile(blockIdx.x, per_xcd, chunk_log2);
    if (li >= n_list) return;
    // every load that does not depend on another goes out before any wait:
    // descriptor and scalars, the tile's stream and rows, own-row vector
    // elements, the partials, then the gathers
    const TileDesc d = desc[li];
    const int done = st->done, max_iter = st->max_iter;
    const double tol2 = st->tol2;
    const Cg1Scalars S = *sc_in;
    Regs t;
    t.load(col, val, d.s, d.e);
    RowPre<T, EPI_DOT> pre;
    pre.load(row_ptr, r_in, static_cast<const T *>(nullptr), d.r0, d.r1, d.s & ~3);  // op = r of own rows
    T w_row[2], s_row[2], p_row[2], x_row[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int j = min(d.r0 + (int)threadIdx.x + i * kBlock, d.r1 - 1);
        w_row[i] = w_in[j];
        s_row[i] = s_in[j];
        p_row[i] = p[j];
        x_row[i] = x[j];
    }
    double pg = 0.0, pd = 0.0;  // this lane's shares of the gamma and delta sums, in sum_partials' order
    if (!S.fresh) {
#pragma unroll 4
        for (int i = (int)threadIdx.x; i < n_part; i += kBlock) {
            pg += gam_in[i];
            pd += del_in[i];
        }
    }
    T rv[Regs::kMaxPass][4], wv[Regs::kMaxPass][4], sv[Regs::kMaxPass][4];
    t.gather([r_in](int c) { return r_in[c]; }, rv);
    t.gather([w_in](int c) { return w_in[c]; }, wv);
    t.gather([s_in](int c) { return s_in[c]; }, sv);
    if (done) return;
    double alpha = S.alpha, beta = S.beta, gamma = S.gamma;
    int iter = S.iter;
    if (!S.fresh) {
        const double g0 = block_sum(pg, sh);
        const double d0 = block_sum(pd, sh2);
        if (threadIdx.x == 0) {
            sums[0] = g0;
            sums[1] = d0;
        }
        __syncthreads();
        const double g = sums[0], dl = sums[1];
        iter += 1;  // the previous launch's iteration, now checked
        beta = g / S.gamma;
        const double den = dl - beta * g / S.alpha;
        alpha = g / den;
        gamma = g;
        // every workgroup takes the same decision from the same sums;
        // workgroup 0 records it
        int32_t stop = 0;
        if (!isfinite(g)) stop = F_BREAKDOWN;
        else if (g <= tol2) stop = F_CONVERGED;
        else if (!(den > 0.0) || !isfinite(den)) stop = F_BREAKDOWN;
        else if (iter >= max_iter) stop = F_MAXITER;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->iter = iter;
            st->rho = g;
            st->rho_new = g;
            st->pq = dl;
            if (stop) {
                st->flags |= stop;
                st->done = 1;
            }
        }
        if (stop) return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc_out->gamma = gamma;
        sc_out->alpha = alpha;
        sc_out->beta = beta;
        sc_out->fresh = 0;
        sc_out->iter = iter;
        st->alpha = alpha;
        st->beta = beta;
    }
    const T a = static_cast<T>(alpha), b = static_cast<T>(beta);
    T xv[Regs::kMaxPass][4];
#pragma unroll
    for (int ps = 0; ps < Regs::kMaxPass; ++ps)
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[ps][j] = fma_t(-a, fma_t(b, sv[ps][j], wv[ps][j]), rv[ps][j]);
    double gp = 0.0;  // r_new.r_new over own rows
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int j = d.r0 + (int)threadIdx.x + i * kBlock;
        const T sn = fma_t(b, s_row[i], w_row[i]);
        const T rn = fma_t(-a, sn, pre.op[i]);
        const T pn = fma_t(b, p_row[i], pre.op[i]);
        if (j < d.r1) {
            s_out[j] = sn;
            r_out[j] = rn;
            p[j] = pn;
            x[j] = fma_t(a, pn, x_row[i]);
            gp += static_cast<double>(rn) * static_cast<double>(rn);
        }
        pre.op[i] = rn;
    }
    t.products(xv, prod);
    const double gt = block_sum(gp, sh2);
    if (threadIdx.x == 0) gam_out[d.seg] = gt;
    __syncthreads();
    tile_rows<T, T, EPI_DOT>(pre, d.r0, d.r1, prod, w_out, del_out, d.seg, sh);
}

// The x/r update of a fused iteration: p_new = r + beta p (as the fused
// product formed it) is written for this workgroup's rows, then x += alpha
// p_new, r -= alpha q and the r.r partial, as k_update_xr.  Workgroup 0
// clears F_FRESH.  The fused path runs on at most 1,024 workgroups, so a
// workgroup's chunk holds at most 1,024 rows, four per lane: the state, the
// p.q partials and all of the lane's vector elements are loaded before any
// is waited for (one memory round trip instead of three).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_xpr(int n, int chunk, T *__restrict__ x, T *__restrict__ r,
                                                       T *__restrict__ p, const T *__restrict__ q, CgState *st,
                                                       const double *__restrict__ part_pq, int n_pq,
                                                       double *__restrict__ part) {
    constexpr int kRows = 4;  // rows per lane: chunk <= kRows * kBlock
    __shared__ double sh[kBlock / kWave];
    __shared__ double pq_all;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    const int done = st->done;
    const double rho_new = st->rho_new, alpha_state = st->alpha, beta = st->beta;
    T xs[kRows], ps[kRows], rs[kRows], qs[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int i = min(lo + (int)threadIdx.x + u * kBlock, n - 1);
        xs[u] = x[i];
        ps[u] = p[i];
        rs[u] = r[i];
        qs[u] = q[i];
    }
    double s = 0.0;  // this lane's share of the p.q sum, in sum_partials' order
    if (n_pq >= 0) {
#pragma unroll 4
        for (int i = (int)threadIdx.x; i < n_pq; i += kBlock) s += part_pq[i];
    }
    if (done) return;
    double alpha = alpha_state;
    if (n_pq >= 0) {
        const double t = block_sum(s, sh);
        if (threadIdx.x == 0) pq_all = t;
        __syncthreads();
        const double pq = pq_all;
        if (!(pq > 0.0) || !isfinite(pq)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) apply_reduction(st, R_ALPHA, pq);
            return;
        }
        alpha = rho_new / pq;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->alpha = alpha;
            st->rho = rho_new;
        }
    }
    const T a = static_cast<T>(alpha);
    const T b = static_cast<T>(beta);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->flags &= ~F_FRESH;
    double dd = 0.0;
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int i = lo + (int)threadIdx.x + u * kBlock;
        if (i < hi) {
            const T pn = fma_t(b, ps[u], rs[u]);
            const T xi = xs[u] + a * pn;
            const T ri = rs[u] - a * qs[u];
            p[i] = pn;
            x[i] = xi;
            r[i] = ri;
            dd += static_cast<double>(ri) * static_cast<double>(ri);
        }
    }
    const double tt = block_sum(dd, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tt;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot_part(int n, int chunk, const T *__restrict__ a,
                                                     const T *__restrict__ b, double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double d = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) d += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    const double t = block_sum(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename D, typename S>
__global__ __launch_bounds__(kBlock) void k_copy(int n, D *__restrict__ d, const S *__restrict__ s) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[i] = static_cast<D>(s[i]);
}

template <typename T> __global__ __launch_bounds__(kBlock) void k_zero(int n, T *__restrict__ d) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[i] = T(0);
}

// r32 = r64 / sqrt(rt2)   (unit-norm right-hand side of the correction solve)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_residual(int n, T *__restrict__ d, const double *__restrict__ s,
                                                           const CgState *st) {
    const double inv = 1.0 / sqrt(st->rt2);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[i] = static_cast<T>(s[i] * inv);
}

// x64 += sqrt(rt2) * d
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_correction(int n, double *__restrict__ x, const T *__restrict__ d,
                                                           const CgState *st) {
    const double sc = sqrt(st->rt2);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        x[i] = x[i] + sc * static_cast<double>(d[i]);
}

// ------------------------------------------- preconditioned CG (bfloat16)
//
// M^-1 r = w D^-1 (2 r - w A~ D^-1 r): a damped two-term Neumann polynomial
// in A~, the bfloat16 copy of A, with D = diag(A) in binary64 and the weight
// w = 1.9 / g, g = max_i sum_j |a~_ij| / sqrt(d_i d_j) (a Gershgorin bound on
// the spectrum of D^-1/2 A~ D^-1/2), so M^-1 = 2w D^-1 - w^2 D^-1 A~ D^-1 is
// symmetric positive definite.  One preconditioner application is one
// bfloat16 SpMV (FP32 vectors and accumulation) between two vector passes.

// dinv_i = 1 / a_ii (duplicates summed); NaN marks a diagonal that is not
// positive and finite.
__global__ __launch_bounds__(kBlock) void k_diag_inv(int n, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, double *__restrict__ dinv) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double d = 0.0;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) d += val[k];
        dinv[i] = (d > 0.0 && isfinite(d)) ? 1.0 / d : __builtin_nan("");
    }
}

// Per workgroup: max over its rows of sum_j |a~_ij| sqrt(dinv_i dinv_j)
// (NaN if any row's is NaN).
__global__ __launch_bounds__(kBlock) void k_gersh(int n, const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col,
                                                  const uint16_t *__restrict__ v16,
                                                  const double *__restrict__ dinv, double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    double m = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double g = 0.0;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            g += fabs(static_cast<double>(__uint_as_float(static_cast<unsigned>(v16[k]) << 16))) *
                 sqrt(dinv[i] * dinv[col[k]]);
        m = (g > m || g != g) ? g : m;   // keeps NaN
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double u = __shfl_xor(m, o);
        m = (u > m || u != u) ? u : m;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t = (sh[w] > t || sh[w] != sh[w]) ? sh[w] : t;
        part[blockIdx.x] = t;
    }
}

// g = max of the partials; w = 1.9 / g, or the bad-diagonal flag.
__global__ __launch_bounds__(kBlock) void k_weight(const double *__restrict__ part, int n, CgState *st) {
    if (threadIdx.x != 0) return;
    double g = 0.0;
    for (int i = 0; i < n; ++i) g = (part[i] > g || part[i] != part[i]) ? part[i] : g;
    if (!(g > 0.0) || !isfinite(g)) {
        st->flags |= F_BADDIAG;
        st->done = 1;
        st->omega = 0.0;
    } else {
        st->omega = 1.9 / g;
    }
}

// t = D^-1 r in FP32 (the bfloat16 product's input)
__global__ __launch_bounds__(kBlock) void k_dinv_f32(int n, float *__restrict__ t, const double *__restrict__ r,
                                                     const double *__restrict__ dinv) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        t[i] = static_cast<float>(dinv[i] * r[i]);
}

// x += alpha p; r -= alpha q; t = D^-1 r (FP32); partial r.r (alpha formed
// here on small systems, as in k_update_xr)
__global__ __launch_bounds__(kBlock) void k_update_xr_pcg(int n, int chunk, double *__restrict__ x,
                                                          double *__restrict__ r, const double *__restrict__ p,
                                                          const double *__restrict__ q,
                                                          const double *__restrict__ dinv, float *__restrict__ t,
                                                          CgState *st, const double *__restrict__ part_pq,
                                                          int n_pq, double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    __shared__ double pq_all;
    if (st->done) return;
    double a;
    if (!form_alpha(st, part_pq, n_pq, sh, &pq_all, a)) return;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double d = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
        const double xi = x[i] + a * p[i];
        const double ri = r[i] - a * q[i];
        x[i] = xi;
        r[i] = ri;
        t[i] = static_cast<float>(dinv[i] * ri);
        d += ri * ri;
    }
    const double tt = block_sum(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tt;
}

// z = w D^-1 (2 r - w s) with s = A~ t; partial r.z
__global__ __launch_bounds__(kBlock) void k_precond_z(int n, int chunk, const double *__restrict__ r,
                                                      const float *__restrict__ s, const double *__restrict__ dinv,
                                                      double *__restrict__ z, const CgState *st,
                                                      double *__restrict__ part, int force) {
    __shared__ double sh[kBlock / kWave];
    if (!force && st->done) return;
    const double w = st->omega;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double d = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
        const double zi = w * dinv[i] * (2.0 * r[i] - w * static_cast<double>(s[i]));
        z[i] = zi;
        d += r[i] * zi;
    }
    const double tt = block_sum(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tt;
}

// ------------------------------------------- preconditioned CG (Jacobi)
//
// M = D = diag(A): z = D^-1 r is fused into the x/r update, and r.r and r.z
// are reduced together, so an iteration takes the launches of plain CG
// (SpMV + p.q; x/r/z update, with alpha formed in it on small systems; the
// r.r / r.z reduction that forms the convergence flag and beta, folded into
// the p update on small systems; p update).

// Per workgroup: how many entries of v are NaN (k_diag_inv marks a diagonal
// that is not positive and finite so).
__global__ __launch_bounds__(kBlock) void k_count_nan(int n, int chunk, const double *__restrict__ v,
                                                      double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double c = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) c += v[i] != v[i] ? 1.0 : 0.0;
    const double t = block_sum(c, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += alpha p; r -= alpha q; z = D^-1 r; partials r.r and r.z
__global__ __launch_bounds__(kBlock) void k_update_xr_jacobi(int n, int chunk, double *__restrict__ x,
                                                             double *__restrict__ r, const double *__restrict__ p,
                                                             const double *__restrict__ q,
                                                             const double *__restrict__ dinv,
                                                             double *__restrict__ z, CgState *st,
                                                             const double *__restrict__ part_pq, int n_pq,
                                                             double *__restrict__ part_rr,
                                                             double *__restrict__ part_rz) {
    __shared__ double sh[kBlock / kWave], sh2[kBlock / kWave];
    __shared__ double pq_all;
    if (st->done) return;
    double a;
    if (!form_alpha(st, part_pq, n_pq, sh, &pq_all, a)) return;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double drr = 0.0, drz = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
        const double xi = x[i] + a * p[i];
        const double ri = r[i] - a * q[i];
        const double zi = dinv[i] * ri;
        x[i] = xi;
        r[i] = ri;
        z[i] = zi;
        drr += ri * ri;
        drz += ri * zi;
    }
    const double trr = block_sum(drr, sh);
    const double trz = block_sum(drz, sh2);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = trr;
        part_rz[blockIdx.x] = trz;
    }
}

// Preconditioned CG: p = z + beta p with the convergence test and beta
// formed in the same launch, as k_update_p_fold does for plain CG: every
// workgroup sums the r.r and r.z partials itself (the order of the
// reduction launches) and workgroup 0 records the step (R_RR, then
// R_RZ_DEFER), so no workgroup reads a field another writes here.
__global__ __launch_bounds__(kBlock) void k_update_p_pcg(int n, double *__restrict__ p,
                                                            const double *__restrict__ z, CgState *st,
                                                            const double *__restrict__ part_rr,
                                                            const double *__restrict__ part_rz, int n_part) {
    __shared__ double sh[kBlock / kWave], sh2[kBlock / kWave];
    __shared__ double rr_all, rz_all;
    if (st->done) return;
    const double a0 = sum_partials(part_rr, n_part, sh);
    const double b0 = sum_partials(part_rz, n_part, sh2);
    if (threadIdx.x == 0) {
        rr_all = a0;
        rz_all = b0;
    }
    __syncthreads();
    const double rr = rr_all, rz = rz_all;
    const double rho = st->rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        apply_reduction(st, R_RR, rr);
        if (!st->done) apply_reduction(st, R_RZ_DEFER, rz);
    }
    if (!isfinite(rr) || rr <= st->tol2 || !(rz > 0.0) || !isfinite(rz)) return;
    const double b = rz / rho;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + b * p[i];
}

// z = D^-1 r and the r.z partial, whatever the done flag (start, restarts)
__global__ __launch_bounds__(kBlock) void k_precond_jacobi(int n, int chunk, const double *__restrict__ r,
                                                           const double *__restrict__ dinv, double *__restrict__ z,
                                                           double *__restrict__ part) {
    __shared__ double sh[kBlock / kWave];
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double d = 0.0;
#pragma unroll 4
    for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
        const double zi = dinv[i] * r[i];
        z[i] = zi;
        d += r[i] * zi;
    }
    const double t = block_sum(d, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The convergence test on r.r, then (unless it stopped) beta from r.z: the
// two reductions k_reduce makes with R_RR and R_RZ, in one launch.
__global__ __launch_bounds__(kBlock) void k_reduce_rr_rz(const double *__restrict__ part_rr,
                                                         const double *__restrict__ part_rz, int n, CgState *st) {
    __shared__ double sh[kBlock / kWave], sh2[kBlock / kWave];
    if (st->done) return;
    const double trr = sum_partials(part_rr, n, sh);
    const double trz = sum_partials(part_rz, n, sh2);
    if (threadIdx.x != 0) return;
    apply_reduction(st, R_RR, trr);
    if (!st->done) apply_reduction(st, R_RZ, trz);
}

// ------------------------------------------------------------ host driver

namespace {

int grid_for(int n) { return std::max(1, std::min(4096, (n + kBlock - 1) / kBlock)); }

// Device workspace allocated stream-ordered (hipMallocAsync on the solve's
// stream, freed with hipFreeAsync), so concurrent solves on different
// streams never synchronise the device through an allocation.  The pinned
// host mirror of the device scalars is either owned here or lent by the
// caller (serving slots keep one per slot).
struct Buffers {
    hipStream_t s;
    std::vector<void *> dev;
    size_t bytes = 0;  // device bytes held
    void *host = nullptr;
    bool own_host = false;
    explicit Buffers(hipStream_t s_) : s(s_) {}
    ~Buffers() {
        for (void *p : dev) (void)hipFreeAsync(p, s);
        if (own_host && host) {
            std::lock_guard<std::mutex> lock(capture_gate());
            (void)hipHostFree(host);
        }
    }
    template <typename T> hipError_t alloc(T **p, size_t n) {
        void *q = nullptr;
        hipError_t e = hipMallocAsync(&q, sizeof(T) * std::max<size_t>(n, 1), s);
        if (e == hipSuccess) {
            dev.push_back(q);
            bytes += sizeof(T) * std::max<size_t>(n, 1);
            *p = static_cast<T *>(q);
        }
        return e;
    }
    hipError_t host_state(void *lent, size_t bytes) {
        if (lent) {
            host = lent;
            return hipSuccess;
        }
        own_host = true;
        std::lock_guard<std::mutex> lock(capture_gate());
        return hipHostMalloc(&host, bytes, hipHostMallocDefault);
    }
};

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

// One CG solve with vectors of type T and values of type V on workspace
// vectors (x, r, p, q).  On entry x holds x0 and `st->bb` holds ||b||^2.
template <typename T, typename V> struct CgCore {
    const DevMatrix &M;
    const V *val;
    int n;
    T *x, *r, *p, *q;
    double *part_seg, *part_vec;
    double *part2;      // first-stage sums of a two-stage reduction
    double *long_ws = nullptr;  // the long rows' piece sums (several workgroups per long row)
    CgState *st;        // device
    CgState *hst;       // pinned host mirror
    int n_wg, chunk, graph_iters;
    hipStream_t s;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    // launch each batch of graph_iters iterations directly on the stream
    // instead of capturing and replaying them (same kernels, same bits)
    bool eager = false;
    // two launches per iteration (k_spmv_pfused + k_update_xpr): the
    // product is plain row tiles (no windows, no long rows) and every
    // workgroup can sum the r.r partials itself
    bool fused = false;

    CgCore(const DevMatrix &M_, const V *val_, int n_, hipStream_t s_) : M(M_), val(val_), n(n_), s(s_) {
        n_wg = std::max(1, std::min(2048, (n + 4 * kBlock - 1) / (4 * kBlock)));
        chunk = (n + n_wg - 1) / n_wg;
        graph_iters = n >= (1 << 20) ? 8 : (n >= (1 << 16) ? 16 : 32);
        fused = n_wg <= kFoldBeta && chunk <= 4 * kBlock && M.block == 1 && M.format == SPMV_FORMAT_CSR &&
                M.n_stream > 0 &&
                M.n_cwin == 0 && M.n_blk == 0 && M.n_long == 0 && M.n_seg == M.n_stream;
    }
    ~CgCore() {
        if (!exec && !graph) return;
        std::lock_guard<std::mutex> lock(capture_gate());
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }

    // Deterministic reduction of n partials into the device scalars: one
    // workgroup for up to 4096 partials, else a fixed-partition first stage
    // over up to kStage1 workgroups and a one-workgroup second stage.
    static constexpr int kStage1 = 256;
    // Up to this many SpMV partials every workgroup of the x/r update sums
    // them itself instead of waiting for a reduction launch (4,096: 398K and
    // 775K rows, 1,920 and 3,745 tiles, 6% and 4% faster per iteration than
    // with a reduction launch; k_reduce sums up to 4,096 partials in the
    // same order, so alpha has the same bits either way).
    static constexpr int kFoldAlpha = 4096;
    // Up to this many r.r partials (systems up to 1,048,576 rows) every
    // workgroup of the p update forms beta itself (measured: -7% per
    // iteration at 398,000 rows, -1.5% at 775,058).
    static constexpr int kFoldBeta = 1024;
    void reduce(const double *part, int n, int mode, hipStream_t t) {
        if (n <= 4096) {
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, t, part, n, st, mode);
            return;
        }
        const int chunk = (n + kStage1 - 1) / kStage1;
        const int nb = (n + chunk - 1) / chunk;
        hipLaunchKernelGGL(k_reduce_stage, dim3(nb), dim3(kBlock), 0, t, part, n, chunk, part2, st, mode);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, t, part2, nb, st, mode);
    }

    template <int NT> void launch_pfused_nt(hipStream_t t, int per_xcd, int grid) {
        hipLaunchKernelGGL((k_spmv_pfused<T, V, NT>), dim3(grid), dim3(kBlock), 0, t, M.stream_desc, M.n_stream,
                           per_xcd, M.xcd_chunk_log2, M.row_ptr, M.col, val, p, r, q, part_seg, st, part_vec, n_wg);
    }

    // one iteration in two launches (three with a reduction launch for alpha)
    hipError_t fused_iteration(hipStream_t t) {
        const int per_xcd = M.xcd_remap && M.n_stream >= 16 ? (M.n_stream + 7) / 8 : 0;
        const int grid = xcd_grid(M.n_stream, per_xcd, M.xcd_chunk_log2);
        switch (M.tile_nnz) {
            case 1024: launch_pfused_nt<1024>(t, per_xcd, grid); break;
            case 2048: launch_pfused_nt<2048>(t, per_xcd, grid); break;
            default: launch_pfused_nt<4096>(t, per_xcd, grid); break;
        }
        const bool fold_alpha = M.n_seg <= kFoldAlpha;
        if (!fold_alpha) reduce(part_seg, M.n_seg, R_ALPHA, t);
        hipLaunchKernelGGL((k_update_xpr<T>), dim3(n_wg), dim3(kBlock), 0, t, n, chunk, x, r, p, q, st, part_seg,
                           fold_alpha ? M.n_seg : -1, part_vec);
        return hipGetLastError();
    }

    hipError_t iteration(hipStream_t t) {
        if (fused) return fused_iteration(t);
        const int *done = &st->done;
        hipError_t e = launch_spmv<V, T, T, T>(M, val, p, q, EPI_DOT, nullptr, part_seg, done, t, long_ws);
        if (e != hipSuccess) return e;
        const bool fold_alpha = M.n_seg <= kFoldAlpha;
        if (!fold_alpha) reduce(part_seg, M.n_seg, R_ALPHA, t);
        hipLaunchKernelGGL((k_update_xr<T>), dim3(n_wg), dim3(kBlock), 0, t, n, chunk, x, r, p, q, st, part_seg,
                           fold_alpha ? M.n_seg : -1, part_vec);
        if (n_wg <= kFoldBeta) {
            hipLaunchKernelGGL((k_update_p_fold<T>), dim3(grid_for(n)), dim3(kBlock), 0, t, n, p, r, st, part_vec,
                               n_wg);
        } else {
            reduce(part_vec, n_wg, R_BETA, t);
            hipLaunchKernelGGL((k_update_p<T>), dim3(grid_for(n)), dim3(kBlock), 0, t, n, p, r, st);
        }
        return hipGetLastError();
    }

    int capture() {
        return capture_with([this](hipStream_t t) { return iteration(t); });
    }

    // Captures graph_iters calls of iter(stream) into one replayable graph,
    // with the capture gate held (one capture at a time in the process, and
    // none during the library's synchronous runtime work).
    double capture_s = 0.0;  // host time spent capturing and instantiating

    template <typename F> int capture_with(F &&iter) {
        std::lock_guard<std::mutex> lock(capture_gate());
        const auto t0 = std::chrono::steady_clock::now();
        struct Timer {
            double &acc;
            std::chrono::steady_clock::time_point t0;
            ~Timer() { acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
        } timer{capture_s, t0};
        hipStream_t cs;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < graph_iters && e == hipSuccess; ++i) e = iter(cs);
            hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return hip_fail(e, "CG graph capture");
        return SPMV_OK;
    }

    int read_state() {
        HIP_TRY(hipMemcpyAsync(hst, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SPMV_OK;
    }

    // r = b - A x and its squared norm into st->rt2 (values of type V)
    hipError_t true_residual(const T *b) {
        hipError_t e = launch_spmv<V, T, T, T>(M, val, x, r, EPI_RESID, b, part_seg, nullptr, s, long_ws);
        if (e != hipSuccess) return e;
        reduce(part_seg, M.n_seg, R_TRUE, s);
        return hipGetLastError();
    }

    // Runs CG to tol (relative to sqrt(st->bb)).  Returns SPMV_OK, ENOTCONV or
    // EBREAK; *iters and *replacements are accumulated.  With confirm = false
    // the recursive residual alone decides (the correction solve of the
    // refinement loop, whose accuracy the binary64 outer residual checks).
    int solve(const T *b, double tol, int max_iter, int *iters, int *replacements, bool confirm = true) {
        hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, tol, max_iter);
        HIP_TRY(true_residual(b));
        reduce(part_seg, M.n_seg, R_RHO0, s);
        if (fused) {
            // p = 0 and beta = 0: the first fused product gathers p_new = r
            hipLaunchKernelGGL((k_zero<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p);
            hipLaunchKernelGGL(k_set_fresh, dim3(1), dim3(1), 0, s, st);
        } else {
            hipLaunchKernelGGL((k_copy<T, T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p, r);
        }
        HIP_TRY(hipGetLastError());
        int rc = read_state();
        if (rc) return rc;
        if (hst->rho <= hst->tol2) return SPMV_OK;
        if (max_iter <= 0) return SPMV_ENOTCONV;
        if (!exec && !eager) {
            rc = capture();
            if (rc) return rc;
        }
        int done_iters = 0;
        for (;;) {
            if (eager) {
                for (int i = 0; i < graph_iters; ++i) HIP_TRY(iteration(s));
            } else {
                HIP_TRY(hipGraphLaunch(exec, s));
            }
            rc = read_state();
            if (rc) return rc;
            done_iters = hst->iter;
            if (hst->flags & F_BREAKDOWN) {
                *iters += done_iters;
                return SPMV_EBREAK;
            }
            if (hst->flags & F_CONVERGED) {
                if (!confirm) break;
                HIP_TRY(true_residual(b));
                rc = read_state();
                if (rc) return rc;
                if (hst->rt2 <= hst->tol2) break;
                // recursive residual drifted from the true one: replace it
                ++*replacements;
                hipLaunchKernelGGL(k_replace, dim3(1), dim3(1), 0, s, st, fused ? 1 : 0);
                if (!fused)
                    hipLaunchKernelGGL((k_update_p_force<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p, r, st);
                HIP_TRY(hipGetLastError());
                rc = read_state();
                if (rc) return rc;
                if (hst->flags & F_MAXITER) {
                    *iters += hst->iter;
                    return SPMV_ENOTCONV;
                }
                continue;
            }
            if ((hst->flags & F_MAXITER) || hst->iter >= max_iter) {
                *iters += hst->iter;
                return SPMV_ENOTCONV;
            }
        }
        *iters += done_iters;
        return SPMV_OK;
    }
};

template <typename T, typename V>
int alloc_core(Buffers &B, CgCore<T, V> &C) {
    HIP_TRY(B.alloc(&C.x, C.n));
    HIP_TRY(B.alloc(&C.r, C.n));
    HIP_TRY(B.alloc(&C.p, C.n));
    HIP_TRY(B.alloc(&C.q, C.n));
    HIP_TRY(B.alloc(&C.part_seg, (size_t)std::max(C.M.n_seg, 1)));
    HIP_TRY(B.alloc(&C.part_vec, (size_t)C.n_wg));
    HIP_TRY(B.alloc(&C.part2, (size_t)CgCore<T, V>::kStage1));
    if (C.M.piece_long) HIP_TRY(B.alloc(&C.long_ws, (size_t)C.M.n_long_pieces));
    HIP_TRY(B.alloc(&C.st, 1));
    return SPMV_OK;
}

// Preconditioned CG: CgCore's buffers and reductions plus z and D^-1, and
// for the bfloat16 polynomial preconditioner the FP32 vectors of its
// product.  Polynomial: eight launches per iteration on the largest systems
// (SpMV + p.q, alpha, x/r update + r.r + t = D^-1 r, convergence, bfloat16
// SpMV, z + r.z, beta, p update), five on small ones, where alpha is formed
// in the x/r update and the convergence test and beta in the p update.
// Jacobi: three to five (see its kernels).
struct PcgCore : CgCore<double, double> {
    double *z = nullptr, *dinv = nullptr, *part_rz = nullptr;
    float *t = nullptr, *sv = nullptr;
    bool jacobi;

    PcgCore(const DevMatrix &M_, int n_, hipStream_t s_, bool jacobi_)
        : CgCore<double, double>(M_, M_.val64, n_, s_), jacobi(jacobi_) {
        fused = false;  // preconditioned iterations have kernels of their own
    }

    hipError_t pcg_iteration(hipStream_t ts) {
        const int *done = &st->done;
        hipError_t e = launch_spmv<double, double, double, double>(M, val, p, q, EPI_DOT, nullptr, part_seg, done, ts,
                                                                     long_ws);
        if (e != hipSuccess) return e;
        if (jacobi) {
            const bool fold_alpha = M.n_seg <= kFoldAlpha;
            if (!fold_alpha) reduce(part_seg, M.n_seg, R_ALPHA, ts);
            hipLaunchKernelGGL(k_update_xr_jacobi, dim3(n_wg), dim3(kBlock), 0, ts, n, chunk, x, r, p, q, dinv, z,
                               st, part_seg, fold_alpha ? M.n_seg : -1, part_vec, part_rz);
            if (n_wg <= kFoldBeta) {
                hipLaunchKernelGGL(k_update_p_pcg, dim3(grid_for(n)), dim3(kBlock), 0, ts, n, p, z, st, part_vec,
                                   part_rz, n_wg);
            } else {
                hipLaunchKernelGGL(k_reduce_rr_rz, dim3(1), dim3(kBlock), 0, ts, part_vec, part_rz, n_wg, st);
                hipLaunchKernelGGL((k_update_p<double>), dim3(grid_for(n)), dim3(kBlock), 0, ts, n, p, z, st);
            }
            return hipGetLastError();
        }
        const bool fold_alpha = M.n_seg <= kFoldAlpha, fold_beta = n_wg <= kFoldBeta;
        if (!fold_alpha) reduce(part_seg, M.n_seg, R_ALPHA, ts);
        hipLaunchKernelGGL(k_update_xr_pcg, dim3(n_wg), dim3(kBlock), 0, ts, n, chunk, x, r, p, q, dinv, t, st,
                           part_seg, fold_alpha ? M.n_seg : -1, part_vec);
        // folded: the convergence test waits for the p update, so on the last
        // iteration the preconditioner runs once more (it writes neither x nor r)
        if (!fold_beta) reduce(part_vec, n_wg, R_RR, ts);
        e = launch_spmv<uint16_t, float, float, float>(M, M.val16, t, sv, EPI_PLAIN, nullptr, nullptr, done, ts,
                                                          long_ws);
        if (e != hipSuccess) return e;
        double *rz = fold_beta ? part_rz : part_vec;
        hipLaunchKernelGGL(k_precond_z, dim3(n_wg), dim3(kBlock), 0, ts, n, chunk, r, sv, dinv, z, st, rz, 0);
        if (fold_beta) {
            hipLaunchKernelGGL(k_update_p_pcg, dim3(grid_for(n)), dim3(kBlock), 0, ts, n, p, z, st, part_vec,
                               part_rz, n_wg);
        } else {
            reduce(part_vec, n_wg, R_RZ, ts);
            hipLaunchKernelGGL((k_update_p<double>), dim3(grid_for(n)), dim3(kBlock), 0, ts, n, p, z, st);
        }
        return hipGetLastError();
    }

    // D^-1 and the polynomial weight (st->omega), or F_BADDIAG
    hipError_t setup() {
        hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(n)), dim3(kBlock), 0, s, n, M.row_ptr, M.col, M.val64, dinv);
        if (jacobi) {
            hipLaunchKernelGGL(k_count_nan, dim3(n_wg), dim3(kBlock), 0, s, n, chunk, dinv, part_vec);
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, part_vec, n_wg, st, (int)R_DIAG);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_gersh, dim3(n_wg), dim3(kBlock), 0, s, n, M.row_ptr, M.col, M.val16, dinv, part_vec);
        hipLaunchKernelGGL(k_weight, dim3(1), dim3(kWave), 0, s, part_vec, n_wg, st);
        return hipGetLastError();
    }

    // From the current r: z = M^-1 r, rho = r.z, p = z (start and restarts)
    hipError_t restart() {
        if (jacobi) {
            hipLaunchKernelGGL(k_precond_jacobi, dim3(n_wg), dim3(kBlock), 0, s, n, chunk, r, dinv, z, part_vec);
            reduce(part_vec, n_wg, R_RZ0, s);
            hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p, z);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_dinv_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, n, t, r, dinv);
        hipError_t e = launch_spmv<uint16_t, float, float, float>(M, M.val16, t, sv, EPI_PLAIN, nullptr, nullptr,
                                                                  nullptr, s, long_ws);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_precond_z, dim3(n_wg), dim3(kBlock), 0, s, n, chunk, r, sv, dinv, z, st, part_vec, 1);
        reduce(part_vec, n_wg, R_RZ0, s);
        hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p, z);
        return hipGetLastError();
    }

    int pcg_solve(const double *b, double tol, int max_iter, int *iters, int *restarts) {
        hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, tol, max_iter);
        HIP_TRY(setup());
        int rc = read_state();
        if (rc) return rc;
        if (hst->flags & F_BADDIAG)
            return fail(SPMV_EBREAK, "preconditioned CG needs a positive finite diagonal");
        HIP_TRY(true_residual(b));
        HIP_TRY(restart());
        rc = read_state();
        if (rc) return rc;
        if (hst->rt2 <= hst->tol2) return SPMV_OK;
        if (hst->flags & F_BREAKDOWN) return SPMV_EBREAK;
        if (max_iter <= 0) return SPMV_ENOTCONV;
        if (!exec) {
            rc = capture_with([this](hipStream_t ts) { return pcg_iteration(ts); });
            if (rc) return rc;
        }
        for (;;) {
            HIP_TRY(hipGraphLaunch(exec, s));
            rc = read_state();
            if (rc) return rc;
            if (hst->flags & F_BREAKDOWN) {
                *iters = hst->iter;
                return SPMV_EBREAK;
            }
            if (hst->flags & F_CONVERGED) {
                HIP_TRY(true_residual(b));
                rc = read_state();
                if (rc) return rc;
                if (hst->rt2 <= hst->tol2) break;
                // the recursive residual drifted: restart from r = b - A x
                ++*restarts;
                HIP_TRY(restart());
                rc = read_state();
                if (rc) return rc;
                if (hst->flags & F_BREAKDOWN) {
                    *iters = hst->iter;
                    return SPMV_EBREAK;
                }
                if (hst->flags & F_MAXITER) {
                    *iters = hst->iter;
                    return SPMV_ENOTCONV;
                }
                continue;
            }
            if ((hst->flags & F_MAXITER) || hst->iter >= max_iter) {
                *iters = hst->iter;
                return SPMV_ENOTCONV;
            }
        }
        *iters = hst->iter;
        return SPMV_OK;
    }
};

}  // namespace

// ------------------------------------------------ one-reduction CG driver
//
// One launch of k_cg1 per iteration, graph_iters (even) of them per graph
// replay: the launch of parity j reads copy j of r, w, s and of the partials
// written by the launch before it, and slot 1 - j of the scalars, and writes
// the other copies, so each replay starts from copy 0 and slot 1.  Start and
// restart (after the recursive r.r met the tolerance but the true residual
// did not): r = b - A x, w = A r with the w.r partials, p = s = 0, and
// k_cg1_start sets slot 1 to alpha0 = r.r / w.r, beta = 0.

// Plain row tiles only, and at most this many of them, so that every
// workgroup can sum the previous launch's partials itself.
constexpr int kCg1MaxTiles = 4096;

bool cg1_eligible(const DevMatrix &M) {
    return M.block == 1 && M.format == SPMV_FORMAT_CSR && M.n_stream > 0 && M.n_cwin == 0 && M.n_blk == 0 &&
           M.n_long == 0 && M.n_seg == M.n_stream && M.n_stream <= kCg1MaxTiles &&
           (M.tile_nnz == 1024 || M.tile_nnz == 2048 || M.tile_nnz == 4096);
}

struct Cg1Core : CgCore<double, double> {
    double *r2 = nullptr, *w[2] = {nullptr, nullptr}, *sv[2] = {nullptr, nullptr};
    double *gam[2] = {nullptr, nullptr}, *del[2] = {nullptr, nullptr};
    Cg1Scalars *sc = nullptr;  // two slots
    Cg1Core(const DevMatrix &M_, int n_, hipStream_t s_) : CgCore<double, double>(M_, M_.val64, n_, s_) {
        fused = false;
    }

    template <int NT> void launch_nt(hipStream_t t, int par, int per_xcd, int grid) {
        const double *r_in = par ? r2 : r;
        double *r_out = par ? r : r2;
        hipLaunchKernelGGL((k_cg1<double, double, NT>), dim3(grid), dim3(kBlock), 0, t, M.stream_desc, M.n_stream,
                           per_xcd, M.xcd_chunk_log2, M.row_ptr, M.col, val, x, p, r_in, w[par], sv[par], r_out,
                           w[1 - par], sv[1 - par], gam[1 - par], del[1 - par], gam[par], del[par], M.n_seg,
                           sc + (1 - par), sc + par, st);
    }

    hipError_t iteration1(hipStream_t t, int par) {
        const int per_xcd = M.xcd_remap && M.n_stream >= 16 ? (M.n_stream + 7) / 8 : 0;
        const int grid = xcd_grid(M.n_stream, per_xcd, M.xcd_chunk_log2);
        switch (M.tile_nnz) {
            case 1024: launch_nt<1024>(t, par, per_xcd, grid); break;
            case 2048: launch_nt<2048>(t, par, per_xcd, grid); break;
            default: launch_nt<4096>(t, par, per_xcd, grid); break;
        }
        return hipGetLastError();
    }

    // r = b - A x (copy 0), w = A r, p = s = 0, slot 1 set; st->rt2 = r.r
    hipError_t start(const double *b) {
        hipError_t e = true_residual(b);
        if (e != hipSuccess) return e;
        e = launch_spmv<double, double, double, double>(M, val, r, w[0], EPI_DOT, nullptr, part_seg, nullptr, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_cg1_start, dim3(1), dim3(kBlock), 0, s, st, sc + 1, part_seg, M.n_seg);
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, p);
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, sv[0]);
        return hipGetLastError();
    }

    int solve1(const double *b, double tol, int max_iter, int *iters, int *restarts) {
        hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, tol, max_iter);
        HIP_TRY(start(b));
        int rc = read_state();
        if (rc) return rc;
        if (hst->rt2 <= hst->tol2) return SPMV_OK;
        if (max_iter <= 0) return SPMV_ENOTCONV;
        if (hst->flags & F_BREAKDOWN) return SPMV_EBREAK;
        if (!exec) {
            int j = 0;
            rc = capture_with([this, &j](hipStream_t t) { return iteration1(t, (j++) & 1); });
            if (rc) return rc;
        }
        for (;;) {
            HIP_TRY(hipGraphLaunch(exec, s));
            rc = read_state();
            if (rc) return rc;
            if (hst->flags & F_BREAKDOWN) {
                *iters += hst->iter;
                return SPMV_EBREAK;
            }
            if (hst->flags & F_CONVERGED) {
                HIP_TRY(true_residual(b));
                rc = read_state();
                if (rc) return rc;
                if (hst->rt2 <= hst->tol2) break;
                ++*restarts;  // the recursive residual drifted from the true one
                HIP_TRY(start(b));
                rc = read_state();
                if (rc) return rc;
                if (hst->flags & F_BREAKDOWN) {
                    *iters += hst->iter;
                    return SPMV_EBREAK;
                }
                if (hst->flags & F_MAXITER) {
                    *iters += hst->iter;
                    return SPMV_ENOTCONV;
                }
                continue;
            }
            if ((hst->flags & F_MAXITER) || hst->iter >= max_iter) {
                *iters += hst->iter;
                return SPMV_ENOTCONV;
            }
        }
        *iters += hst->iter;
        return SPMV_OK;
    }
};

// ------------------------------------------------------- solver cache
struct CgCache {
    uint64_t serial = 0;  // the matrix handle's serial (0: empty)
    int mode = -1;
    hipStream_t s = nullptr;
    void *pinned = nullptr;
    std::unique_ptr<Buffers> B;
    std::unique_ptr<CgCore<double, double>> C;
    std::unique_ptr<Cg1Core> C1;
    // the same handle and mode; the stream and a lent pinned mirror may
    // differ (the last solve synchronised its stream, so the workspace is idle)
    bool matches(const spmv_matrix *A, int m, void *pn) const {
        return serial == A->serial && mode == m && (pn == pinned || (pn && pinned));
    }
    // the cores first: their graphs are destroyed before the buffers they use
    void clear() {
        C.reset();
        C1.reset();
        B.reset();
        serial = 0;
        mode = -1;
    }
};

void cg_cache_free(CgCache *c) {
    if (!c) return;
    c->clear();
    delete c;
}

size_t cg_cache_bytes(const CgCache *c) { return c && c->B ? c->B->bytes : 0; }

// The workspace and core of a solve: the cached ones when the cache holds
// this (matrix, mode, stream, pinned mirror), else new ones, which go into
// the cache when there is one.
template <typename Core, typename Make>
static int acquire_core(CgCache *cache, std::unique_ptr<Core> CgCache::*slot, const spmv_matrix *A, int mode,
                        hipStream_t s, void *pinned, std::unique_ptr<Buffers> &ownB, std::unique_ptr<Core> &ownC,
                        Core *&core, Make &&make) {
    if (cache && (cache->*slot) && cache->matches(A, mode, pinned)) {
        core = (cache->*slot).get();
        // this solve's stream and pinned mirror (the captured graph uses neither)
        core->s = s;
        cache->B->s = s;
        cache->s = s;
        if (pinned) {
            cache->B->host = pinned;
            cache->pinned = pinned;
            core->hst = static_cast<CgState *>(pinned);
        }
        return SPMV_OK;
    }
    if (cache) cache->clear();
    ownB.reset(new (std::nothrow) Buffers(s));
    if (!ownB) return fail(SPMV_ENOMEM, "host allocation failed");
    int rc = make(*ownB, ownC);
    if (rc) return rc;
    HIP_TRY(ownB->host_state(pinned, 2 * sizeof(CgState)));
    ownC->hst = static_cast<CgState *>(ownB->host);
    core = ownC.get();
    if (cache) {
        cache->serial = A->serial;
        cache->mode = mode;
        cache->s = s;
        cache->pinned = pinned;
        cache->B = std::move(ownB);
        cache->*slot = std::move(ownC);
    }
    return SPMV_OK;
}

static int cg_fp64_body(CgCore<double, double> &C, const double *b, double *x, double tol, int max_iter,
                        cg_info *info, hipStream_t s) {
    const int n = C.n;
    const double capture0 = C.capture_s;
    // ||b||^2
    hipLaunchKernelGGL((k_dot_part<double>), dim3(C.n_wg), dim3(kBlock), 0, s, n, C.chunk, b, b, C.part_vec);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, C.part_vec, C.n_wg, C.st, (int)R_BB);
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, C.x, x);
    HIP_TRY(hipGetLastError());
    int rc = C.read_state();
    if (rc) return rc;
    if (C.hst->bb == 0.0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) info->rel_residual = 0.0;
        return SPMV_OK;
    }
    int iters = 0, repl = 0;
    rc = C.solve(b, tol, max_iter, &iters, &repl);
    if (rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) return rc;
    int rc2;
    HIP_TRY(C.true_residual(b));
    if ((rc2 = C.read_state())) return rc2;
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, C.x);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->refinements = repl;
        info->graph_seconds = C.capture_s - capture0;
        info->rel_residual = std::sqrt(C.hst->rt2 / C.hst->bb);
    }
    if (rc == SPMV_ENOTCONV) return fail(rc, "CG did not reach tol = %g within %d iterations", tol, max_iter);
    if (rc == SPMV_EBREAK) return fail(rc, "CG breakdown (p.q <= 0 or not finite): matrix not SPD?");
    return SPMV_OK;
}

static int cg_fp64(const spmv_matrix *A, const double *b, double *x, double tol, int max_iter, cg_info *info,
                   hipStream_t s, void *pinned, CgCache *cache) {
    const DevMatrix &M = A->M;
    std::unique_ptr<Buffers> ownB;
    std::unique_ptr<CgCore<double, double>> ownC;
    CgCore<double, double> *C = nullptr;
    int rc = acquire_core(cache, &CgCache::C, A, CG_FP64, s, pinned, ownB, ownC, C,
                          [&](Buffers &B, std::unique_ptr<CgCore<double, double>> &c) {
                              c.reset(new (std::nothrow) CgCore<double, double>(M, M.val64, M.n_rows, s));
                              if (!c) return fail(SPMV_ENOMEM, "host allocation failed");
                              return alloc_core(B, *c);
                          });
    if (!rc) rc = cg_fp64_body(*C, b, x, tol, max_iter, info, s);
    // a solve that failed on the device leaves its workspace in no known state
    if (cache && rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) cache->clear();
    return rc;
}

static int cg1_body(Cg1Core &C, const double *b, double *x, double tol, int max_iter, cg_info *info,
                    hipStream_t s) {
    const int n = C.n;
    const double capture0 = C.capture_s;
    hipLaunchKernelGGL((k_dot_part<double>), dim3(C.n_wg), dim3(kBlock), 0, s, n, C.chunk, b, b, C.part_vec);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, C.part_vec, C.n_wg, C.st, (int)R_BB);
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, C.x, x);
    HIP_TRY(hipGetLastError());
    int rc = C.read_state();
    if (rc) return rc;
    if (C.hst->bb == 0.0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) info->rel_residual = 0.0;
        return SPMV_OK;
    }
    int iters = 0, restarts = 0;
    rc = C.solve1(b, tol, max_iter, &iters, &restarts);
    if (rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) return rc;
    int rc2;
    HIP_TRY(C.true_residual(b));
    if ((rc2 = C.read_state())) return rc2;
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, C.x);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->refinements = restarts;
        info->graph_seconds = C.capture_s - capture0;
        info->rel_residual = std::sqrt(C.hst->rt2 / C.hst->bb);
    }
    if (rc == SPMV_ENOTCONV) return fail(rc, "CG did not reach tol = %g within %d iterations", tol, max_iter);
    if (rc == SPMV_EBREAK) return fail(rc, "CG breakdown (w.r - beta r.r / alpha <= 0 or not finite): matrix not SPD?");
    return SPMV_OK;
}

static int cg_fp64_one_reduction(const spmv_matrix *A, const double *b, double *x, double tol, int max_iter,
                                 cg_info *info, hipStream_t s, void *pinned, CgCache *cache) {
    const DevMatrix &M = A->M;
    if (!cg1_eligible(M))
        return fail(SPMV_ENOTSUP,
                    "one-reduction CG needs a CSR handle of plain row tiles (no windows, no row longer than a "
                    "tile) with at most %d tiles (this one: %d plain tiles, %d window tiles, %d ring blocks, %d long "
                    "rows)",
                    kCg1MaxTiles, M.n_stream, M.n_cwin, M.n_blk, M.n_long);
    const int n = M.n_rows;
    std::unique_ptr<Buffers> ownB;
    std::unique_ptr<Cg1Core> ownC;
    Cg1Core *C = nullptr;
    int rc = acquire_core(cache, &CgCache::C1, A, CG_FP64_ONE_REDUCTION, s, pinned, ownB, ownC, C,
                          [&](Buffers &B, std::unique_ptr<Cg1Core> &c) {
                              c.reset(new (std::nothrow) Cg1Core(M, n, s));
                              if (!c) return fail(SPMV_ENOMEM, "host allocation failed");
                              int r = alloc_core(B, *c);
                              if (r) return r;
                              HIP_TRY(B.alloc(&c->r2, (size_t)n));
                              for (int k = 0; k < 2; ++k) {
                                  HIP_TRY(B.alloc(&c->w[k], (size_t)n));
                                  HIP_TRY(B.alloc(&c->sv[k], (size_t)n));
                                  HIP_TRY(B.alloc(&c->gam[k], (size_t)M.n_seg));
                                  HIP_TRY(B.alloc(&c->del[k], (size_t)M.n_seg));
                              }
                              HIP_TRY(B.alloc(&c->sc, 2));
                              return (int)SPMV_OK;
                          });
    if (!rc) rc = cg1_body(*C, b, x, tol, max_iter, info, s);
    if (cache && rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) cache->clear();
    return rc;
}

// ------------------------------------------------- allocation-free FP64 CG
//
// cg_solve_noalloc runs cg_fp64's kernels, in the same order, on a
// workspace that is a file-scope device array instead of stream-ordered
// allocations: r, p, q and the SpMV partials (n_seg <= n) for up to
// kNoallocMaxRows rows, the per-workgroup partials, the two-stage reduction's
// first stage and the device scalars.  The caller's x is the iterate itself.
// Iterations are launched directly (no graph to instantiate) and the scalar
// state is read into pageable host memory, so a solve calls no allocating
// runtime routine.  One array per device, shared by every call on it.
constexpr int kNoallocMaxRows = 1 << 19;
constexpr size_t kNoallocPartVec = 2048, kNoallocPart2 = 256, kNoallocState = 16;
constexpr size_t kNoallocWords = 4 * (size_t)kNoallocMaxRows + kNoallocPartVec + kNoallocPart2 + kNoallocState;
static_assert(sizeof(CgState) <= kNoallocState * sizeof(double), "scalar state slot too small");

static __device__ __align__(256) double scratch[kNoallocWords];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};

// The device address of this device's scratch array.  Resolved once per
// device (with that device current) on its first call; in host code the
// array's name is not a device address.
int scratch_of(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SPMV_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return SPMV_OK;
}
}  // namespace

static int cg_fp64_noalloc(const spmv_matrix *A, const double *b, double *x, double tol, int max_iter,
                           cg_info *info, hipStream_t s, double *scr) {
    const DevMatrix &M = A->M;
    const int n = M.n_rows;
    const size_t N = kNoallocMaxRows;
    CgCore<double, double> C(M, M.val64, n, s);
    C.eager = true;
    C.x = x;
    C.r = scr;
    C.p = scr + N;
    C.q = scr + 2 * N;
    C.part_seg = scr + 3 * N;
    C.part_vec = scr + 4 * N;
    C.part2 = scr + 4 * N + kNoallocPartVec;
    C.st = reinterpret_cast<CgState *>(scr + 4 * N + kNoallocPartVec + kNoallocPart2);
    CgState host_state{};
    C.hst = &host_state;
    // ||b||^2
    hipLaunchKernelGGL((k_dot_part<double>), dim3(C.n_wg), dim3(kBlock), 0, s, n, C.chunk, b, b, C.part_vec);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, C.part_vec, C.n_wg, C.st, (int)R_BB);
    HIP_TRY(hipGetLastError());
    int rc = C.read_state();
    if (rc) return rc;
    if (C.hst->bb == 0.0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) info->rel_residual = 0.0;
        return SPMV_OK;
    }
    int iters = 0, repl = 0;
    rc = C.solve(b, tol, max_iter, &iters, &repl);
    if (rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) return rc;
    int rc2;
    HIP_TRY(C.true_residual(b));
    if ((rc2 = C.read_state())) return rc2;
    if (info) {
        info->iterations = iters;
        info->refinements = repl;
        info->graph_seconds = C.capture_s;
        info->rel_residual = std::sqrt(C.hst->rt2 / C.hst->bb);
    }
    if (rc == SPMV_ENOTCONV) return fail(rc, "CG did not reach tol = %g within %d iterations", tol, max_iter);
    if (rc == SPMV_EBREAK) return fail(rc, "CG breakdown (p.q <= 0 or not finite): matrix not SPD?");
    return SPMV_OK;
}

// Iterative refinement whose correction solves read the FP32 values; T is
// the correction solve's vector and accumulation type (float, or double for
// products that round only the stored values).
template <typename T>
static int cg_mixed(const spmv_matrix *A, const double *b, double *x, double tol, int max_iter, cg_info *info,
                    hipStream_t s, double inner_tol, void *pinned) {
    const DevMatrix &M = A->M;
    const int n = M.n_rows;
    Buffers B(s);
    // outer (binary64) residual machinery reuses a CgCore for its buffers
    CgCore<double, double> O(M, M.val64, n, s);
    CgCore<T, float> I(M, M.val32, n, s);
    int rc = alloc_core(B, O);
    if (!rc) rc = alloc_core(B, I);
    if (rc) return rc;
    HIP_TRY(B.host_state(pinned, 2 * sizeof(CgState)));
    O.hst = static_cast<CgState *>(B.host);
    I.hst = O.hst + 1;
    hipLaunchKernelGGL((k_dot_part<double>), dim3(O.n_wg), dim3(kBlock), 0, s, n, O.chunk, b, b, O.part_vec);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, O.part_vec, O.n_wg, O.st, (int)R_BB);
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, O.x, x);
    HIP_TRY(hipGetLastError());
    rc = O.read_state();
    if (rc) return rc;
    const double bb = O.hst->bb;
    if (bb == 0.0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) info->rel_residual = 0.0;
        return SPMV_OK;
    }
    T *rhs = nullptr;  // the correction solve's right-hand side (kept intact)
    HIP_TRY(B.alloc(&rhs, (size_t)n));
    int iters = 0, outer = 0, repl = 0;
    int status = SPMV_ENOTCONV;
    for (;;) {
        HIP_TRY(O.true_residual(b));
        rc = O.read_state();
        if (rc) return rc;
        if (O.hst->rt2 <= tol * tol * bb) {
            status = SPMV_OK;
            break;
        }
        if (iters >= max_iter || outer >= 200) break;
        // correction solve A32 d = r / ||r|| from d = 0; its "b" is I.r after scaling
        hipLaunchKernelGGL((k_scale_residual<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, I.q, O.r, O.st);
        hipLaunchKernelGGL((k_zero<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, I.x);
        hipLaunchKernelGGL((k_dot_part<T>), dim3(I.n_wg), dim3(kBlock), 0, s, n, I.chunk, I.q, I.q, I.part_vec);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, I.part_vec, I.n_wg, I.st, (int)R_BB);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_copy<T, T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, rhs, I.q);
        int it_inner = 0;
        rc = I.solve(rhs, inner_tol, max_iter - iters, &it_inner, &repl, false);
        iters += it_inner;
        if (rc == SPMV_EBREAK) {
            status = SPMV_EBREAK;
            break;
        }
        if (rc != SPMV_OK && rc != SPMV_ENOTCONV) return rc;
        hipLaunchKernelGGL((k_add_correction<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, O.x, I.x, O.st);
        HIP_TRY(hipGetLastError());
        ++outer;
    }
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, O.x);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->refinements = outer;
        info->graph_seconds = O.capture_s + I.capture_s;
        info->rel_residual = std::sqrt(O.hst->rt2 / bb);
    }
    if (status == SPMV_ENOTCONV) return fail(status, "mixed CG did not reach tol = %g within %d iterations", tol, max_iter);
    if (status == SPMV_EBREAK) return fail(status, "CG breakdown in the correction solve");
    return SPMV_OK;
}



static int cg_pcg(const spmv_matrix *A, const double *b, double *x, double tol, int max_iter, cg_info *info,
                  hipStream_t s, void *pinned, bool jacobi) {
    const DevMatrix &M = A->M;
    const int n = M.n_rows;
    Buffers B(s);
    PcgCore C(M, n, s, jacobi);
    int rc = alloc_core(B, C);
    if (rc) return rc;
    HIP_TRY(B.alloc(&C.z, (size_t)n));
    HIP_TRY(B.alloc(&C.dinv, (size_t)n));
    HIP_TRY(B.alloc(&C.part_rz, (size_t)C.n_wg));
    if (!jacobi) {
        HIP_TRY(B.alloc(&C.t, (size_t)n));
        HIP_TRY(B.alloc(&C.sv, (size_t)n));
    }
    HIP_TRY(B.host_state(pinned, 2 * sizeof(CgState)));
    C.hst = static_cast<CgState *>(B.host);
    hipLaunchKernelGGL((k_dot_part<double>), dim3(C.n_wg), dim3(kBlock), 0, s, n, C.chunk, b, b, C.part_vec);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, C.part_vec, C.n_wg, C.st, (int)R_BB);
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, C.x, x);
    HIP_TRY(hipGetLastError());
    rc = C.read_state();
    if (rc) return rc;
    if (C.hst->bb == 0.0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) info->rel_residual = 0.0;
        return SPMV_OK;
    }
    int iters = 0, restarts = 0;
    rc = C.pcg_solve(b, tol, max_iter, &iters, &restarts);
    if (rc != SPMV_OK && rc != SPMV_ENOTCONV && rc != SPMV_EBREAK) return rc;
    const bool bad_diag = rc == SPMV_EBREAK && (C.hst->flags & F_BADDIAG);
    int rc2;
    HIP_TRY(C.true_residual(b));
    if ((rc2 = C.read_state())) return rc2;
    hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, C.x);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->refinements = restarts;
        info->graph_seconds = C.capture_s;
        info->rel_residual = std::sqrt(C.hst->rt2 / C.hst->bb);
    }
    if (rc == SPMV_ENOTCONV) return fail(rc, "PCG did not reach tol = %g within %d iterations", tol, max_iter);
    if (bad_diag) return fail(rc, "preconditioned CG needs a positive finite diagonal");
    if (rc == SPMV_EBREAK) return fail(rc, "PCG breakdown (p.q or r.z <= 0 or not finite): matrix not SPD?");
    return SPMV_OK;
}

int cg_run(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter, int32_t mode,
           cg_info *info, hipStream_t s, void *pinned_state, CgCache **cache) {
    auto t0 = std::chrono::steady_clock::now();
    if (info) std::memset(info, 0, sizeof *info);
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    if (A->M.block != 1) return fail(SPMV_ENOTSUP, "cg_solve needs a scalar CSR handle");
    if (A->M.n_rows != A->M.n_cols) return fail(SPMV_EINVAL, "CG needs a square matrix (%d x %d)", A->M.n_rows, A->M.n_cols);
    if (!(tol >= 0.0) || max_iter < 0) return fail(SPMV_EINVAL, "tol must be >= 0 and max_iter >= 0");
    if (mode != CG_FP64 && mode != CG_MIXED_FP32 && mode != CG_PCG_BF16 && mode != CG_MIXED_FP32V &&
        mode != CG_PCG_JACOBI && mode != CG_FP64_ONE_REDUCTION)
        return fail(SPMV_EINVAL, "unknown CG mode %d", mode);
    if ((mode == CG_MIXED_FP32 || mode == CG_MIXED_FP32V) && !A->M.val32)
        return fail(SPMV_ENOTSUP, "mixed-precision CG needs the FP32 copy (create with SPMV_VALUES_FP32)");
    if (mode == CG_PCG_BF16 && !A->M.val16)
        return fail(SPMV_ENOTSUP, "CG_PCG_BF16 needs the BF16 copy (create with SPMV_VALUES_BF16)");
    if ((mode == CG_PCG_BF16 || mode == CG_PCG_JACOBI) && A->M.format != SPMV_FORMAT_CSR)
        return fail(SPMV_ENOTSUP, "preconditioned CG needs a CSR handle (the diagonal is read from CSR rows)");
    const int n = A->M.n_rows;
    if (n == 0) return SPMV_OK;
    if (!b || !x) return fail(SPMV_EINVAL, "b or x is NULL");
    if (reinterpret_cast<uintptr_t>(b) < reinterpret_cast<uintptr_t>(x) + sizeof(double) * n &&
        reinterpret_cast<uintptr_t>(x) < reinterpret_cast<uintptr_t>(b) + sizeof(double) * n)
        return fail(SPMV_EINVAL, "b and x overlap");
    int dev_prev = -1;
    {
        hipError_t e = hipGetDevice(&dev_prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (dev_prev != A->device) {
            e = hipSetDevice(A->device);
            if (e != hipSuccess) return hip_fail(e, "making the matrix's device current");
        } else {
            dev_prev = -1;
        }
    }
    int rc;
    CgCache *cc = nullptr;
    if (cache && (mode == CG_FP64 || mode == CG_FP64_ONE_REDUCTION)) {
        if (!*cache) *cache = new (std::nothrow) CgCache();
        cc = *cache;
    }
    if (mode == CG_FP64) {
        rc = cg_fp64(A, b, x, tol, max_iter, info, s, pinned_state, cc);
    } else if (mode == CG_FP64_ONE_REDUCTION) {
        rc = cg_fp64_one_reduction(A, b, x, tol, max_iter, info, s, pinned_state, cc);
    } else if (mode == CG_PCG_BF16 || mode == CG_PCG_JACOBI) {
        rc = cg_pcg(A, b, x, tol, max_iter, info, s, pinned_state, mode == CG_PCG_JACOBI);
    } else {
        // each correction solve reduces the residual by the inner tolerance,
        // so r = ceil(log tol / log 1e-4) refinements of 0.6 tol^(1/r) reach
        // tol without overshooting it (2.8e-4 at tol = 1e-10: 0.875 s against
        // 0.903 s with 1e-4 on the 16M-row mesh matrix, three refinements each)
        const char *env = std::getenv("SPMV_CG_INNER_TOL");
        const double env_tol = env ? std::strtod(env, nullptr) : 0.0;
        double inner = 1e-4;
        if (env_tol > 0.0 && env_tol < 1.0) {
            inner = env_tol;
        } else if (tol > 0.0 && tol < 1.0) {
            const double r = std::max(1.0, std::ceil(std::log(tol) / std::log(1e-4)));
            inner = 0.6 * std::pow(tol, 1.0 / r);
        }
        rc = mode == CG_MIXED_FP32 ? cg_mixed<float>(A, b, x, tol, max_iter, info, s, inner, pinned_state)
                                   : cg_mixed<double>(A, b, x, tol, max_iter, info, s, inner, pinned_state);
    }
    if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // namespace spmvlib

extern "C" int cg_solve(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter,
                        int32_t mode, cg_info *info, void *stream) {
    spmvlib::clear_error();
    return spmvlib::cg_run(A, b, x, tol, max_iter, mode, info, static_cast<hipStream_t>(stream), nullptr);
}

extern "C" int cg_solve_noalloc(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter,
                                int32_t mode, cg_info *info, void *stream) {
    using namespace spmvlib;
    clear_error();
    auto t0 = std::chrono::steady_clock::now();
    if (info) std::memset(info, 0, sizeof *info);
    if (!A) return fail(SPMV_EINVAL, "matrix handle is NULL");
    if (mode != CG_FP64) return fail(SPMV_ENOTSUP, "cg_solve_noalloc runs CG_FP64 only (mode %d)", mode);
    if (A->M.block != 1) return fail(SPMV_ENOTSUP, "cg_solve_noalloc needs a scalar CSR handle");
    if (A->M.n_rows != A->M.n_cols)
        return fail(SPMV_EINVAL, "CG needs a square matrix (%d x %d)", A->M.n_rows, A->M.n_cols);
    if (A->M.n_rows > kNoallocMaxRows || A->M.n_seg > kNoallocMaxRows)
        return fail(SPMV_EINVAL, "n = %d exceeds the allocation-free solver's scratch of %d rows", A->M.n_rows,
                    kNoallocMaxRows);
    if (!(tol >= 0.0) || max_iter < 0) return fail(SPMV_EINVAL, "tol must be >= 0 and max_iter >= 0");
    const int n = A->M.n_rows;
    if (n == 0) return SPMV_OK;
    if (!b || !x) return fail(SPMV_EINVAL, "b or x is NULL");
    if (reinterpret_cast<uintptr_t>(b) < reinterpret_cast<uintptr_t>(x) + sizeof(double) * n &&
        reinterpret_cast<uintptr_t>(x) < reinterpret_cast<uintptr_t>(b) + sizeof(double) * n)
        return fail(SPMV_EINVAL, "b and x overlap");
    int dev_prev = -1;
    {
        hipError_t e = hipGetDevice(&dev_prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (dev_prev != A->device) {
            e = hipSetDevice(A->device);
            if (e != hipSuccess) return hip_fail(e, "making the matrix's device current");
        } else {
            dev_prev = -1;
        }
    }
    double *scr = nullptr;
    int rc = scratch_of(A->device, &scr);
    if (rc == SPMV_OK) rc = cg_fp64_noalloc(A, b, x, tol, max_iter, info, static_cast<hipStream_t>(stream), scr);
    if (dev_prev >= 0) (void)hipSetDevice(dev_prev);
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
