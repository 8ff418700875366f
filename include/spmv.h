/*
 * spmv.h -- C ABI of the MI355X (gfx950) sparse matrix-vector product and
 * conjugate-gradient library for finite-volume mesh matrices.
 *
 * The operation (paper Sec. 2 and Sec. 4.2): y = A x for a square or
 * rectangular sparse matrix A stored in CSR -- binary64 coefficients and
 * 4-byte column indices -- where row i is mesh cell i and its column indices
 * are the neighbouring cells, so the product gathers x indirectly.  The paper
 * expresses the call as a task spmv(double *A, int *cols, double *x,
 * double *b) that reads A, cols and x and produces b (Sec. 3.2); here the
 * matrix is uploaded once and kept resident (the matrix is constant over the
 * simulation and its transfer is a preprocessing cost, Secs. 2 and 3.1), and
 * each product is an asynchronous call on a HIP stream.
 *
 * Conventions for every entry point:
 *  - Return value: SPMV_OK (0) or a negative spmv_status.  A human-readable
 *    message for the calling thread's last failure is spmv_last_error().
 *  - Errors detectable on the host (bad sizes, bad CSR, null or aliasing
 *    pointers) are returned synchronously and nothing is launched.  Device
 *    failures are returned as SPMV_EDEVICE when the HIP runtime reports them.
 *  - Vectors (x, y, b, X, Y) are caller-owned DEVICE pointers (for example
 *    torch tensors' data_ptr()), contiguous, properly aligned for their type.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Products are asynchronous on that stream; CG solves synchronise on it.
 *  - Matrix handles are immutable after creation: concurrent products with
 *    one handle on different streams are allowed.  spmv_destroy requires that
 *    no work using the handle is still in flight.
 *  - The library holds no global state besides the per-thread error message,
 *    per-device properties and one process-wide lock; it needs no init call.
 *    CG solves capture their iterations into HIP graphs.  HIP refuses some
 *    runtime calls from other threads while a stream is being captured (work
 *    on the legacy null stream, and with it some synchronous allocation,
 *    free and copy calls), and the refused call also breaks the capture.  The
 *    library's own such calls (matrix creation and destruction, pinned host
 *    buffers, graph set-up and teardown) take the lock, as do its captures,
 *    and its uploads never use the null stream, so library calls from any
 *    number of threads do not collide.  A caller that submits null-stream
 *    work from another thread during a CG solve can still make that solve
 *    fail with SPMV_EDEVICE; give such work a stream of its own.
 */
#ifndef PAPER_2107_12371_AMD_SPMV_H
#define PAPER_2107_12371_AMD_SPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spmv_status {
    SPMV_OK = 0,
    SPMV_EINVAL = -1,   /* invalid argument or malformed CSR */
    SPMV_ENOMEM = -2,   /* host or device allocation failed */
    SPMV_EDEVICE = -3,  /* HIP runtime error */
    SPMV_ENOTCONV = -4, /* iterative solve did not reach tol within max_iter */
    SPMV_EBUDGET = -5,  /* serving: request exceeds the device-memory budget */
    SPMV_ENOTSUP = -6,  /* operation not available for this handle */
    SPMV_EBREAK = -7    /* CG breakdown: p.q <= 0 or not finite (A not SPD) */
} spmv_status;

typedef struct spmv_matrix spmv_matrix;

/* ------------------------------------------------------------ create flags */
#define SPMV_VALUES_FP32 0x1u   /* also keep an FP32 copy of the values */
#define SPMV_VALUES_BF16 0x2u   /* also keep a BF16 copy of the values */
#define SPMV_NO_XCD_REMAP 0x4u  /* keep launch order = tile order (no XCD grouping) */
#define SPMV_XCD_CONTIGUOUS 0x10u /* 3x3 block CSR: deal one contiguous range of tiles to each
                                     XCD even when the matrix takes 256 MB or more (where the
                                     default deals chunks of 16 tiles in turn; scalar CSR:
                                     spmv_params.xcd_chunk = -2) */
#define SPMV_DEVICE_PTRS 0x8u   /* row_ptr, col_idx and values are device (or managed)
                                   arrays of the current device, holding n_rows + 1, nnz
                                   and nnz elements (9 nnz_blocks values for block CSR);
                                   they are copied to the host for the plan, then
                                   uploaded as host arrays are.  A pointer the runtime
                                   does not know as device memory is SPMV_EINVAL */

/* x-window policy.  The GPU counterparts of the paper's vector cache
 * (Sec. 5.1): x words a tile needs are staged in LDS with contiguous loads
 * and the tile's entries address them with short window-relative indices
 * (12 bits packed per lane for 2048-entry tiles, 16 bits otherwise; the
 * paper shortens its indices to 16 bits). */
#define SPMV_WINDOW_AUTO 0 /* compact per-tile windows wherever they fit (default):
                              the tile's distinct columns merged into at most 64
                              runs, at most tile_nnz staged words; other tiles
                              gather x directly.  With the default tile_nnz, AUTO
                              builds windows only for matrices of at least 512 MB
                              (smaller ones are served from cache); products of
                              every value precision use them */
#define SPMV_WINDOW_OFF 1  /* direct L2 gathers everywhere */
#define SPMV_WINDOW_RING 2 /* the paper's circular cache literally: one workgroup
                              walks a block of adjacent tiles, staging only the
                              words (colend_{i-1}, colend_i] into an LDS ring */

/* Analysis parameters; zero fields take the defaults (shown). */
typedef struct spmv_params {
    int32_t tile_nnz;      /* row-tile capacity: 1024, 2048 or 4096; a tile holds
                              at most tile_nnz - 3 stored entries; longer rows take
                              the long-row path (0: chosen from nnz; with AUTO
                              windows 2048 when windows cover most tiles) */
    int32_t tile_rows;     /* max rows per tile, <= 512 (0: 512) */
    int32_t window_mode;   /* SPMV_WINDOW_* (0: AUTO) */
    int32_t ring_words;    /* RING: LDS ring capacity in x words, a power of two
                              in [256, 8192] (0: 4096) */
    int32_t window_block;  /* RING: adjacent tiles walked by one workgroup
                              (0: chosen from the tile count) */
    int32_t window_gap;    /* AUTO: column gaps up to this many words are staged
                              inside a run rather than starting a new run (0: 64) */
    int32_t kernel;        /* direct-gather kernel: 0 auto, 1 one workgroup per
                              tile, 2 pipelined persistent workgroups, 3 persistent
                              wavefront tiles (tile_nnz 1024, <= 128 rows) */
    int32_t format;        /* SPMV_FORMAT_* (0: CSR row tiles) */
    int32_t sell_sigma;    /* SELL: rows are sorted by length inside windows of
                              this many rows, a multiple of 64 (0: 4096; 64 keeps
                              the row order) */
    int32_t xcd_chunk;     /* CSR row tiles: how tiles are dealt to the 8 XCDs
                              (each has its own L2).  c (a power of two <= 4096):
                              chunks of c consecutive tiles dealt to the XCDs in
                              turn, so all XCDs work near the same rows and share
                              one band of x in the memory-side cache; -2: one
                              contiguous range of tiles per XCD, whose L2 holds
                              its band; -1: no grouping (same as
                              SPMV_NO_XCD_REMAP).  0: chunks of 16 for matrices of
                              at least 256 MB (beyond the memory-side cache), -2
                              for smaller ones */
    int32_t long_rows;     /* rows longer than a tile: 0 (default) sums their
                              pieces of 16,384 entries on a workgroup each wherever
                              the product has scratch for the pieces' sums (see
                              spmv_apply_ws), 1: one workgroup per row always.
                              Same bits either way. */
} spmv_params;

/* Storage formats of a scalar handle. */
#define SPMV_FORMAT_CSR 0  /* CSR in row tiles, optional LDS windows (all of the above) */
#define SPMV_FORMAT_SELL 1 /* sliced ELLPACK, SELL-C-sigma with C = 64 (the paper's
                              sliced ELLPACK, Sec. 4.2, one wavefront lane per row):
                              rows of at most 255 entries are sorted by length
                              inside windows of sell_sigma rows and cut into slices
                              of 64 rows stored column-major, padded to the slice's
                              longest row; padding is masked, never multiplied.
                              Longer rows take the long-row path.  The tile and
                              window fields are ignored. */

/* Summary of a handle's analysis plan and resident storage. */
typedef struct spmv_info {
    int32_t n_rows, n_cols;
    int64_t nnz;
    int32_t tile_nnz, tile_rows;
    int32_t n_tiles;        /* all row segments (stream tiles + long rows) */
    int32_t n_stream_tiles; /* tiles on the direct-gather path */
    int32_t n_long_rows;    /* rows longer than tile_nnz */
    int32_t n_window_tiles; /* tiles on an LDS-window path (ring or compact) */
    int32_t n_window_blocks; /* RING: blocks of adjacent tiles */
    int32_t ring_words;
    int64_t window_words;   /* x words staged into LDS per product */
    int64_t n_runs;         /* compact windows: column runs over all tiles */
    int32_t has_fp32, has_bf16;
    int64_t device_bytes;   /* bytes of device memory held by the handle */
    int32_t block_size;     /* 1: scalar CSR, 3: 3x3 block CSR (n_rows/n_cols/nnz count blocks) */
    int32_t format;         /* SPMV_FORMAT_* of a scalar handle */
    int32_t n_slices;       /* SELL: slices of 64 rows */
    int64_t sell_entries;   /* SELL: stored slots including padding (long rows excluded) */
    int32_t n_long_pieces;  /* pieces of 16,384 stored entries over the long rows */
    int64_t workspace_bytes; /* spmv_workspace_bytes of the handle */
    int32_t y_scratch_ok;   /* 1: binary64 products split the long rows using the output
                               vector as scratch (the rows of its longest run without a long
                               row hold 8 bytes per piece) */
} spmv_info;

/*
 * spmv_create: validate a host CSR matrix, build the analysis plan and copy
 * everything the products need to device memory.
 *   n_rows, n_cols  >= 0
 *   nnz             stored entries, 0 <= nnz <= 2^31 - 2^16 (the kernels'
 *                   32-bit entry offsets reach a tile past the last entry)
 *   row_ptr         int32[n_rows + 1]: row_ptr[0] = 0, non-decreasing,
 *                   row_ptr[n_rows] = nnz
 *   col_idx         int32[nnz], each in [0, n_cols); unsorted columns and
 *                   duplicate (row, col) entries are accepted (all are summed)
 *   values          double[nnz] (any values, including NaN/Inf)
 *                   (host arrays, or device arrays with SPMV_DEVICE_PTRS)
 *   flags           SPMV_VALUES_FP32 | SPMV_VALUES_BF16 | SPMV_NO_XCD_REMAP |
 *                   SPMV_DEVICE_PTRS
 *   params          NULL for defaults
 *   out             receives the new handle (NULL on failure)
 * The caller keeps ownership of its arrays.  The device is the current HIP
 * device.  Errors: SPMV_EINVAL (malformed input), SPMV_ENOMEM, SPMV_EDEVICE.
 */
int spmv_create(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                const int32_t *col_idx, const double *values, uint32_t flags,
                const spmv_params *params, spmv_matrix **out);

/* Release a handle and its device memory (no work may be in flight). NULL is a no-op. */
int spmv_destroy(spmv_matrix *A);

int spmv_get_info(const spmv_matrix *A, spmv_info *info);

/*
 * spmv_apply: y = A x in binary64 (paper Secs. 2, 4.2).  x: device
 * double[n_cols]; y: device double[n_rows], fully overwritten (never read).
 * x and y must not overlap (SPMV_EINVAL).  Each y_i is summed in a fixed
 * order that depends only on the handle, so results are bitwise reproducible
 * and independent of concurrent work.  Per row the result meets
 * |y_i - exact_i| <= gamma_m * sum_k |a_ik||x_k| (m = row length).
 * The call only enqueues kernels on `stream` (no allocation, copy, memset or
 * synchronisation), so a caller may record it into a HIP graph by stream
 * capture and replay it; the same holds for the other spmv_apply_* calls
 * and spmv_spmm / bsr3_spmm.  On a matrix without stored entries (nnz = 0)
 * these calls only fill y with zeros: x is never read and may be NULL.
 */
int spmv_apply(const spmv_matrix *A, const double *x, double *y, void *stream);

/*
 * Rows longer than a tile (spmv_info.n_long_rows) are summed in pieces of
 * 16,384 stored entries: per piece, lane-strided fused multiply-adds and a
 * fixed-shape workgroup sum in binary64; per row, the pieces' sums added in
 * piece order in binary64 (paper Sec. 2: the row's products summed, here in
 * an order fixed by the row's length alone).  Each piece can run on a
 * workgroup of its own, its sum going to scratch memory that a second launch
 * adds up, so a matrix with a few very long rows (a dense coupling row, a
 * global constraint) spreads them over the whole GPU; otherwise one
 * workgroup walks a row's pieces.  The bits are the same either way.  The
 * products (spmv_apply and its FP32/BF16 forms, spmv_spmm with k = 1, the
 * solvers) take the scratch from the output vector itself: the longest run
 * of rows without a long row, which the same call writes only afterwards,
 * when it holds 8 bytes per piece (spmv_info.y_scratch_ok).  Where it does
 * not, spmv_apply_ws takes the scratch from the caller.
 *
 * spmv_workspace_bytes: device bytes that spmv_apply_ws needs for the handle:
 * 8 per long-row piece when some row has more than one piece, else 0.
 * Errors: SPMV_EINVAL (NULL argument).
 *
 * spmv_apply_ws: spmv_apply with the long rows' pieces on a workgroup each
 * and their sums in the caller's workspace, also where the output has no
 * room for them (spmv_info.y_scratch_ok = 0); with spmv_params.long_rows = 1
 * the handle keeps one workgroup per row here too.
 *   ws        caller-owned device memory of at least ws_bytes bytes, 8-byte
 *             aligned, holding the pieces' sums between the two launches;
 *             not to be shared by products that may run at the same time
 *             (a product on another stream, another caller).  NULL when
 *             spmv_workspace_bytes is 0.
 *   ws_bytes  >= spmv_workspace_bytes(A), else SPMV_EINVAL; ws must not
 *             overlap x or y (SPMV_EINVAL).
 * Otherwise as spmv_apply (including capture into a HIP graph).  On block-
 * CSR handles and on handles without such rows it is spmv_apply.
 */
int spmv_workspace_bytes(const spmv_matrix *A, size_t *bytes);
int spmv_apply_ws(const spmv_matrix *A, const double *x, double *y, void *ws, size_t ws_bytes, void *stream);

/* y = A32 x with the FP32 copy of the values, FP32 x/y, FP32 accumulation
 * (needs SPMV_VALUES_FP32, else SPMV_ENOTSUP). */
int spmv_apply_f32(const spmv_matrix *A, const float *x, float *y, void *stream);

/* y = A32 x with FP32 values but binary64 x, y and accumulation
 * (needs SPMV_VALUES_FP32). */
int spmv_apply_f32v(const spmv_matrix *A, const double *x, double *y, void *stream);

/* y = A16 x with the BF16 copy of the values, FP32 x/y, FP32 accumulation
 * (needs SPMV_VALUES_BF16). */
int spmv_apply_bf16(const spmv_matrix *A, const float *x, float *y, void *stream);

/* ------------------------------------------------------ 3x3 block CSR */
/*
 * spmv_create_bsr3: a matrix of dense 3x3 blocks in block-CSR form, as
 * produced by coupled three-component operators on a mesh (velocity u, v, w
 * per cell; paper Sec. 2: row i = cell i, its blocks = neighbour cells).
 *   n_block_rows, n_block_cols >= 0; nnz_blocks stored blocks,
 *              0 <= nnz_blocks <= (2^31 - 2^16) / 9
 *   brow_ptr   int32[n_block_rows + 1] (same rules as CSR row_ptr)
 *   bcol_idx   int32[nnz_blocks] in [0, n_block_cols)
 *   bvalues    double[9 * nnz_blocks], each block row-major
 *              (host arrays, or device arrays with SPMV_DEVICE_PTRS)
 *   flags      SPMV_VALUES_FP32 keeps an FP32 copy; SPMV_NO_XCD_REMAP;
 *              SPMV_DEVICE_PTRS
 * The scalar matrix is (3 n_block_rows) x (3 n_block_cols).  spmv_apply and
 * spmv_apply_f32 on such a handle compute the k = 1 product; cg_solve,
 * spmv_apply_f32v and spmv_apply_bf16 return SPMV_ENOTSUP.
 */
int spmv_create_bsr3(int32_t n_block_rows, int32_t n_block_cols, int64_t nnz_blocks,
                     const int32_t *brow_ptr, const int32_t *bcol_idx, const double *bvalues,
                     uint32_t flags, spmv_matrix **out);

/*
 * spmv_spmm: Y = A X for a scalar CSR handle with k >= 1 right-hand sides
 * (paper Sec. 2: the product of the solver, here applied to k vectors at
 * once, e.g. the k vectors of one serving request).
 *   X  device double[n_cols * k], row-major (the k values of one row of X
 *      are contiguous)
 *   Y  device double[n_rows * k], row-major, fully overwritten
 * The values are read once for all k columns.  Every output is summed as
 * spmv_apply sums a row, so column j of Y equals spmv_apply of column j of
 * X bit for bit.  X and Y must not overlap (SPMV_EINVAL), k >= 1.
 * SPMV_ENOTSUP on block-CSR handles (bsr3_spmm) and SELL-format handles.
 */
int spmv_spmm(const spmv_matrix *A, int32_t k, const double *X, double *Y, void *stream);

/*
 * bsr3_spmm: Y = A X for a block-CSR handle with k >= 1 right-hand sides.
 *   X  device double[(3 n_block_cols) * k], row-major (the k values of one
 *      scalar row are contiguous)
 *   Y  device double[(3 n_block_rows) * k], row-major, fully overwritten
 * Each output is summed over the row's blocks in ascending order, then over
 * the block's three columns; column j of Y equals the k = 1 product of
 * column j of X bit for bit.  X and Y must not overlap.  SPMV_ENOTSUP on a
 * scalar CSR handle.
 */
int bsr3_spmm(const spmv_matrix *A, int32_t k, const double *X, double *Y, void *stream);

/* bsr3_spmm with the FP32 copy of the blocks, FP32 X/Y and FP32 accumulation
 * (needs SPMV_VALUES_FP32). */
int bsr3_spmm_f32(const spmv_matrix *A, int32_t k, const float *X, float *Y, void *stream);

/* ------------------------------------------------------------------- CG */
#define CG_FP64 0       /* binary64 values, vectors, dots and scalars */
#define CG_MIXED_FP32 1 /* iterative refinement: binary64 residual r = b - A x
                           with binary64 values; inner CG with FP32 values,
                           FP32 vectors and FP32 SpMV accumulation, dots and
                           scalar recurrences in binary64 (needs SPMV_VALUES_FP32).
                           Each correction solve stops at a relative recursive
                           residual of 0.6 tol^(1/r), r = ceil(log tol / log 1e-4)
                           the number of refinements it plans for (2.8e-4 at
                           tol = 1e-10), or at the value of the environment
                           variable SPMV_CG_INNER_TOL when it is set to a
                           number in (0, 1) (other values are ignored) */
#define CG_PCG_BF16 2   /* CG preconditioned with a polynomial in the bfloat16
                           copy A~ of A: M^-1 = w D^-1 (2I - w A~ D^-1), D =
                           diag(A), w = 1.9 / max_i sum_j |a~_ij| / sqrt(d_i d_j)
                           (M^-1 symmetric positive definite); binary64 iterate,
                           residual, dots and scalars, one bfloat16 SpMV with
                           FP32 vectors per iteration (needs SPMV_VALUES_BF16 and
                           a CSR-format handle; SPMV_EBREAK if a diagonal entry is
                           not positive) */
#define CG_MIXED_FP32V 3 /* the refinement of CG_MIXED_FP32 with an inner CG that
                           reads the FP32 values but keeps binary64 vectors and
                           binary64 SpMV accumulation (needs SPMV_VALUES_FP32) */
#define CG_PCG_JACOBI 4  /* CG preconditioned with M = D = diag(A) (duplicates
                           summed), all in binary64 (needs a CSR-format handle;
                           SPMV_EBREAK if a diagonal entry is not positive and
                           finite) */
#define CG_FP64_ONE_REDUCTION 5 /* binary64 CG with one reduction phase per
                           iteration (Chronopoulos-Gear: w = A r and s = A p
                           carried by recurrence, r.r and w.r taken together),
                           one launch per iteration; the same Krylov iterates
                           as CG_FP64 in exact arithmetic, and restarts from the
                           true residual when the recursive one has drifted
                           (counted in cg_info.refinements).  For small systems,
                           whose iterations are bound by launch latency: needs a
                           CSR handle of plain row tiles (the default plan of a
                           matrix under 512 MB, or window_mode SPMV_WINDOW_OFF;
                           no row longer than a tile) with at most 4,096 tiles,
                           else SPMV_ENOTSUP */

typedef struct cg_info {
    int32_t iterations;        /* total CG iterations (inner iterations for MIXED) */
    int32_t refinements;       /* outer refinement steps (MIXED), residual replacements (FP64),
                                  restarts from the true residual (PCG) */
    double rel_residual;       /* true ||b - A x||_2 / ||b||_2 in binary64 at exit */
    double seconds;            /* wall time of the solve on the host clock */
    double graph_seconds;      /* part of seconds spent capturing and instantiating the
                                  iteration graph (0 for cg_solve_noalloc) */
} cg_info;

/*
 * cg_solve: solve A x = b for symmetric positive definite A with conjugate
 * gradients (the paper's "linear solver", Sec. 2; Hestenes-Stiefel 1952).
 *   b          device double[n]   (A must be square, n = n_rows)
 *   x          device double[n], in: initial guess, out: last iterate
 *   tol        stop when ||b - A x||_2 <= tol * ||b||_2 (true residual)
 *   max_iter   iteration cap (total inner iterations for MIXED)
 *   mode       CG_FP64, CG_MIXED_FP32, CG_PCG_BF16, CG_MIXED_FP32V or CG_PCG_JACOBI
 *   info       optional, filled on return (also on ENOTCONV / EBREAK)
 * b = 0 gives x = 0 and 0 iterations.  Returns SPMV_ENOTCONV when the cap is
 * reached (x is the last iterate).  Blocks the host until done; work runs on
 * `stream`, reductions are two-stage in a fixed order (reproducible).
 */
int cg_solve(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter,
             int32_t mode, cg_info *info, void *stream);

/*
 * cg_solve_noalloc: cg_solve in CG_FP64 mode that allocates nothing -- for
 * callers that cannot allocate device or pinned host memory or instantiate
 * graphs (tight serving loops, harnesses that forbid allocation after
 * start-up).  Same arguments, results and errors as cg_solve with
 * mode = CG_FP64, bit for bit: the same kernels run in the same order, with
 * the iterations launched directly on `stream` instead of replayed from a
 * captured graph.
 *   mode       must be CG_FP64 (else SPMV_ENOTSUP)
 *   A          a scalar CSR handle with at most 524,288 rows (2^19; larger:
 *              SPMV_EINVAL)
 * The workspace (r, p, q, the partial sums and the scalar state; x itself
 * is the caller's) is one device array of the library, 16.8 MB, held on
 * each GPU the library runs on until the process ends; it is located on a
 * device's first call.  Every call on one GPU uses that GPU's array, so
 * calls that overlap on one GPU (from several threads or streams) race and
 * must be serialised by the caller.  Blocks the host until done; not
 * capturable into a graph (it reads the scalar state after each batch of
 * iterations).
 */
int cg_solve_noalloc(const spmv_matrix *A, const double *b, double *x, double tol, int32_t max_iter,
                     int32_t mode, cg_info *info, void *stream);

/* ------------------------------------------------------------- serving */
/*
 * A request server over resident matrices with continuous batching.
 * Requests (k SpMVs, or a CG solve) are submitted at any time from any
 * thread; a scheduler thread admits them as device memory and solver slots
 * free up, uploading a registered matrix on first use and evicting the least
 * recently used idle matrices to stay within hbm_budget_bytes (a request
 * that has waited 50 ms for memory is admitted before any younger one, so
 * small requests cannot starve a large one).  Admitted SpMV
 * requests join the next round, in which one multi-matrix kernel launch
 * covers all of the round's vectors, or, with persistent_wgs > 0, the round
 * is queued to one long-lived multi-matrix kernel that works the tiles of
 * every queued round as they arrive (the analogue of a task queue feeding
 * accelerator kernels, paper Sec. 3.2); CG requests run on solver slots
 * (one stream each, graph-captured iterations) concurrently with the rounds.
 * The device workspace and captured iteration graph of each FP64 solve are
 * kept per matrix (up to hbm_budget_bytes / 16 in all, least recently used
 * dropped first, dropped with an evicted matrix, outside hbm_budget_bytes),
 * so a later solve on the same matrix from any slot only replays.
 * A request's result is bitwise identical alone and in any mix.
 * Input and output buffers of at least 4 MB move between the caller's
 * (pageable) memory and the device through two pinned host buffers of
 * 16 MB per lane (allocated on the lane's first such request, freed by
 * srv_destroy), in chunks whose DMA overlaps the host copy of the next one,
 * the host copies split over a few copy threads of the server.
 * Latency is measured from srv_submit until the result is in `out`.
 */
typedef struct spmv_server spmv_server;

#define SRV_SPMV 0   /* out[j*n_rows..] = A in[j*n_cols..] for j < k */
#define SRV_CG 1     /* out = x with A x = in (x0 = 0), stop at tol */

typedef struct srv_config {
    uint64_t hbm_budget_bytes; /* resident matrices + request buffers (0: 200 GiB) */
    int32_t n_slots;           /* concurrent CG solves, <= 64 (0: 8) */
    int32_t cg_mode;           /* CG_FP64 or CG_MIXED_FP32 for solve requests */
    int32_t max_round_tiles;   /* cap on workgroups per SpMV round (0: 2^20) */
    int32_t preload;           /* 1: upload each matrix in the background as it is added, while it
                                  fits in the free budget without evicting (0: on first request) */
    int32_t n_lanes;           /* SpMV rounds in flight at once, each on its own stream, <= 16 (0: 4) */
    int32_t persistent_wgs;    /* > 0: SpMV rounds run on one persistent multi-matrix kernel of this
                                  many worker workgroups (plus one that watches the queue; capped at
                                  what the device holds at once), which lanes feed through a queue
                                  in host memory; 0: one launch per round */
    int32_t persist_idle_us;   /* the persistent kernel ends after this long without work and is
                                  launched again when work comes, <= 10^7 (0: 20000) */
    int32_t cg1_max_rows;      /* with cg_mode CG_FP64, solves on matrices of at most this many rows
                                  use CG_FP64_ONE_REDUCTION (faster per iteration on small systems;
                                  0: never) */
} srv_config;

typedef struct srv_result {
    int32_t done;         /* 1 when finished */
    int32_t status;       /* SPMV_OK or the error (SPMV_EBUDGET, SPMV_ENOTCONV, ...) */
    int32_t iterations;   /* CG iterations */
    int32_t op;           /* SRV_SPMV or SRV_CG */
    double rel_residual;  /* CG: true relative residual */
    double latency_s;     /* submit -> result in the caller's buffer */
    double queue_s;       /* submit -> admission (budget, a free CG slot) */
    double wait_s;        /* admission -> an SpMV lane or CG slot starts on it (matrix upload,
                             a free lane, the round it joins) */
    /* Measured with HIP events on the lane's or slot's stream (-1 if the
     * request did not run): */
    double copy_in_s;     /* input vectors to the device, with their buffers' allocation */
    double compute_s;     /* device work: the round's multi-matrix launch (shared by the
                             round's requests), or the whole CG solve */
    double copy_out_s;    /* results back to the caller's buffer */
    double graph_s;       /* CG: capturing and instantiating the iteration graph (host clock,
                             part of compute_s) */
    double dev_begin_s, dev_end_s; /* the device work's interval, in seconds on one device
                             clock per server (comparable across requests) */
    double kernel_s;      /* SpMV on the persistent kernel: its busy time on the round, from
                             the round's first claimed tile to its last (device clock, part of
                             compute_s); -1 otherwise */
    char message[160];    /* why the request failed; empty when status is SPMV_OK */
} srv_result;

typedef struct srv_stats {
    int64_t submitted, completed, failed, rounds, uploads, evictions;
    int64_t used_bytes, peak_bytes; /* budget accounting */
    double p50_s, p99_s, mean_s, max_s; /* latency of completed requests */
    double wall_s;          /* first submit -> last completion */
    double throughput_rps;  /* completed / wall_s */
    int64_t persist_launches; /* launches of the persistent kernel (0 without one) */
    int64_t solver_reuses;    /* CG solves that replayed a kept solver (no capture) */
    int64_t solver_cached_bytes; /* device bytes of the kept solvers */
} srv_stats;

/* Creates the server on the current device (cfg NULL: defaults). */
int srv_create(const srv_config *cfg, spmv_server **out);
/* Registers a host CSR matrix (copied).  It is uploaded by the server's
 * upload thread, on its first request or, with cfg.preload, at once if it
 * fits.  *matrix_id is its handle for srv_submit.  Validation as in
 * spmv_create.  A failed upload fails the requests that waited for it, with
 * its message; the next request on the matrix tries again. */
int srv_add_matrix(spmv_server *srv, int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                   const int32_t *col_idx, const double *values, int32_t *matrix_id);
/* Submits a request.  in/out are HOST buffers (SRV_SPMV: k*n_cols in,
 * k*n_rows out, vector-major; SRV_CG: n in (b), n out (x)) that must stay
 * valid until the request is done.  k is ignored for SRV_CG.  Returns at once
 * with a ticket.  SPMV_EINVAL for bad ids, sizes or pointers. */
int srv_submit(spmv_server *srv, int32_t matrix_id, int32_t op, int32_t k, const double *in, double *out,
               double tol, int32_t max_iter, uint64_t *ticket);
/* Non-blocking status of a ticket. */
int srv_poll(spmv_server *srv, uint64_t ticket, srv_result *res);
/* Blocks until the ticket is done (res may be NULL). */
int srv_wait(spmv_server *srv, uint64_t ticket, srv_result *res);
/* Blocks until every submitted request is done and no upload is running. */
int srv_drain(spmv_server *srv);
int srv_get_stats(spmv_server *srv, srv_stats *st);
/* Drains, stops the threads and frees everything. */
int srv_destroy(spmv_server *srv);

/*
 * srv_policy_simulate: replays the server's admission policy on the host
 * (no GPU), for tests.  Matrices need mat_bytes[i] when resident.  Op t is
 * an admission (op_kind 0) or a release (1) of a request on matrix op_mat[t]
 * holding op_extra[t] bytes of buffers, (2) a failed upload of a resident
 * matrix, which leaves it not resident (its requests are released with 1),
 * or (3) a preload, which makes the matrix resident only if it fits in the
 * free budget (verdict 0) and otherwise does nothing (verdict 1).  Per op:
 * verdict (0 admit, 1 wait, 2 never; -1 for releases and failed uploads),
 * number of evicted matrices, whether the matrix is uploaded, and the bytes
 * in use afterwards.  Unknown kinds: SPMV_EINVAL.
 */
int srv_policy_simulate(uint64_t budget, int32_t n_mats, const uint64_t *mat_bytes, int32_t n_ops,
                        const int32_t *op_kind, const int32_t *op_mat, const uint64_t *op_extra,
                        int32_t *verdict, int32_t *n_evicted, int32_t *uploaded, uint64_t *used);

/*
 * spmv_calibrate_read: reads buf (device double[n], 16-byte aligned, n even)
 * once with a plain streaming kernel of n_blocks workgroups of 256 lanes,
 * storing each workgroup's sum of the values in partials (device
 * double[n_blocks]).  Timing it over a buffer far larger than the caches
 * gives the HBM read rate a streaming kernel reaches on this part, the
 * practical ceiling against which the products are also reported.
 * Asynchronous on `stream`.  SPMV_EINVAL for bad sizes, alignment or NULL.
 */
int spmv_calibrate_read(const double *buf, int64_t n, double *partials, int32_t n_blocks, void *stream);

/* Thread-local message describing the calling thread's last failure ("" if none). */
const char *spmv_last_error(void);

/* ------------------------------------------------ host-only plan inspection */
/*
 * spmv_plan_inspect: run the analysis plan on host arrays without touching
 * the GPU (for tests and tools).  Validates like spmv_create.  Outputs are
 * optional (NULL skips); size them from a first call's *n_tiles_out and
 * info->n_runs:
 *   seg_bound   int32[n_tiles + 1] row boundaries of the tiles
 *   seg_kind    int32[n_tiles]: 0 direct-gather tile, 1 long row,
 *               2 ring-window tile, 3 compact-window tile
 *   win_off     int32[n_tiles]: ring: first x word staged before the tile;
 *               compact: index of the tile's first run
 *   win_cnt     int32[n_tiles]: ring: x words staged; compact: number of runs
 *   win_block   int32[n_tiles]: ring block id, -1 otherwise
 *   runs        int32[2 * n_runs]: compact runs (first column, window position)
 *   lidx        uint16[nnz]: compact tiles: each entry's window position
 *   lidx12      uint32[768 * (number of tiles of kind 3)], filled only when
 *               the tile capacity is 2048: the same positions as the device
 *               reads them, 12 bits each; for the t-th compact tile (in row
 *               order) lane l < 256 owns words 3*(256 t + l) .. +2 holding
 *               entry s4 + 1024 p + 4 l + j (s4 = first entry rounded down
 *               to a multiple of 4, p < 2, j < 4) in bits [12 m, 12 m + 12),
 *               m = 4 p + j; entries outside the tile hold 0
 *   info        plan summary (device_bytes is an estimate)
 */
int spmv_plan_inspect(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                      const int32_t *col_idx, const spmv_params *params, int32_t *n_tiles_out,
                      int32_t *seg_bound, int32_t *seg_kind, int32_t *win_off, int32_t *win_cnt,
                      int32_t *win_block, int32_t *runs, uint16_t *lidx, uint32_t *lidx12,
                      spmv_info *info);

/*
 * spmv_sell_inspect: the SELL-C-sigma layout spmv_create builds for
 * SPMV_FORMAT_SELL, on host arrays and without the GPU (for tests and
 * tools).  Validates like spmv_create.  Outputs are optional (NULL skips);
 * size them from a first call's counts:
 *   n_slices_out, n_entries_out (padded slice entries), n_long_out
 *   perm       int32[64 * n_slices]: row of each slot (slice-major, lane-minor),
 *              -1 for the empty slots of the last slice
 *   len        uint8[64 * n_slices]: entries of each slot's row (0 if empty)
 *   slice_ptr  int32[n_slices + 1]: first entry of each slice; a slice of width
 *              w holds entry j of lane l at slice_ptr[s] + 64 j + l
 *   col        int32[n_entries + entries of the long rows]: columns; padding
 *              repeats the row's last column (0 for an empty row); the long
 *              rows follow the slices in CSR order
 *   long_rows  int32[n_long]: rows longer than 255 entries, ascending
 */
int spmv_sell_inspect(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                      const int32_t *col_idx, int32_t sigma, int32_t *n_slices_out, int64_t *n_entries_out,
                      int32_t *n_long_out, int32_t *perm, uint8_t *len, int32_t *slice_ptr, int32_t *col,
                      int32_t *long_rows);

#ifdef __cplusplus
}
#endif
#endif
