/*
 * hmat.h -- C ABI of an MI355X (gfx950) library for the mixed-precision
 * H-matrix-vector product and the BiCGSTAB solve that repeats it.
 *
 * Method: Ooi, Iwashita, Fukaya, Ida, Yokota, "Effect of Mixed Precision
 * Computing on H-Matrix Vector Multiplication in BEM Analysis",
 * arXiv:1911.00093.  An H-matrix is a partition M of the N x N index set
 * into blocks I_m x J_m (Sec. 2, Eqs. 1-2); each block is either kept dense
 * or stored as a low-rank product V_m W_m (Eqs. 3-4).  The product
 * y = A~ x is the sum of the block products scattered into y (Eqs. 5-8),
 * a low-rank block being applied in two steps z_m = W_m x_m, y^_m = V_m z_m
 * (Eqs. 9-10).  The precision variants are those of Sec. 3 / Table 1.
 *
 * Conventions used by every entry point:
 *  - Indices are 0-based and half-open: a block covers rows
 *    [row0, row0 + nrows) and columns [col0, col0 + ncols).  The paper writes
 *    them 1-based and inclusive (i_m^(s) .. i_m^(e), Sec. 2); contiguous
 *    ranges mean the matrix is given in cluster (permuted) order, and every
 *    vector crossing this ABI is in that order too.
 *  - "host" pointers point to CPU memory, "device" pointers to memory of the
 *    current HIP device.  `stream` is a hipStream_t passed as void*
 *    (NULL = the null stream).
 *  - Every function returns an hmat_status; on failure a thread-local
 *    message is available from hmat_last_error().  No function aborts or
 *    throws across the ABI.
 *  - The library never allocates device memory for matrices, vectors or
 *    solver state: the caller passes device buffers sized by hmat_plan() and
 *    hmat_solver_workspace_bytes().  It allocates small host-side handle
 *    state only.
 */
#ifndef HMAT_H
#define HMAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef enum {
    HMAT_OK = 0,
    HMAT_E_ARG = 1,        /* a null pointer, a size out of range, a bad enum value */
    HMAT_E_LAYOUT = 2,     /* the blocks do not form a partition (Eqs. 1-2 violated) */
    HMAT_E_WORKSPACE = 3,  /* a caller buffer is too small or misaligned */
    HMAT_E_HIP = 4,        /* a HIP runtime call failed */
    HMAT_E_BREAKDOWN = 5,  /* BiCGSTAB breakdown: rho = 0, r~^T v = 0 or omega = 0 (Alg. 1) */
    HMAT_E_NOCONV = 6,     /* BiCGSTAB did not reach the tolerance within maxiter */
    HMAT_E_NONFINITE = 7,  /* a NaN or Inf appeared in the solver's residual */
    HMAT_E_NOMEM = 8       /* host memory allocation failed */
} hmat_status;

/* Thread-local description of the last failure in this thread ("" if none). */
const char *hmat_last_error(void);

/* ------------------------------------------------------------ precision */
/* Storage and arithmetic types, Table 1 of the paper (Sec. 3.1-3.3), plus one
 * addition that the paper does not make:
 *  M1_*  original structure V_m W_m (Sec. 3.1)
 *  M2_*  extended structure V'_m D_m W'_m, D_m FP64 (Sec. 3.2, Eqs. 11-16)
 *  M3    per-term split of the M2 structure by the constant c (Sec. 3.3,
 *        Eqs. 17-20): terms with d_i >= d_max 10^-c FP64, the rest FP32;
 *        dense blocks FP64
 *  BF16_SCALED  low-rank factors in bfloat16 with one power-of-two FP32
 *        scale per factor and block, dense blocks FP32, z in FP64 (not from
 *        the paper).
 * Double: FP64 matrix and source vector.  Single: FP32 matrix, source vector
 * rounded to FP32 before each product (Sec. 3.5).  Mixed: FP32 matrix, FP64
 * source vector.  The result vector is FP64 in every variant, and every
 * product and sum is carried out in FP64 after upcasting the stored values;
 * z_m is rounded to FP32 in M1_SINGLE / M1_MIXED, where Table 1 stores it in
 * FP32. */
typedef enum {
    HMAT_M1_DOUBLE = 0,
    HMAT_M1_SINGLE = 1,
    HMAT_M1_MIXED = 2,
    HMAT_M2_DOUBLE = 3,
    HMAT_M2_SINGLE = 4,
    HMAT_M2_MIXED = 5,
    HMAT_M3 = 6,
    HMAT_BF16_SCALED = 7
} hmat_precision;

enum { HMAT_DENSE = 0, HMAT_LOWRANK = 1 };

/* ---------------------------------------------------- block description */
/* An FP64 H-matrix as produced by a cluster tree and ACA (or any other
 * source).  All arrays are host memory of length nblocks and are only read
 * during the call they are passed to.
 *  data + offset[m] holds, for a dense block, the nrows x ncols block in
 *  column-major order; for a low-rank block of rank r, V_m (nrows x r,
 *  column-major) immediately followed by the transpose of W_m (ncols x r,
 *  column-major).  0 <= r <= min(nrows, ncols) (Eq. 3). */
typedef struct {
    int64_t n;                /* matrix order N */
    int64_t nblocks;
    const int64_t *row0, *nrows, *col0, *ncols;
    const int32_t *kind;      /* HMAT_DENSE or HMAT_LOWRANK */
    const int32_t *rank;      /* ignored for dense blocks */
    const int64_t *offset;    /* element offset into data */
    const double *data;
    int64_t ndata;            /* number of doubles readable at data */
} hmat_blocks;

typedef struct {
    int32_t precision;        /* hmat_precision */
    int32_t c;                /* Method 3 split constant (Eqs. 19-20); the paper uses -1, 1..7 */
    int32_t nrhs_max;         /* largest nrhs later passed to hmat_matvec, >= 1 */
    int32_t drop;             /* 0, or t in 1..15 (Methods 2 and 3 only): omit every low-rank term
                                 whose D_m entry d_i is below d_max 10^-t of its block, i.e. delete
                                 that column of V' and row of W' (the deletion Sec. 4.5 proposes for
                                 terms much smaller than the largest; not a measured variant of the
                                 paper) */
    int32_t dense_split;      /* 0, or 1 (Method 3 only): split the dense leaves like the low-rank
                                 terms, the other proposal of Sec. 4.5: column j of a dense block is
                                 stored in FP32 when its largest magnitude is below the block's
                                 largest times 10^-c, in FP64 otherwise (ties FP64, as Eq. 20) */
    int32_t reserved;         /* 0 */
} hmat_build_opts;

typedef struct {
    uint64_t device_bytes;    /* size of the device buffer hmat_build needs */
    uint64_t matrix_bytes;    /* stored matrix values after conversion */
    uint64_t algorithmic_bytes; /* bytes one product must move at nrhs = 1:
                                   matrix values + D_m scales + x + y */
    int64_t nblocks_dense, nblocks_lowrank;
    int64_t max_rank;
    int64_t terms_fp64, terms_fp32, terms_bf16; /* low-rank terms per storage type */
} hmat_plan_info;

typedef struct hmat_s *hmat_t;

/* Validate a block description and size the device buffer for it.
 * Pure host code; needs no GPU.  Checks that every block lies inside the
 * matrix, that the blocks are pairwise disjoint and cover all of it
 * (Eqs. 1-2; else HMAT_E_LAYOUT), that ranks satisfy Eq. 3 and that all data
 * offsets are in range (else HMAT_E_ARG).  `out` receives the sizes. */
int hmat_plan(const hmat_blocks *blocks, const hmat_build_opts *opts, hmat_plan_info *out);

/* Convert the FP64 blocks to the requested variant (Sec. 4.1.3: the matrix is
 * generated in FP64 and converted afterwards; Methods 2 and 3 decompose in
 * FP64 before rounding) and pack them into the caller's device buffer
 * `dev_mem` (256-byte aligned, at least plan.device_bytes bytes).  The copy
 * is enqueued on `stream` and completed before the call returns, so the
 * host arrays may be freed afterwards.  The handle does not own dev_mem: the
 * caller keeps it alive until hmat_destroy and frees it afterwards.  The
 * buffer also holds the per-handle product workspace, so two products with
 * the same handle must not run concurrently on different streams. */
int hmat_build(const hmat_blocks *blocks, const hmat_build_opts *opts, void *dev_mem, uint64_t dev_bytes,
               void *stream, hmat_t *out);

/* y = A~ x (Eq. 5) for nrhs right-hand sides.  x and y are device arrays of
 * FP64, column-major n x nrhs with leading dimension ld >= n; y is
 * overwritten and may alias x.  1 <= nrhs <= nrhs_max of the build.
 * Asynchronous on `stream`; no host synchronisation.
 * A handle built with nrhs_max > 1 stores its blocks for the matrix cores
 * and multiplies 16 right-hand sides per pass on the FP64 matrix cores:
 * every stored value is widened exactly to FP64 and meets the same FP64
 * operands as with nrhs_max = 1, so the arithmetic is the same (exact
 * products, FP64 sums, Table 1 roundings of x and z); only the summation
 * order differs. */
int hmat_matvec(hmat_t h, const double *x, double *y, int64_t nrhs, int64_t ld, void *stream);

/* Tuning of a handle's launch configuration (not from the paper), timed on
 * the handle's own blocks; the fastest choice is kept for later products of
 * that handle.  Results are unchanged by the choice (same arithmetic, same
 * summation order; the solver's fused inner products are kept per row chunk,
 * so its iterations do not change either).
 *  Multi-right-hand-side handles (nrhs_max > 1): for each stage-1 storage
 *  class and for stage 2, the column blocks loaded per batch (1, 2, 4) and
 *  the grid (0 persistent at full occupancy, 1 at half occupancy, 2 one wave
 *  per work unit).
 *  Single-vector handles (nrhs_max = 1): for each stage-1 storage class the
 *  grid (0 one wave per item, 1 persistent at full occupancy, 2 at half), and
 *  for stage 2 the grid (0 persistent at full occupancy, 1 at half, 2 one
 *  workgroup per row chunk) and the operand tile, the panel columns whose
 *  operands are staged in LDS per pass (1024, 2048 or 4096).
 * x: device, n x min(16, nrhs_max) FP64 column-major (ld = n), the timing
 * input; y (same shape) receives products.  reps: timed launches per choice
 * (1 .. 1000).  Synchronises `stream`. */
typedef struct {
    int32_t stage1_batch[3];  /* per storage class FP64 / FP32 / BF16 (0: no items; 1 on single-vector handles) */
    int32_t stage1_grid[3];   /* grid mode per storage class (see above) */
    int32_t stage2_batch, stage2_grid;  /* batch (0 on single-vector handles) and grid mode of stage 2 */
    double ms_fixed;          /* one product with the configuration before tuning */
    double ms_tuned;          /* one product with the chosen configuration */
    int32_t stage2_tile;      /* single-vector handles: operand tile chosen (0 otherwise) */
    int32_t reserved;
} hmat_tune_info;

int hmat_autotune(hmat_t h, const double *x, double *y, int32_t reps, hmat_tune_info *info, void *stream);

/* Apply a launch configuration without timing (a choice hmat_autotune made
 * for another handle of the same blocks, kept by the caller): the fields
 * hmat_autotune fills, read as above (ms_fixed / ms_tuned ignored).  Single-
 * vector handles read stage1_grid, stage2_grid and stage2_tile;
 * multi-right-hand-side handles stage1_batch (classes with items),
 * stage1_grid, stage2_batch and stage2_grid.  HMAT_E_ARG for a value out of
 * range; results are unchanged by any valid choice. */
int hmat_set_tuning(hmat_t h, const hmat_tune_info *cfg);

/* Independent systems batched into one handle (not from the paper): system
 * k (a full H-matrix of order n_k, blocks as in hmat_blocks) occupies the
 * index range [off_k, off_k + n_k) of a block-diagonal operator, off_0 = 0,
 * off_{k+1} = off_k + n_k; each system's blocks must partition its own
 * n_k x n_k index set (Eqs. 1-2 per system).  One product then covers the
 * blocks of every system in the same launches.  `systems` is a host array
 * of `count` descriptions, only read during the call.  Vectors of a batched
 * handle are the systems' vectors concatenated in this order. */
int hmat_plan_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts, hmat_plan_info *out);
int hmat_build_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts, void *dev_mem,
                       uint64_t dev_bytes, void *stream, hmat_t *out);
/* Plan once, build from the kept plan (not from the paper; setup only).
 * hmat_plan_keep and hmat_plan_keep_batched check and size exactly as
 * hmat_plan and hmat_plan_batched do (same errors, same `out`, which may be
 * NULL) and also keep the plan, returned in *plan (NULL on error);
 * hmat_build_kept then does what hmat_build / hmat_build_batched do with
 * that plan (same buffer rules, errors and result) without planning again:
 * a plan scans every low-rank factor for the Method 2 scales (Eqs. 13-16),
 * which otherwise runs once for the caller's sizing and again in the build.
 * A kept plan points into the caller's block arrays and values (for a
 * batch, into each system's arrays; the `systems` array itself is only read
 * during the call): they must stay alive and unchanged until the last
 * build from it.  A plan is only read by a build and may serve several,
 * each into its own buffer.  hmat_plan_release frees a plan (NULL is
 * ignored); handles built from it stay valid. */
typedef struct hmat_kept_plan_s *hmat_kept_plan_t;
int hmat_plan_keep(const hmat_blocks *blocks, const hmat_build_opts *opts, hmat_plan_info *out,
                   hmat_kept_plan_t *plan);
int hmat_plan_keep_batched(const hmat_blocks *systems, int64_t count, const hmat_build_opts *opts,
                           hmat_plan_info *out, hmat_kept_plan_t *plan);
int hmat_build_kept(hmat_kept_plan_t plan, void *dev_mem, uint64_t dev_bytes, void *stream, hmat_t *out);
int hmat_plan_release(hmat_kept_plan_t plan);

/* System boundaries of a handle: *count systems, offsets[0..count] (host,
 * capacity >= count + 1; offsets may be NULL to query the count). */
int hmat_system_offsets(hmat_t h, int64_t *offsets, int64_t capacity, int64_t *count);

/* Release the host-side handle state (not the caller's device buffer). */
int hmat_destroy(hmat_t h);

/* The packed image hmat_build would upload, written into host memory (pure
 * host code, no GPU: for inspection and for checking the layout on the CPU).
 * `image` receives image_bytes bytes (pass NULL to query the sizes; else
 * HMAT_E_WORKSPACE if `bytes` is smaller); `out` the offsets of its parts.
 * The layout is the library's internal one (single-vector handles: per
 * storage class the values in consumption order, 32-bit gather indices,
 * then the row-chunk and stage-1 item descriptors, the stage-1 reduction
 * table and the D_m scales); hmat_build copies exactly these bytes to the
 * start of its device buffer. */
typedef struct {
    uint64_t image_bytes;
    uint64_t off_vals[3], bytes_vals[3];  /* per storage class FP64 / FP32 / BF16 */
    uint64_t off_gidx[3], bytes_gidx[3];
    uint64_t off_chunks, off_items, off_zinfo, off_dscale;
    int64_t n, nchunks, nitems, zlen;
    int64_t zw0;              /* z entries [zw0, zlen) are finished by the stage-1 reduction */
    int32_t x32, z32;         /* x rounded to FP32 (Single variants); z rounded to FP32 (M1-Single/Mixed) */
    int32_t layout;           /* 0 single-vector, 1 multi-right-hand-side */
    int32_t reserved;
} hmat_image_info;
int hmat_pack_host(const hmat_blocks *blocks, const hmat_build_opts *opts, void *image, uint64_t bytes,
                   hmat_image_info *out);

#define HMAT_SIZE_CLASSES 8
typedef struct {
    int64_t n, nblocks, nblocks_dense, nblocks_lowrank, max_rank;
    int64_t row_chunks;       /* stage-2 work units (row ownership) */
    int64_t column_groups;    /* stage-1 groups of low-rank factors sharing J_m */
    int64_t stage1_items;     /* stage-1 work units */
    int64_t z_len;            /* number of z_m entries */
    uint64_t bytes_dense;     /* stored dense values */
    uint64_t bytes_v;         /* stored V'_m values */
    uint64_t bytes_w;         /* stored W'_m values */
    uint64_t bytes_packed;    /* values incl. row padding as laid out in HBM */
    uint64_t bytes_index;     /* gather indices and descriptors */
    uint64_t algorithmic_bytes;        /* per product at nrhs = 1 (see hmat_plan_info) */
    uint64_t stage1_algorithmic_bytes; /* W' values + x reads + z writes */
    uint64_t stage2_algorithmic_bytes; /* dense + V' values + x/z reads + y writes */
    int32_t precision;
    int32_t c;
    /* stored values per storage class (FP64, FP32, BF16): dense columns and
     * low-rank terms of that class, V'_m and W'_m rows together */
    uint64_t bytes_class[3];
    /* blocks per size class of their larger side max(#I, #J): class k holds
     * sides in (2^(k+3), 2^(k+4)] (class 0: <= 16; the last class: > 1024) */
    int64_t blocks_dense_by_size[HMAT_SIZE_CLASSES];
    int64_t blocks_lowrank_by_size[HMAT_SIZE_CLASSES];
} hmat_stats;

int hmat_get_stats(hmat_t h, hmat_stats *out);

/* ------------------------------------------------------------- solver */
/* Right preconditioner K for hmat_bicgstab (a fixed linear map; not from the
 * paper).  HMAT_PRECOND_JACOBI inverts every dense diagonal block of the
 * handle's FP64 source blocks (up to 256 rows; hmat_batched_inverse on the
 * GPU, inside hmat_precond_create, which fails with HMAT_E_ARG naming the
 * first singular block) and applies y_tau = A_tautau^{-1} x_tau on each;
 * rows of no diagonal dense block pass through unchanged. */
typedef struct hmat_precond_s *hmat_precond_t;
enum { HMAT_PRECOND_NONE = 0, HMAT_PRECOND_JACOBI = 1, HMAT_PRECOND_LEARNED = 2 };

/* Device bytes hmat_precond_create needs for `blocks`. */
int hmat_precond_plan(const hmat_blocks *blocks, int32_t kind, uint64_t *device_bytes);
int hmat_precond_create(const hmat_blocks *blocks, int32_t kind, void *dev_mem, uint64_t dev_bytes, void *stream,
                        hmat_precond_t *out);
/* HMAT_PRECOND_LEARNED: on every dense diagonal block tau (m <= 64 rows, in
 * the order of `blocks`), K_tau = diag(A_tautau)^{-1} + (1/s_tau) U V^T with
 * s_tau the mean of A_tautau's diagonal and U, V the 64 x 16 factors the MLP
 * below predicts for that leaf (rows >= m ignored).  uv: device FP32, one
 * HMAT_MLP_OUT row per diagonal block (U then V, row-major), copied into
 * dev_mem.  Size dev_mem with hmat_precond_plan(blocks, HMAT_PRECOND_LEARNED).
 * Fails with HMAT_E_ARG when a diagonal block exceeds 64 rows. */
int hmat_precond_create_learned(const hmat_blocks *blocks, const float *uv, void *dev_mem, uint64_t dev_bytes,
                                void *stream, hmat_precond_t *out);

/* The dense diagonal blocks a preconditioner acts on, in its order: block
 * index, first row, rows (host arrays of capacity entries; may be NULL to
 * query *count). */
int hmat_precond_leaves(const hmat_blocks *blocks, int32_t kind, int64_t *block, int64_t *row0, int64_t *rows,
                        int64_t capacity, int64_t *count);

/* y = K x for one vector (device FP64, length n); y must not alias x. */
int hmat_precond_apply(hmat_precond_t p, const double *x, double *y, void *stream);
int hmat_precond_destroy(hmat_precond_t p);

typedef struct {
    double tol;               /* relative residual |r|/|b| to reach (Sec. 4.1.3 uses 1e-6) */
    int64_t maxiter;          /* iterations of Algorithm 1's loop */
    int32_t poll_every;       /* read the device status every this many iterations (>= 1) */
    int32_t use_graph;        /* 1: capture one iteration in a HIP graph and replay it */
    hmat_precond_t precond;   /* NULL: no preconditioner */
    double *history;          /* host, maxiter + 1 entries, or NULL: |r_i|/|b| per iteration */
    double refine;            /* 0, or also check the FP64 true residual whenever |r|/|b| < refine x the
                                 last true residual; a failed check restarts (not in the paper) */
} hmat_solve_opts;

typedef struct {
    int32_t status;           /* HMAT_OK, HMAT_E_BREAKDOWN, HMAT_E_NOCONV or HMAT_E_NONFINITE */
    int32_t restarts;         /* restarts after a failed true-residual check */
    int64_t iterations;
    int64_t matvecs;          /* products with h_iter */
    int64_t matvecs_fp64;     /* products with h_fp64 (true residuals) */
    double rel_res;           /* final recurrence |r|/|b| */
    double true_rel_res;      /* final |b - A~64 x| / |b| */
} hmat_solve_info;

/* Device bytes of solver workspace for order n. */
uint64_t hmat_solver_workspace_bytes(int64_t n);

/* BiCGSTAB (Sec. 3.5, Algorithm 1) with h_iter as the operator and every
 * vector and scalar in FP64 on the device.  x holds x_0 on entry and the
 * solution on return (device, length n); b is a device vector.  The
 * iteration stops when |s|/|b| or |r|/|b| < tol; convergence is then
 * confirmed with the true residual b - A~ x computed with h_fp64 (Sec. 4.1.3;
 * h_fp64 may equal h_iter).  If that check fails the iteration restarts from
 * the current x with r = r~ = the true residual.  b = 0 gives x = 0.
 * `work` is a device buffer of hmat_solver_workspace_bytes(n) bytes.
 * Synchronises `stream` before returning; `info` is filled in every case. */
int hmat_bicgstab(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, const hmat_solve_opts *opts,
                  hmat_solve_info *info, void *work, uint64_t work_bytes, void *stream);

/* hmat_bicgstab for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, bit for bit, with the solver workspace taken from a static
 * device array that the library holds on every GPU it runs on (about 39 MB
 * per GPU, kept until the process ends) instead of a `work` argument.  The
 * caller still passes b, x, the handles and opts as for hmat_bicgstab.
 * Limits: the order n must not exceed hmat_bicgstab_noalloc_max_n()
 * (524,288; larger orders fail with HMAT_E_WORKSPACE before any work is
 * queued) and opts->use_graph must be 0 (HMAT_E_ARG: instantiating a graph
 * allocates).  Nothing is allocated on the device: no hipMalloc, hipFree or
 * allocating library call.  Every call on one GPU uses that GPU's single
 * array, so calls that overlap on one GPU (other host threads, other
 * streams) race and must be serialised by the caller; the solver initialises
 * every workspace entry it reads, so the previous call's contents never
 * matter.  The first call on a device looks up the array's device address
 * with that device current (HMAT_E_HIP if that fails). */
int64_t hmat_bicgstab_noalloc_max_n(void);
int hmat_bicgstab_noalloc(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, const hmat_solve_opts *opts,
                          hmat_solve_info *info, void *stream);

/* Restarted GMRES(restart) (the further solver Sec. 5 names; the textbook
 * method, not from the paper): Arnoldi with classical Gram-Schmidt applied
 * twice, Givens rotations, right preconditioning x = K u (opts->precond, or
 * none), every vector and scalar FP64 on the device.  A cycle of at most
 * `restart` steps (1..128) uses h_iter; it ends when the residual estimate
 * |g_{j+1}|/|b| falls below tol, the basis is full, the Krylov space
 * contains the solution or opts->maxiter steps have run; then x is updated
 * and the true residual b - A~ x is computed with h_fp64 (Sec. 4.1.3): below
 * tol the solve is done, else the next cycle starts from that residual.
 * iterations = steps (one h_iter product each); matvecs counts the h_iter
 * products (the initial residual and one per step), matvecs_fp64 the cycles'
 * true residuals, restarts the cycles after the first, rel_res the last
 * estimate.  opts->refine must be 0; opts->history receives the estimate
 * after every step.  x holds x_0 on entry.  `work`: device, 256-byte
 * aligned, hmat_gmres_workspace_bytes(n, restart) bytes.  Synchronises
 * `stream` before returning; `info` is filled in every case. */
uint64_t hmat_gmres_workspace_bytes(int64_t n, int32_t restart);
int hmat_gmres(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, int32_t restart, const hmat_solve_opts *opts,
               hmat_solve_info *info, void *work, uint64_t work_bytes, void *stream);

/* Outcome of one recurrence of the batched solver. */
typedef struct {
    int32_t status;           /* HMAT_OK, HMAT_E_BREAKDOWN, HMAT_E_NOCONV or HMAT_E_NONFINITE */
    int32_t restarts;
    int64_t iterations;
    double rel_res;           /* final |r|/|b| (the true one once converged) */
    double true_rel_res;      /* |b - A~64 x| / |b| at the end */
    int64_t products;         /* products with h_iter that covered this recurrence's system */
} hmat_batch_result;

/* Device bytes of workspace hmat_bicgstab_batched needs for handle h and nrhs
 * right-hand sides (0 on bad arguments or when the host is out of memory). */
uint64_t hmat_bicgstab_batched_workspace_bytes(hmat_t h, int64_t nrhs);

/* BiCGSTAB (Sec. 3.5, Algorithm 1) on every system of a batched handle for
 * nrhs right-hand sides at once: nsys x nrhs independent recurrences, each
 * with its own FP64 scalars, the same stopping rule and FP64 true-residual
 * confirmation (Sec. 4.1.3) as hmat_bicgstab, and the same restart on a
 * failed check.  A recurrence that converges or breaks down stops while the
 * others continue; the products still run over all nrhs columns, but on
 * multi-right-hand-side handles (nrhs_max > 1) an iteration's products skip
 * the systems none of whose recurrences is iterating (results[].products
 * counts the products that covered each system).
 * b, x: device, n x nrhs with column k at offset k * n (column-major, the
 * layout of hmat_matvec with ld = n); x holds x_0 on entry.  1 <= nrhs <=
 * min(16, nrhs_max of both handles).  h_fp64 (may be NULL = h_iter) must
 * have the same systems.  opts->precond and opts->history must be NULL;
 * opts->use_graph = 1 captures one iteration in a HIP graph on an internal
 * stream and replays it on `stream`.  results: host, nsys x nrhs entries,
 * system-major (entry s * nrhs + k).  summary (may be NULL): status = the
 * first failing status, iterations and restarts = maxima, matvecs = batched
 * products launched.  Returns HMAT_OK when every recurrence converged.  Synchronises
 * `stream` before returning. */
int hmat_bicgstab_batched(hmat_t h_iter, hmat_t h_fp64, const double *b, double *x, int64_t nrhs,
                          const hmat_solve_opts *opts, hmat_batch_result *results, hmat_solve_info *summary,
                          void *work, uint64_t work_bytes, void *stream);

/* ------------------------------------- learned leaf map (not in the paper) */
/* A small MLP predicts, from the geometry of one leaf cluster (at most 64
 * panels in cluster order), the factors U, V of the learned preconditioner
 * above.  Input: per panel p the offset of its centroid from the leaf's mean
 * centroid divided by the diagonal of the leaf's centroid box (3), its unit
 * normal (3) and its area over the mean area (1), zero beyond the m panels,
 * then a mask of m ones (64 x 7 + 64 = 512).  Layers: 512 -> 128 -> 128 ->
 * 2048, ReLU after the first two.  Parameters: one FP32 device array of
 * HMAT_MLP_PARAMS floats, W1 (512 x 128, row-major), b1, W2 (128 x 128), b2,
 * W3 (128 x 2048), b3; H = relu(X W + b).  Training minimises the batch mean
 * of |K_tau - A_tautau^{-1}|_F^2 / |A_tautau^{-1}|_F^2 with Adam. */
#define HMAT_MLP_LEAF 64
#define HMAT_MLP_RANK 16
#define HMAT_MLP_IN 512
#define HMAT_MLP_HIDDEN 128
#define HMAT_MLP_OUT 2048
#define HMAT_MLP_PARAMS (512 * 128 + 128 + 128 * 128 + 128 + 128 * 2048 + 2048)

/* Features of one leaf (host): centroids and normals m x 3 row-major, areas
 * m (FP64, cluster order, 1 <= m <= 64); out: 512 floats. */
int hmat_leaf_features(int64_t m, const double *centroids, const double *normals, const double *areas, float *out);

/* The fixed parts of the learned map of one leaf (host): a is the dense
 * diagonal block A_tautau (m x m column-major, FP64, 1 <= m <= 64); dinv
 * receives 64 floats, 1 / A_ii for i < m and 0 beyond, and *sinv the float
 * 1 / s_tau = m / sum_i A_ii (the reciprocal of the mean self term), both
 * computed in FP64 and rounded once, the same values the preconditioner
 * applies in FP64.  HMAT_E_ARG for a zero diagonal entry. */
int hmat_leaf_scales(int64_t m, const double *a, float *dinv, float *sinv);

/* Batched exact FP64 inverse of small dense square matrices on the GPU, in
 * place: the inverses A_tautau^{-1} of the dense diagonal leaves that
 * block-Jacobi applies and that the learned map is trained against
 * (Gauss-Jordan elimination with partial pivoting, every operation in FP64;
 * one workgroup per matrix, orders up to 128 held in LDS).
 *   count      number of matrices, 0 .. 2^31-1.
 *   off, dim   device arrays of count entries: matrix q has order dim[q] and
 *              starts at a + off[q] (elements), stored m x m column-major
 *              (row-major storage gives the inverse in row-major: the
 *              inverse of the transpose is the transposed inverse).
 *              Matrices must not overlap.
 *   max_dim    (host) the largest order present, 1 .. 256; it sizes the
 *              launch's LDS.
 *   a          device FP64, overwritten by the inverses.
 *   first_bad  device int64 (one word): set to count, then to the smallest q
 *              whose order lies outside 1 .. max_dim or whose elimination
 *              meets a pivot that is zero or NaN (such a matrix holds
 *              unspecified values afterwards; every other matrix is
 *              inverted).
 * Asynchronous on `stream`; allocates nothing.  HMAT_E_ARG for null
 * pointers, count < 0 or max_dim outside 1 .. 256; HMAT_E_HIP if a launch
 * fails.  The caller owns every buffer. */
int hmat_batched_inverse(int64_t count, const int64_t *off, const int32_t *dim, int32_t max_dim, double *a,
                         int64_t *first_bad, void *stream);

/* Device workspace of the MLP calls for `batch` samples. */
uint64_t hmat_mlp_workspace_bytes(int64_t batch);

/* out (device, batch x 2048) = MLP(x) for x (device, batch x 512). */
int hmat_mlp_forward(const float *params, const float *x, int64_t batch, float *out, void *work,
                     uint64_t work_bytes, void *stream);

/* Batch mean loss and its gradient for the samples idx[0 .. batch) (device
 * int32; an entry outside [0, nsamples) counts as an empty sample) of a
 * training set on the device: x (nsamples x 512), ainv
 * (nsamples x 64 x 64, row-major, the exact inverse in the leading m x m
 * corner, FP32), dinv (nsamples x 64: 1 / A_ii), sinv (nsamples: 1 / s_tau),
 * m (nsamples, int32, clamped to 0..64).  grad: HMAT_MLP_PARAMS floats (overwritten, same
 * layout as params); loss: one float (overwritten).  Deterministic. */
int hmat_mlp_loss_grad(const float *params, const float *x, const float *ainv, const float *dinv, const float *sinv,
                       const int32_t *m, int64_t nsamples, const int32_t *idx, int64_t batch, float *grad, float *loss,
                       void *work, uint64_t work_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) of
 * number t >= 1 with rate lr on params and its moments m1, m2 (device FP32,
 * HMAT_MLP_PARAMS each). */
int hmat_mlp_adam(float *params, float *m1, float *m2, const float *grad, int64_t t, float lr, void *stream);

/* ------------------------------------------------------------ assembly */
/* Setup step (untimed; not the product path): build an FP64 H-matrix for the
 * BEM collocation problem on a triangle mesh -- cluster tree (bisection of
 * the centroid box across its longest side), admissible block partition
 * (min(diam) <= eta dist), dense leaves and partially pivoted ACA to the
 * relative tolerance eps on the admissible blocks.  The paper only names
 * ACA (Sec. 1) and leaves generation to the library it extends
 * (Sec. 4.1.3).  Entries: A_ij = a_j / (4 pi |c_i - c_j|), A_ii = sqrt(a_i/pi)/2.
 * centroids: host, n x 3 row-major; areas: host, n; original panel order. */
typedef struct {
    int64_t leaf;             /* largest leaf cluster */
    double eta;               /* admissibility constant */
    double eps;               /* ACA relative tolerance */
    int32_t threads;          /* host threads (0: all hardware threads) */
    int32_t reserved;
} hmat_assemble_opts;

typedef struct hmat_assembly_s *hmat_assembly_t;

int hmat_assemble_bem(int64_t n, const double *centroids, const double *areas, const hmat_assemble_opts *opts,
                      hmat_assembly_t *out);
/* The same H-matrix built with its entries and ACA on the GPU (the paper's
 * Sec. 4.5 outlook; generation itself is Sec. 4.1.3's FP64 step): cluster
 * tree and partition on the host as above, then one workgroup per admissible
 * block runs the partially pivoted ACA of hmat_assemble_bem with the same
 * operations in the same order (residual rows and columns term by term,
 * every norm and inner product summed in index order, no fused multiply-add),
 * and a second kernel evaluates the dense blocks and writes the factors in
 * the host layout; the result is copied back into an assembly identical, bit
 * for bit, to hmat_assemble_bem's.  rank_cap (1..127, 0: 48) bounds the
 * ranks kept on the device per block; a block whose ACA has not stopped
 * by then (and cannot yet be known to end dense) is redone on the host.
 * Device memory: the library allocates its scratch on the current device
 * (about 8 (#I + #J) rank_cap bytes per admissible block plus the result) and
 * frees it before returning; HMAT_E_NOMEM if that fails.  Work is queued on
 * `stream` and the call synchronises it before returning. */
int hmat_assemble_bem_gpu(int64_t n, const double *centroids, const double *areas, const hmat_assemble_opts *opts,
                          int32_t rank_cap, void *stream, hmat_assembly_t *out);

/* Several meshes at once (independent systems, e.g. the systems of a
 * batched build): mesh s has n[s] panels, centroids[s] (n[s] x 3 row-major)
 * and areas[s], all host; out[s] receives its assembly, the same, bit for
 * bit, as hmat_assemble_bem_gpu (and hmat_assemble_bem) gives for that mesh
 * alone.  The meshes' admissible blocks share one ACA launch and their blocks
 * one emit launch, so small meshes fill the GPU together.  Each handle's
 * stats report its own block counts and the batch's phase times.  On error
 * every out[s] is null. */
int hmat_assemble_bem_gpu_batched(int64_t count, const int64_t *n, const double *const *centroids,
                                  const double *const *areas, const hmat_assemble_opts *opts, int32_t rank_cap,
                                  void *stream, hmat_assembly_t *out);

/* What an assembly did (either path). */
typedef struct {
    int64_t blocks;          /* blocks of the partition */
    int64_t lowrank;         /* blocks stored low rank */
    int64_t host_blocks;     /* blocks whose entries were computed on the host */
    int32_t rank_cap;        /* device path: ranks kept per block (0: host path) */
    int32_t reserved;
    uint64_t device_bytes;   /* device path: scratch allocated */
    double ms_partition;     /* cluster tree and partition (host) */
    double ms_fill;          /* entries and ACA: host threads, or the device path from upload to copy-back */
    double ms_aca, ms_emit;  /* device path: the two kernels (HIP events) */
    double ms_copy;          /* device path: result copied to the host */
    double ms_upload;        /* device path: scratch allocated, mesh and descriptors uploaded */
} hmat_assembly_stats;
int hmat_assembly_get_stats(hmat_assembly_t a, hmat_assembly_stats *stats);

/* Fill `view` with pointers into the assembly (valid until hmat_assembly_free). */
int hmat_assembly_blocks(hmat_assembly_t a, hmat_blocks *view);
/* perm[k] = original panel index at cluster position k (length n). */
const int64_t *hmat_assembly_perm(hmat_assembly_t a);
int hmat_assembly_free(hmat_assembly_t a);

/* ---------------------------------------------------------- diagnostics */
/* Kernel timing (not from the paper): while enabled, hmat_matvec records
 * HIP events on its stream around each of its three kernels (stage 1,
 * stage-1 reduction, stage 2).  hmat_kernel_times waits for the recorded
 * events, writes the average duration in milliseconds of each kernel over
 * the products since the previous call into avg_ms[0..2], the number of
 * products into *count, and resets the averages.  Enabling adds event
 * records between the kernels but does not change what they compute. */
int hmat_set_profiling(hmat_t h, int32_t enable);
int hmat_kernel_times(hmat_t h, double *avg_ms, int64_t *count);

/* Bandwidth calibration kernels (device pointers, 16-byte aligned, bytes a
 * multiple of 16), asynchronous on `stream`.  hmat_stream_read reads
 * `bytes` with 16-byte non-temporal loads, one contiguous range per
 * workgroup and eight loads in flight per thread, the fastest plain read
 * measured on MI355X (sink: one device double, written only to keep the
 * loads alive);
 * hmat_stream_copy copies `bytes` from src to dst. */
int hmat_stream_read(const void *src, uint64_t bytes, double *sink, void *stream);
int hmat_stream_copy(void *dst, const void *src, uint64_t bytes, void *stream);

/* Vectors between the original panel order and the cluster (permuted)
 * order every other entry point uses: y[k] = x[perm[k]], or with inverse != 0
 * y[perm[k]] = x[k], for each of nrhs columns (column j at offset j * n).
 * perm: device int64, a permutation of 0..n-1 (the one hmat_assembly_perm
 * returns, copied to the device); x, y: device FP64, must not alias.
 * Asynchronous on `stream`. */
int hmat_permute(int64_t n, const int64_t *perm, const double *x, double *y, int64_t nrhs, int32_t inverse,
                 void *stream);

/* Library version string. */
const char *hmat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H */
