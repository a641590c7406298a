/*
 * libprcg: conjugate-gradient solvers for sparse symmetric positive definite
 * systems A x = b on one AMD MI355X (gfx950), following
 *   T. Chen and E. Carson, "Predict-and-recompute conjugate gradient
 *   variants", SIAM J. Sci. Comput. 42(5), 2020.
 *
 * The problem is the paper's: A is n-by-n, sparse, symmetric positive
 * definite (Section 1); an optional SPD preconditioner M is used only through
 * products with M^{-1} (Section 1, preconditioned variants); the inputs are
 * exactly HS-CG's, (A, M, b, x0), and no variant has a tuning parameter.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments named as device arrays are device pointers on the device
 *   that was current when the matrix handle was created (for instance the
 *   data pointer of a torch CUDA tensor).  `info`, `history`, `iters`,
 *   `status` and `sys_row_offset` are host pointers.
 * - Ownership: the library never keeps a caller pointer after a call
 *   returns.  prcg_create_csr copies the matrix; a handle owns all of its
 *   device memory and prcg_destroy releases it.
 * - Streams: all device work is enqueued on the stream given at creation
 *   (NULL = the default stream).  Solves return after the work is finished;
 *   the host waits once per batch of iterations, never once per iteration.
 * - Concurrency: a handle is not thread-safe; distinct handles may be used
 *   from different threads.
 * - Errors: every function returns a prcg_status.  Negative codes are caller
 *   or system errors: after PRCG_EINVAL nothing was written, after
 *   PRCG_EDEVICE outputs are unspecified.  Non-negative codes are numerical
 *   outcomes and come with a valid x.  prcg_last_error() describes the last
 *   non-OK status of the calling thread.
 * - Arithmetic is IEEE double precision throughout; indices are int32, so
 *   n and nnz are below 2^31.
 */
#ifndef PRCG_H
#define PRCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prcg_matrix_s* prcg_matrix;
typedef struct prcg_batch_s* prcg_batch;

/* The variants.
 *   PRCG_HS      Alg. 1, Hestenes-Stiefel CG: one product, inner products
 *                nu_k and mu_k, two synchronisations per iteration.
 *   PRCG_PR      Alg. 2, predict-and-recompute CG: nu'_k from
 *                eq. nuk_simplified predicts beta_k; mu, sigma, gamma and the
 *                recomputed nu share one reduction.
 *   PRCG_PIPE_PR Alg. 3, pipelined predict-and-recompute CG: recurrences for
 *                s, s~, w', w~'; the products u = A s~ and w = A r~ (the
 *                recompute of w') read A once and overlap the reduction.
 *   PRCG_M       M-CG (Appendix D): PR-CG with nu'_k = -nu_{k-1} + alpha^2 gamma.
 *   PRCG_PIPE_M  pipe-PR-M-CG (Appendix D): pipe-PR-CG with the M-CG nu'.
 *   PRCG_GV      GV-CG (Appendix D), the Ghysels-Vanroose pipelined CG the
 *                paper compares against: recurrences for w, s, u and
 *                mu_k = eta_k - (beta_k / alpha_{k-1}) nu_k; one product
 *                t = A w~ per iteration overlaps the reduction.
 *   PRCG_PR_NORECOMPUTE  the ablation of Section 2: PR-CG that keeps the
 *                predicted nu'_k as nu_k (eq. nuk_norecomp) instead of
 *                recomputing it; it loses accuracy and is for study only.
 *   PRCG_PIPE_PR_NOWRECOMPUTE  the second ablation of Section 2: pipe-PR-CG
 *                that keeps w'_k (and w~'_k) as w_k instead of recomputing
 *                w_k = A r~_k; the product computes u = A s~ only.
 *   PRCG_CG      CG-CG (Appendix D), the Chronopoulos-Gear variant: w = A r~
 *                each iteration, nu_k and eta_k = <r~_k, w_k> in one
 *                reduction, mu_k = eta_k - (beta_k / alpha_{k-1}) nu_k.
 *   PRCG_PR_UNSIMPLIFIED  PR-CG predicting nu'_{k+1} with the four terms of
 *                eq. nuk: delta_k = <s~_k, r_k> joins the reduction instead
 *                of being taken equal to sigma_k = <r~_k, s_k> (Appendix C
 *                discusses when the two differ).  Without a preconditioner
 *                it computes exactly what PRCG_PR does; for study.
 * The batched solver runs the first five. */
typedef enum {
    PRCG_HS = 0,
    PRCG_PR = 1,
    PRCG_PIPE_PR = 2,
    PRCG_M = 3,
    PRCG_PIPE_M = 4,
    PRCG_GV = 5,
    PRCG_PR_NORECOMPUTE = 6,
    PRCG_PIPE_PR_NOWRECOMPUTE = 7,
    PRCG_CG = 8,
    PRCG_PR_UNSIMPLIFIED = 9
} prcg_variant;

/* Preconditioners: none (M = I) or Jacobi (M^{-1} = diag(A)^{-1}). */
typedef enum { PRCG_PRECOND_NONE = 0, PRCG_PRECOND_JACOBI = 1 } prcg_precond;

typedef enum {
    PRCG_OK = 0,             /* converged: ||r_k|| <= tol * ||b||, x = x_k            */
    PRCG_NOT_CONVERGED = 1,  /* k reached maxit; x = x_maxit                           */
    PRCG_BREAKDOWN = 2,      /* nu_k <= 0, mu_k <= 0, nu' <= 0 or a non-finite scalar  */
    PRCG_EINVAL = -1,        /* invalid argument or matrix                            */
    PRCG_ENOMEM = -2,        /* device or host allocation failed                      */
    PRCG_EDEVICE = -3        /* a HIP call failed                                     */
} prcg_status;

/* Outcome of one solve.  relres_updated = ||r_k|| / ||b|| with r_k the
 * recursively updated residual; relres_true = ||b - A x_k|| / ||b||,
 * computed once at exit.  Both are 0 when b = 0. */
typedef struct {
    int32_t iters;
    int32_t status;
    double relres_updated;
    double relres_true;
} prcg_info;

/* Storage the library chose for a matrix (informational). */
typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t stored_entries;   /* value slots of the SpMV layout, padding included    */
    int32_t format;           /* 0 = SELL-64 (one row per lane), 1 = vector CSR      */
    int32_t lanes_per_row;    /* 1 for SELL-64, L for vector CSR                     */
    int32_t grid;             /* workgroups of the row-parallel kernels              */
    int32_t block;            /* threads per workgroup                               */
    int64_t matrix_bytes;     /* bytes of the SpMV layout read by one product        */
    double aligned_slices_frac; /* SELL-64: share of slots in offset-aligned slices,
                                   which store one column offset per slot and slice
                                   instead of a column index per entry              */
    int32_t kernels;          /* kernel structure in use (PRCG_KERNELS_*; AUTO is
                                 reported as the structure it chose)              */
    int32_t stage2;           /* two-pass stage-2 reductions in one-workgroup
                                 kernels of their own: bit 0 HS-CG, bit 1 PR-CG
                                 and M-CG                                         */
    int64_t streamed_entries; /* SELL-64: value slots read with nontemporal loads
                                 (offset-aligned slices past the first 128 MiB of
                                 values, which stay cacheable between products)   */
} prcg_matrix_props;

/* Options (prcg_set_option).
 *   PRCG_OPT_KERNELS  kernel structure of an iteration:
 *     PRCG_KERNELS_AUTO (default): FUSED for HS-CG and the PR-CG forms when
 *       A is stored as SELL-64 and the row-parallel kernels have fewer than
 *       2048 workgroups (below 8192 row groups of 256 by the default grid),
 *       for pipe-PR-CG only below 64 workgroups; TWO_PASS otherwise.
 *       prcg_get_props reports the structure chosen for HS-CG and PR-CG.
 *     PRCG_KERNELS_FUSED: PR-CG and pipe-PR-CG run one kernel per
 *       iteration, HS-CG two; the sparse product recomputes the new
 *       direction at neighbouring rows from double-buffered vectors, with
 *       the owner's exact operations.  Needs the SELL-64 layout; matrices
 *       stored as vector CSR use the two-pass structure.
 *     PRCG_KERNELS_TWO_PASS: an update kernel and a product kernel
 *       per reduction (PR: 2, pipe-PR: 2, HS: 3 kernels per iteration), with
 *       stage 2 of each reduction (the sum of the per-workgroup partials)
 *       placed by size: HS-CG and PR-CG as STAGE2 from 2048 workgroups
 *       up, else as REDUNDANT; pipe-PR-CG always as REDUNDANT.
 *     PRCG_KERNELS_TWO_PASS_REDUNDANT: stage 2 runs redundantly in every
 *       workgroup of the kernel that consumes the totals (pipe-PR-CG: in
 *       workgroup 0 of the product kernel, before its share of the
 *       product, so that the reduction overlaps the others' products).
 *     PRCG_KERNELS_TWO_PASS_STAGE2: every stage-2 reduction in a
 *       one-workgroup kernel of its own (PR and pipe-PR: 3, HS: 5 kernels per
 *       iteration).
 *     PRCG_KERNELS_TWO_PASS_LAST: stage 2 run by the last workgroup of the
 *       kernel that writes the partials (an atomic ticket counter picks it;
 *       no workgroup waits for another).  Slower on MI355X: the fence that
 *       publishes each workgroup's partials to the other XCDs writes back
 *       its L2.
 *     PRCG_KERNELS_TEXTBOOK: HS-CG as one kernel per line of Alg. 1 (AXPYs,
 *       preconditioner, each inner product, a one-workgroup reduction
 *       kernel per synchronisation, the product): the unfused baseline.
 *       Other variants run TWO_PASS under this setting.
 *   All two-pass placements add the partials in the same fixed order:
 *   results are bitwise identical across them.
 *   PRCG_OPT_GRID  largest number of workgroups of the row-parallel kernels
 *     (8..16384; the actual count is a multiple of 8), or 0 (the default):
 *     by size, one 256-row group per workgroup from 8192 groups (2M rows)
 *     up (at most 16384 workgroups), else at most 1024. */
typedef enum { PRCG_OPT_KERNELS = 0, PRCG_OPT_GRID = 1 } prcg_option;
typedef enum {
    PRCG_KERNELS_FUSED = 0,
    PRCG_KERNELS_TWO_PASS = 1,
    PRCG_KERNELS_TWO_PASS_STAGE2 = 2,
    PRCG_KERNELS_TEXTBOOK = 3,
    PRCG_KERNELS_TWO_PASS_LAST = 4,
    PRCG_KERNELS_TWO_PASS_REDUNDANT = 5,
    PRCG_KERNELS_AUTO = 6
} prcg_kernels;

/*
 * Create a matrix handle from CSR arrays (Section 1: A sparse SPD).
 *   n, nnz    1 <= n < 2^31, 0 <= nnz < 2^31.
 *   row_ptr   device int32[n+1]: row_ptr[0] = 0, non-decreasing,
 *             row_ptr[n] = nnz.
 *   col_idx   device int32[nnz]: 0 <= col < n.  Any order within a row;
 *             duplicates are summed.  Each row is summed in stored order.
 *   values    device float64[nnz].
 *   precond   PRCG_PRECOND_JACOBI needs every diagonal entry (summed over
 *             duplicates) to be > 0.
 *   hip_stream  hipStream_t cast to void*, or NULL.
 * The arrays are copied (and re-laid-out for the SpMV); the caller may free
 * them afterwards.  Symmetry and definiteness are preconditions, not
 * checked; violating them shows up as PRCG_BREAKDOWN or PRCG_NOT_CONVERGED.
 * Returns PRCG_EINVAL for an invalid structure (nothing is allocated then).
 */
prcg_status prcg_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* values, prcg_precond precond, void* hip_stream,
                            prcg_matrix* out);

/* Replace the values of A (same sparsity pattern, CSR order as at
 * creation; device float64[nnz]) and refresh the Jacobi diagonal. */
prcg_status prcg_set_values(prcg_matrix A, const double* values);

/* Set an option of A (see prcg_option); results of later solves are
 * bitwise repeatable for a fixed option set. */
prcg_status prcg_set_option(prcg_matrix A, int32_t option, int32_t value);

/* Change the stream used by later calls on A. */
prcg_status prcg_set_stream(prcg_matrix A, void* hip_stream);

/* y = A x (device float64[n] each; x and y must not overlap).  The product
 * of Section 3 eq. Ax: each row summed in stored order with fused
 * multiply-adds.  Non-finite entries of x: the SELL-64 layout pads rows to
 * their slice's width with zero slots, which multiply 0 by an entry of x in
 * the row's own system (offset-aligned slices: the column row + offset,
 * clamped into range; packed slices: the row itself), so a non-finite x at
 * such a column makes y_i NaN where a product over the stored entries alone
 * would stay finite.  Finite x gives the same result either way. */
prcg_status prcg_spmv(prcg_matrix A, const double* x, double* y);

/*
 * Solve A x = b with one variant (Algs. 1-3, Appendix D), starting from the
 * initialisation of Appendix D.
 *   b        device float64[n].
 *   x        device float64[n]; x_0 on entry, the final iterate on exit.
 *   tol      >= 0.  Stops at the first k with ||r_k|| <= tol * ||b|| (r_k
 *            the updated residual).  tol = 0 runs exactly maxit iterations
 *            unless the method breaks down.
 *   maxit    >= 0.
 *   info     host, nullable.
 *   history  host, nullable, maxit+1 doubles: history[k] = ||r_k|| / ||b||
 *            for k = 0..iters (entries past iters are left untouched).
 * b = 0 gives x = 0, iters = 0, PRCG_OK.  Breakdown (the paper notes the
 * methods break down when nu turns negative): nu_k <= 0, mu_k <= 0 or a
 * non-finite scalar after the reduction of iteration k returns x_k; a
 * predicted nu'_{k+1} <= 0 makes iteration k+1 the last one (its x and r
 * updates do not involve nu'), which returns x_{k+1} with PRCG_OK if its
 * residual meets tol, else PRCG_BREAKDOWN.
 * Inner products are reduced deterministically: the same call on the same
 * device gives bitwise identical results.
 */
prcg_status prcg_solve(prcg_matrix A, prcg_variant v, const double* b, double* x, double tol,
                       int32_t maxit, prcg_info* info, double* history);

/*
 * prcg_solve for callers that cannot allocate device memory: code that runs
 * between graph captures, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and bits as prcg_solve on the same
 * handle, but the call allocates nothing: the partial sums, the scalar
 * state and the residual history live in a fixed device array of the
 * library (about 2.8 MB per device, held from the first such call until the
 * process ends), and the iterations are launched directly instead of
 * through an instantiated graph.  The handle (created beforehand) still
 * owns the vectors.
 *   maxit    0 <= maxit <= PRCG_NOALLOC_MAX_ITERS, else PRCG_EINVAL (nothing
 *            written): the history array holds PRCG_NOALLOC_MAX_ITERS + 1
 *            entries.
 * Every call on one device shares that device's array and leaves its
 * contents behind: calls that overlap on one device (from several threads
 * or streams) race and give undefined results.
 */
#define PRCG_NOALLOC_MAX_ITERS 65536
prcg_status prcg_solve_noalloc(prcg_matrix A, prcg_variant v, const double* b, double* x, double tol,
                               int32_t maxit, prcg_info* info, double* history);

/*
 * Per-kernel device time of `iters` iterations of variant v on A, from
 * x0 = 0 with b = (1, ..., 1) and tol = 0 (so every iteration does its full
 * work; PRCG_EDEVICE if the run ends early).  Each launch carries dispatch
 * start/stop timestamps (hipExtLaunchKernelGGL events) and runs on the
 * handle's own non-blocking stream after A's stream has drained, so the
 * times are kernel execution times.  Overwrites the solver state of A.
 *   ms_per_launch  host float64[capacity]: average milliseconds per launch
 *                  of each kernel of one iteration, in launch order.
 *   names          host, nullable, char[capacity][48]: kernel names.
 *   capacity       entries of ms_per_launch / names; PRCG_EINVAL (nothing
 *                  written) if an iteration has more kernels (at most 10).
 *   nkernels       host: number of kernels per iteration.
 */
prcg_status prcg_time_kernels(prcg_matrix A, prcg_variant v, int32_t iters, double* ms_per_launch,
                              char (*names)[48], int32_t capacity, int32_t* nkernels);

/* Describe the storage chosen for A. */
prcg_status prcg_get_props(prcg_matrix A, prcg_matrix_props* props);

/*
 * Batched solve of nsys independent systems stored as one block-diagonal
 * matrix (not in the paper; the block-diagonal structure is the only
 * assumption).  Two modes (prcg_batch_set_mode): a persistent kernel in
 * which each workgroup takes the next-largest unsolved system from a queue
 * and runs its whole solve with workgroup-local reductions, and (PR-CG,
 * M-CG) a lockstep mode in which every iteration is three launches over the
 * row groups of all systems still running.
 *   blockdiag       a handle created by prcg_create_csr (no column index
 *                   may leave its block; checked here).
 *   sys_row_offset  host int64[nsys+1]: system s owns rows
 *                   [off[s], off[s+1]); off[0] = 0, strictly increasing,
 *                   off[nsys] = n.
 */
prcg_status prcg_create_batch(prcg_matrix blockdiag, int32_t nsys, const int64_t* sys_row_offset,
                              prcg_batch* out);

/* Solve every system of the batch with variant v, same semantics per system
 * as prcg_solve (the matrix handle's preconditioner applies).  b, x: device
 * float64[n]; x holds x_0 on entry.  iters, status: host int32[nsys],
 * nullable.  Returns the largest per-system status (OK < NOT_CONVERGED <
 * BREAKDOWN).  The first call with a variant runs the autotuner, each
 * candidate timed with HIP events on this batch:
 *   persistent launch: threads per workgroup (256, 512, 1024) x workgroups
 *     per compute unit (1, 2, 4, 8; at most 2048 threads per compute unit)
 *     x slices multiplied together per wavefront in the product (1 or 2),
 *     a few iterations of every system each;
 *   lockstep row groups (PR-CG, M-CG): 8, 16 or 32 slices of 64 rows per
 *     group (2, 4 or 8 slices per wavefront), each with three launches per
 *     iteration and, where allowed, with the fused iteration
 *     (prcg_batch_set_fusion), the initialisation and 32 iterations each;
 *   mode (PR-CG, M-CG, unless set): one whole solve in each, the faster kept.
 * prcg_batch_set_config and prcg_batch_set_fusion fix any of these
 * instead.  The persistent launch
 * and chunks of lockstep iterations are captured in HIP graphs.
 * Reductions are deterministic for a fixed configuration (threads per
 * workgroup and group size set the order of a system's sums; the number of
 * slices in flight does not): a configuration the autotuner picks can differ
 * between processes, so fix it for results that must agree bit for bit
 * across processes. */
prcg_status prcg_solve_batched(prcg_batch B, prcg_variant v, const double* b, double* x, double tol,
                               int32_t maxit, int32_t* iters, int32_t* status);

/* The configuration the batched solver's autotuner chose for variant v
 * (0, 0 before the first prcg_solve_batched with that variant): threads per
 * workgroup (64 per wavefront) and workgroups of the persistent launch.
 * The environment variable PRCG_BATCH_CONFIG="threads,per_cu" (threads in
 * 256/512/1024, 1 <= per_cu <= 8) fixes it instead. */
prcg_status prcg_batch_config(prcg_batch B, prcg_variant v, int32_t* threads, int32_t* grid);

/* Fix parts of the batched configuration for later solves (0 leaves a part
 * to the autotuner); forgets earlier choices.
 *   threads           0, 256, 512 or 1024 threads per persistent workgroup
 *   per_cu            0..8 persistent workgroups per compute unit
 *                     (threads x per_cu <= 2048)
 *   slices_in_flight  0, 1 or 2 slices multiplied together per wavefront
 *   group_slices      0, 8, 16 or 32 slices per lockstep row group
 * PRCG_EINVAL for other values. */
prcg_status prcg_batch_set_config(prcg_batch B, int32_t threads, int32_t per_cu, int32_t slices_in_flight,
                                  int32_t group_slices);

/* The batch's storage and the configuration in use for variant v (zeros
 * for parts not chosen yet). */
typedef struct {
    int64_t n;                /* rows of all systems                                  */
    int64_t stored_entries;   /* value slots of the batch's SELL-64 slices            */
    int64_t matrix_bytes;     /* bytes of those slices read by one product of all
                                 systems (values, packed columns, offsets, metadata) */
    int64_t groups;           /* lockstep row groups of the size in use               */
    int64_t uniform_groups;   /* of which uniform (one width and offset list)         */
    int32_t nsys;
    int32_t mode;             /* PRCG_BATCH_PERSISTENT / _LOCKSTEP, 0 if undecided    */
    int32_t threads;          /* persistent: threads per workgroup                    */
    int32_t grid;             /* persistent: workgroups                               */
    int32_t slices_in_flight; /* persistent: slices multiplied together per wavefront */
    int32_t group_slices;     /* lockstep: slices per row group (PR-CG, M-CG)         */
    int32_t fused;            /* lockstep: 1 when iterations run fused                */
} prcg_batch_props;
prcg_status prcg_batch_get_props(prcg_batch B, prcg_variant v, prcg_batch_props* props);

/* How the batched solver runs PR-CG and M-CG (HS-CG and the pipelined
 * variants always run persistent):
 *   PRCG_BATCH_PERSISTENT  one persistent kernel, a workgroup per system;
 *   PRCG_BATCH_LOCKSTEP    three launches per iteration (one when fused:
 *     prcg_batch_set_fusion) over the row groups
 *     (8, 16 or 32 slices of 64 rows of one system) of every system still
 *     running: the
 *     vector update, the product with one partial per group of each inner
 *     product, then one workgroup per system that sums its partials in a
 *     fixed order and takes the scalar step (Alg. 2); the host checks every
 *     16 iterations whether a system is still running;
 *   PRCG_BATCH_AUTO (default)  the faster of the two on the first solve. */
typedef enum { PRCG_BATCH_AUTO = 0, PRCG_BATCH_PERSISTENT = 1, PRCG_BATCH_LOCKSTEP = 2 } prcg_batch_mode_t;

/* Lockstep iterations of PR-CG and M-CG (with or without the Jacobi
 * preconditioner) may run fused, one launch per iteration: a workgroup
 * updates x, r and p of its row group, multiplies the new p (recomputing it
 * at the rows outside the group that the stencil reaches, held in LDS) and
 * writes its partials; the last workgroup of each system to finish (an
 * atomic ticket per system) takes the system's stage 2 and scalar step.
 * Without a preconditioner eight vector words per row move instead of ten
 * (with Jacobi, twelve instead of fifteen).  Allowed for a group table
 * whose groups are all offset-aligned with one offset list each, of at most
 * 7 slots, at 8 or 16 slices per group, when the stencil span (largest
 * minus smallest column offset, 0 included) is at most 6656 rows (8 slices)
 * or 5120 (16 slices), so that a workgroup's LDS stays within 64 KB.  The
 * results equal those of three launches bit for bit.
 *   PRCG_BATCH_FUSION_AUTO  the autotuner times both (default);
 *   PRCG_BATCH_FUSION_OFF   three launches per iteration;
 *   PRCG_BATCH_FUSION_ON    fused only: where no group table allows it, a
 *                           solve with PR-CG or M-CG fails with PRCG_EINVAL
 *                           unless the mode is PRCG_BATCH_PERSISTENT. */
typedef enum {
    PRCG_BATCH_FUSION_AUTO = 0,
    PRCG_BATCH_FUSION_OFF = 1,
    PRCG_BATCH_FUSION_ON = 2
} prcg_batch_fusion_t;

/* Request a fusion setting (PRCG_BATCH_FUSION_*) for later solves; forgets
 * the lockstep group size chosen before.  PRCG_EINVAL for an unknown
 * setting. */
prcg_status prcg_batch_set_fusion(prcg_batch B, int32_t fusion);

/* Request a mode (PRCG_BATCH_*) for later solves; forgets earlier choices.
 * PRCG_EINVAL for an unknown mode. */
prcg_status prcg_batch_set_mode(prcg_batch B, int32_t mode);

/* The mode in use for variant v (PRCG_BATCH_PERSISTENT or _LOCKSTEP; 0
 * before the first prcg_solve_batched with that variant). */
prcg_status prcg_batch_mode(prcg_batch B, prcg_variant v, int32_t* mode);

/*
 * Adjoint of a solve (not in the paper): for L(x) with x = A^{-1} b and
 * gx = dL/dx, solves A lambda = gx with variant v (A is symmetric, so
 * A^T = A) and returns
 *   gb     device float64[n], nullable:   dL/db = lambda;
 *   gvals  device float64[nnz], nullable: dL/dA_e = -lambda[row(e)] * x[col(e)]
 *          for every stored entry e, in the CSR order given at creation.
 *   x      device float64[n]: the forward solution.
 *   info   host, nullable: outcome of the adjoint solve.
 */
prcg_status prcg_adjoint(prcg_matrix A, prcg_variant v, const double* x, const double* gx, double* gb,
                         double* gvals, double tol, int32_t maxit, prcg_info* info);

void prcg_destroy(prcg_matrix A);
void prcg_batch_destroy(prcg_batch B);
const char* prcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRCG_H */
