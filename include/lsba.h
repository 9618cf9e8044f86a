/*
 * lsba.h -- C ABI of the MI355X (gfx950) adaptively restarted block Krylov
 * solver library (liblsba.so).
 *
 * The library solves A X = B for a large sparse A (n x n, CSR) and a block of
 * s right-hand sides (n x s) with restarted block FOM or block GMRES, built on
 * a block Arnoldi cycle with one of the low-synchronization block Gram-Schmidt
 * skeletons of K. Lund, "Adaptively restarted block Krylov subspace methods
 * with low-synchronization skeletons":
 *
 *   - problem statement A X = B ........................... Sec. 2, eq. (AX=B)
 *   - classical block inner product X^T Y ................. Sec. 2.2, Table 1
 *   - skeletons BMGS-SVL / BMGS-LTS ....................... Sec. 3.2, Alg. 5
 *   - skeletons BMGS-CWY / BMGS-ICWY ...................... Sec. 3.3, Alg. 6
 *   - skeleton BCGSI+LS ................................... Sec. 3.4, Alg. 7
 *   - muscles (IntraOrtho) CholQR / HouseQR ............... Sec. 2.3, Sec. 5
 *   - BFOM / BGMRES as modified BFOM ...................... Sec. 2.4.1, eq. Xm
 *   - cospatial restarts, residual estimate ............... Sec. 2.4.2, Thm. 1,
 *                                                           eq. normF_Rm
 *   - adaptive restarting on a Cholesky breakdown ......... Sec. 4
 *   - loss of orthogonality ||I - V^T V||_2 ............... Sec. 2.3, eq. loo
 *   - counts of A-calls, basis applications, syncs ........ Sec. 2.1, Sec. 5
 *   - ILU(0) right preconditioning ........................ Sec. 5 (tests on
 *                                                           matrices from
 *                                                           applications)
 *
 * Real double-precision arithmetic (the conjugate transpose of the paper is
 * the plain transpose).  Every step of the solve runs in the library's own
 * HIP kernels on one GPU.
 *
 * Conventions
 *   Layout.    Blocks of right-hand sides and solutions are n x s, row-major:
 *              element (i, c) is at ptr[i * ld + c], ld >= s.
 *   CSR.       row_ptr is int64 [n+1] with row_ptr[0] = 0 and row_ptr[n] = nnz,
 *              non-decreasing; col_idx is int32 [nnz] with 0 <= col < n;
 *              values is double [nnz].  Column order inside a row is free.
 *   Memory.    Pointer arguments are host pointers when the matching
 *              `on_device` argument is 0, and device pointers (on the
 *              context's device) when it is 1.  Inputs stay owned by the
 *              caller; the library copies what it keeps.  Handles are owned by
 *              the caller and released only by their _destroy function.
 *   Streams.   All device work of a context is issued on its stream.  Calls
 *              on one context must come from one host thread at a time.
 *   Errors.    A negative lsba_status means the call failed and wrote no
 *              output; lsba_last_error() then holds a message.  A positive
 *              status from lsba_solve means X holds the last iterate and the
 *              result is valid.
 *   Limits.    1 <= s <= 32, 1 <= m <= 128, n >= 1, n * s < 2^31.
 */
#ifndef LSBA_H
#define LSBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSBA_OK = 0,                /* converged: residual estimate / ||B||_F <= tol            */
  LSBA_NOT_CONVERGED = 1,     /* max_cycles or max_iters reached; X = last iterate         */
  LSBA_BREAKDOWN = 2,         /* Cholesky flag with no final column left (Sec. 4); X kept  */
  LSBA_ERR_ARG = -1,          /* invalid argument (null pointer, bad size, bad enum)      */
  LSBA_ERR_OOM = -2,          /* device or host allocation failed                         */
  LSBA_ERR_HIP = -3,          /* a HIP runtime call failed                                */
  LSBA_ERR_UNSUPPORTED = -4,  /* valid but not supported combination                      */
  LSBA_ERR_BUSY = -5          /* the serving queue is full                                */
} lsba_status;

typedef enum { LSBA_FOM = 0, LSBA_GMRES = 1 } lsba_method;       /* modification none / harmonic */

typedef enum {
  LSBA_BCGSI_LS = 0,          /* Alg. 7 */
  LSBA_BMGS_SVL = 1,          /* Alg. 5, Schreiber-Van Loan T update */
  LSBA_BMGS_LTS = 2,          /* Alg. 5, lower-triangular-solve T update */
  LSBA_BMGS_CWY = 3,          /* Alg. 6, compact WY */
  LSBA_BMGS_ICWY = 4,         /* Alg. 6, inverse compact WY */
  LSBA_BCGS_PIP = 5,          /* Alg. 3, one fused inner product + Pythagorean Cholesky */
  LSBA_BMGS = 6,              /* Alg. 2, the block MGS baseline: k + 1 syncs at step k */
  LSBA_BCGS_PIO = 7           /* Alg. 4, inner product + IntraOrtho of [W 0; 0 H]: 2 syncs/step */
} lsba_skeleton;

/* LSBA_GLOBAL selects the global block paradigm as a whole (Sec. 2.2,
   Table 1): every block inner product is (1/s) trace(X^T Y) I_s and the
   muscle is the global scaling ||X||_F / sqrt(s) I_s (the paper forces that
   muscle in the global paradigm).  Not available with LSBA_BCGS_PIO. */
/* LSBA_MGS_SVL / LSBA_MGS_LTS are the column-wise low-sync MGS muscles
   (Sec. 5; the column versions of Alg. 5, 3 s - 2 syncs per call), the
   muscles the paper pairs with BMGS-SVL / BMGS-LTS; they also serve the
   cycle start of every other skeleton but BCGS-PIO. */
typedef enum {
  LSBA_CHOLQR = 0,
  LSBA_HOUSEQR = 1,
  LSBA_GLOBAL = 2,
  LSBA_MGS_SVL = 3,
  LSBA_MGS_LTS = 4
} lsba_muscle;

typedef enum {
  LSBA_FP64 = 0,              /* every step in FP64                                        */
  LSBA_MIXED = 1              /* inner solves with an FP32 basis: FP32 SpMM, Gram products
                                 (FP32 products, FP64 cross-lane sums) and projections on the
                                 vector units; FP64 Cholesky (shifted retry) and Hessenberg
                                 steps; FP64 outer iterative refinement on B - A X            */
} lsba_precision;

enum {
  LSBA_REC_LOO = 1u,          /* record ||I - V_{1:j+1}^T V_{1:j+1}||_2 after every column  */
  LSBA_REC_TRUE_RES = 2u      /* compute the final FP64 true residual ||B - A X||_F/||B||_F  */
};

typedef struct {
  uint32_t struct_size;       /* sizeof(lsba_params); set by lsba_params_default            */
  int32_t method;             /* lsba_method                                               */
  int32_t skeleton;           /* lsba_skeleton                                             */
  int32_t muscle;             /* lsba_muscle (IntraOrtho at each cycle start; every step
                                 for BMGS-SVL/LTS)                                           */
  int32_t precision;          /* lsba_precision                                            */
  int32_t m;                  /* maximum basis size per cycle (block columns)              */
  double tol;                 /* stop when residual estimate / ||B||_F <= tol              */
  int32_t max_cycles;         /* restart cycles allowed                                    */
  int64_t max_iters;          /* total block columns allowed (<= 0: unlimited)             */
  int32_t max_refine;         /* LSBA_MIXED: outer refinement steps allowed                */
  double inner_tol;           /* LSBA_MIXED: relative tolerance of each inner solve, loosened
                                 so that no inner solve aims below tol / 2 overall          */
  uint32_t record;            /* LSBA_REC_* bit set                                        */
  int32_t force_flag_cycle;   /* test hook: raise the Cholesky flag at this cycle (1-based) */
  int32_t force_flag_step;    /*   ... and this skeleton loop step k (0 = first IntraOrtho);
                                 -1 disables the hook                                        */
} lsba_params;

typedef struct lsba_context lsba_context;
typedef struct lsba_operator lsba_operator;
typedef struct lsba_result lsba_result;

/* Fill *p with defaults: BGMRES, BCGSI+LS, CholQR, FP64, m = 20, tol = 1e-8,
 * max_cycles = 50, max_iters = 0, max_refine = 20, inner_tol = 1e-4, record = 0,
 * force flag off.  Returns LSBA_ERR_ARG for p == NULL. */
lsba_status lsba_params_default(lsba_params* p);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * issue work on (not owned), or NULL to let the library create and own one.
 * On success *ctx receives the handle. */
lsba_status lsba_context_create(int device, void* hip_stream, lsba_context** ctx);
void lsba_context_destroy(lsba_context* ctx);
/* Message of the last failed call on ctx (or of the last failed context
 * creation when ctx is NULL).  Owned by the library. */
const char* lsba_last_error(const lsba_context* ctx);
const char* lsba_status_string(lsba_status st);

/* Device-time statistics per kernel class.  While timing is enabled, HIP
 * events are recorded on the launching stream around every kernel launch of
 * the selected classes; elapsed times and the launches' algorithmic bytes (the block
 * and CSR data the method must read and write, not the implementation's extra
 * traffic) are accumulated per class.  Launches queued after the step that
 * ended a cycle find nothing to do: they count with their (short) durations
 * and zero bytes. */
typedef enum {
  LSBA_K_SPMM = 0,            /* W = A V (block SpMM)                                       */
  LSBA_K_GRAM = 1,            /* Gram products, split-n stage                                */
  LSBA_K_GRAM_REDUCE = 2,     /* Gram products, fixed-order reduction stage (0 bytes)        */
  LSBA_K_UPDATE = 3,          /* fused block updates / projections / basis applications      */
  LSBA_K_SMALL = 4,           /* small dense steps (0 bytes)                                 */
  LSBA_K_RESIDUAL = 5,        /* FP64 true residual B - A X                                  */
  LSBA_K_PRECOND = 6          /* ILU(0) triangular sweeps (one launch per level or run of
                                 chained levels)                                             */
} lsba_kernel_kind;
/* Time the kernel classes whose bits (1u << lsba_kernel_kind) are set in
 * kind_mask (LSBA_TIME_ALL: every class; 0: timing off).  Launches of other
 * classes are not bracketed by events, so timing one class perturbs the run
 * least.  Either way the statistics are cleared. */
#define LSBA_TIME_ALL 0x7Fu
lsba_status lsba_context_set_timing(lsba_context* ctx, uint32_t kind_mask);
/* Launch count, summed device milliseconds and summed algorithmic bytes of a
 * kernel class since timing was enabled (all zero when disabled). */
lsba_status lsba_context_kernel_stats(const lsba_context* ctx, int32_t kind, int64_t* launches,
                                      double* total_ms, double* total_bytes);
/* Summed algorithmic floating-point operations of a kernel class's timed
 * launches (2 per multiply-add of the products the method needs: the Gram
 * 2 n (p s)(q s), an update 2 n s^2 per coefficient block it applies, the
 * SpMM 2 nnz s; 0 for the other classes). */
lsba_status lsba_context_kernel_flops(const lsba_context* ctx, int32_t kind, double* total_flops);

/* Cycle replay.  A cycle's launch sequence depends only on host values fixed
 * for a solve (buffer and operator pointers, sizes, method, skeleton, muscle,
 * restart length).  With enable = 1 it is captured into a hipGraph on first
 * use and replayed with one launch per cycle; the context keeps up to 8 such
 * graphs, keyed by those values, and drops them all when a cached buffer is
 * freed or this setting changes.  enable = 0 (the default) launches every
 * kernel individually, which on ROCm keeps the three streams' kernels
 * overlapping best.  Results are bitwise the same either way; while kernel
 * timing is enabled cycles are always launched individually. */
lsba_status lsba_context_set_graphs(lsba_context* ctx, int enable);

/* Copy a CSR matrix (layout above) into device memory owned by the operator.
 * Validates the row pointer (monotone, row_ptr[0] = 0, row_ptr[n] = nnz) and
 * the column range; an invalid matrix gives LSBA_ERR_ARG. */
lsba_status lsba_operator_create_csr(lsba_context* ctx, int64_t n, int64_t nnz,
                                     const int64_t* row_ptr, const int32_t* col_idx,
                                     const double* values, int on_device, lsba_operator** op);
/* Free an operator.  Destroying its context first is allowed: the context
 * then releases the operator's device memory, and this call only frees the
 * handle. */
void lsba_operator_destroy(lsba_operator* op);

/* Solve A X = B from X_0 = 0 (eq. Xm).  B and X are n x s row-major with
 * leading dimensions ldb, ldx >= s; host or device per `on_device`.  Blocks
 * until the solve ends.  *res receives a result handle for every status >= 0
 * (and for no negative status). */
lsba_status lsba_solve(lsba_context* ctx, const lsba_operator* op, const lsba_params* prm,
                       int32_t s, const double* B, int64_t ldb, double* X, int64_t ldx,
                       int on_device, lsba_result** res);

/* ---------------------------------------------------------------- ILU(0)
 * Incomplete LU factorization with no fill (the preconditioner of the
 * paper's tests on matrices from applications, Sec. 5): L unit lower
 * triangular and U upper triangular on A's stored pattern with
 * (L U)_ij = a_ij for every stored (i, j) -- Gaussian elimination in row
 * order with every update outside the pattern dropped.  Rows and columns are
 * used in the order given; explicit zeros count as stored entries.
 * Factorization and every application run on the device, one dependency
 * level of rows at a time (levels are computed on the host from the pattern
 * once, at creation). */
typedef struct lsba_precond lsba_precond;

/* Factor op's matrix.  Every row must store its diagonal entry and no column
 * twice, and n < 2^31 - 1 (else LSBA_ERR_ARG); a zero or non-finite pivot
 * u_ii is LSBA_ERR_ARG with the row in lsba_last_error; LSBA_ERR_OOM when the
 * factors' device memory cannot be allocated.  The factors are device memory owned by
 * the handle; op may be destroyed afterwards.  Destroying the context first
 * releases the factors (lsba_precond_destroy then frees only the handle). */
lsba_status lsba_precond_create_ilu0(lsba_context* ctx, const lsba_operator* op,
                                     lsba_precond** pc);
void lsba_precond_destroy(lsba_precond* pc);

/* Z = M^{-1} Y = U^{-1} (L^{-1} Y) for an n x s block (1 <= s <= 32;
 * row-major, leading dimensions ldy, ldz >= s; host or device per on_device;
 * Z may equal Y).  Blocks until done. */
lsba_status lsba_precond_apply(lsba_context* ctx, const lsba_precond* pc, int32_t s,
                               const double* Y, int64_t ldy, double* Z, int64_t ldz,
                               int on_device);

/* Copy the factors to host arrays in CSR form on A's pattern with each row's
 * columns ascending: row_ptr [n+1], col_idx [nnz], values [nnz]; entries left
 * of the diagonal are L's multipliers (L's unit diagonal is not stored), the
 * diagonal and the entries right of it are U. */
lsba_status lsba_precond_factors(const lsba_precond* pc, int64_t* row_ptr, int32_t* col_idx,
                                 double* values);

/* Size, stored entries and number of dependency levels of the forward (L)
 * and backward (U) sweeps; any output pointer may be NULL. */
lsba_status lsba_precond_info(const lsba_precond* pc, int64_t* n, int64_t* nnz,
                              int32_t* levels_lower, int32_t* levels_upper);

/* lsba_solve with right preconditioning: the restart cycles run on A M^{-1}
 * (each basis block goes through M^{-1} before the SpMM) and X = M^{-1} Y
 * for the cycles' solution Y.  The residual of A M^{-1} Y = B is B - A X, so
 * tol, the residual history and the true residual mean what they mean
 * without M.  pc must come from ctx and have op's size (it may be the
 * factorization of another matrix of that size).  FP64 form only
 * (LSBA_MIXED: LSBA_ERR_UNSUPPORTED). */
lsba_status lsba_solve_precond(lsba_context* ctx, const lsba_operator* op,
                               const lsba_precond* pc, const lsba_params* prm, int32_t s,
                               const double* B, int64_t ldb, double* X, int64_t ldx,
                               int on_device, lsba_result** res);

/* Variant of lsba_solve for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree or other device / pinned-memory allocator.  Its
 * workspace (copies of B and X, the basis of m + 1 blocks, U, W, Gram
 * partials, the small dense state, norm partials) is carved from a 64 MiB
 * device array of the library, one per device, reserved when the library's
 * code is loaded on that device and held until the process ends; a problem
 * whose workspace exceeds it gives LSBA_ERR_ARG (nothing is written).  B and
 * X are device pointers (n x s, row-major, leading dimensions ldb, ldx >= s).
 * FP64 form only (LSBA_MIXED: LSBA_ERR_UNSUPPORTED).  Results are exactly
 * those of lsba_solve with the same arguments; the result handle is host
 * memory as there.  Kernel timing and cycle replay are suspended during the
 * call.  All calls on one device share that device's array: calls that
 * overlap in time on one device (several contexts or host threads) race and
 * must be serialised by the caller.  Every value the solve reads from the
 * array is written by the same call first.  Blocks until the solve ends. */
lsba_status lsba_solve_noalloc(lsba_context* ctx, const lsba_operator* op, const lsba_params* prm,
                               int32_t s, const double* B, int64_t ldb, double* X, int64_t ldx,
                               lsba_result** res);

/* Result getters.  Arrays are library-owned host memory, valid until
 * lsba_result_destroy.  res_hist[i] is the residual estimate (eq. normF_Rm)
 * over ||B||_F after the i-th final block column, over all cycles (for the
 * mixed form: of the inner solves, in order).  loo_hist is NULL unless
 * LSBA_REC_LOO was set.  cycle_len[c] is the number of final columns of cycle
 * c and m_after[c] the basis size allowed after it (the adaptive restart
 * shrinks it, Sec. 4). */
lsba_status lsba_result_status(const lsba_result* r);
int64_t lsba_result_iters(const lsba_result* r);
const double* lsba_result_res_hist(const lsba_result* r);
const double* lsba_result_loo_hist(const lsba_result* r);
int32_t lsba_result_cycles(const lsba_result* r);
const int32_t* lsba_result_cycle_len(const lsba_result* r);
const int32_t* lsba_result_m_after(const lsba_result* r);
/* A-calls, basis applications and syncs as the paper counts them (Sec. 5). */
void lsba_result_counts(const lsba_result* r, int64_t* a_calls, int64_t* v_apps, int64_t* syncs);
/* ||B - A X||_F / ||B||_F in FP64 (NaN unless LSBA_REC_TRUE_RES or LSBA_MIXED). */
double lsba_result_true_relres(const lsba_result* r);
/* Error of a solution against a reference solution, e.g. the FP64 CPU
 * oracle's X on the same inputs: lsba_result_set_err_vs_ref forms
 * ||X - Xref||_F / ||Xref||_F in FP64 on the context's device (fixed-order
 * reductions; X and Xref n x s row-major with leading dimensions ldx, ldr,
 * host or device memory per on_device; neither is modified) and stores it
 * in r; lsba_result_err_vs_ref returns it, NaN until set.  The library does
 * not compute the reference itself. */
lsba_status lsba_result_set_err_vs_ref(lsba_context* ctx, lsba_result* r, int64_t n, int32_t s,
                                       const double* X, int64_t ldx, const double* Xref,
                                       int64_t ldr, int on_device);
double lsba_result_err_vs_ref(const lsba_result* r);
/* Outer refinement steps taken (LSBA_MIXED), else 0. */
int32_t lsba_result_refine_steps(const lsba_result* r);
/* Device time of the solve in milliseconds (HIP events around the whole solve). */
double lsba_result_gpu_ms(const lsba_result* r);
void lsba_result_destroy(lsba_result* r);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent FP64 solves (requests) on one device.
 * A server owns max_slots slots; each slot has its own streams, events,
 * pinned staging memory and stream-ordered device buffers.  An admitted
 * request keeps its basis, Hessenberg and control state on the device in its
 * slot; its restart cycles are queued one at a time by lsba_server_poll, so
 * the cycles of all admitted requests run concurrently on the GPU.  Requests
 * are admitted in arrival order when a slot is free and the sum of the
 * admitted requests' footprints (lsba_solve_footprint) stays within the byte
 * budget.  Each request computes exactly what lsba_solve computes for it
 * (same kernels, same fixed-order reductions): its X, histories and counts do
 * not depend on what else runs.  Progress happens only inside
 * lsba_server_poll; a server is used by one host thread at a time.  The
 * operators must outlive the requests that use them. */
typedef struct lsba_server lsba_server;

/* Device bytes an FP64 solve of an n-row operator with s right-hand sides
 * holds while it runs (B, X, basis of m + 1 blocks, U, W, Gram partials,
 * small dense state, norm workspaces); 0 for invalid arguments. */
uint64_t lsba_solve_footprint(int64_t n, int32_t s, const lsba_params* params);

/* Create a server on ctx's device.  hbm_budget_bytes > 0 bounds the summed
 * footprints of the admitted requests; 1 <= max_slots <= 64. */
lsba_status lsba_server_create(lsba_context* ctx, uint64_t hbm_budget_bytes, int32_t max_slots,
                               lsba_server** out);

/* Queue a request.  B (n x s, row-major, ld ldb; host memory, or device
 * memory if on_device) is copied into pinned host memory (the call returns
 * once the copy is done); *ticket identifies the request.
 * The parameters are validated as in lsba_solve; the serving form runs FP64
 * only (LSBA_MIXED: LSBA_ERR_UNSUPPORTED).  A footprint above the budget is
 * LSBA_ERR_OOM (it could never be admitted). */
lsba_status lsba_server_submit(lsba_server* srv, const lsba_operator* op,
                               const lsba_params* params, int32_t s, const double* B,
                               int64_t ldb, int on_device, uint64_t* ticket);

/* Progress engine: advance every slot whose queued work has completed (the
 * upload of B and its norm, a restart cycle, or the end of a request: true
 * residual and download of X into pinned memory) and queue the next step,
 * then admit queued requests; it only queries events and never waits for
 * the GPU.
 * Writes up to cap tickets of requests finished since the last report to
 * done[] and their number to *n_done (the rest are reported by later calls). */
lsba_status lsba_server_poll(lsba_server* srv, uint64_t* done, int32_t cap, int32_t* n_done);

/* Copy a finished request's X (n x s, ld ldx; device memory if on_device) and
 * hand over its result (the caller destroys it with lsba_result_destroy).
 * The ticket is then forgotten.  A request that has not finished:
 * LSBA_ERR_BUSY; an unknown ticket: LSBA_ERR_ARG.  Returns the result's status. */
lsba_status lsba_server_fetch(lsba_server* srv, uint64_t ticket, double* X, int64_t ldx,
                              int on_device, lsba_result** out);

/* Requests running and queued now, footprint bytes of the running ones, and
 * the largest number of requests that ran at once. */
lsba_status lsba_server_stats(const lsba_server* srv, int32_t* active, int32_t* queued,
                              uint64_t* bytes_in_use, int32_t* peak_active);

/* Wait for the device work of every slot and free everything, including
 * requests not yet fetched. */
void lsba_server_destroy(lsba_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* LSBA_H */
