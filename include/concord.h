/*
 * concord.h - C-ABI of the MI355X (gfx950) proximal-gradient solver for the
 * CONCORD / PseudoNet sparse inverse-covariance estimator.
 *
 * The problem (paper Section 2, eq. (1), and Algorithm 1): given data
 * X in R^{n x p} (or its sample covariance S = X^T X / n) and tuning
 * parameters lambda1, lambda2 >= 0, minimise over symmetric Omega
 *
 *   F(Omega) = f(Omega) + lambda1 * sum_{i != j} |omega_ij|,
 *   f(Omega) = -sum_i log omega_ii + 1/2 tr(Omega S Omega)
 *              + lambda2/2 ||Omega||_F^2
 *
 * by proximal gradient with backtracking line search (step sizes
 * tau = 1, 1/2, 1/4, ..., restarted at 1 every iteration).  f is eq. (1)'s
 * smooth part at (2 lambda1, 2 lambda2), halved; with this scaling the
 * gradient G = -(Omega_D)^{-1} + 1/2 (W + W^T) + lambda2 Omega (W = Omega S)
 * of Algorithm 1 is exactly f's gradient.  The soft threshold of eq. (2) is
 * applied to off-diagonal entries only (the l1 term covers Omega_X only).
 *
 * Two forms of the products (Section 3):
 *   CONCORD_COV  (Algorithm 2): S formed once, W = Omega S per iterate;
 *   CONCORD_OBS  (Algorithm 3): Y = Omega X^T per iterate, W = Y X / n.
 *
 * Conventions for every entry point:
 *   - Return value: 0 = OK, > 0 = warning, < 0 = error (codes below).  No C++
 *     exception crosses this boundary.  concord_last_error() describes the
 *     last failure of a handle.
 *   - All array arguments named dev_* or documented as "device" are device
 *     (HBM) pointers of the handle's device.  Host pointers are named host_*.
 *   - Work is ordered on the handle's stream (concord_config.stream).  Calls
 *     that return values to the host synchronise that stream.
 *   - A handle may be used by one host thread at a time.
 *   - The caller owns every buffer it passes; inputs are copied into the
 *     library's own layout before the call returns (in stream order), so the
 *     caller may free them afterwards.  The library owns Omega, its
 *     workspace and all intermediate products; they are freed by
 *     concord_destroy().
 *   - Asynchronous HIP errors surface as CONCORD_EHIP at the next
 *     synchronising call.
 */
#ifndef CONCORD_H
#define CONCORD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define CONCORD_OK            0
#define CONCORD_WMAXITER      1   /* concord_solve: max_iter reached before tol */
#define CONCORD_EINVAL       -1   /* bad argument: lambda < 0, tol <= 0, dims, dtype, shape */
#define CONCORD_ENOMEM       -2   /* device allocation failed (or alloc_fn returned NULL) */
#define CONCORD_EHIP         -3   /* HIP runtime error (message in last_error) */
#define CONCORD_ENOTPD       -4   /* a supplied Omega has a diagonal entry <= 0 */
#define CONCORD_ENONFINITE   -5   /* NaN or Inf in X, S or Omega */
#define CONCORD_ELINESEARCH  -6   /* max_backtracks step sizes all rejected; Omega kept */
#define CONCORD_ENODATA      -7   /* step/solve/objective before concord_set_data */

/* ---- enums ---- */
#define CONCORD_COV 0
#define CONCORD_OBS 1
#define CONCORD_AUTO 2   /* concord_create picks COV or OBS: Lemma 3.1's work priced with rates
                            measured on the device (see concord_suggest_variant); the handle
                            then runs that form (concord_variant_of) */

#define CONCORD_FP64   0   /* products and storage in FP64 */
#define CONCORD_FP32   1   /* products in FP32 (FP32 MFMA / FP32 FMA), FP64 reductions */
#define CONCORD_BF16X3 2   /* dense contractions as BF16 hi/lo split (hi*hi + hi*lo + lo*hi)
                              on BF16 MFMA with FP32 accumulation; sparse products in FP32;
                              FP64 reductions */

#define CONCORD_F64 0
#define CONCORD_F32 1

#define CONCORD_DATA_X 0   /* observations X, n x p */
#define CONCORD_DATA_S 1   /* sample covariance S, p x p symmetric (Cov only) */

#define CONCORD_GRAD_MASKED 0   /* d f / d Omega on the stored entries of Omega only */
#define CONCORD_GRAD_DENSE  1   /* d f / d Omega as a dense p x p array */

typedef struct concord_ctx concord_ctx;

/* Device-memory allocator bridge (e.g. a framework's caching allocator).
   alloc returns `bytes` of device memory of the handle's device usable on
   `stream` (the hipStream_t the handle orders its work on), or NULL on
   failure, which the library reports as CONCORD_ENOMEM.  free returns a block
   obtained from alloc with the same size; the library has synchronised
   `stream` before it frees, so no queued work of its own still uses the block.
   `user` is passed through unchanged.  Both may be called from any host
   thread that calls into the library. */
typedef void* (*concord_alloc_fn)(void* user, size_t bytes, void* stream);
typedef void (*concord_free_fn)(void* user, void* ptr, size_t bytes, void* stream);

typedef struct concord_config {
    int64_t p;              /* number of variables, >= 1 */
    int64_t n;              /* number of observations, >= 1 (ignored when S is supplied) */
    int32_t variant;        /* CONCORD_COV, CONCORD_OBS or CONCORD_AUTO */
    int32_t precision;      /* CONCORD_FP64, CONCORD_FP32 or CONCORD_BF16X3 */
    void*   stream;         /* hipStream_t to order all work on; NULL = null stream */
    int32_t device;         /* HIP device ordinal; -1 = the current device */
    int32_t max_backtracks; /* step-size reductions allowed per iteration (default 60) */
    int32_t trial_batch;    /* step sizes evaluated together per launch, 1..8 (default 8) */
    int32_t use_graph;      /* 1: the handle works on a stream of its own (ordered after
                               `stream` at every call) and replays each iteration's common
                               path (contraction, candidates, first trial batch, accept) as
                               one captured HIP graph; 0 (default): direct launches */
    int32_t no_screen;      /* Cov: 1 = the refresh forms every tile pair of M (the plain
                               product of Algorithm 2); 0 (default) = exact tile screening
                               (see concord_refresh_screen_stats) when p > 448 (smaller
                               problems refresh every pair).  Same results either way. */
    int32_t reserved;       /* set to 0 */
    /* Step sizes of the backtracking search (Algorithm 1: tau = 1, 1/2, 1/4, ...):
       every iteration tries tau0, tau0 * shrink, tau0 * shrink^2, ... (each a
       product formed left to right in FP64), restarting at tau0. */
    double  tau0;           /* > 0, default 1 */
    double  shrink;         /* in (0, 1), default 0.5 */
    /* Device memory for the handle's workspace: both NULL (default) = hipMalloc /
       hipFree; otherwise both must be set.  Every device buffer the handle owns
       (data layout, Omega, candidates, products, partial sums) comes from
       alloc_fn and goes back through free_fn. */
    concord_alloc_fn alloc_fn;
    concord_free_fn  free_fn;
    void*   alloc_user;     /* passed to alloc_fn / free_fn */
} concord_config;

/* Per-iteration record (Algorithm 1, one pass of the outer loop). */
typedef struct concord_step_info {
    int64_t k;            /* iterations completed after this step */
    double  tau;          /* accepted step size */
    int32_t n_trials;     /* step sizes tried, as the sequential search would count (1 = tau 1) */
    int32_t n_batches;    /* trial launches used */
    double  f;            /* smooth value at the new iterate (FP64) */
    double  F;            /* full objective at the new iterate (FP64) */
    int64_t nnz;          /* stored entries of the new iterate (both triangles + diagonal) */
    double  delta_fro;    /* ||Omega^{k+1} - Omega^k||_F */
    int64_t n_candidates; /* |A|: entries the step could make nonzero this iteration */
    double  lhs;          /* difference-form left side of the test at the accepted tau */
    double  rhs;          /* ||Delta||^2 / (2 tau) */
} concord_step_info;

typedef struct concord_solve_info {
    int64_t iters;        /* accepted iterations */
    double  f, F;         /* objective at the returned iterate */
    int64_t nnz;
    int32_t status;       /* same value the call returns */
    int32_t reserved;
} concord_solve_info;

/* Fill *cfg with defaults: variant COV, precision FP64, stream NULL,
   device -1, max_backtracks 60, trial_batch 8, use_graph 0, tau0 1,
   shrink 0.5, no allocator bridge, p = n = 0. */
void concord_config_init(concord_config* cfg);

/* Create a handle for problems of size p (and n).  Allocates the workspace
   for X/S, Omega and the products on cfg->device (through cfg->alloc_fn when
   set).  Omega starts at I (Algorithm 1, first line).  Errors: EINVAL (p < 1,
   n < 1 when needed, unknown variant/precision, trial_batch outside 1..8,
   tau0 <= 0, shrink outside (0, 1), only one of alloc_fn / free_fn set),
   ENOMEM (an allocation failed or alloc_fn returned NULL; everything allocated
   so far has been returned), EHIP. */
int concord_create(const concord_config* cfg, concord_ctx** out);

/* Load the data (device pointer, row-major, leading dimension ld >= cols).
   kind = CONCORD_DATA_X: rows = n, cols = p; copied to the library layout
     X^T (p x n, variable-major) in the handle's precision (plus BF16 hi/lo
     planes for CONCORD_BF16X3).  For Cov, S = X^T X / n is then formed on
     the GPU (Algorithm 2, once).
   kind = CONCORD_DATA_S (Cov only): rows = cols = p; the library stores
     (S + S^T) / 2, rounded once to its precision, so the stored S is exactly
     symmetric (a symmetric S, e.g. one with rounding-level asymmetry from a
     library GEMM, changes by at most one rounding; an exactly symmetric S is
     stored unchanged).  The Cov products rely on that exact symmetry.
   dtype: CONCORD_F64 or CONCORD_F32.  Resets Omega to I and k to 0.
   Errors: EINVAL (shape/dtype/kind mismatch, S with Obs), ENONFINITE
   (NaN/Inf in the input; X is checked while it is copied, so after this
   error for an X the handle holds no data and calls that need data return
   ENODATA until a set_data succeeds; a rejected S leaves the handle as it
   was), EHIP. */
int concord_set_data(concord_ctx* ctx, int32_t kind, const void* dev_data, int32_t dtype,
                     int64_t rows, int64_t cols, int64_t ld);

/* Replace the iterate by a caller-supplied symmetric CSR matrix: the starting
   point Omega^0 of Algorithm 1 (its first line sets Omega^0 = I; any positive-
   diagonal symmetric start is as valid for the method), used for warm starts
   along a lambda path (Section 5) and to resume from a checkpoint.  Device arrays: row_ptr int64[p+1] (row_ptr[0] = 0),
   col int32[nnz] (sorted and unique within each row, both triangles, the
   diagonal present in every row), val[nnz] of dtype.  Symmetry is the
   caller's promise and is not checked.  Sets k to 0.
   Errors: EINVAL (bad row_ptr/col, missing diagonal), ENOTPD (diagonal <= 0),
   ENONFINITE, ENOMEM, EHIP. */
int concord_set_omega(concord_ctx* ctx, int64_t nnz, const int64_t* dev_row_ptr,
                      const int32_t* dev_col, const void* dev_val, int32_t dtype);

/* Omega <- I, k <- 0: the initialisation of Algorithm 1 (its first line) and of
   Algorithms 2 and 3. */
int concord_reset(concord_ctx* ctx);

/* One outer iteration of Algorithm 1 (Algorithm 2 or 3 for the products):
   gradient, then the backtracking search tau = 1, 1/2, ... with the
   sufficient-decrease test, then accept.  Trials whose diagonal is not
   positive are rejected.  The test is evaluated in the exact difference
   form  sum_i [x_i - log1p x_i] + 1/2 tr(D S D) + lambda2/2 ||D||^2
   <= ||D||^2 / (2 tau)  with D = Omega+ - Omega, x_i = D_ii / omega_ii, in
   FP64; it equals the paper's test f(Omega+) <= f(Omega) + <G, D> +
   ||D||^2/(2 tau) identically.  trial_batch step sizes are evaluated per
   launch and the first passing one (in the order 1, 1/2, ...) is taken,
   which is the sequential search's choice.
   info may be NULL.  Errors: EINVAL (lambda < 0), ENODATA, ELINESEARCH
   (Omega and k unchanged), EHIP. */
int concord_step(concord_ctx* ctx, double lambda1, double lambda2, concord_step_info* info);

/* As concord_step, but the step size is forced: tau = tau0 * shrink^(trials-1)
   (2^-(trials-1) with the defaults) is
   accepted without the test (its terms are still reported).  trials >= 1.
   Used to replay a reference run's step sizes.  Errors as concord_step, plus
   ENOTPD if the forced step leaves a diagonal entry <= 0. */
int concord_step_replay(concord_ctx* ctx, double lambda1, double lambda2, int32_t trials,
                        concord_step_info* info);

/* Iterate concord_step until |F_new - F_old| < tol * |F_old| (checked after
   each accepted step) or max_iter steps (Algorithm 1's stopping rule "using
   epsilon", read as a relative change of the full objective).  tol = 0 runs
   exactly max_iter steps.  Returns OK when tol was met, WMAXITER when
   max_iter was reached first (OK when tol = 0), or an error of
   concord_step.  info may be NULL. */
int concord_solve(concord_ctx* ctx, double lambda1, double lambda2, double tol, int64_t max_iter,
                  concord_solve_info* info);

/* Screening statistics of the Cov refresh (this library's exact screening; not part
   of the paper's method, which forms every entry of W = Omega S).  The refresh bounds
   |M_ij| over each pair of 64 x 64 tiles (I, J), I <= J, by
     ( max_i sum_k |omega_ik| smax(k/64, J) + max_j sum_k |omega_jk| smax(k/64, I) ) / 2
   with smax(K, L) the largest |S| of tile (K, L), and skips the pair's S loads when
   the bound (widened by the FMA chains' rounding and 1%) is at most lambda1; the
   skipped pairs' candidate words are provably empty, so results are unchanged.
   This call runs the refresh once at the current iterate for lambda1 and writes the
   number of tile pairs, T (T + 1) / 2 with T = ceil(p / 64), and the number that
   loaded S (diagonal pairs always do; with no_screen set, or p <= 448, every pair
   does).  Host pointers; either may be NULL.
   Errors: EINVAL (null handle, Obs handle, lambda1 < 0), ENODATA, ENOMEM, EHIP. */
int concord_refresh_screen_stats(concord_ctx* ctx, double lambda1, int64_t* host_pairs,
                                 int64_t* host_active);

/* f and F at the current iterate, FP64 (host pointers; either may be NULL).
   f is the smooth value Algorithm 1 evaluates before each search (the
   log-diagonal, trace and Frobenius terms; Algorithm 2 forms the trace from
   W = Omega S, Algorithm 3 from ||Omega X^T||^2 / n), F adds the l1 term of
   eq. (1) over the off-diagonal entries.  Errors: EINVAL, ENODATA, EHIP. */
int concord_objective(concord_ctx* ctx, double lambda1, double lambda2, double* host_f,
                      double* host_F);

/* Copy the current iterate out as CSR (same layout as concord_set_omega): the
   estimate Algorithm 1 returns (its output) after the last accepted step.
   Always writes *host_nnz.  If dev_row_ptr is NULL only the size is
   returned; otherwise dev_row_ptr (p+1), dev_col and dev_val (capacity >=
   *host_nnz as returned by a sizing call) are filled.  dtype: F64 or F32. */
int concord_get_omega(concord_ctx* ctx, int64_t* host_nnz, int64_t* dev_row_ptr,
                      int32_t* dev_col, void* dev_val, int32_t dtype);

/* Candidate set of the last step and the gradient on it (Algorithm 1's
   gradient step and prox argument).  A = supp(Omega^k) U {i != j : |G_ij| >
   lambda1 restricted to where omega_ij = 0} U diag holds every entry the
   step's soft threshold (eq. (2)) could leave nonzero at any step size; for
   each entry the call returns omega^k_ij and G_ij = (W + W^T)_ij / 2 +
   lambda2 omega^k_ij - [i == j] / omega^k_ii at the iterate Omega^k the step
   started from (W = Omega^k S).  Layout: CSR over p rows, row_ptr int64[p+1],
   col int32 (sorted), omega and grad double[nnz]; device arrays.  Always
   writes *host_nnz = |A|; with dev_row_ptr NULL only the size is returned.
   The set belongs to the last successful concord_step / concord_step_replay
   / step of concord_solve on this handle.  Errors: EINVAL, ENODATA (no step
   since the iterate or the data was last set), EHIP. */
int concord_get_candidates(concord_ctx* ctx, int64_t* host_nnz, int64_t* dev_row_ptr,
                           int32_t* dev_col, double* dev_omega, double* dev_grad);

/* Number of completed iterations of the current iterate. */
int64_t concord_iterations(const concord_ctx* ctx);

/* Differentiation form (Obs products).  Smooth value at the current iterate
   with the loaded X:  f = -sum log omega_ii + ||Omega X^T||_F^2 / (2n)
   + lambda2/2 ||Omega||_F^2, in FP64 (host pointer).  Y = Omega X^T is not
   stored.  Requires CONCORD_OBS and X.  Errors: EINVAL, ENODATA, EHIP. */
int concord_smooth_value(concord_ctx* ctx, double lambda2, double* host_f);

/* ---- entry point that allocates nothing ----
   For callers that cannot allocate device memory: code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc.  The value of
   concord_smooth_value, f = -sum_i log omega_ii + ||Omega X^T||_F^2 / (2n) +
   lambda2/2 ||Omega||_F^2, for an iterate and data the caller passes, without a
   handle: the partial sums live in a per-device array of the library of
   CONCORD_NOALLOC_SCRATCH_BYTES (each device the call runs on holds it until the
   process ends).  The call allocates and frees no device memory and does not
   synchronise: f is written to dev_f in stream order.
     p, n: sizes; the problem must fit the array: 8 * (4 + ceil(n / c)) * p bytes
       plus a few KB, c = 256 (F32) or 128 (F64) columns.
     dev_Xt: X^T, p x n row-major, leading dimension ldx >= n (a multiple of 4 for
       F32, of 2 for F64), 16-byte aligned; dtype F32 (FP32 products, the FP32 form)
       or F64.
     dev_row_ptr int64[p+1], dev_col int32[nnz] (sorted per row, diagonal present),
       dev_val double[nnz]: the iterate in CSR, as concord_set_omega takes it (not
       validated here).
     dev_f: one double of device memory.  stream: hipStream_t, NULL = null stream.
   Every call on a device uses that device's one array, which keeps the last call's
   contents: calls that overlap on one device race (order them, e.g. on one stream).
   Errors (decided before any launch): EINVAL (sizes, null pointers, alignment,
   lambda2 < 0 or not finite, problem larger than the array), EHIP. */
#define CONCORD_NOALLOC_SCRATCH_BYTES (32u << 20)
int concord_smooth_value_noalloc(int64_t p, int64_t n, const void* dev_Xt, int64_t ldx,
                                 int32_t dtype, int64_t nnz, const int64_t* dev_row_ptr,
                                 const int32_t* dev_col, const double* dev_val, double lambda2,
                                 double* dev_f, void* stream);

/* Gradients of concord_smooth_value at the current iterate.
   dev_dOmega: mode MASKED -> val-shaped array (nnz of the iterate, CSR
     order, dtype) holding G_ij on the stored entries; mode DENSE -> p x p
     row-major (ld = p) holding G.  G is the gradient over symmetric
     matrices, G = -(Omega_D)^{-1} + 1/2 (Omega S + S Omega) + lambda2 Omega
     (a symmetric perturbation E_ij + E_ji changes f by 2 G_ij).  NULL skips it.
     The iterate must be symmetric in pattern and values (as concord_set_omega
     requires): each unordered pair is computed once and written to both of
     its entries, so in MASKED mode an entry whose mirror is not stored is
     left unwritten.
   dev_dX: n x p row-major (ld = p) receiving d f / d X = (Omega Y)^T / n
     with Y = Omega X^T recomputed here.  NULL skips it.
   dtype: F64 or F32 for both outputs.  Errors: EINVAL, ENODATA, EHIP. */
int concord_gradient(concord_ctx* ctx, double lambda2, int32_t mode, void* dev_dOmega,
                     void* dev_dX, int32_t dtype);

/* ---- batched lambda path (Section 5 solves a grid of lambda values; Section S.3.1) ----
   Many independent Cov problems (Algorithm 2), each solved at every lambda1 of a path
   from Omega = I with the stopping rule of concord_solve, all at once on one device:
   every phase of an iteration (candidates, trials and decision, emission, the refresh
   of W = Omega S and the objective, the stopping test) is one launch over all solves
   still running, with the control state of every solve (iteration, step-size index,
   phase, objective) in device memory and no host decision between phases.  Up to
   iters_per_launch iterations are captured as one HIP graph and replayed until every
   solve has stopped; the host reads two counters per replay.  The refresh is
   lambda-stacked: each tile pair any solve of an instance keeps is processed once for
   all of that instance's lambda1 values, which read the same S tiles.
   Each solve's iterates are bitwise those of the single solver (concord_solve on a Cov
   handle of the same precision, trial batch, tau0, shrink and max_backtracks).
   S = X_b^T X_b / n_b is formed for every instance (MFMA, the autotuned contraction of
   its shape) by the first concord_batch_solve and kept for later calls. */
typedef struct concord_batch concord_batch;
typedef struct concord_batch_config {
    int32_t precision;        /* CONCORD_FP32 (default), CONCORD_FP64 or CONCORD_BF16X3 products
                                 (as concord_config.precision in the Cov form) */
    int32_t device;           /* -1 = the current device */
    void*   stream;           /* hipStream_t; NULL = null stream */
    int32_t max_backtracks;   /* 60 */
    int32_t trial_batch;      /* 1..8, default 8 */
    double  tau0, shrink;     /* 1, 0.5 (as concord_config) */
    int32_t iters_per_launch; /* iterations per graph replay, 1..64 (default 4) */
    int32_t use_graph;        /* 1 (default): replay captured iterations; 0: direct launches */
    concord_alloc_fn alloc_fn;   /* device memory bridge, as in concord_config */
    concord_free_fn  free_fn;
    void*   alloc_user;
} concord_batch_config;
void concord_batch_config_init(concord_batch_config* cfg);

/* count instances; instance b has p_b variables and data X_b (device, n_b x p_b
   row-major with leading dimension ld_b, FP32 for the FP32 form, FP64 for FP64),
   borrowed until the first concord_batch_solve has formed its S.  Every instance is
   solved at every lambda1 in host_lambda1[0 .. n_l1 - 1].  cfg may be NULL (defaults).
   Errors: EINVAL (count or n_l1 < 1, p, n < 1, ld < p, null data, lambda1 < 0, bad
   config), ENOMEM, EHIP. */
int concord_batch_create(const concord_batch_config* cfg, int32_t count, const int64_t* host_p,
                         const int64_t* host_n, const void* const* host_dev_X,
                         const int64_t* host_ld, int32_t n_l1, const double* host_lambda1,
                         concord_batch** out);
/* Solve every (instance, lambda1) with lambda2, tol and max_iter (concord_solve's rule),
   each from Omega = I.  Per solve s = b * n_l1 + l (host arrays of count * n_l1, any
   may be NULL): accepted iterations, F at the estimate, and the solve's status
   (CONCORD_OK, CONCORD_WMAXITER or CONCORD_ELINESEARCH).  Returns the largest warning,
   or the first error.  Errors: EINVAL, ENOMEM, EHIP. */
int concord_batch_solve(concord_batch* b, double lambda2, double tol, int64_t max_iter,
                        int64_t* host_iters, double* host_F, int32_t* host_status);
/* The estimate of (instance, l1_index) as CSR (layout of concord_get_omega, values
   double); with dev_row_ptr NULL only *host_nnz is written. */
int concord_batch_get_omega(concord_batch* b, int32_t instance, int32_t l1_index,
                            int64_t* host_nnz, int64_t* dev_row_ptr, int32_t* dev_col,
                            double* dev_val);
/* Counters of the last concord_batch_solve: graph replays (or direct iteration
   groups), host synchronisations, iterations launched (the longest solve's count plus
   the replays' idle tail), milliseconds forming S and iterating. */
typedef struct concord_batch_stats {
    int64_t launches, host_syncs, iterations_launched, regrows;
    double  s_ms, iterate_ms;
} concord_batch_stats;
int concord_batch_stats_get(const concord_batch* b, concord_batch_stats* out);
const char* concord_batch_last_error(const concord_batch* b);
void concord_batch_destroy(concord_batch* b);

/* Per-kernel-class timing (HIP events recorded on the handle's stream around
   each launch group; read at the synchronisation points the solver already
   has).  Classes: */
#define CONCORD_PROF_DENSE 0   /* MFMA SYR2K (Obs gradient) / SYRK (Cov, once) */
#define CONCORD_PROF_SPMM  1   /* product refresh at the accepted iterate + objective sums */
#define CONCORD_PROF_CAND  2   /* gradient + candidate set */
#define CONCORD_PROF_TRIAL 3   /* step-size trials + test sums + decision */
#define CONCORD_PROF_EMIT  4   /* CSR emission of the accepted iterate */
#define CONCORD_PROF_REFRESH 5 /* Cov: the refresh kernel alone (the tile pairs kept by the
                                  screening) at the accepted iterate; its screening and the
                                  objective sums stay in CONCORD_PROF_SPMM, which then times
                                  two intervals per refresh */
#define CONCORD_PROF_NCLASS 6
typedef struct concord_profile {
    double  ms[8];        /* accumulated milliseconds per class */
    int64_t launches[8];  /* timed launch groups per class */
} concord_profile;
/* on != 0 starts timing and clears the counters; on = 0 stops it. */
int concord_set_profiling(concord_ctx* ctx, int32_t on);
int concord_get_profile(const concord_ctx* ctx, concord_profile* host_out);
/* Tile variant the library's autotuner picked for this handle's dense contraction
   (Obs: the gradient SYR2K of Algorithm 3; Cov: the S = X^T X / n SYRK of
   Algorithm 2).  The first contraction of a shape times every variant of the
   precision form and keeps the fastest for the rest of the process (all variants
   give bitwise the same result).  Writes the variant's name, NUL-terminated and
   truncated to host_cap bytes, into host_name (may be null) and returns its index,
   -1 if the shape has not been tuned yet (or the form has a single variant and was
   never tuned), or CONCORD_EINVAL for a null handle. */
int concord_contraction_variant(const concord_ctx* ctx, char* host_name, int32_t host_cap);

/* ---- choice of the product form (Section 3, Lemma 3.1; Section S.1; Section 4) ----
   Lemma 3.1 counts F_Cov = 2np^2 + 2dp^2(st+1) and F_Obs = 2np^2 s + 2dnp(st+1)
   flops for s iterations with t step sizes tried per iteration and d nonzeros
   per row of Omega on average; paper_choice is the form with fewer flops.
   Section 4 notes that the two terms run at very different rates (sparse-dense
   products far slower per flop than dense ones), so choice prices the work this
   library does, with dense_tflops the useful rate of its dense contraction and
   hbm_gbps its memory rate:
     Cov: S once (symmetric: n p^2 flops) + per iteration the refresh of
          W = Omega S, which reads the S tiles of the kept tile pairs
          (screen_fraction of them; 1 = no screening, an upper bound) and writes
          and reads the candidate threshold words (p^2 / 4 bytes);
     Obs: per iteration the symmetric rank-2n contraction (2 n p^2 flops) and the
          write and read of its dense result (2 p^2 elements) and of Y (2 p n).
   dense_tflops / hbm_gbps <= 0 select built-in MI355X figures for `precision`
   (BF16 split 330, FP32 125, FP64 60 TFLOP/s useful; 3200 GB/s); screen_fraction
   <= 0 selects 1.  Host-only: no GPU is touched.
   Errors: EINVAL (p, n < 1; d, t, s < 0; precision). */
typedef struct concord_variant_estimate {
    int32_t paper_choice;   /* CONCORD_COV or CONCORD_OBS by flop count */
    int32_t choice;         /* CONCORD_COV or CONCORD_OBS by modelled time */
    double  cov_flops, obs_flops;
    double  cov_seconds, obs_seconds;
} concord_variant_estimate;
int concord_suggest_variant(int64_t p, int64_t n, double d, double t, double s, int32_t precision,
                            double dense_tflops, double hbm_gbps, double screen_fraction,
                            concord_variant_estimate* out);

/* Rates of this library measured on `device` (-1: current) for `precision`, once per
   process and cached: the useful FP rate of the dense symmetric contraction on a
   p = 4096, K = 2048 problem (its autotuned tile variant) and the device-to-device
   copy rate of 256 MiB (bytes read + written per second).  CONCORD_AUTO prices
   concord_suggest_variant with them (d = 5, t = 3, s = 30, screen_fraction 1).
   Output pointers may be NULL.  Errors: EINVAL (precision), ENOMEM, EHIP. */
int concord_measure_rates(int32_t device, int32_t precision, double* host_dense_tflops,
                          double* host_hbm_gbps);

/* The product form a handle runs (CONCORD_COV or CONCORD_OBS; for a CONCORD_AUTO
   handle, the one concord_create picked), or CONCORD_EINVAL for a null handle. */
int32_t concord_variant_of(const concord_ctx* ctx);

/* Description of the last error on this handle ("" if none). Never NULL. */
const char* concord_last_error(const concord_ctx* ctx);

/* Free the handle and everything it owns.  NULL is accepted. */
void concord_destroy(concord_ctx* ctx);

/* Library version string. */
const char* concord_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CONCORD_H */
