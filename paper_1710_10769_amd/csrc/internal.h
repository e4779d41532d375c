// Internal declarations shared by the HIP translation units of libconcord.
// Nothing here is part of the C-ABI (include/concord.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace concord {

// Dense element storage forms.
enum Store : int {
    ST_F64 = 0,   // double
    ST_F32 = 1,   // float
    ST_B16P = 2,  // packed pair (bf16 hi | bf16 lo << 16); value = hi + lo
};

// Operand planes of the MFMA symmetric contraction.
enum GemmKind : int {
    GK_F64 = 0,    // FP64 MFMA 16x16x4
    GK_F32 = 1,    // FP32 MFMA 32x32x2
    GK_BF16X3 = 2, // BF16 MFMA 32x32x16, hi*hi + hi*lo + lo*hi
};

constexpr int ROW_PAD = 256;   // dense operands are allocated with rows padded to this
constexpr int K_PAD = 64;      // and their K (column) dimension padded to this

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// BF16 hi/lo operand planes are K-blocked: blocks of KBLK elements (32 bytes) of K,
// and within a block all rows back to back, so element (row, k) sits at
//   (k / KBLK) * kblk_stride(prow) + row * KBLK + k % KBLK
// with prow = round_up(rows, ROW_PAD).  One K stage of a 256-row tile is then one
// contiguous 8 KB run per plane, and the contraction's loads use whole cache lines.
constexpr int KBLK = 16;
__host__ __device__ inline int64_t kblk_stride(int64_t prow) { return prow * KBLK; }
__host__ __device__ inline int64_t kblk_index(int64_t row, int64_t k, int64_t stride) {
    return (k / KBLK) * stride + row * KBLK + k % KBLK;
}

// ---- launchers (all asynchronous on `stream`) ----

// C = alpha * (P Q^T + Q P^T)  (syr2k)  or  alpha * P P^T  (syrk, Q ignored),
// over the upper-triangle tiles only, written symmetrically (both triangles,
// bitwise symmetric).  P and Q hold prow x ldk operands (prow = round_up(p,
// ROW_PAD), zero rows beyond p; ldk a multiple of K_PAD, zero columns beyond the
// true K).  For GK_BF16X3, P0/P1 and Q0/Q1 are the hi/lo planes (uint16 bf16 bits)
// in the K-blocked layout above; otherwise P0/Q0 are row-major float (GK_F32) or
// double (GK_F64) with row stride ldk.
// out_store: ST_F32, ST_F64 or ST_B16P.
// Optional second output of the contraction: threshold words of the next candidate
// set (p x nwords uint64, nwords = ceil(p/64)); bit j of word w of row i is set iff
// i == j or |C_ij| > lam1 for the stored value.  bits == nullptr: not requested.
// Only the direct-to-LDS BF16-split variants write it; *wrote (host, optional) tells
// whether the variant that ran did (else the caller runs the full candidate pass).  A
// variant that writes the words stores C's upper triangle only (i <= j; the lower one is
// not written): the candidate pass then reads C_ij as C[min(i,j)][max(i,j)].
struct ThreshOut {
    double lam1 = 0.0;
    uint64_t* bits = nullptr;
    int64_t nwords = 0;
    int* wrote = nullptr;
};
hipError_t launch_gemm_sym(int kind, bool syr2k, const void* P0, const void* P1,
                           const void* Q0, const void* Q1, int64_t ldk, int64_t p,
                           double alpha, void* C, int out_store, int64_t ldc,
                           hipStream_t stream, ThreshOut th = ThreshOut());

// Tuned variant index for a shape (-1 if not tuned yet) and its name.
int gemm_sym_choice(int kind, bool syr2k, int64_t p, int64_t ldk, const char** name);

// X (rows x cols, ld, F64 or F32) -> Xt (cols x ldo) in `store` (F64/F32);
// optionally bf16 hi/lo planes (hi, lo may be null), K-blocked with block stride
// kbs elements.  Sets *flag (int) to 1 if any entry of X is NaN/Inf (the
// transposed data is written regardless).
hipError_t launch_transpose_in(const void* X, int x_is_f64, int64_t rows, int64_t cols,
                               int64_t ld, void* Xt, int store, int64_t ldo, uint16_t* hi,
                               uint16_t* lo, int64_t kbs, int* flag, hipStream_t stream);

// (S + S^T) / 2 of a square p x p (ld) F64/F32 matrix into `store` layout with ldo,
// exactly symmetric in the stored type (a symmetric S is copied unchanged).
hipError_t launch_sym_copy(const void* S, int s_is_f64, int64_t p, int64_t ld, void* out,
                           int store, int64_t ldo, hipStream_t stream);

// Non-finite detector: sets *flag (int) to 1 if any of the rows x cols (ld)
// entries is NaN/Inf.
hipError_t launch_check_finite(const void* A, int is_f64, int64_t rows, int64_t cols,
                               int64_t ld, int* flag, hipStream_t stream);

// ---- sparse side ----

struct Csr {
    int64_t* rowptr;  // p+1
    int32_t* col;     // cap
    double* val;      // cap
};

// Y = Omega B (B: K x N dense, ldb, store), rows < p written to C (ldc) in
// `cstore` (F64/F32) unless C is null; hi/lo planes written if non-null, K-blocked
// with block stride kbs elements.
// sq_part (if non-null) receives sum_j Y_ij^2 per (row, column-chunk) in FP64
// as sq_part[chunk * p + row]; nchunks returned through *nchunks_out.
// `gate` (device int, may be null): kernel does nothing unless *gate != 0.
hipError_t launch_spmm(const Csr& A, int64_t p, const void* B, int bstore, int64_t ldb,
                       int64_t ncols, void* C, int cstore, int64_t ldc, uint16_t* hi,
                       uint16_t* lo, int64_t kbs, double* sq_part, const int* gate,
                       hipStream_t stream);
int spmm_nchunks(int bstore, int64_t ncols);

// Candidate set of one iteration.
struct Cand {
    int64_t* rowptr;  // p+1
    int32_t* col;     // cap
    double* omega;    // cap: current omega_ij (0 off the support)
    double* grad;     // cap: G_ij
};

// Candidate bitmap and counts from threshold words written by launch_cov_refresh for
// the same iterate and lambda1: ORs supp(Omega_i) into row i's words (in place) and
// writes cnt[i] = |A_i|; the result equals launch_cand_count's.
// With tmask (the kept-tile bits of a screened Cov refresh, T x ceil(T/64) uint64) only
// the words of kept tiles and the support's words are read; words outside both are stale
// and never read.
hipError_t launch_cand_merge(const Csr& om, int64_t p, uint64_t* bitmap, int64_t nwords,
                             int64_t* cnt, hipStream_t stream, const uint64_t* tmask = nullptr);

// Count pass: for every row, A_i = {j != i : |M_ij| > lam1} U supp(Omega_i) U {i}.
// Writes the candidate bitmap (p x nwords64 uint64, row-major, word w bit b
// covers column 64*w+b) and cnt[i] = |A_i|.
hipError_t launch_cand_count(const void* M, int mstore, int64_t ldm, const Csr& om, int64_t p,
                             double lam1, uint64_t* bitmap, int64_t nwords, int64_t* cnt,
                             hipStream_t stream);
// Fill pass: writes A (sorted columns) with omega and G = M + lam2*omega - [i==j]/omega_ii.
// With M null (Cov form) it writes the columns and omega only; launch_cand_grad_cov then
// writes G.  m_upper: only M's upper triangle is stored (M_ij read at [min][max]).
hipError_t launch_cand_fill(const void* M, int mstore, int64_t ldm, const Csr& om, int64_t p,
                            double lam2, const uint64_t* bitmap, int64_t nwords,
                            const Cand& A, int64_t cap, const int* overflow,
                            hipStream_t stream, const uint64_t* tmask = nullptr,
                            bool m_upper = false);

// Cov form: G on the candidates of A (filled for the same iterate), with M_ij gathered
// from S and the CSR rows i and j of Omega; bitwise the value the Cov refresh tests.
hipError_t launch_cand_grad_cov(const Csr& om, int64_t p, const void* S, int sstore, int64_t lds,
                                double lam2, const Cand& A, const int* overflow,
                                hipStream_t stream);

constexpr int SCAN_CHUNK = 2048;   // entries per scan chunk (8 per thread of a 256-thread block)

// Exclusive scan of cnt[0..p) into out[0..p] (out[p] = total); sets
// *overflow = 1 if total > cap (overflow may be null), and copies the total to
// *total_out (may be null).  Two launches (chunk sums into
// ws, scan_ws_len(p) int64, then per-chunk scans); integer, so deterministic.
hipError_t launch_scan(const int64_t* cnt, int64_t p, int64_t* out, int64_t cap, int* overflow,
                       int64_t* ws, hipStream_t stream, int64_t* total_out = nullptr);
// int64 workspace length launch_scan needs for p rows.
int64_t scan_ws_len(int64_t p);

struct DevState;
// Cov trials of problems with at least this many rows run 8 lanes per row (8 rows per
// wave); smaller ones a wave per row.  The batched solver makes the same choice per solve.
constexpr int64_t COV_TRIAL_GROUP_MIN_P = 1024;
// Column splits of the Obs quadratic term in launch_trial (1 for Cov).
int trial_splits(int variant, int bstore, int64_t ncols);
// Trial evaluation for `m` step sizes tau_q = tau0 * shrink^q (q < m) at once (tau_q
// formed by q successive multiplications).
// Per row partials part[((q*4 + t) * S + s) * p + row] for column split s < S =
// trial_splits(...), t = 0: sum x - log1p x over the
// diagonal, 1: ||Delta_i||^2, 2: quadratic term of row i, 3: 1 if the
// diagonal entry is <= 0.  Obs quadratic: ||Delta_i X^T||^2 (B = Xt, ncols = n); a row
// with a single candidate (i, j) takes it as delta^2 xn2[j] when xn2 (the squared row norms
// of X^T, launch_row_norm2) is given.  Cov quadratic: sum_{j,k in A_i} Delta_ij S_jk
// Delta_ik (B = S).
hipError_t launch_trial(const Cand& A, int64_t p, double tau0, double shrink, int m, double lam1,
                        int variant, const void* B, int bstore, int64_t ldb, int64_t ncols,
                        const double* xn2, double* part, const struct DevState* st,
                        hipStream_t stream);
// out[j] = sum_c B[j * ldb + c]^2 over c < ncols, in FP64 (B FP64 or FP32, row-major,
// ldb and ncols multiples of 4).
hipError_t launch_row_norm2(const void* B, int bstore, int64_t ldb, int64_t ncols, int64_t p,
                            double* out, hipStream_t stream);

// Deterministic FP64 column sums in[c * rows + r] -> out[c], c < ncol, and in the same
// launch the step that uses them.  ws holds at least ncol * COLSUM_MAXSEG doubles
// (segment sums); st->ticket must be 0 (it is 0 again when the launch completes).
constexpr int COLSUM_MAXSEG = 256;
// Trial sums (ncol = 4m, out[q*4 + t]), then the decision: the first passing q (or the
// forced one) is written to the state.
hipError_t launch_colsum_decide(const double* in, int64_t rows, int ncol, double* out,
                                double* ws, int m, double tau0, double shrink, int q_base,
                                double lam2, double inv_n, int forced_q, DevState* st,
                                hipStream_t stream);
// Objective sums (ncol = 4 + nysq), then, when gated on, copied into st->obj.
hipError_t launch_colsum_obj(const double* in, int64_t rows, int ncol, double* out, double* ws,
                             int nysq, const int* gate, DevState* st, hipStream_t stream);

// Emission: new CSR from A at the chosen step (state->accepted_q).
// grouped: 8 lanes per row (Cov problems of at least COV_TRIAL_GROUP_MIN_P rows; same
// results as a wave per row).
hipError_t launch_emit_count(const Cand& A, int64_t p, double lam1, const DevState* st,
                             int64_t* cnt, hipStream_t stream, bool grouped = false);
hipError_t launch_emit_fill(const Cand& A, int64_t p, double lam1, const DevState* st,
                            const Csr& out, hipStream_t stream, bool grouped = false);

// Objective partials of a CSR iterate.  part[t * p + row]: t = 0 sum of log
// of the diagonal, 1 sum of squares, 2 off-diagonal sum of |v|, 3 sum of
// W_ij * omega_ij over the stored entries (only if W non-null).
hipError_t launch_obj_parts(const Csr& om, int64_t p, const void* W, int wstore, int64_t ldw,
                            double* part, const int* gate, hipStream_t stream);
// Cov form: the same partials, t = 3 as sum_j M_ij omega_ij with M gathered from S on
// the support of Omega (no dense M).
hipError_t launch_obj_parts_cov(const Csr& om, int64_t p, const void* S, int sstore, int64_t lds,
                                double* part, const int* gate, hipStream_t stream);

// f = -obj[0] + 1/2 obj[4] / n + lam2/2 obj[1] from the objective sums in st->obj (the
// smooth value of the differentiation form), written to *f (device) in stream order.
hipError_t launch_smooth_finish(const DevState* st, int64_t n, double lam2, double* f,
                                hipStream_t stream);

// Identity CSR (omega = I) into `om`.
hipError_t launch_identity(const Csr& om, int64_t p, hipStream_t stream);

// Cov refresh: forms M = (W + W^T) / 2 with W = Omega S (S: p x p, row stride
// lds >= 64 * nwords, `sstore`; M in FP64 for an FP64 S, FP32 otherwise) tile pair by
// tile pair over the upper triangle and writes the threshold words
// {j : j == i or |M_ij| > lam1} of every row into tbits (p x nwords, nwords =
// ceil(p/64); see launch_cand_merge).  M is not stored.  smax (T x T, T = nwords) holds
// the largest |S| of each 64 x 64 tile (launch_tile_max); pairs whose bound on |M|
// stays at or below lam1 skip their S loads.  Gated like launch_spmm.  If `active` is
// non-null, every pair that loads S adds one to it (a diagnostic: one atomic per pair).
// Workspace (see refresh_ws_sizes): per row tile the screened column-tile list, and the
// list of kept pairs with its count.
struct RefreshWs {
    int* lcnt;      // T
    int* lK;        // T * 64
    double* lW;     // T * 64
    int* lcmax;     // T
    int* plist;     // T (T + 1) / 2
    int* pcount;    // 1
    uint64_t* tmask;  // T * ceil(T / 64): bit (I, J) = tile pair {I, J} kept
};
hipError_t launch_cov_refresh(const Csr& A, int64_t p, const void* S, int sstore, int64_t lds,
                              const double* smax, double lam1, uint64_t* tbits, int64_t nwords,
                              const RefreshWs& ws, const int* gate, hipStream_t stream,
                              unsigned long long* active = nullptr, bool screen = true);
// The two halves of launch_cov_refresh: the screening (row-tile lists, the list of kept
// pairs, the words zeroed) and the refresh of the kept pairs (smax null: no screening in
// the refresh either).  screen = false keeps every pair (the unscreened product).
hipError_t launch_cov_screen(const Csr& A, int64_t p, int sstore, const double* smax,
                             double lam1, uint64_t* tbits, int64_t nwords, const RefreshWs& ws,
                             const int* gate, hipStream_t stream, bool screen = true);
hipError_t launch_cov_refresh_pairs(const Csr& A, int64_t p, const void* S, int sstore,
                                    int64_t lds, const double* smax, double lam1,
                                    uint64_t* tbits, int64_t nwords, const RefreshWs& ws,
                                    const int* gate, hipStream_t stream,
                                    unsigned long long* active = nullptr);
// smax[I * T + J] = max |S| over tile (I, J), T = ceil(p / 64), as the refresh reads S.
hipError_t launch_tile_max(const void* S, int sstore, int64_t p, int64_t lds, double* out,
                           hipStream_t stream);

// Differentiation form.
// Masked gradient on the stored entries and Omega Y (d f / d X^T times n) in one row
// pass (Y = Omega X^T, p x ld rows): d_ij = <Y_j, Xt_i> goes to D at entry (i, j), per
// column block cb at offset cb * nnz (grad_col_blocks(store, n) blocks; D holds that many
// times nnz doubles); oy (p x ld, may be null) receives Omega Y.  launch_grad_combine
// then finds d_ji at the mirror entry and writes G_ij = (d_ij + d_ji) / (2n) + lam2 w_ij -
// [i == j] / w_ii to out (nnz, FP64 or FP32).  The pattern must be symmetric (an entry
// whose mirror is not stored gets an unspecified value).
int grad_col_blocks(int store, int64_t n);
hipError_t launch_grad_rows(const Csr& om, int64_t p, int64_t nnz, const void* Y, const void* Xt,
                            int store, int64_t ld, int64_t n, double* D, void* oy,
                            hipStream_t stream);
hipError_t launch_grad_combine(const Csr& om, int64_t p, int64_t nnz, int ncb, const double* D,
                               int64_t n, double lam2, void* out, int out_f64,
                               hipStream_t stream);
hipError_t launch_gather_dense_grad(const void* M, int mstore, int64_t ldm, const Csr& om,
                                    int64_t p, double lam2, void* out, int out_f64,
                                    hipStream_t stream);
hipError_t launch_transpose_out(const void* Yt, int store, int64_t p, int64_t n, int64_t ld,
                                double scale, void* out, int out_f64, hipStream_t stream);
hipError_t launch_csr_validate(const int64_t* rowptr, const int32_t* col, const void* val,
                               int val_f64, int64_t p, int64_t nnz, int* flags,
                               hipStream_t stream);
hipError_t launch_csr_import(const int32_t* col, const void* val, int val_f64, int64_t nnz,
                             int32_t* col_out, double* val_out, hipStream_t stream);
hipError_t launch_csr_export(const double* val, int64_t nnz, void* out, int out_f64,
                             hipStream_t stream);

// Smooth value f and full objective F from the objective sums o[] of an iterate
// (o[0] sum of log omega_ii, o[1] sum of squares, o[2] off-diagonal sum of |omega_ij|,
// o[3] sum M o Omega (Cov), o[4] ||Y||^2 (Obs)):
//   f = -o[0] + 1/2 quad + lam2/2 o[1],  quad = o[4] / n (Obs) or o[3] (Cov),
//   F = f + lam1 o[2].
// One definition for host and device code, without contraction into FMAs, so the
// batched solves' stopping tests see bitwise the values the single solver computes.
__host__ __device__ inline void objective_value(const double* o, bool obs, double dn,
                                                double lam1, double lam2, double* f,
                                                double* F) {
#pragma clang fp contract(off)
    const double quad = obs ? o[4] / dn : o[3];
    const double fv = -o[0] + 0.5 * quad + 0.5 * lam2 * o[1];
    *f = fv;
    *F = fv + lam1 * o[2];
}

// Device-side solver state (one per handle, in device memory).
struct DevState {
    double f, F;            // at the current iterate
    double sums[16 * 4];    // per-q trial sums of the last batch
    double tau;             // accepted step size
    double lhs, rhs, dd;    // test terms at the accepted step
    double obj[5];          // objective sums at the last evaluated iterate:
                            // log-diagonal, sum of squares, off-diagonal |.|,
                            // sum W o Omega (Cov), ||Y||^2 (Obs)
    int64_t n_cand;         // |A| of the last candidate pass (its scan's total)
    int64_t nnz_next;       // stored entries of the emitted iterate (its scan's total)
    int accepted_q;         // -1: none passed yet in this iteration
    int accepted;           // 1 once a step is accepted (gate of the accept kernels)
    int nonpos;             // forced step leaves the domain
    int overflow;           // candidate capacity exceeded
    unsigned ticket;        // blocks finished in the running column-sum launch (0 between)
    double fval;            // smooth value written by launch_smooth_finish
};

// ---- batched solves (many Cov problems and lambda1 values in one set of launches) ----
//
// One SolveDesc per (instance, lambda1) solve, in device memory; the solves of one
// instance share its S.  Every phase kernel walks work items (solve, local block) of the
// solves that still run, from tables a plan kernel builds at the start of each iteration,
// with a fixed grid whose blocks loop over the items (no host decision between phases).
struct SolveCtl {
    int cur;            // CSR buffer holding the iterate
    int phase;          // BPH_* below
    int q_base;         // first step-size index of the next trial batch
    int status;         // CONCORD_OK, CONCORD_WMAXITER, CONCORD_ELINESEARCH (when done)
    int grow;           // 1: the candidate capacity was exceeded; the host regrows
    int pad_;
    int64_t k;          // accepted iterations
    double F;           // full objective at the iterate
};
enum { BPH_CAND = 0, BPH_TRIAL = 1, BPH_DONE = 2 };

struct SolveDesc {
    int64_t p, nwords;
    int T, inst, screen, grouped;   // tile rows; instance; exact screening; 8 lanes per trial row
    const void* S;
    int64_t lds;
    const double* smax;
    Csr om[2];
    Cand A;
    int64_t a_cap;
    int64_t* cnt;
    uint64_t* bitmap;
    double* part;       // 4 * MAXQ * p trial partials, then 4 * p objective partials
    double* tsums;      // 64
    double* osums;      // 64
    double* colws;      // 4 * MAXQ * COLSUM_MAXSEG
    int64_t* scanws;    // scan_ws_len(p)
    RefreshWs rws;
    DevState* st;
    SolveCtl* ctl;
    double lam1;
};

// Per-instance lists of the tile pairs any of its solves keeps in a refresh (the
// lambda-stacked refresh walks each listed pair once for all of them).
struct InstDesc {
    int T, nsolve, first;   // tile rows, solves of the instance (consecutive from `first`)
    int screen;
    int* ulist;             // T (T + 1) / 2 pair indices
    int* ucount;            // 1
    uint32_t* ubits;        // ceil(T (T + 1) / 2 / 32): pair already listed
};

// Work tables of one iteration.  off[ph][a] = first item of active solve act[a] in phase
// ph (a = 0 .. nact), for the static phases; roff[i] the same for the refresh over the
// instances.  status[0] = solves still running, status[1] = solves asking for more
// candidate capacity.
// Row phases: BP_ROW every solve's rows (WPB per item), BP_ROWU the same for the solves
// whose per-row kernels run a wave per row, BP_ROWG 8 lanes per row (WPB * 8 rows per item)
// for the others, so a phase of one form walks no items of the other.
enum { BP_ROW = 0, BP_ROWU, BP_ROWG, BP_SCAN, BP_COLT, BP_COLO, BP_SROWS, BP_SPAIRS, BP_SOLVE, BP_N };
struct BatchPlan {
    int nact;
    int* act;      // nsolve
    int* off;      // BP_N * (nsolve + 1)
    int* roff;     // ninst + 1
    int* status;   // 2
};

struct BatchArgs {
    int nsolve, ninst, maxT;   // maxT: largest tile-row count (dynamic LDS of two phases)
    // which launches can have work at all (fixed at batch creation): solves with a wave per
    // trial row, solves with 8 lanes per row, screened solves, solves of more than one
    // scan chunk; an iteration leaves out the launches of a form no solve uses
    int any_rowu, any_rowg, any_screen, any_multichunk;
    int bstore;            // S storage (ST_F64 or ST_F32)
    int tb, total;         // step sizes per trial batch, max_backtracks + 1
    int64_t max_iter;
    double lam2, tol, tau0, shrink;
};

// Iteration of every running solve (the plan, candidates, trials and decision, emission,
// the stacked refresh and objective of the accepted iterates, the stopping test), as
// kernel launches on `stream` that read all control state from the device (graph
// capturable).  init = true instead evaluates the products, threshold words and
// objective of every solve's current iterate (the start, Omega = I).
hipError_t launch_batch_iteration(const SolveDesc* sd, const InstDesc* idesc, const BatchPlan& pl,
                                  const BatchArgs& a, bool init, int grid, hipStream_t stream);

}  // namespace concord
