// Host driver and C-ABI of libconcord (see include/concord.h).
//
// One outer iteration (Algorithm 1; products per Algorithm 2 or 3):
//   [Obs]  M = (Y X + (Y X)^T) / (2n)          gemm_sym, syr2k, MFMA
//   [Cov]  M = (W + W^T) / 2, W = Omega S      (already formed at accept)
//   A      = candidates of the prox step       cand_count + scan + cand_fill
//   trials tau0 * 2^-q, q < trial_batch         trial + colsum + decide
//   accept Omega+ (CSR emission), products and objective at Omega+ (gated on
//          the device-side decision), one host synchronisation per batch.
//
// The backtracking line search restarts at tau = 1 every iteration.  A batch
// evaluates several step sizes of the sequence 1, 1/2, 1/4, ... in one pass
// and accepts the first passing one, which is exactly the step the sequential
// search of Algorithm 1 would accept.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/concord.h"
#include "internal.h"

using namespace concord;

namespace {

constexpr int MAXQ = 8;

__global__ void state_reset_kernel(DevState* st) {
    if (threadIdx.x == 0) {
        st->accepted_q = -1;
        st->accepted = 0;
        st->nonpos = 0;
        st->overflow = 0;
    }
}

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) *p = v;
}

__global__ void set_int_kernel(int* p, int v) {
    if (threadIdx.x == 0) *p = v;
}

}  // namespace

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Device memory of a handle: the caller's allocator bridge when one is configured,
// else hipMalloc / hipFree.
struct DevAlloc {
    concord_alloc_fn afn = nullptr;
    concord_free_fn ffn = nullptr;
    void* user = nullptr;
};

struct concord_ctx {
    int64_t p = 0, n = 0;
    int variant = CONCORD_COV, precision = CONCORD_FP64;
    hipStream_t stream = nullptr;
    int device = 0;
    int max_bt = 60, tb = 8;
    double tau0 = 1.0, shrink = 0.5;   // step sizes tau0 * shrink^q
    DevAlloc alloc;
    std::string err;

    int64_t prow = 0, ldk = 0, ldp = 0;
    int dstore = ST_F64;   // Xt / Y / M element storage
    int sstore = ST_F64;   // S storage (Cov)
    int gkind = GK_F64;

    bool has_data = false;

    void* Xt = nullptr;
    uint16_t* Xt_hi = nullptr;
    uint16_t* Xt_lo = nullptr;
    void* Y = nullptr;
    uint16_t* Y_hi = nullptr;
    uint16_t* Y_lo = nullptr;
    void* S = nullptr;
    double* smax = nullptr;   // Cov: largest |S| of each 64 x 64 tile (T x T)
    unsigned long long* d_active = nullptr;   // screening statistics counter
    RefreshWs rws = {};                         // Cov refresh screening workspace
    void* M = nullptr;
    double* xn2 = nullptr;     // Obs: squared row norms of Xt (FP64), for one-candidate trial rows
    bool xn2_valid = false;

    Csr om[2] = {};
    int64_t om_cap[2] = {0, 0};
    int cur = 0;
    int64_t nnz = 0;
    int64_t k = 0;

    Cand A = {};
    int64_t a_cap = 0;
    int64_t a_nnz = -1;          // |A| of the last accepted step (-1: none since the iterate was set)
    int64_t* cnt = nullptr;
    uint64_t* bitmap = nullptr;
    int64_t nwords = 0;

    double* part = nullptr;
    int64_t part_elems = 0;
    double* sums = nullptr;      // 64
    double* objsums = nullptr;   // 64 + chunks
    double* colsum_ws = nullptr; // (max columns) * COLSUM_MAXSEG segment sums
    int64_t* scan_ws = nullptr;  // chunk sums of launch_scan
    DevState* st = nullptr;
    DevState* st_host = nullptr; // pinned
    int* d_one = nullptr;
    int* d_flags = nullptr;      // 8 ints

    bool prod_valid = false;     // products and objective sums valid for om[cur]
    double obj[5] = {0, 0, 0, 0, 0};
    // Cov: the candidate bitmap holds, for om[cur], at least the threshold words for
    // lambda1 = bits_lam1 (written by the refresh at acceptance, or by a full pass)
    bool bits_valid = false;
    double bits_lam1 = -1.0;

    std::vector<DevBuf> allocs;

    // graph replay of the common step path
    bool use_graph = false;
    bool screen = true;   // Cov refresh: exact tile screening
    hipStream_t user_stream = nullptr;   // caller's stream when the handle runs on its own
    hipEvent_t enter_ev = nullptr;
    int64_t gen = 0;                     // bumped whenever a captured buffer is reallocated
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        double lam1 = -1, lam2 = -1;
        int64_t gen = -1;
        bool merge = false;   // candidate pass captured: merge of threshold words or full
    } graphs[2];

    // profiling
    bool prof = false;
    hipEvent_t ev[16][2] = {};
    int ev_cls[16] = {};
    int nrec = 0;
    int open_slot = -1;
    double prof_ms[8] = {};
    int64_t prof_cnt[8] = {};
};

namespace {

const char* kVersion = "concord-mi355x 0.1 (gfx950)";

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);   // a bad device fails at the first call
    }
    ~DeviceGuard() {
        int now = -1;
        (void)hipGetDevice(&now);
        if (prev >= 0 && now != prev) (void)hipSetDevice(prev);
    }
};

int fail(concord_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCK(ctx, expr)                                                                 \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, e_ == hipErrorOutOfMemory ? CONCORD_ENOMEM : CONCORD_EHIP,  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Return one device block to where it came from (the stream has been synchronised).
void release(concord_ctx* c, const DevBuf& b) {
    if (!b.ptr) return;
    if (c->alloc.ffn) c->alloc.ffn(c->alloc.user, b.ptr, b.bytes, (void*)c->stream);
    else (void)hipFree(b.ptr);
}

int dalloc(concord_ctx* c, void** out, size_t bytes, bool zero) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (c->alloc.afn) {
        *out = c->alloc.afn(c->alloc.user, bytes, (void*)c->stream);
        if (!*out)
            return fail(c, CONCORD_ENOMEM,
                        "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(out, bytes);
        if (e != hipSuccess) {
            *out = nullptr;
            (void)hipGetLastError();   // clear the sticky error of the failed allocation
            return fail(c, CONCORD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    c->allocs.push_back(DevBuf{*out, bytes});
    if (zero) {
        hipError_t e = hipMemsetAsync(*out, 0, bytes, c->stream);
        if (e != hipSuccess) return fail(c, CONCORD_EHIP, "hipMemsetAsync failed");
    }
    return CONCORD_OK;
}

void dfree(concord_ctx* c, void* p) {
    if (!p) return;
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i].ptr == p) {
            // work queued on the stream may still read the block (hipFree would wait for
            // the device; a caller's allocator need not)
            (void)hipStreamSynchronize(c->stream);
            release(c, c->allocs[i]);
            // the record goes too: a handle that allocates per call (the differentiation
            // form's backward) keeps a list as long as its live blocks, not its calls
            c->allocs[i] = c->allocs.back();
            c->allocs.pop_back();
            return;
        }
}

template <typename T>
int dalloc_t(concord_ctx* c, T** out, size_t count, bool zero = false) {
    void* v = nullptr;
    int rc = dalloc(c, &v, count * sizeof(T), zero);
    *out = (T*)v;
    return rc;
}

int elem_bytes(int store) { return store == ST_F64 ? 8 : 4; }

// capacity for candidate / iterate arrays.  The new arrays are allocated before the old
// ones are released, so a failed allocation leaves the handle as it was; growing the
// current iterate's arrays keeps its entries.
int ensure_csr_cap(concord_ctx* c, int which, int64_t cap) {
    if (c->om_cap[which] >= cap) return CONCORD_OK;
    Csr& o = c->om[which];
    int32_t* ncol = nullptr;
    double* nval = nullptr;
    int rc;
    if ((rc = dalloc_t(c, &ncol, cap))) return rc;
    if ((rc = dalloc_t(c, &nval, cap))) {
        dfree(c, ncol);
        return rc;
    }
    if (which == c->cur && o.col && c->nnz > 0) {
        HIPCK(c, hipMemcpyAsync(ncol, o.col, (size_t)c->nnz * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, c->stream));
        HIPCK(c, hipMemcpyAsync(nval, o.val, (size_t)c->nnz * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
    }
    dfree(c, o.col);
    dfree(c, o.val);
    o.col = ncol;
    o.val = nval;
    c->om_cap[which] = cap;
    c->gen += 1;
    return CONCORD_OK;
}

int ensure_cand_cap(concord_ctx* c, int64_t cap) {
    if (c->a_cap >= cap) return CONCORD_OK;
    int32_t* ncol = nullptr;
    double* nom = nullptr;
    double* ngr = nullptr;
    int rc;
    if ((rc = dalloc_t(c, &ncol, cap)) || (rc = dalloc_t(c, &nom, cap)) ||
        (rc = dalloc_t(c, &ngr, cap))) {
        dfree(c, ncol);
        dfree(c, nom);
        dfree(c, ngr);
        return rc;
    }
    dfree(c, c->A.col);
    dfree(c, c->A.omega);
    dfree(c, c->A.grad);
    c->A.col = ncol;
    c->A.omega = nom;
    c->A.grad = ngr;
    c->a_cap = cap;
    c->gen += 1;
    return CONCORD_OK;
}

void prof_begin(concord_ctx* c, int cls) {
    if (!c->prof || c->nrec >= 16) return;
    const int s = c->nrec++;
    c->ev_cls[s] = cls;
    (void)hipEventRecord(c->ev[s][0], c->stream);   // if it fails, prof_collect skips the sample
    c->open_slot = s;
}

void prof_end(concord_ctx* c) {
    if (!c->prof || c->open_slot < 0) return;
    (void)hipEventRecord(c->ev[c->open_slot][1], c->stream);
    c->open_slot = -1;
}

// after a stream synchronisation: fold the recorded intervals into the totals
void prof_collect(concord_ctx* c) {
    if (!c->prof) return;
    for (int s = 0; s < c->nrec; ++s) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[s][0], c->ev[s][1]) == hipSuccess) {
            c->prof_ms[c->ev_cls[s]] += ms;
            c->prof_cnt[c->ev_cls[s]] += 1;
        }
    }
    c->nrec = 0;
}

// When the handle runs on its own stream, make it wait for the caller's stream.
int enter(concord_ctx* c) {
    if (!c->use_graph) return CONCORD_OK;
    HIPCK(c, hipEventRecord(c->enter_ev, c->user_stream));
    HIPCK(c, hipStreamWaitEvent(c->stream, c->enter_ev, 0));
    return CONCORD_OK;
}

int sync_state(concord_ctx* c) {
    HIPCK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    return CONCORD_OK;
}

// Dense p x p work buffers (M for Obs, the candidate bitmap) are allocated on first
// use, so handles used only for the differentiation form never hold them.  The Cov
// form never stores M (the refresh writes threshold words; the gradient is gathered
// on the candidates).
int ensure_dense(concord_ctx* c) {
    int rc;
    if (c->variant == CONCORD_OBS && !c->M &&
        (rc = dalloc(c, &c->M, (size_t)c->p * c->ldp * elem_bytes(c->dstore), true)))
        return rc;
    if (!c->bitmap && (rc = dalloc_t(c, &c->bitmap, (size_t)c->p * c->nwords, true))) return rc;
    if (c->variant == CONCORD_OBS && !c->xn2_valid) {
        // once per data set, before any step (the differentiation form never needs them)
        if (!c->xn2 && (rc = dalloc_t(c, &c->xn2, (size_t)c->p, false))) return rc;
        HIPCK(c, launch_row_norm2(c->Xt, c->dstore, c->ldk, c->ldk, c->p, c->xn2, c->stream));
        c->xn2_valid = true;
    }
    return CONCORD_OK;
}

// Screening pays for its three launches only with enough tile pairs: below 8 tile rows
// (p <= 448, at most 36 pairs) every refresh covers every pair.
bool screen_now(const concord_ctx* c) { return c->screen && (c->p + 63) / 64 >= 8; }

// Products and objective sums at om[which], gated on `gate` (device int).  Cov: the
// objective gathers M on the support; with bits_lam1 >= 0 the refresh writes the
// candidate threshold words of om[which] for that lambda1.
int products_at(concord_ctx* c, int which, const int* gate, double bits_lam1 = -1.0) {
    if (c->variant == CONCORD_COV) {
        int rc = ensure_dense(c);
        if (rc) return rc;
    }
    const Csr& O = c->om[which];
    const int64_t p = c->p;
    int nysq = 0;
    if (c->variant == CONCORD_OBS && c->precision != CONCORD_BF16X3 && !c->Y) {
        int rc = dalloc(c, &c->Y, (size_t)c->prow * c->ldk * elem_bytes(c->dstore), true);
        if (rc) return rc;
    }
    prof_begin(c, CONCORD_PROF_SPMM);
    if (c->variant == CONCORD_OBS) {
        const bool split = c->precision == CONCORD_BF16X3;
        const int nch = spmm_nchunks(c->dstore, c->ldk);
        // sq parts go after the 4 objective columns in `part`
        double* sq = c->part + 4 * p;
        HIPCK(c, launch_spmm(O, p, c->Xt, c->dstore, c->ldk, c->ldk, split ? nullptr : c->Y,
                             c->dstore, c->ldk, split ? c->Y_hi : nullptr,
                             split ? c->Y_lo : nullptr, kblk_stride(c->prow), sq, gate,
                             c->stream));
        nysq = nch;
        HIPCK(c, launch_obj_parts(O, p, nullptr, c->dstore, 0, c->part, gate, c->stream));
    } else {
        if (bits_lam1 >= 0.0) {
            // the refresh kernel alone gets its own timing class
            const bool scr = screen_now(c);
            HIPCK(c, launch_cov_screen(O, p, c->sstore, c->smax, bits_lam1, c->bitmap, c->nwords,
                                       c->rws, gate, c->stream, scr));
            prof_end(c);
            prof_begin(c, CONCORD_PROF_REFRESH);
            HIPCK(c, launch_cov_refresh_pairs(O, p, c->S, c->sstore, c->ldp, scr ? c->smax : nullptr,
                                              bits_lam1, c->bitmap, c->nwords, c->rws, gate,
                                              c->stream));
            prof_end(c);
            prof_begin(c, CONCORD_PROF_SPMM);
        }
        HIPCK(c, launch_obj_parts_cov(O, p, c->S, c->sstore, c->ldp, c->part, gate, c->stream));
    }
    HIPCK(c, launch_colsum_obj(c->part, p, 4 + nysq, c->objsums, c->colsum_ws, nysq, gate, c->st,
                               c->stream));
    prof_end(c);
    return CONCORD_OK;
}

// bits_lam1 >= 0 (a step about to run with that lambda1): the Cov refresh also writes
// the candidate threshold words for it.
int ensure_products(concord_ctx* c, double bits_lam1 = -1.0) {
    if (c->prod_valid) return CONCORD_OK;
    hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(64), 0, c->stream, c->st);
    const bool bits = c->variant == CONCORD_COV && bits_lam1 >= 0.0;
    int rc = products_at(c, c->cur, c->d_one, bits ? bits_lam1 : -1.0);
    if (rc) return rc;
    if (bits) {
        c->bits_valid = true;
        c->bits_lam1 = bits_lam1;
    }
    if ((rc = sync_state(c))) return rc;
    for (int i = 0; i < 5; ++i) c->obj[i] = c->st_host->obj[i];
    c->prod_valid = true;
    return CONCORD_OK;
}

void objective_from(const concord_ctx* c, const double* o, double lam1, double lam2, double* f,
                    double* F) {
    objective_value(o, c->variant == CONCORD_OBS, (double)c->n, lam1, lam2, f, F);
}

// tau0 * shrink^q as the trial kernels form it: q successive multiplications
double step_size(const concord_ctx* c, int q) {
    double t = c->tau0;
    for (int i = 0; i < q; ++i) t *= c->shrink;
    return t;
}

int set_identity(concord_ctx* c) {
    int rc = ensure_csr_cap(c, c->cur, c->p);
    if (rc) return rc;
    HIPCK(c, launch_identity(c->om[c->cur], c->p, c->stream));
    c->nnz = c->p;
    c->k = 0;
    c->a_nnz = -1;
    c->prod_valid = false;
    c->bits_valid = false;
    return CONCORD_OK;
}

int do_step(concord_ctx* c, double lam1, double lam2, int forced_trials, concord_step_info* info) {
    if (!c) return CONCORD_EINVAL;
    if (!(lam1 >= 0.0) || !(lam2 >= 0.0) || !std::isfinite(lam1) || !std::isfinite(lam2))
        return fail(c, CONCORD_EINVAL, "lambda1 and lambda2 must be finite and >= 0");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    if (forced_trials > c->max_bt + 1)
        return fail(c, CONCORD_EINVAL, "forced trial count exceeds max_backtracks + 1");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    int rc = ensure_dense(c);
    if (rc) return rc;
    if ((rc = ensure_products(c, lam1))) return rc;
    const int64_t p = c->p;
    c->a_nnz = -1;   // the candidate set is rebuilt below; valid again once a step is accepted

    const int nxt = c->cur ^ 1;
    const double inv_n = c->variant == CONCORD_OBS ? 1.0 / (double)c->n : 1.0;
    const void* TB = c->variant == CONCORD_OBS ? c->Xt : c->S;
    const int tbstore = c->variant == CONCORD_OBS ? c->dstore : c->sstore;
    const int64_t tld = c->variant == CONCORD_OBS ? c->ldk : c->ldp;
    const int forced_q = forced_trials >= 1 ? forced_trials - 1 : -1;
    const int total = c->max_bt + 1;   // step sizes 1 .. 2^-max_bt

    int obs_bits = 0;   // the Obs contraction wrote the candidate threshold words
    // gradient-side dense product (Obs): M = (Y X + (Y X)^T) / (2n)
    auto enqueue_gemm = [&]() -> int {
        if (c->variant != CONCORD_OBS) return CONCORD_OK;
        const bool split = c->precision == CONCORD_BF16X3;
        const void* P0 = split ? (const void*)c->Y_hi : c->Y;
        const void* P1 = split ? (const void*)c->Y_lo : nullptr;
        const void* Q0 = split ? (const void*)c->Xt_hi : c->Xt;
        const void* Q1 = split ? (const void*)c->Xt_lo : nullptr;
        prof_begin(c, CONCORD_PROF_DENSE);
        // the epilogue of the tuned variant may also write this iteration's candidate
        // threshold words (obs_bits says whether it did)
        ThreshOut th;
        th.lam1 = lam1;
        th.bits = c->bitmap;
        th.nwords = c->nwords;
        th.wrote = &obs_bits;
        HIPCK(c, launch_gemm_sym(c->gkind, true, P0, P1, Q0, Q1, c->ldk, p, 0.5 / (double)c->n,
                                 c->M, c->dstore, c->ldp, c->stream, th));
        prof_end(c);
        return CONCORD_OK;
    };
    // candidate set A of this iteration: the support is merged into threshold words
    // already written for this lambda1 by the Obs contraction's epilogue (this step) or
    // by the Cov refresh of the accepted step; otherwise a full pass over M (Obs) or a
    // refresh of the words at the current iterate (Cov).
    auto merge_now = [&]() {
        return c->variant == CONCORD_OBS ? obs_bits != 0 : (c->bits_valid && c->bits_lam1 == lam1);
    };
    auto enqueue_cands = [&]() -> int {
        const bool merge = merge_now();
        hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(64), 0, c->stream, c->st);
        prof_begin(c, CONCORD_PROF_CAND);
        const bool cov = c->variant == CONCORD_COV;
        if (cov && !merge)
            HIPCK(c, launch_cov_refresh(c->om[c->cur], p, c->S, c->sstore, c->ldp, c->smax, lam1,
                                        c->bitmap, c->nwords, c->rws, c->d_one, c->stream,
                                        nullptr, screen_now(c)));
        // the screened refresh leaves the words of screened-out tiles stale: merge and fill
        // read only kept tiles and support words
        const uint64_t* tm = cov && screen_now(c) ? c->rws.tmask : nullptr;
        if (merge || cov)
            HIPCK(c, launch_cand_merge(c->om[c->cur], p, c->bitmap, c->nwords, c->cnt, c->stream,
                                       tm));
        else
            HIPCK(c, launch_cand_count(c->M, c->dstore, c->ldp, c->om[c->cur], p, lam1,
                                       c->bitmap, c->nwords, c->cnt, c->stream));
        HIPCK(c, launch_scan(c->cnt, p, c->A.rowptr, c->a_cap, &c->st->overflow, c->scan_ws,
                             c->stream, &c->st->n_cand));
        // a contraction that wrote the threshold words stored M's upper triangle only
        HIPCK(c, launch_cand_fill(cov ? nullptr : c->M, c->dstore, c->ldp, c->om[c->cur], p, lam2,
                                  c->bitmap, c->nwords, c->A, c->a_cap, &c->st->overflow,
                                  c->stream, tm, !cov && merge));
        if (cov)
            HIPCK(c, launch_cand_grad_cov(c->om[c->cur], p, c->S, c->sstore, c->ldp, lam2, c->A,
                                          &c->st->overflow, c->stream));
        prof_end(c);
        return CONCORD_OK;
    };
    // one batch of step sizes tau0 * 2^-q, q < m, then emission, products and
    // objective at Omega+ (gated on the device-side decision) and the read-back
    auto enqueue_batch = [&](int q_base, int m) -> int {
        const double tau0 = step_size(c, q_base);
        prof_begin(c, CONCORD_PROF_TRIAL);
        HIPCK(c, launch_trial(c->A, p, tau0, c->shrink, m, lam1, c->variant, TB, tbstore, tld,
                              c->variant == CONCORD_OBS ? c->ldk : 0, c->xn2, c->part, c->st,
                              c->stream));
        const int S = trial_splits(c->variant, tbstore, c->variant == CONCORD_OBS ? c->ldk : 0);
        HIPCK(c, launch_colsum_decide(c->part, (int64_t)S * p, 4 * m, c->sums, c->colsum_ws, m,
                                      tau0, c->shrink, q_base, lam2, inv_n, forced_q, c->st,
                                      c->stream));
        prof_end(c);
        prof_begin(c, CONCORD_PROF_EMIT);
        const bool grp = c->variant == CONCORD_COV && p >= COV_TRIAL_GROUP_MIN_P;
        HIPCK(c, launch_emit_count(c->A, p, lam1, c->st, c->cnt, c->stream, grp));
        HIPCK(c, launch_scan(c->cnt, p, c->om[nxt].rowptr, c->om_cap[nxt], nullptr, c->scan_ws,
                             c->stream, &c->st->nnz_next));
        HIPCK(c, launch_emit_fill(c->A, p, lam1, c->st, c->om[nxt], c->stream, grp));
        prof_end(c);
        int rc2 = products_at(c, nxt, &c->st->accepted,
                              c->variant == CONCORD_COV ? lam1 : -1.0);
        if (rc2) return rc2;
        HIPCK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost,
                                c->stream));
        return CONCORD_OK;
    };

    // Common path as one graph launch: contraction, candidates and the first batch.
    // Used after the first iteration of a handle (the contraction's tile variant is
    // chosen by timing on its first call, which cannot happen inside a capture).
    const int m0 = std::min(c->tb, total);
    bool first_done = false;
    if (c->use_graph && !c->prof && forced_q < 0 && c->k > 0) {
        if ((rc = ensure_csr_cap(c, nxt, c->a_cap))) return rc;
        if ((rc = ensure_csr_cap(c, c->cur, c->a_cap))) return rc;
        concord_ctx::StepGraph& sg = c->graphs[c->cur];
        // Obs: the tuned variant (fixed after the first step) decides; Cov: the state
        const bool merge = c->variant == CONCORD_OBS ? sg.merge : merge_now();
        if (!sg.exec || sg.lam1 != lam1 || sg.lam2 != lam2 || sg.gen != c->gen ||
            sg.merge != merge) {
            if (sg.exec) {
                (void)hipGraphExecDestroy(sg.exec);
                sg.exec = nullptr;
            }
            hipGraph_t g = nullptr;
            HIPCK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            int rc1 = enqueue_gemm();
            if (!rc1) rc1 = enqueue_cands();
            if (!rc1) rc1 = enqueue_batch(0, m0);
            hipError_t ec = hipStreamEndCapture(c->stream, &g);
            if (rc1) {
                if (g) (void)hipGraphDestroy(g);
                return rc1;
            }
            HIPCK(c, ec);
            hipError_t ei = hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCK(c, ei);
            sg.lam1 = lam1;
            sg.lam2 = lam2;
            sg.gen = c->gen;
            sg.merge = c->variant == CONCORD_OBS ? obs_bits != 0 : merge;
        }
        HIPCK(c, hipGraphLaunch(sg.exec, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
        prof_collect(c);
        first_done = true;
    } else {
        if ((rc = enqueue_gemm())) return rc;
    }

    for (int attempt = 0; attempt < 8; ++attempt) {
        int q_base = forced_q >= 0 ? forced_q : 0, batches = 0;
        bool overflow = false, accepted = false;
        if (!first_done) {
            if ((rc = enqueue_cands())) return rc;
            if ((rc = ensure_csr_cap(c, nxt, c->a_cap))) return rc;
        }
        while (q_base < total) {
            const int m = forced_q >= 0 ? 1 : std::min(c->tb, total - q_base);
            if (first_done) {
                first_done = false;   // the graph ran candidates and this batch
            } else {
                if ((rc = enqueue_batch(q_base, m))) return rc;
                HIPCK(c, hipStreamSynchronize(c->stream));
                prof_collect(c);
            }
            ++batches;
            if (c->st_host->overflow) { overflow = true; break; }
            if (c->st_host->accepted_q >= 0) { accepted = true; break; }
            if (forced_q >= 0) break;
            q_base += m;
        }
        if (overflow) {
            const int64_t need = c->st_host->n_cand;
            if ((rc = ensure_cand_cap(c, need + need / 2 + 1024))) return rc;
            continue;
        }
        // the candidate pass ran for (om[cur], lam1); an accepted step's refresh rewrote
        // the threshold words for (om[nxt], lam1)
        if (c->variant == CONCORD_COV) {
            c->bits_valid = true;
            c->bits_lam1 = lam1;
        }
        if (c->st_host->nonpos)
            return fail(c, CONCORD_ENOTPD, "replayed step leaves a diagonal entry <= 0");
        if (!accepted)
            return fail(c, CONCORD_ELINESEARCH,
                        "line search exhausted max_backtracks; iterate unchanged");
        const DevState& s = *c->st_host;
        c->cur = nxt;
        c->nnz = c->st_host->nnz_next;
        c->k += 1;
        c->a_nnz = c->st_host->n_cand;
        for (int i = 0; i < 5; ++i) c->obj[i] = s.obj[i];
        c->prod_valid = true;
        if (info) {
            info->k = c->k;
            info->tau = s.tau;
            info->n_trials = s.accepted_q + 1;
            info->n_batches = batches;
            objective_from(c, c->obj, lam1, lam2, &info->f, &info->F);
            info->nnz = c->nnz;
            info->delta_fro = std::sqrt(s.dd);
            info->n_candidates = c->st_host->n_cand;
            info->lhs = s.lhs;
            info->rhs = s.rhs;
        }
        return CONCORD_OK;
    }
    return fail(c, CONCORD_ENOMEM, "candidate capacity did not converge");
}

// Rates for CONCORD_AUTO, measured once per (device, precision) and cached: the useful
// rate of the dense symmetric contraction (syr2k, p = 4096, K = 2048, zero operands; the
// tuner picks its variant on the first call) and the device copy rate of 256 MiB.
std::mutex g_rate_mu;
std::map<std::pair<int, int>, std::pair<double, double>> g_rates;

int measured_rates(int dev, int precision, double (&out)[2]) {
    std::lock_guard<std::mutex> lk(g_rate_mu);
    auto it = g_rates.find({dev, precision});
    if (it != g_rates.end()) {
        out[0] = it->second.first;
        out[1] = it->second.second;
        return CONCORD_OK;
    }
    DeviceGuard g(dev);
    const int64_t p = 4096, K = 2048;
    const int kind = precision == CONCORD_FP64 ? GK_F64 : (precision == CONCORD_FP32 ? GK_F32 : GK_BF16X3);
    const int ostore = precision == CONCORD_FP64 ? ST_F64 : ST_F32;
    const size_t eb = precision == CONCORD_FP64 ? 8 : (precision == CONCORD_FP32 ? 4 : 2);
    const size_t op = (size_t)p * K * eb, cb = (size_t)p * p * (ostore == ST_F64 ? 8 : 4);
    const size_t copy_bytes = (size_t)256 << 20;
    void *P0 = nullptr, *P1 = nullptr, *C = nullptr, *src = nullptr, *dst = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&](int rc) {
        if (st) (void)hipStreamSynchronize(st);
        for (void* q : {P0, P1, C, src, dst})
            if (q) (void)hipFree(q);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
        return rc;
    };
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return cleanup(CONCORD_EHIP);
    if (hipMalloc(&P0, op) != hipSuccess || hipMalloc(&P1, op) != hipSuccess ||
        hipMalloc(&C, cb) != hipSuccess || hipMalloc(&src, copy_bytes) != hipSuccess ||
        hipMalloc(&dst, copy_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(CONCORD_ENOMEM);
    }
    if (hipMemsetAsync(P0, 0, op, st) != hipSuccess || hipMemsetAsync(P1, 0, op, st) != hipSuccess ||
        hipMemsetAsync(src, 0, copy_bytes, st) != hipSuccess)
        return cleanup(CONCORD_EHIP);
    const bool split = kind == GK_BF16X3;
    auto gemm = [&]() {
        return launch_gemm_sym(kind, true, P0, split ? P1 : nullptr, P1, split ? P0 : nullptr, K, p,
                               1.0, C, ostore, p, st);
    };
    float ms_g = 0.f, ms_c = 0.f;
    if (gemm() != hipSuccess || gemm() != hipSuccess) return cleanup(CONCORD_EHIP);   // tune, warm
    if (hipEventRecord(e0, st) != hipSuccess) return cleanup(CONCORD_EHIP);
    for (int r = 0; r < 3; ++r)
        if (gemm() != hipSuccess) return cleanup(CONCORD_EHIP);
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms_g, e0, e1) != hipSuccess)
        return cleanup(CONCORD_EHIP);
    if (hipMemcpyAsync(dst, src, copy_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipEventRecord(e0, st) != hipSuccess)
        return cleanup(CONCORD_EHIP);
    for (int r = 0; r < 3; ++r)
        if (hipMemcpyAsync(dst, src, copy_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return cleanup(CONCORD_EHIP);
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms_c, e0, e1) != hipSuccess)
        return cleanup(CONCORD_EHIP);
    out[0] = 3.0 * 2.0 * (double)K * (double)p * (double)p / (ms_g * 1e-3) / 1e12;
    out[1] = 3.0 * 2.0 * (double)copy_bytes / (ms_c * 1e-3) / 1e9;
    g_rates[{dev, precision}] = {out[0], out[1]};
    return cleanup(CONCORD_OK);
}

}  // namespace

extern "C" {

void concord_config_init(concord_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->variant = CONCORD_COV;
    cfg->precision = CONCORD_FP64;
    cfg->stream = nullptr;
    cfg->device = -1;
    cfg->max_backtracks = 60;
    cfg->trial_batch = 8;
    cfg->tau0 = 1.0;
    cfg->shrink = 0.5;
}

const char* concord_version(void) { return kVersion; }

const char* concord_last_error(const concord_ctx* ctx) {
    if (!ctx) return "null handle";
    return ctx->err.c_str();
}

int concord_set_profiling(concord_ctx* c, int32_t on) {
    if (!c) return CONCORD_EINVAL;
    DeviceGuard g(c->device);
    if (on && !c->ev[0][0]) {
        for (int s = 0; s < 16; ++s)
            for (int t = 0; t < 2; ++t) HIPCK(c, hipEventCreate(&c->ev[s][t]));
    }
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->nrec = 0;
    c->open_slot = -1;
    for (int i = 0; i < 8; ++i) { c->prof_ms[i] = 0.0; c->prof_cnt[i] = 0; }
    c->prof = on != 0;
    return CONCORD_OK;
}

int concord_get_profile(const concord_ctx* c, concord_profile* out) {
    if (!c || !out) return CONCORD_EINVAL;
    for (int i = 0; i < 8; ++i) { out->ms[i] = c->prof_ms[i]; out->launches[i] = c->prof_cnt[i]; }
    return CONCORD_OK;
}

int concord_contraction_variant(const concord_ctx* c, char* name, int32_t cap) {
    if (!c) return CONCORD_EINVAL;
    const char* nm = "untuned";
    const int v = gemm_sym_choice(c->gkind, c->variant == CONCORD_OBS, c->p, c->ldk, &nm);
    if (name && cap > 0) {
        std::snprintf(name, (size_t)cap, "%s", nm);
    }
    return v;
}

void concord_destroy(concord_ctx* ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (int s = 0; s < 16; ++s)
            for (int t = 0; t < 2; ++t)
                if (ctx->ev[s][t]) (void)hipEventDestroy(ctx->ev[s][t]);
        for (auto& sg : ctx->graphs)
            if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
        if (ctx->use_graph) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipStreamDestroy(ctx->stream);
            if (ctx->enter_ev) (void)hipEventDestroy(ctx->enter_ev);
        }
        for (const DevBuf& a : ctx->allocs) release(ctx, a);
        if (ctx->st_host) (void)hipHostFree(ctx->st_host);
    }
    delete ctx;
}

int concord_create(const concord_config* cfg, concord_ctx** out) {
    if (!out) return CONCORD_EINVAL;
    *out = nullptr;
    if (!cfg) return CONCORD_EINVAL;
    if (cfg->p < 1 || cfg->p > (int64_t)1 << 30) return CONCORD_EINVAL;
    if (cfg->variant != CONCORD_COV && cfg->variant != CONCORD_OBS && cfg->variant != CONCORD_AUTO)
        return CONCORD_EINVAL;
    if (cfg->precision < CONCORD_FP64 || cfg->precision > CONCORD_BF16X3) return CONCORD_EINVAL;
    if ((cfg->variant == CONCORD_OBS || cfg->variant == CONCORD_AUTO) && cfg->n < 1)
        return CONCORD_EINVAL;
    if (cfg->n < 0) return CONCORD_EINVAL;
    if (cfg->trial_batch < 1 || cfg->trial_batch > MAXQ) return CONCORD_EINVAL;
    if (cfg->max_backtracks < 0 || cfg->max_backtracks > 1000) return CONCORD_EINVAL;
    if (!(cfg->tau0 > 0.0) || !std::isfinite(cfg->tau0)) return CONCORD_EINVAL;
    if (!(cfg->shrink > 0.0 && cfg->shrink < 1.0)) return CONCORD_EINVAL;
    if ((cfg->alloc_fn == nullptr) != (cfg->free_fn == nullptr)) return CONCORD_EINVAL;

    int dev = cfg->device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return CONCORD_EHIP;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) return CONCORD_EHIP;

    int variant = cfg->variant;
    if (variant == CONCORD_AUTO) {
        // Lemma 3.1's work priced with this device's measured rates (the kept fraction of
        // the Cov refresh is unknown before S exists: 1, an upper bound on Cov's cost)
        double r[2];
        const int rc0 = measured_rates(dev, cfg->precision, r);
        if (rc0) return rc0;
        concord_variant_estimate est;
        if (concord_suggest_variant(cfg->p, cfg->n, 5.0, 3.0, 30.0, cfg->precision, r[0], r[1], 1.0,
                                    &est) != CONCORD_OK)
            return CONCORD_EINVAL;
        variant = est.choice;
    }
    concord_ctx* c = new concord_ctx();
    c->p = cfg->p;
    c->n = cfg->n;
    c->variant = variant;
    c->precision = cfg->precision;
    c->stream = (hipStream_t)cfg->stream;
    c->device = dev;
    c->max_bt = cfg->max_backtracks;
    c->tb = cfg->trial_batch;
    c->tau0 = cfg->tau0;
    c->shrink = cfg->shrink;
    c->alloc.afn = cfg->alloc_fn;
    c->alloc.ffn = cfg->free_fn;
    c->alloc.user = cfg->alloc_user;
    c->use_graph = cfg->use_graph != 0;
    c->screen = cfg->no_screen == 0;
    DeviceGuard g(dev);
    if (c->use_graph) {
        // captures need a stream of our own (the caller's may be the null stream)
        c->user_stream = c->stream;
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->enter_ev, hipEventDisableTiming) != hipSuccess) {
            c->use_graph = false;
            c->stream = c->user_stream;
        }
    }

    c->dstore = c->precision == CONCORD_FP64 ? ST_F64 : ST_F32;
    c->sstore = c->precision == CONCORD_FP64 ? ST_F64 : (c->precision == CONCORD_FP32 ? ST_F32 : ST_B16P);
    c->gkind = c->precision == CONCORD_FP64 ? GK_F64 : (c->precision == CONCORD_FP32 ? GK_F32 : GK_BF16X3);
    const int64_t p = c->p;
    c->prow = round_up(p, ROW_PAD);
    c->ldk = round_up(c->n > 0 ? c->n : 1, K_PAD);
    c->ldp = round_up(p, 64);
    c->nwords = (p + 63) / 64;

    auto bail = [&](int rc) {
        concord_destroy(c);
        return rc;
    };
    int rc;
    const size_t eb = elem_bytes(c->dstore);
    const bool split = c->precision == CONCORD_BF16X3;
    if (c->n > 0) {
        if ((rc = dalloc(c, &c->Xt, (size_t)c->prow * c->ldk * eb, true))) return bail(rc);
        if (split) {
            if ((rc = dalloc_t(c, &c->Xt_hi, (size_t)c->prow * c->ldk, true))) return bail(rc);
            if ((rc = dalloc_t(c, &c->Xt_lo, (size_t)c->prow * c->ldk, true))) return bail(rc);
        }
    }
    if (c->variant == CONCORD_OBS) {
        if (split) {
            if ((rc = dalloc_t(c, &c->Y_hi, (size_t)c->prow * c->ldk, true))) return bail(rc);
            if ((rc = dalloc_t(c, &c->Y_lo, (size_t)c->prow * c->ldk, true))) return bail(rc);
        }
        // the FP64/FP32 Y is allocated by the first solver step (a handle used only for
        // the differentiation form never holds it)
    } else {
        if ((rc = dalloc(c, &c->S, (size_t)p * c->ldp * (c->sstore == ST_F64 ? 8 : 4), true)))
            return bail(rc);
        const int64_t T = (p + 63) / 64;
        if ((rc = dalloc_t(c, &c->smax, (size_t)(T * T), true))) return bail(rc);
        RefreshWs& r = c->rws;
        if ((rc = dalloc_t(c, &r.lcnt, (size_t)T, true)) || (rc = dalloc_t(c, &r.lK, (size_t)T * 64, true)) ||
            (rc = dalloc_t(c, &r.lW, (size_t)T * 64, true)) || (rc = dalloc_t(c, &r.lcmax, (size_t)T, true)) ||
            (rc = dalloc_t(c, &r.plist, (size_t)(T * (T + 1) / 2), true)) ||
            (rc = dalloc_t(c, &r.pcount, 1, true)) ||
            (rc = dalloc_t(c, &r.tmask, (size_t)(T * ((T + 63) / 64)), true)))
            return bail(rc);
    }
    for (int w = 0; w < 2; ++w)
        if ((rc = dalloc_t(c, &c->om[w].rowptr, p + 1, true))) return bail(rc);
    const int64_t cap0 = 8 * p + 1024;
    if ((rc = ensure_csr_cap(c, 0, cap0)) || (rc = ensure_csr_cap(c, 1, cap0))) return bail(rc);
    if ((rc = dalloc_t(c, &c->A.rowptr, p + 1, true))) return bail(rc);
    if ((rc = ensure_cand_cap(c, cap0))) return bail(rc);
    if ((rc = dalloc_t(c, &c->cnt, p + 1, true))) return bail(rc);
    const int nch = c->variant == CONCORD_OBS ? spmm_nchunks(c->dstore, c->ldk) : 0;
    c->part_elems = (int64_t)std::max(4 * MAXQ * 8, 4 + nch) * p;   // trials: up to 8 column splits
    if ((rc = dalloc_t(c, &c->part, c->part_elems, true))) return bail(rc);
    if ((rc = dalloc_t(c, &c->sums, 64, true))) return bail(rc);
    if ((rc = dalloc_t(c, &c->objsums, 64 + nch, true))) return bail(rc);
    if ((rc = dalloc_t(c, &c->scan_ws, (size_t)scan_ws_len(p), true))) return bail(rc);
    if ((rc = dalloc_t(c, &c->colsum_ws, (size_t)std::max(4 * MAXQ, 4 + nch) * COLSUM_MAXSEG, true)))
        return bail(rc);
    if ((rc = dalloc_t(c, &c->st, 1, true))) return bail(rc);
    if ((rc = dalloc_t(c, &c->d_one, 1, false))) return bail(rc);
    if ((rc = dalloc_t(c, &c->d_flags, 8, true))) return bail(rc);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, c->d_one, 1);
    if (hipHostMalloc((void**)&c->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        return bail(CONCORD_ENOMEM);
    if ((rc = set_identity(c))) return bail(rc);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(CONCORD_EHIP);
    *out = c;
    return CONCORD_OK;
}

int concord_set_data(concord_ctx* c, int32_t kind, const void* dev_data, int32_t dtype,
                     int64_t rows, int64_t cols, int64_t ld) {
    if (!c) return CONCORD_EINVAL;
    if (!dev_data) return fail(c, CONCORD_EINVAL, "null data pointer");
    if (dtype != CONCORD_F64 && dtype != CONCORD_F32) return fail(c, CONCORD_EINVAL, "dtype");
    if (ld < cols) return fail(c, CONCORD_EINVAL, "ld < cols");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    const int is64 = dtype == CONCORD_F64;
    if (kind == CONCORD_DATA_X) {
        if (rows != c->n || cols != c->p)
            return fail(c, CONCORD_EINVAL, "X must be n x p as configured");
    } else if (kind == CONCORD_DATA_S) {
        if (c->variant != CONCORD_COV) return fail(c, CONCORD_EINVAL, "S is accepted by Cov only");
        if (rows != c->p || cols != c->p) return fail(c, CONCORD_EINVAL, "S must be p x p");
    } else {
        return fail(c, CONCORD_EINVAL, "unknown data kind");
    }
    // X: the non-finite check rides on the transpose into the library layout, so a
    // rejected X leaves the handle without data; S is checked before it is copied.
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, c->d_flags, 0);
    if (kind == CONCORD_DATA_X) {
        const bool split = c->precision == CONCORD_BF16X3;
        c->xn2_valid = false;
        HIPCK(c, launch_transpose_in(dev_data, is64, rows, cols, ld, c->Xt, c->dstore, c->ldk,
                                     split ? c->Xt_hi : nullptr, split ? c->Xt_lo : nullptr,
                                     kblk_stride(c->prow), c->d_flags, c->stream));
    } else {
        HIPCK(c, launch_check_finite(dev_data, is64, rows, cols, ld, c->d_flags, c->stream));
    }
    int hflag = 0;
    HIPCK(c, hipMemcpyAsync(&hflag, c->d_flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (hflag) {
        if (kind == CONCORD_DATA_X) {
            c->has_data = false;
            c->prod_valid = false;
            c->bits_valid = false;
        }
        return fail(c, CONCORD_ENONFINITE, "data holds NaN or Inf");
    }

    if (kind == CONCORD_DATA_X) {
        const bool split = c->precision == CONCORD_BF16X3;
        if (c->variant == CONCORD_COV) {
            const void* P0 = split ? (const void*)c->Xt_hi : c->Xt;
            const void* P1 = split ? (const void*)c->Xt_lo : nullptr;
            prof_begin(c, CONCORD_PROF_DENSE);
            HIPCK(c, launch_gemm_sym(c->gkind, false, P0, P1, nullptr, nullptr, c->ldk, c->p,
                                     1.0 / (double)c->n, c->S, c->sstore, c->ldp, c->stream));
            prof_end(c);
        }
    } else {
        HIPCK(c, launch_sym_copy(dev_data, is64, c->p, ld, c->S, c->sstore, c->ldp, c->stream));
    }
    if (c->variant == CONCORD_COV)
        HIPCK(c, launch_tile_max(c->S, c->sstore, c->p, c->ldp, c->smax, c->stream));
    c->has_data = true;
    int rc = set_identity(c);
    if (rc) return rc;
    HIPCK(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    return CONCORD_OK;
}

int concord_set_omega(concord_ctx* c, int64_t nnz, const int64_t* dev_row_ptr,
                      const int32_t* dev_col, const void* dev_val, int32_t dtype) {
    if (!c) return CONCORD_EINVAL;
    if (nnz < c->p || !dev_row_ptr || !dev_col || !dev_val)
        return fail(c, CONCORD_EINVAL, "bad CSR arguments");
    if (dtype != CONCORD_F64 && dtype != CONCORD_F32) return fail(c, CONCORD_EINVAL, "dtype");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, c->d_flags, 0);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, c->d_flags + 1, 0);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, c->stream, c->d_flags + 2, 0);
    HIPCK(c, launch_csr_validate(dev_row_ptr, dev_col, dev_val, dtype == CONCORD_F64, c->p, nnz,
                                 c->d_flags, c->stream));
    int hf[3] = {0, 0, 0};
    HIPCK(c, hipMemcpyAsync(hf, c->d_flags, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (hf[0]) return fail(c, CONCORD_EINVAL, "CSR structure invalid (row_ptr, sorted columns or diagonal)");
    if (hf[2]) return fail(c, CONCORD_ENONFINITE, "Omega holds NaN or Inf");
    if (hf[1]) return fail(c, CONCORD_ENOTPD, "Omega has a diagonal entry <= 0");
    int rc;
    if ((rc = ensure_csr_cap(c, c->cur, nnz))) return rc;
    if ((rc = ensure_cand_cap(c, std::max<int64_t>(c->a_cap, 2 * nnz)))) return rc;
    Csr& o = c->om[c->cur];
    HIPCK(c, hipMemcpyAsync(o.rowptr, dev_row_ptr, (c->p + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToDevice, c->stream));
    HIPCK(c, launch_csr_import(dev_col, dev_val, dtype == CONCORD_F64, nnz, o.col, o.val, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->nnz = nnz;
    c->k = 0;
    c->a_nnz = -1;
    c->prod_valid = false;
    c->bits_valid = false;
    return CONCORD_OK;
}

int concord_reset(concord_ctx* c) {
    if (!c) return CONCORD_EINVAL;
    DeviceGuard g(c->device);
    int rc = set_identity(c);
    if (rc) return rc;
    HIPCK(c, hipStreamSynchronize(c->stream));
    return CONCORD_OK;
}

int concord_step(concord_ctx* c, double lam1, double lam2, concord_step_info* info) {
    return do_step(c, lam1, lam2, 0, info);
}

int concord_step_replay(concord_ctx* c, double lam1, double lam2, int32_t trials,
                        concord_step_info* info) {
    if (!c) return CONCORD_EINVAL;
    if (trials < 1) return fail(c, CONCORD_EINVAL, "trials must be >= 1");
    return do_step(c, lam1, lam2, trials, info);
}

int concord_solve(concord_ctx* c, double lam1, double lam2, double tol, int64_t max_iter,
                  concord_solve_info* info) {
    if (!c) return CONCORD_EINVAL;
    if (!(tol >= 0.0) || max_iter < 0) return fail(c, CONCORD_EINVAL, "tol must be >= 0, max_iter >= 0");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    int rc = ensure_products(c, lam1);
    if (rc) return rc;
    double f, F_old;
    objective_from(c, c->obj, lam1, lam2, &f, &F_old);
    int status = tol > 0.0 ? CONCORD_WMAXITER : CONCORD_OK;
    int64_t it = 0;
    for (; it < max_iter; ++it) {
        concord_step_info si;
        rc = do_step(c, lam1, lam2, 0, &si);
        if (rc < 0) { status = rc; break; }
        const double F_new = si.F;
        if (tol > 0.0 && std::fabs(F_new - F_old) < tol * std::fabs(F_old)) {
            status = CONCORD_OK;
            ++it;
            break;
        }
        F_old = F_new;
    }
    if (info) {
        info->iters = c->k;
        objective_from(c, c->obj, lam1, lam2, &info->f, &info->F);
        info->nnz = c->nnz;
        info->status = status;
    }
    return status;
}

int concord_refresh_screen_stats(concord_ctx* c, double lam1, int64_t* host_pairs,
                                 int64_t* host_active) {
    if (!c) return CONCORD_EINVAL;
    if (c->variant != CONCORD_COV) return fail(c, CONCORD_EINVAL, "screening is a Cov refresh");
    if (!(lam1 >= 0.0) || !std::isfinite(lam1)) return fail(c, CONCORD_EINVAL, "lambda1 must be >= 0");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    int rc = ensure_dense(c);
    if (rc) return rc;
    if (!c->d_active && (rc = dalloc_t(c, &c->d_active, 1, false))) return rc;
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, c->stream, c->d_active, 0ull);
    HIPCK(c, launch_cov_refresh(c->om[c->cur], c->p, c->S, c->sstore, c->ldp, c->smax, lam1,
                                c->bitmap, c->nwords, c->rws, c->d_one, c->stream, c->d_active,
                                screen_now(c)));
    unsigned long long act = 0;
    HIPCK(c, hipMemcpyAsync(&act, c->d_active, sizeof(act), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    // the words now belong to (current iterate, lam1)
    c->bits_valid = true;
    c->bits_lam1 = lam1;
    const int64_t T = (c->p + 63) / 64;
    if (host_pairs) *host_pairs = T * (T + 1) / 2;
    if (host_active) *host_active = (int64_t)act;
    return CONCORD_OK;
}

int concord_objective(concord_ctx* c, double lam1, double lam2, double* host_f, double* host_F) {
    if (!c) return CONCORD_EINVAL;
    if (!(lam1 >= 0.0) || !(lam2 >= 0.0)) return fail(c, CONCORD_EINVAL, "lambda must be >= 0");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    int rc = ensure_products(c);
    if (rc) return rc;
    double f, F;
    objective_from(c, c->obj, lam1, lam2, &f, &F);
    if (host_f) *host_f = f;
    if (host_F) *host_F = F;
    return CONCORD_OK;
}

int concord_get_omega(concord_ctx* c, int64_t* host_nnz, int64_t* dev_row_ptr, int32_t* dev_col,
                      void* dev_val, int32_t dtype) {
    if (!c || !host_nnz) return CONCORD_EINVAL;
    *host_nnz = c->nnz;
    if (!dev_row_ptr) return CONCORD_OK;
    if (!dev_col || !dev_val) return fail(c, CONCORD_EINVAL, "col/val must be given with row_ptr");
    if (dtype != CONCORD_F64 && dtype != CONCORD_F32) return fail(c, CONCORD_EINVAL, "dtype");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    const Csr& o = c->om[c->cur];
    HIPCK(c, hipMemcpyAsync(dev_row_ptr, o.rowptr, (c->p + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToDevice, c->stream));
    HIPCK(c, hipMemcpyAsync(dev_col, o.col, c->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice,
                            c->stream));
    HIPCK(c, launch_csr_export(o.val, c->nnz, dev_val, dtype == CONCORD_F64, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return CONCORD_OK;
}

int concord_get_candidates(concord_ctx* c, int64_t* host_nnz, int64_t* dev_row_ptr,
                           int32_t* dev_col, double* dev_omega, double* dev_grad) {
    if (!c || !host_nnz) return CONCORD_EINVAL;
    if (c->a_nnz < 0) return fail(c, CONCORD_ENODATA, "no step since the iterate was set");
    *host_nnz = c->a_nnz;
    if (!dev_row_ptr) return CONCORD_OK;
    if (!dev_col || !dev_omega || !dev_grad)
        return fail(c, CONCORD_EINVAL, "col/omega/grad must be given with row_ptr");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    const size_t n = (size_t)c->a_nnz;
    HIPCK(c, hipMemcpyAsync(dev_row_ptr, c->A.rowptr, (c->p + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToDevice, c->stream));
    if (n) {
        HIPCK(c, hipMemcpyAsync(dev_col, c->A.col, n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                c->stream));
        HIPCK(c, hipMemcpyAsync(dev_omega, c->A.omega, n * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
        HIPCK(c, hipMemcpyAsync(dev_grad, c->A.grad, n * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream));
    }
    HIPCK(c, hipStreamSynchronize(c->stream));
    return CONCORD_OK;
}

int64_t concord_iterations(const concord_ctx* c) { return c ? c->k : -1; }

int concord_suggest_variant(int64_t p, int64_t n, double d, double t, double s, int32_t precision,
                            double dense_tflops, double hbm_gbps, double screen_fraction,
                            concord_variant_estimate* out) {
    if (!out || p < 1 || n < 1 || !(d >= 0.0) || !(t >= 0.0) || !(s >= 0.0)) return CONCORD_EINVAL;
    if (precision < CONCORD_FP64 || precision > CONCORD_BF16X3) return CONCORD_EINVAL;
    const double P = (double)p, N = (double)n;
    // Lemma 3.1
    out->cov_flops = 2.0 * N * P * P + 2.0 * d * P * P * (s * t + 1.0);
    out->obs_flops = 2.0 * N * P * P * s + 2.0 * d * N * P * (s * t + 1.0);
    out->paper_choice = out->cov_flops < out->obs_flops ? CONCORD_COV : CONCORD_OBS;
    // the same work priced as this library does it
    const double rate = (dense_tflops > 0.0 ? dense_tflops
                         : precision == CONCORD_BF16X3 ? 330.0
                         : precision == CONCORD_FP32 ? 125.0 : 60.0) * 1e12;
    const double bw = (hbm_gbps > 0.0 ? hbm_gbps : 3200.0) * 1e9;
    const double b = precision == CONCORD_FP64 ? 8.0 : 4.0;
    const double f = screen_fraction > 0.0 ? std::min(screen_fraction, 1.0) : 1.0;
    out->cov_seconds = N * P * P / rate + s * (f * P * P * b + 0.25 * P * P) / bw;
    out->obs_seconds = s * (2.0 * N * P * P / rate + (2.0 * P * P * b + 2.0 * P * N * b) / bw);
    out->choice = out->cov_seconds < out->obs_seconds ? CONCORD_COV : CONCORD_OBS;
    return CONCORD_OK;
}

int32_t concord_variant_of(const concord_ctx* c) { return c ? c->variant : CONCORD_EINVAL; }

int concord_measure_rates(int32_t device, int32_t precision, double* host_dense_tflops,
                          double* host_hbm_gbps) {
    if (precision < CONCORD_FP64 || precision > CONCORD_BF16X3) return CONCORD_EINVAL;
    int dev = device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return CONCORD_EHIP;
    double r[2] = {0.0, 0.0};
    const int rc = measured_rates(dev, precision, r);
    if (rc) return rc;
    if (host_dense_tflops) *host_dense_tflops = r[0];
    if (host_hbm_gbps) *host_hbm_gbps = r[1];
    return CONCORD_OK;
}

int concord_smooth_value(concord_ctx* c, double lam2, double* host_f) {
    if (!c) return CONCORD_EINVAL;
    if (c->variant != CONCORD_OBS) return fail(c, CONCORD_EINVAL, "differentiation form needs Obs");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    if (!(lam2 >= 0.0)) return fail(c, CONCORD_EINVAL, "lambda2 must be >= 0");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    // ||Omega X^T||^2 reduced per row and column chunk by the SpMM without writing Y,
    // the other sums per row, fixed-order column sums, then f on the device
    const Csr& O = c->om[c->cur];
    const int64_t p = c->p;
    const int nch = spmm_nchunks(c->dstore, c->ldk);
    HIPCK(c, launch_spmm(O, p, c->Xt, c->dstore, c->ldk, c->ldk, nullptr, c->dstore, c->ldk,
                         nullptr, nullptr, 0, c->part + 4 * p, nullptr, c->stream));
    HIPCK(c, launch_obj_parts(O, p, nullptr, c->dstore, 0, c->part, nullptr, c->stream));
    HIPCK(c, launch_colsum_obj(c->part, p, 4 + nch, c->objsums, c->colsum_ws, nch, nullptr, c->st,
                               c->stream));
    HIPCK(c, launch_smooth_finish(c->st, c->n, lam2, &c->st->fval, c->stream));
    int rc = sync_state(c);
    if (rc) return rc;
    if (host_f) *host_f = c->st_host->fval;
    return CONCORD_OK;
}

int concord_gradient(concord_ctx* c, double lam2, int32_t mode, void* dev_dOmega, void* dev_dX,
                     int32_t dtype) {
    if (!c) return CONCORD_EINVAL;
    if (c->variant != CONCORD_OBS) return fail(c, CONCORD_EINVAL, "differentiation form needs Obs");
    if (!c->has_data) return fail(c, CONCORD_ENODATA, "no data: call concord_set_data first");
    if (!(lam2 >= 0.0)) return fail(c, CONCORD_EINVAL, "lambda2 must be >= 0");
    if (mode != CONCORD_GRAD_MASKED && mode != CONCORD_GRAD_DENSE)
        return fail(c, CONCORD_EINVAL, "mode");
    if (dtype != CONCORD_F64 && dtype != CONCORD_F32) return fail(c, CONCORD_EINVAL, "dtype");
    if (c->precision == CONCORD_BF16X3)
        return fail(c, CONCORD_EINVAL, "differentiation form supports FP64 and FP32");
    DeviceGuard g(c->device);
    if (int rc0 = enter(c)) return rc0;
    const Csr& O = c->om[c->cur];
    const int out64 = dtype == CONCORD_F64;
    const int64_t p = c->p, nnz = c->nnz;
    const size_t dense_bytes = (size_t)c->prow * c->ldk * elem_bytes(c->dstore);
    // Buffers of this call only, in one block from one allocation (returned before the
    // call ends): Y when the handle holds none, Omega Y before its transpose, and the half
    // d_ij of every masked entry.
    const bool masked = dev_dOmega && mode == CONCORD_GRAD_MASKED;
    const bool need_y = !(c->prod_valid && c->Y);
    const int ncb = grad_col_blocks(c->dstore, c->n);
    auto a256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t ya = need_y && !c->Y ? a256(dense_bytes) : 0;
    const size_t oa = dev_dX ? a256(dense_bytes) : 0;
    const size_t da = masked ? a256((size_t)std::max<int64_t>(nnz, 1) * ncb * sizeof(double)) : 0;
    void* blk = nullptr;
    auto done = [&](int rc) {
        dfree(c, blk);
        return rc;
    };
    int rc;
    if (ya + oa + da && (rc = dalloc(c, &blk, ya + oa + da, false))) return rc;
    char* const base = (char*)blk;
    void* ybuf = ya ? base : nullptr;
    void* oy = oa ? base + ya : nullptr;
    double* D = da ? (double*)(base + ya + oa) : nullptr;
    // Y = Omega X^T: kept only by a solver whose products are current; otherwise
    // recomputed here (the forward pass reduces ||Y||^2 without storing Y).  Omega Y needs
    // no clearing (every column that is read is written); a fresh Y gets zero columns
    // n .. ldk - 1, which the row pass's last chunk and the dense contraction's K loop read.
    void* Y = c->Y;
    if (need_y) {
        if (!Y) {
            Y = ybuf;
            const size_t eb = elem_bytes(c->dstore);
            if (c->ldk > c->n)
                HIPCK(c, hipMemset2DAsync((char*)Y + (size_t)c->n * eb, (size_t)c->ldk * eb, 0,
                                          (size_t)(c->ldk - c->n) * eb, (size_t)p, c->stream));
        }
        HIPCK(c, launch_spmm(O, p, c->Xt, c->dstore, c->ldk, c->ldk, Y, c->dstore, c->ldk, nullptr,
                             nullptr, 0, nullptr, c->d_one, c->stream));
    }
    if (masked) {
        // the half d_ij of every entry and, when d f / d X is wanted too, Omega Y, from one
        // gather of the rows Y_j
        HIPCK(c, launch_grad_rows(O, p, nnz, Y, c->Xt, c->dstore, c->ldk, c->n, D, oy,
                                  c->stream));
        HIPCK(c, launch_grad_combine(O, p, nnz, ncb, D, c->n, lam2, dev_dOmega, out64,
                                     c->stream));
    } else {
        if (dev_dOmega) {   // dense G: the contraction of Algorithm 3 at the current iterate
            if ((rc = ensure_dense(c))) return done(rc);
            HIPCK(c, launch_gemm_sym(c->gkind, true, Y, nullptr, c->Xt, nullptr, c->ldk, p,
                                     0.5 / (double)c->n, c->M, c->dstore, c->ldp, c->stream));
            HIPCK(c, launch_gather_dense_grad(c->M, c->dstore, c->ldp, O, p, lam2, dev_dOmega,
                                              out64, c->stream));
        }
        if (dev_dX)
            HIPCK(c, launch_spmm(O, p, Y, c->dstore, c->ldk, c->ldk, oy, c->dstore, c->ldk,
                                 nullptr, nullptr, 0, nullptr, c->d_one, c->stream));
    }
    // d f / d X = (Omega Y)^T / n, written transposed (n x p)
    if (dev_dX)
        HIPCK(c, launch_transpose_out(oy, c->dstore, p, c->n, c->ldk, 1.0 / (double)c->n, dev_dX,
                                      out64, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return done(CONCORD_OK);
}

}  // extern "C"
