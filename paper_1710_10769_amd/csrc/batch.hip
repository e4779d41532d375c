// Batched lambda path over independent Cov problems (see include/concord.h).
//
// Execution: a pool of worker threads, each with its own HIP stream (default
// priority) on the batch's device, pulls instances from a shared queue ordered
// by decreasing p (largest first, so the tail of the batch is short).  A worker
// forms S = X^T X / n once per instance (MFMA), then solves every lambda1 of
// the path from Omega = I with the single-problem solver on its stream, and
// copies each estimate into batch-owned CSR buffers.  Independent instances
// thus overlap on the GPU instead of serialising on launch latency and on the
// host synchronisation of each step.  A worker keeps its solver handles for the
// whole call, one per (p, n) it has met, and loads the next instance of the same
// shape into the same handle: no device allocation or free (a free waits for
// every stream of the device) between instances of one shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/concord.h"

struct BatchResult {
    int64_t nnz = 0;
    int64_t cap = 0;
    int64_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    int64_t iters = 0;
    double F = 0.0;
};

struct concord_batch {
    int count = 0, n_l1 = 0;
    int device = 0;
    std::vector<int64_t> p, n, ld;
    std::vector<const void*> X;
    std::vector<double> lambda1;
    std::vector<BatchResult> res;
    hipStream_t stream = nullptr;   // caller's stream (result copies)
    int workers = 8;
    std::string err;
};

namespace {
int bfail(concord_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}
void free_result(BatchResult& r) {
    if (r.rowptr) (void)hipFree(r.rowptr);
    if (r.col) (void)hipFree(r.col);
    if (r.val) (void)hipFree(r.val);
    r = BatchResult();
}

// A worker's solver handles, one per problem shape.
struct HandlePool {
    struct Entry {
        int64_t p, n;
        concord_ctx* c;
    };
    std::vector<Entry> e;
    ~HandlePool() {
        for (auto& x : e) concord_destroy(x.c);
    }
};

// One instance, every lambda1, on `stream`, in the worker's handle of that shape
// (created on first use).  Returns a status and a message.
int solve_instance(concord_batch* b, int i, hipStream_t stream, double lam2, double tol,
                   int64_t max_iter, std::string* msg, HandlePool& pool) {
    concord_ctx* c = nullptr;
    for (auto& x : pool.e)
        if (x.p == b->p[i] && x.n == b->n[i]) c = x.c;
    if (!c) {
        concord_config cfg;
        concord_config_init(&cfg);
        cfg.p = b->p[i];
        cfg.n = b->n[i];
        cfg.variant = CONCORD_COV;
        cfg.precision = CONCORD_FP32;
        cfg.stream = stream;
        cfg.device = b->device;
        const int rc0 = concord_create(&cfg, &c);
        if (rc0) {
            *msg = "concord_create failed for instance " + std::to_string(i);
            return rc0;
        }
        pool.e.push_back({b->p[i], b->n[i], c});
    }
    // set_data starts the instance from Omega = I with k = 0
    int rc = concord_set_data(c, CONCORD_DATA_X, b->X[i], CONCORD_F32, b->n[i], b->p[i], b->ld[i]);
    int worst = CONCORD_OK;
    for (int l = 0; rc >= 0 && l < b->n_l1; ++l) {
        if ((rc = concord_reset(c))) break;
        concord_solve_info si;
        rc = concord_solve(c, b->lambda1[l], lam2, tol, max_iter, &si);
        if (rc < 0) break;
        worst = std::max(worst, rc);
        BatchResult& r = b->res[(size_t)i * b->n_l1 + l];
        int64_t nnz = 0;
        concord_get_omega(c, &nnz, nullptr, nullptr, nullptr, CONCORD_F64);
        if (!r.rowptr || nnz > r.cap) {
            free_result(r);
            if (hipMalloc((void**)&r.rowptr, (b->p[i] + 1) * sizeof(int64_t)) != hipSuccess ||
                hipMalloc((void**)&r.col, std::max<int64_t>(nnz, 1) * sizeof(int32_t)) != hipSuccess ||
                hipMalloc((void**)&r.val, std::max<int64_t>(nnz, 1) * sizeof(double)) != hipSuccess) {
                rc = CONCORD_ENOMEM;
                break;
            }
            r.cap = nnz;
        }
        rc = concord_get_omega(c, &nnz, r.rowptr, r.col, r.val, CONCORD_F64);
        if (rc) break;
        r.nnz = nnz;
        r.iters = si.iters;
        r.F = si.F;
        rc = CONCORD_OK;
    }
    if (rc < 0) *msg = std::string("instance ") + std::to_string(i) + ": " + concord_last_error(c);
    return rc < 0 ? rc : worst;
}
}  // namespace

extern "C" {

void concord_batch_destroy(concord_batch* b) {
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& r : b->res) free_result(r);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete b;
}

const char* concord_batch_last_error(const concord_batch* b) {
    return b ? b->err.c_str() : "null handle";
}

int concord_batch_create(int32_t count, const int64_t* host_p, const int64_t* host_n,
                         const void* const* host_dev_X, const int64_t* host_ld, int32_t n_l1,
                         const double* host_lambda1, void* stream, concord_batch** out) {
    if (!out) return CONCORD_EINVAL;
    *out = nullptr;
    if (count < 1 || n_l1 < 1 || !host_p || !host_n || !host_dev_X || !host_ld || !host_lambda1)
        return CONCORD_EINVAL;
    for (int l = 0; l < n_l1; ++l)
        if (!(host_lambda1[l] >= 0.0)) return CONCORD_EINVAL;
    for (int i = 0; i < count; ++i)
        if (host_p[i] < 1 || host_n[i] < 1 || host_ld[i] < host_p[i] || !host_dev_X[i])
            return CONCORD_EINVAL;
    concord_batch* b = new concord_batch();
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return CONCORD_EHIP;
    }
    b->count = count;
    b->n_l1 = n_l1;
    b->stream = (hipStream_t)stream;
    b->p.assign(host_p, host_p + count);
    b->n.assign(host_n, host_n + count);
    b->ld.assign(host_ld, host_ld + count);
    b->X.assign(host_dev_X, host_dev_X + count);
    b->lambda1.assign(host_lambda1, host_lambda1 + n_l1);
    b->res.resize((size_t)count * n_l1);
    if (const char* w = std::getenv("CONCORD_BATCH_WORKERS")) b->workers = std::max(1, atoi(w));
    // the inputs were produced on the caller's stream: make them visible to the workers' streams
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        delete b;
        return CONCORD_EHIP;
    }
    *out = b;
    return CONCORD_OK;
}

int concord_batch_solve(concord_batch* b, double lambda2, double tol, int64_t max_iter,
                        int64_t* host_iters, double* host_F) {
    if (!b) return CONCORD_EINVAL;
    if (!(lambda2 >= 0.0) || !(tol >= 0.0) || max_iter < 0)
        return bfail(b, CONCORD_EINVAL, "lambda2, tol must be >= 0");
    std::vector<int> order(b->count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->p[a] > b->p[c]; });
    std::atomic<int> next(0);
    std::mutex mu;
    int status = CONCORD_OK;
    std::string first_err;
    auto worker = [&]() {
        (void)hipSetDevice(b->device);
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            std::lock_guard<std::mutex> g(mu);
            if (status >= 0) { status = CONCORD_EHIP; first_err = "stream creation failed"; }
            return;
        }
        {
            HandlePool pool;   // destroyed before the stream its handles use
            for (;;) {
                {
                    std::lock_guard<std::mutex> g(mu);
                    if (status < 0) break;
                }
                const int k = next.fetch_add(1);
                if (k >= b->count) break;
                std::string msg;
                const int rc = solve_instance(b, order[k], s, lambda2, tol, max_iter, &msg, pool);
                std::lock_guard<std::mutex> g(mu);
                if (rc < 0 && status >= 0) { status = rc; first_err = msg; }
                else if (rc > status && status >= 0) status = rc;
            }
            (void)hipStreamSynchronize(s);
        }
        (void)hipStreamDestroy(s);
    };
    const int nw = std::min(b->workers, b->count);
    std::vector<std::thread> pool;
    for (int t = 0; t < nw; ++t) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
    if (status < 0) return bfail(b, status, first_err);
    for (int i = 0; i < b->count; ++i)
        for (int l = 0; l < b->n_l1; ++l) {
            const BatchResult& r = b->res[(size_t)i * b->n_l1 + l];
            if (host_iters) host_iters[(size_t)i * b->n_l1 + l] = r.iters;
            if (host_F) host_F[(size_t)i * b->n_l1 + l] = r.F;
        }
    return status;
}

int concord_batch_get_omega(concord_batch* b, int32_t instance, int32_t l1_index,
                            int64_t* host_nnz, int64_t* dev_row_ptr, int32_t* dev_col,
                            double* dev_val) {
    if (!b || !host_nnz) return CONCORD_EINVAL;
    if (instance < 0 || instance >= b->count || l1_index < 0 || l1_index >= b->n_l1)
        return bfail(b, CONCORD_EINVAL, "index out of range");
    const BatchResult& r = b->res[(size_t)instance * b->n_l1 + l1_index];
    *host_nnz = r.nnz;
    if (!dev_row_ptr) return CONCORD_OK;
    if (!r.rowptr) return bfail(b, CONCORD_ENODATA, "not solved yet");
    if (!dev_col || !dev_val) return bfail(b, CONCORD_EINVAL, "col/val must be given with row_ptr");
    if (hipMemcpyAsync(dev_row_ptr, r.rowptr, (b->p[instance] + 1) * sizeof(int64_t),
                       hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(dev_col, r.col, r.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync(dev_val, r.val, r.nnz * sizeof(double), hipMemcpyDeviceToDevice,
                       b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, CONCORD_EHIP, "copy failed");
    return CONCORD_OK;
}

}  // extern "C"
