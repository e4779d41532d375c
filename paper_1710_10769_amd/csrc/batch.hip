// Batched lambda path over independent Cov problems (see include/concord.h).
//
// Each instance keeps its own handle (its S formed once on the GPU from X);
// every lambda1 of the path is solved from Omega = I with the single-problem
// solver, and the estimate is kept in batch-owned CSR buffers.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/concord.h"

struct BatchResult {
    int64_t nnz = 0;
    int64_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

struct concord_batch {
    int count = 0, n_l1 = 0;
    std::vector<concord_ctx*> ctx;
    std::vector<double> lambda1;
    std::vector<int64_t> p;
    std::vector<BatchResult> res;
    hipStream_t stream = nullptr;
    std::string err;
};

namespace {
int bfail(concord_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}
void free_result(BatchResult& r) {
    if (r.rowptr) hipFree(r.rowptr);
    if (r.col) hipFree(r.col);
    if (r.val) hipFree(r.val);
    r = BatchResult();
}
}  // namespace

extern "C" {

void concord_batch_destroy(concord_batch* b) {
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    for (auto* c : b->ctx) concord_destroy(c);
    for (auto& r : b->res) free_result(r);
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
    concord_batch* b = new concord_batch();
    b->count = count;
    b->n_l1 = n_l1;
    b->stream = (hipStream_t)stream;
    b->lambda1.assign(host_lambda1, host_lambda1 + n_l1);
    b->res.resize((size_t)count * n_l1);
    for (int i = 0; i < count; ++i) {
        concord_config cfg;
        concord_config_init(&cfg);
        cfg.p = host_p[i];
        cfg.n = host_n[i];
        cfg.variant = CONCORD_COV;
        cfg.precision = CONCORD_FP32;
        cfg.stream = stream;
        concord_ctx* c = nullptr;
        int rc = concord_create(&cfg, &c);
        if (rc) {
            concord_batch_destroy(b);
            return rc;
        }
        b->ctx.push_back(c);
        b->p.push_back(host_p[i]);
        rc = concord_set_data(c, CONCORD_DATA_X, host_dev_X[i], CONCORD_F32, host_n[i], host_p[i],
                              host_ld[i]);
        if (rc) {
            concord_batch_destroy(b);
            return rc;
        }
    }
    *out = b;
    return CONCORD_OK;
}

int concord_batch_solve(concord_batch* b, double lambda2, double tol, int64_t max_iter,
                        int64_t* host_iters, double* host_F) {
    if (!b) return CONCORD_EINVAL;
    if (!(lambda2 >= 0.0) || !(tol >= 0.0) || max_iter < 0)
        return bfail(b, CONCORD_EINVAL, "lambda2, tol must be >= 0");
    int worst = CONCORD_OK;
    for (int i = 0; i < b->count; ++i) {
        concord_ctx* c = b->ctx[i];
        for (int l = 0; l < b->n_l1; ++l) {
            int rc = concord_reset(c);
            if (rc) return bfail(b, rc, concord_last_error(c));
            concord_solve_info si;
            rc = concord_solve(c, b->lambda1[l], lambda2, tol, max_iter, &si);
            if (rc < 0) return bfail(b, rc, concord_last_error(c));
            if (rc > worst) worst = rc;
            BatchResult& r = b->res[(size_t)i * b->n_l1 + l];
            int64_t nnz = 0;
            concord_get_omega(c, &nnz, nullptr, nullptr, nullptr, CONCORD_F64);
            if (nnz > r.nnz || !r.rowptr) {
                free_result(r);
                if (hipMalloc((void**)&r.rowptr, (b->p[i] + 1) * sizeof(int64_t)) != hipSuccess ||
                    hipMalloc((void**)&r.col, nnz * sizeof(int32_t)) != hipSuccess ||
                    hipMalloc((void**)&r.val, nnz * sizeof(double)) != hipSuccess)
                    return bfail(b, CONCORD_ENOMEM, "result allocation failed");
            }
            rc = concord_get_omega(c, &nnz, r.rowptr, r.col, r.val, CONCORD_F64);
            if (rc) return bfail(b, rc, concord_last_error(c));
            r.nnz = nnz;
            if (host_iters) host_iters[(size_t)i * b->n_l1 + l] = si.iters;
            if (host_F) host_F[(size_t)i * b->n_l1 + l] = si.F;
        }
    }
    return worst;
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
    hipMemcpyAsync(dev_row_ptr, r.rowptr, (b->p[instance] + 1) * sizeof(int64_t),
                   hipMemcpyDeviceToDevice, b->stream);
    hipMemcpyAsync(dev_col, r.col, r.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, b->stream);
    hipMemcpyAsync(dev_val, r.val, r.nnz * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, CONCORD_EHIP, "copy failed");
    return CONCORD_OK;
}

}  // extern "C"
