// concord_smooth_value_noalloc (see include/concord.h): the smooth value of the
// differentiation form for a caller's iterate and data, for callers that cannot
// allocate device memory.  Its partial sums live in `scratch`, a file-scope device array
// (one copy per device, held until the process ends); the kernels are those of
// concord_smooth_value, so the two entry points give the same value.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/concord.h"
#include "internal.h"

using namespace concord;

namespace {

static __device__ __align__(256) unsigned char scratch[CONCORD_NOALLOC_SCRATCH_BYTES];

// Device address of each device's scratch, looked up once per device with that device
// current.  In host code `scratch` names a host-side stand-in, never the device memory.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

hipError_t device_scratch(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// the column-sum launch counts finished blocks from zero
__global__ void ticket_reset_kernel(DevState* st) {
    if (threadIdx.x == 0) st->ticket = 0u;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int concord_smooth_value_noalloc(int64_t p, int64_t n, const void* dev_Xt, int64_t ldx,
                                            int32_t dtype, int64_t nnz, const int64_t* dev_row_ptr,
                                            const int32_t* dev_col, const double* dev_val,
                                            double lambda2, double* dev_f, void* stream) {
    if (p < 1 || n < 1 || nnz < p || !dev_Xt || !dev_row_ptr || !dev_col || !dev_val || !dev_f)
        return CONCORD_EINVAL;
    if (dtype != CONCORD_F64 && dtype != CONCORD_F32) return CONCORD_EINVAL;
    if (!(lambda2 >= 0.0) || !std::isfinite(lambda2)) return CONCORD_EINVAL;
    const int store = dtype == CONCORD_F64 ? ST_F64 : ST_F32;
    const int64_t vw = dtype == CONCORD_F64 ? 2 : 4;   // elements per 16-byte chunk load
    if (ldx < n || ldx % vw != 0 || ((uintptr_t)dev_Xt & 15) != 0) return CONCORD_EINVAL;
    // scratch layout: state | objective sums | segment sums | per-row partials
    const int nch = spmm_nchunks(store, n);
    const size_t o_sums = align256(sizeof(DevState));
    const size_t o_ws = o_sums + align256(sizeof(double) * (size_t)(64 + nch));
    const size_t o_part = o_ws + align256(sizeof(double) * (size_t)(4 + nch) * COLSUM_MAXSEG);
    const size_t need = o_part + sizeof(double) * (size_t)(4 + nch) * (size_t)p;
    if (need > (size_t)CONCORD_NOALLOC_SCRATCH_BYTES) return CONCORD_EINVAL;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CONCORD_EHIP;
    unsigned char* base = nullptr;
    if (device_scratch(dev, &base) != hipSuccess) return CONCORD_EHIP;
    DevState* st = (DevState*)base;
    double* sums = (double*)(base + o_sums);
    double* ws = (double*)(base + o_ws);
    double* part = (double*)(base + o_part);
    hipStream_t s = (hipStream_t)stream;

    // the iterate's arrays as the kernels read them (read only; the cast drops const)
    Csr O{const_cast<int64_t*>(dev_row_ptr), const_cast<int32_t*>(dev_col),
          const_cast<double*>(dev_val)};
    hipLaunchKernelGGL(ticket_reset_kernel, dim3(1), dim3(64), 0, s, st);
    if (hipGetLastError() != hipSuccess ||
        launch_spmm(O, p, dev_Xt, store, ldx, n, nullptr, store, ldx, nullptr, nullptr, 0,
                    part + 4 * p, nullptr, s) != hipSuccess ||
        launch_obj_parts(O, p, nullptr, store, 0, part, nullptr, s) != hipSuccess ||
        launch_colsum_obj(part, p, 4 + nch, sums, ws, nch, nullptr, st, s) != hipSuccess ||
        launch_smooth_finish(st, n, lambda2, dev_f, s) != hipSuccess)
        return CONCORD_EHIP;
    return CONCORD_OK;
}
