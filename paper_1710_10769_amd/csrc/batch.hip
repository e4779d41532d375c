// Batched lambda path over independent Cov problems (see include/concord.h).
//
// All solves live on the device at once.  Per solve: its CSR iterates, candidate set,
// bitmap, partial sums, DevState and SolveCtl (iteration, phase, step-size index,
// objective, status); per instance: S, its tile maxima and the list of tile pairs its
// solves keep in a refresh.  One iteration of every running solve is a fixed sequence
// of launches (launch_batch_iteration) whose kernels read the per-solve control from
// device memory, so iterations_per_launch of them are captured once as a HIP graph and
// replayed until no solve runs; the host reads two counters after each replay and steps
// in only to grow a solve's candidate arrays.  The device memory is one arena (through
// the caller's allocator bridge when configured), carved per instance and per solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/concord.h"
#include "internal.h"

using namespace concord;

namespace {

constexpr int MAXQ_B = 8;    // step sizes per trial batch at most (the trial kernels' MAXQ)
constexpr int NSIDE = 4;     // streams forming the instances' S concurrently
constexpr int GRID_MAX = 2048;   // blocks of a phase kernel at most (they loop over work items)

struct Block {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// byte layout of the arena: every region 256-byte aligned
struct Layout {
    size_t bytes = 0;
    size_t add(size_t b) {
        const size_t at = bytes;
        bytes += (b + 255) / 256 * 256;
        return at;
    }
};

}  // namespace

struct concord_batch {
    concord_batch_config cfg;
    int device = 0;
    hipStream_t user = nullptr;     // caller's stream
    hipStream_t work = nullptr;     // the batch's own stream (graphs are captured on it)
    hipStream_t side[NSIDE] = {};
    hipEvent_t ev_fork = nullptr, ev_join[NSIDE] = {};
    int count = 0, n_l1 = 0, nsolve = 0;
    int sstore = ST_F32, dstore = ST_F32, gkind = GK_F32;
    int maxT = 1;
    int grid = 64;                  // blocks of every phase kernel: the row blocks of all solves, capped
    std::vector<int64_t> p, n, ld;
    std::vector<const void*> X;
    std::vector<double> lambda1;
    std::vector<Block> blocks;      // every device allocation
    unsigned char* arena = nullptr;
    std::vector<SolveDesc> hsd;
    std::vector<InstDesc> hid;
    std::vector<int64_t> om_cap;    // capacity of each solve's CSR and candidate arrays
    std::vector<char> own_arrays;   // 1: the solve's arrays were regrown (separate blocks)
    SolveDesc* dsd = nullptr;
    InstDesc* did = nullptr;
    SolveCtl* dctl = nullptr;
    DevState* dst = nullptr;
    int* dflag = nullptr;           // NSIDE non-finite flags of the S formation
    BatchPlan plan = {};
    int* hstatus = nullptr;         // pinned copy of plan.status
    std::vector<SolveCtl> hctl;
    bool s_ready = false;
    hipGraphExec_t gexec = nullptr;
    BatchArgs gargs = {};
    int g_iters = 0;
    concord_batch_stats stats = {};
    std::string err;
};

namespace {

int bfail(concord_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}

#define BHIP(b, expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bfail(b, e_ == hipErrorOutOfMemory ? CONCORD_ENOMEM : CONCORD_EHIP,   \
                         std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

int balloc(concord_batch* b, void** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (b->cfg.alloc_fn) {
        *out = b->cfg.alloc_fn(b->cfg.alloc_user, bytes, (void*)b->work);
        if (!*out) return bfail(b, CONCORD_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else if (hipMalloc(out, bytes) != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return bfail(b, CONCORD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b->blocks.push_back(Block{*out, bytes});
    return CONCORD_OK;
}

void bfree(concord_batch* b, void* ptr) {
    if (!ptr) return;
    for (auto& blk : b->blocks)
        if (blk.ptr == ptr) {
            (void)hipStreamSynchronize(b->work);
            if (b->cfg.free_fn) b->cfg.free_fn(b->cfg.alloc_user, blk.ptr, blk.bytes, (void*)b->work);
            else (void)hipFree(blk.ptr);
            blk.ptr = nullptr;
        }
}

int64_t tiles(int64_t p) { return (p + 63) / 64; }

// The instances' S (and tile maxima) on NSIDE streams, largest first: transpose X into a
// zeroed variable-major scratch, the symmetric rank-n product on MFMA, the tile maxima.
int form_s(concord_batch* b) {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t eb = b->dstore == ST_F64 ? 8 : 4;
    const bool split = b->gkind == GK_BF16X3;   // BF16 hi/lo planes of X^T for the product
    size_t xt_elems = 0;
    for (int i = 0; i < b->count; ++i)
        xt_elems = std::max(xt_elems, (size_t)round_up(b->p[i], ROW_PAD) *
                                          (size_t)round_up(b->n[i], K_PAD));
    void* xt[NSIDE] = {};
    void* xh[NSIDE] = {};
    void* xl[NSIDE] = {};
    auto release = [&]() {
        for (int s = 0; s < NSIDE; ++s) {
            bfree(b, xt[s]);
            bfree(b, xh[s]);
            bfree(b, xl[s]);
        }
    };
    int rc;
    for (int s = 0; s < NSIDE; ++s)
        if ((rc = balloc(b, &xt[s], xt_elems * eb)) ||
            (split && ((rc = balloc(b, &xh[s], xt_elems * 2)) || (rc = balloc(b, &xl[s], xt_elems * 2))))) {
            release();
            return rc;
        }
    std::vector<int> order(b->count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->p[a] > b->p[c]; });
    BHIP(b, hipMemsetAsync(b->dflag, 0, NSIDE * sizeof(int), b->work));
    BHIP(b, hipEventRecord(b->ev_fork, b->work));
    for (int s = 0; s < NSIDE; ++s) BHIP(b, hipStreamWaitEvent(b->side[s], b->ev_fork, 0));
    for (int k = 0; k < b->count; ++k) {
        const int i = order[k], s = k % NSIDE;
        hipStream_t st = b->side[s];
        const int64_t p = b->p[i], n = b->n[i];
        const int64_t ldk = round_up(n, K_PAD), prow = round_up(p, ROW_PAD);
        const InstDesc& id = b->hid[i];
        const SolveDesc& d0 = b->hsd[id.first];
        const size_t ne = (size_t)prow * ldk;
        BHIP(b, hipMemsetAsync(xt[s], 0, ne * eb, st));
        if (split) {
            BHIP(b, hipMemsetAsync(xh[s], 0, ne * 2, st));
            BHIP(b, hipMemsetAsync(xl[s], 0, ne * 2, st));
        }
        BHIP(b, launch_transpose_in(b->X[i], b->dstore == ST_F64, n, p, b->ld[i], xt[s], b->dstore,
                                    ldk, (uint16_t*)xh[s], (uint16_t*)xl[s], kblk_stride(prow),
                                    b->dflag + s, st));
        // the first contraction of a shape times the tile variants (events on its stream):
        // the other streams are drained first so that their kernels do not share the chip
        // with the timed runs
        if (b->gkind != GK_F64 && gemm_sym_choice(b->gkind, false, p, ldk, nullptr) < 0)
            for (int o = 0; o < NSIDE; ++o)
                if (o != s) BHIP(b, hipStreamSynchronize(b->side[o]));
        BHIP(b, launch_gemm_sym(b->gkind, false, split ? xh[s] : xt[s], split ? xl[s] : nullptr,
                                nullptr, nullptr, ldk, p, 1.0 / (double)n,
                                const_cast<void*>(d0.S), b->sstore, d0.lds, st));
        BHIP(b, launch_tile_max(d0.S, b->sstore, p, d0.lds, const_cast<double*>(d0.smax), st));
    }
    for (int s = 0; s < NSIDE; ++s) {
        BHIP(b, hipEventRecord(b->ev_join[s], b->side[s]));
        BHIP(b, hipStreamWaitEvent(b->work, b->ev_join[s], 0));
    }
    int hflag[NSIDE] = {};
    BHIP(b, hipMemcpyAsync(hflag, b->dflag, sizeof(hflag), hipMemcpyDeviceToHost, b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    release();
    for (int s = 0; s < NSIDE; ++s)
        if (hflag[s]) return bfail(b, CONCORD_ENONFINITE, "data holds NaN or Inf");
    b->s_ready = true;
    b->stats.s_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return CONCORD_OK;
}

// Grow the candidate (and iterate) arrays of the solves that asked for more: their
// current iterate is copied over; the descriptors on the device are updated.
int regrow(concord_batch* b) {
    std::vector<DevState> st(b->nsolve);
    BHIP(b, hipMemcpyAsync(b->hctl.data(), b->dctl, b->nsolve * sizeof(SolveCtl),
                           hipMemcpyDeviceToHost, b->work));
    BHIP(b, hipMemcpyAsync(st.data(), b->dst, b->nsolve * sizeof(DevState), hipMemcpyDeviceToHost,
                           b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    int rc;
    for (int s = 0; s < b->nsolve; ++s) {
        SolveCtl& c = b->hctl[s];
        if (!c.grow) continue;
        SolveDesc& d = b->hsd[s];
        const int64_t need = st[s].n_cand;
        const int64_t cap = need + need / 2 + 1024;
        void *acol, *aom, *agr, *c0, *v0, *c1, *v1;
        if ((rc = balloc(b, &acol, cap * 4)) || (rc = balloc(b, &aom, cap * 8)) ||
            (rc = balloc(b, &agr, cap * 8)) || (rc = balloc(b, &c0, cap * 4)) ||
            (rc = balloc(b, &v0, cap * 8)) || (rc = balloc(b, &c1, cap * 4)) ||
            (rc = balloc(b, &v1, cap * 8)))
            return rc;
        const int64_t old = b->om_cap[s];
        void* nc[2] = {c0, c1};
        void* nv[2] = {v0, v1};
        BHIP(b, hipMemcpyAsync(nc[c.cur], d.om[c.cur].col, old * 4, hipMemcpyDeviceToDevice, b->work));
        BHIP(b, hipMemcpyAsync(nv[c.cur], d.om[c.cur].val, old * 8, hipMemcpyDeviceToDevice, b->work));
        if (b->own_arrays[s]) {
            bfree(b, d.A.col); bfree(b, d.A.omega); bfree(b, d.A.grad);
            for (int w = 0; w < 2; ++w) { bfree(b, d.om[w].col); bfree(b, d.om[w].val); }
        }
        d.A.col = (int32_t*)acol;
        d.A.omega = (double*)aom;
        d.A.grad = (double*)agr;
        for (int w = 0; w < 2; ++w) {
            d.om[w].col = (int32_t*)nc[w];
            d.om[w].val = (double*)nv[w];
        }
        d.a_cap = cap;
        b->om_cap[s] = cap;
        b->own_arrays[s] = 1;
        c.grow = 0;
        b->stats.regrows += 1;
    }
    BHIP(b, hipMemcpyAsync(b->dsd, b->hsd.data(), b->nsolve * sizeof(SolveDesc),
                           hipMemcpyHostToDevice, b->work));
    BHIP(b, hipMemcpyAsync(b->dctl, b->hctl.data(), b->nsolve * sizeof(SolveCtl),
                           hipMemcpyHostToDevice, b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    return CONCORD_OK;
}

}  // namespace

extern "C" {

void concord_batch_config_init(concord_batch_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->precision = CONCORD_FP32;
    cfg->device = -1;
    cfg->max_backtracks = 60;
    cfg->trial_batch = 8;
    cfg->tau0 = 1.0;
    cfg->shrink = 0.5;
    cfg->iters_per_launch = 4;
    cfg->use_graph = 1;
}

void concord_batch_destroy(concord_batch* b) {
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    if (b->work) (void)hipStreamSynchronize(b->work);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (auto& blk : b->blocks)
        if (blk.ptr) {
            if (b->cfg.free_fn) b->cfg.free_fn(b->cfg.alloc_user, blk.ptr, blk.bytes, (void*)b->work);
            else (void)hipFree(blk.ptr);
        }
    if (b->hstatus) (void)hipHostFree(b->hstatus);
    for (int s = 0; s < NSIDE; ++s) {
        if (b->side[s]) (void)hipStreamDestroy(b->side[s]);
        if (b->ev_join[s]) (void)hipEventDestroy(b->ev_join[s]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->work) (void)hipStreamDestroy(b->work);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete b;
}

const char* concord_batch_last_error(const concord_batch* b) {
    return b ? b->err.c_str() : "null handle";
}

int concord_batch_stats_get(const concord_batch* b, concord_batch_stats* out) {
    if (!b || !out) return CONCORD_EINVAL;
    *out = b->stats;
    return CONCORD_OK;
}

int concord_batch_create(const concord_batch_config* cfg_in, int32_t count, const int64_t* host_p,
                         const int64_t* host_n, const void* const* host_dev_X,
                         const int64_t* host_ld, int32_t n_l1, const double* host_lambda1,
                         concord_batch** out) {
    if (!out) return CONCORD_EINVAL;
    *out = nullptr;
    concord_batch_config cfg;
    if (cfg_in) cfg = *cfg_in;
    else concord_batch_config_init(&cfg);
    if (count < 1 || n_l1 < 1 || !host_p || !host_n || !host_dev_X || !host_ld || !host_lambda1)
        return CONCORD_EINVAL;
    if (cfg.precision != CONCORD_FP32 && cfg.precision != CONCORD_FP64 &&
        cfg.precision != CONCORD_BF16X3)
        return CONCORD_EINVAL;
    if (cfg.trial_batch < 1 || cfg.trial_batch > MAXQ_B || cfg.max_backtracks < 0 ||
        cfg.max_backtracks > 1000 || cfg.iters_per_launch < 1 || cfg.iters_per_launch > 64)
        return CONCORD_EINVAL;
    if (!(cfg.tau0 > 0.0) || !(cfg.shrink > 0.0 && cfg.shrink < 1.0)) return CONCORD_EINVAL;
    if ((cfg.alloc_fn == nullptr) != (cfg.free_fn == nullptr)) return CONCORD_EINVAL;
    for (int l = 0; l < n_l1; ++l)
        if (!(host_lambda1[l] >= 0.0)) return CONCORD_EINVAL;
    for (int i = 0; i < count; ++i)
        if (host_p[i] < 1 || host_p[i] > (int64_t)1 << 24 || host_n[i] < 1 ||
            host_ld[i] < host_p[i] || !host_dev_X[i])
            return CONCORD_EINVAL;
    if ((int64_t)count * n_l1 > (1 << 20)) return CONCORD_EINVAL;

    concord_batch* b = new concord_batch();
    b->cfg = cfg;
    int dev = cfg.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        delete b;
        return CONCORD_EHIP;
    }
    b->device = dev;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
    auto bail = [&](int rc) {
        concord_batch_destroy(b);
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    };
    b->user = (hipStream_t)cfg.stream;
    if (hipStreamCreateWithFlags(&b->work, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess)
        return bail(CONCORD_EHIP);
    for (int s = 0; s < NSIDE; ++s)
        if (hipStreamCreateWithFlags(&b->side[s], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_join[s], hipEventDisableTiming) != hipSuccess)
            return bail(CONCORD_EHIP);
    if (hipHostMalloc((void**)&b->hstatus, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return bail(CONCORD_ENOMEM);
    b->count = count;
    b->n_l1 = n_l1;
    b->nsolve = count * n_l1;
    // the single solver's stores: X^T in FP64 or FP32, S in FP64, FP32 or BF16 hi/lo pairs
    const bool f64 = cfg.precision == CONCORD_FP64;
    const bool split = cfg.precision == CONCORD_BF16X3;
    b->dstore = f64 ? ST_F64 : ST_F32;
    b->sstore = f64 ? ST_F64 : (split ? ST_B16P : ST_F32);
    b->gkind = f64 ? GK_F64 : (split ? GK_BF16X3 : GK_F32);
    b->p.assign(host_p, host_p + count);
    b->n.assign(host_n, host_n + count);
    b->ld.assign(host_ld, host_ld + count);
    b->X.assign(host_dev_X, host_dev_X + count);
    b->lambda1.assign(host_lambda1, host_lambda1 + n_l1);

    // ---- arena layout ----
    const int N = b->nsolve;
    const size_t sb = f64 ? 8 : 4;
    Layout L;
    struct InstOff { size_t S, smax, ulist, ucount, ubits; };
    struct SolveOff {
        size_t rp0, rp1, c0, v0, c1, v1, arp, acol, aom, agr, cnt, bitmap, part, tsums, osums,
               colws, scanws, lcnt, lK, lW, lcmax, plist, pcount, tmask;
    };
    std::vector<InstOff> io(count);
    std::vector<SolveOff> so(N);
    b->om_cap.assign(N, 0);
    b->own_arrays.assign(N, 0);
    for (int i = 0; i < count; ++i) {
        const int64_t p = b->p[i], T = tiles(p), nt = T * (T + 1) / 2;
        b->maxT = std::max<int>(b->maxT, (int)T);
        io[i].S = L.add((size_t)p * round_up(p, 64) * sb);
        io[i].smax = L.add((size_t)T * T * 8);
        io[i].ulist = L.add((size_t)nt * 4);
        io[i].ucount = L.add(4);
        io[i].ubits = L.add((size_t)((nt + 31) / 32) * 4);
        for (int l = 0; l < n_l1; ++l) {
            const int s = i * n_l1 + l;
            const int64_t cap = 8 * p + 1024, nw = T;
            b->om_cap[s] = cap;
            SolveOff& o = so[s];
            o.rp0 = L.add((p + 1) * 8); o.rp1 = L.add((p + 1) * 8);
            o.c0 = L.add(cap * 4); o.v0 = L.add(cap * 8); o.c1 = L.add(cap * 4); o.v1 = L.add(cap * 8);
            o.arp = L.add((p + 1) * 8); o.acol = L.add(cap * 4); o.aom = L.add(cap * 8);
            o.agr = L.add(cap * 8); o.cnt = L.add((p + 1) * 8);
            o.bitmap = L.add((size_t)p * nw * 8);
            o.part = L.add((size_t)(4 * MAXQ_B + 4) * p * 8);
            o.tsums = L.add(64 * 8); o.osums = L.add(64 * 8);
            o.colws = L.add((size_t)4 * MAXQ_B * COLSUM_MAXSEG * 8);
            o.scanws = L.add((size_t)scan_ws_len(p) * 8);
            o.lcnt = L.add(T * 4); o.lK = L.add(T * 64 * 4); o.lW = L.add(T * 64 * 8);
            o.lcmax = L.add(T * 4); o.plist = L.add(nt * 4); o.pcount = L.add(4);
            o.tmask = L.add((size_t)T * ((T + 63) / 64) * 8);
        }
    }
    int64_t row_blocks = 0;
    for (int i = 0; i < count; ++i) row_blocks += (int64_t)n_l1 * ((b->p[i] + 3) / 4);
    b->grid = (int)std::min<int64_t>(GRID_MAX, std::max<int64_t>(64, row_blocks));
    const size_t o_st = L.add((size_t)N * sizeof(DevState));
    const size_t o_ctl = L.add((size_t)N * sizeof(SolveCtl));
    const size_t o_act = L.add((size_t)N * 4);
    const size_t o_off = L.add((size_t)BP_N * (N + 1) * 4);
    const size_t o_roff = L.add((size_t)(count + 1) * 4);
    const size_t o_status = L.add(4 * 4);
    const size_t o_sd = L.add((size_t)N * sizeof(SolveDesc));
    const size_t o_id = L.add((size_t)count * sizeof(InstDesc));
    const size_t o_flag = L.add(NSIDE * 4);
    void* arena = nullptr;
    int rc;
    if ((rc = balloc(b, &arena, L.bytes))) return bail(rc);
    b->arena = (unsigned char*)arena;
    if (hipMemsetAsync(arena, 0, L.bytes, b->work) != hipSuccess) return bail(CONCORD_EHIP);
    unsigned char* A = b->arena;
    b->dst = (DevState*)(A + o_st);
    b->dctl = (SolveCtl*)(A + o_ctl);
    b->dsd = (SolveDesc*)(A + o_sd);
    b->did = (InstDesc*)(A + o_id);
    b->dflag = (int*)(A + o_flag);
    b->plan.act = (int*)(A + o_act);
    b->plan.off = (int*)(A + o_off);
    b->plan.roff = (int*)(A + o_roff);
    b->plan.status = (int*)(A + o_status);
    b->hsd.resize(N);
    b->hid.resize(count);
    b->hctl.assign(N, SolveCtl{});
    for (int i = 0; i < count; ++i) {
        const int64_t p = b->p[i], T = tiles(p);
        InstDesc& id = b->hid[i];
        id.T = (int)T;
        id.nsolve = n_l1;
        id.first = i * n_l1;
        id.screen = T >= 8 ? 1 : 0;   // as the single solver: no screening below 8 tile rows
        id.ulist = (int*)(A + io[i].ulist);
        id.ucount = (int*)(A + io[i].ucount);
        id.ubits = (uint32_t*)(A + io[i].ubits);
        for (int l = 0; l < n_l1; ++l) {
            const int s = i * n_l1 + l;
            const SolveOff& o = so[s];
            SolveDesc& d = b->hsd[s];
            d.p = p;
            d.nwords = T;
            d.T = (int)T;
            d.inst = i;
            d.screen = id.screen;
            d.grouped = p >= COV_TRIAL_GROUP_MIN_P ? 1 : 0;   // the single solver's choice
            d.S = A + io[i].S;
            d.lds = round_up(p, 64);
            d.smax = (const double*)(A + io[i].smax);
            d.om[0] = Csr{(int64_t*)(A + o.rp0), (int32_t*)(A + o.c0), (double*)(A + o.v0)};
            d.om[1] = Csr{(int64_t*)(A + o.rp1), (int32_t*)(A + o.c1), (double*)(A + o.v1)};
            d.A = Cand{(int64_t*)(A + o.arp), (int32_t*)(A + o.acol), (double*)(A + o.aom),
                       (double*)(A + o.agr)};
            d.a_cap = b->om_cap[s];
            d.cnt = (int64_t*)(A + o.cnt);
            d.bitmap = (uint64_t*)(A + o.bitmap);
            d.part = (double*)(A + o.part);
            d.tsums = (double*)(A + o.tsums);
            d.osums = (double*)(A + o.osums);
            d.colws = (double*)(A + o.colws);
            d.scanws = (int64_t*)(A + o.scanws);
            d.rws.lcnt = (int*)(A + o.lcnt);
            d.rws.lK = (int*)(A + o.lK);
            d.rws.lW = (double*)(A + o.lW);
            d.rws.lcmax = (int*)(A + o.lcmax);
            d.rws.plist = (int*)(A + o.plist);
            d.rws.pcount = (int*)(A + o.pcount);
            d.rws.tmask = (uint64_t*)(A + o.tmask);
            d.st = b->dst + s;
            d.ctl = b->dctl + s;
            d.lam1 = b->lambda1[l];
        }
    }
    if (hipMemcpyAsync(b->dsd, b->hsd.data(), N * sizeof(SolveDesc), hipMemcpyHostToDevice, b->work) != hipSuccess ||
        hipMemcpyAsync(b->did, b->hid.data(), count * sizeof(InstDesc), hipMemcpyHostToDevice, b->work) != hipSuccess ||
        hipStreamSynchronize(b->work) != hipSuccess)
        return bail(CONCORD_EHIP);
    // the inputs were produced on the caller's stream
    if (hipStreamSynchronize(b->user) != hipSuccess) return bail(CONCORD_EHIP);
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = b;
    return CONCORD_OK;
}

int concord_batch_solve(concord_batch* b, double lambda2, double tol, int64_t max_iter,
                        int64_t* host_iters, double* host_F, int32_t* host_status) {
    if (!b) return CONCORD_EINVAL;
    if (!(lambda2 >= 0.0) || !std::isfinite(lambda2) || !(tol >= 0.0) || max_iter < 0)
        return bfail(b, CONCORD_EINVAL, "lambda2, tol must be >= 0, max_iter >= 0");
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    struct Restore {
        int prev;
        ~Restore() {
            if (prev >= 0) (void)hipSetDevice(prev);
        }
    } restore{prev};
    b->stats = concord_batch_stats{};
    BHIP(b, hipEventRecord(b->ev_fork, b->user));
    BHIP(b, hipStreamWaitEvent(b->work, b->ev_fork, 0));
    int rc;
    if (!b->s_ready && (rc = form_s(b))) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    const int N = b->nsolve;
    // every solve from Omega = I: control and search state cleared, then the products,
    // threshold words and objective of the start
    BHIP(b, hipMemsetAsync(b->dctl, 0, N * sizeof(SolveCtl), b->work));
    BHIP(b, hipMemsetAsync(b->dst, 0, N * sizeof(DevState), b->work));
    BatchArgs a{};
    a.nsolve = N;
    a.ninst = b->count;
    a.maxT = b->maxT;
    a.bstore = b->sstore;
    a.tb = b->cfg.trial_batch;
    a.total = b->cfg.max_backtracks + 1;
    a.max_iter = max_iter;
    a.lam2 = lambda2;
    a.tol = tol;
    a.tau0 = b->cfg.tau0;
    a.shrink = b->cfg.shrink;
    for (int s = 0; s < N; ++s) {
        const SolveDesc& d = b->hsd[s];
        a.any_rowu |= d.grouped ? 0 : 1;
        a.any_rowg |= d.grouped ? 1 : 0;
        a.any_screen |= d.screen ? 1 : 0;
        a.any_multichunk |= d.p > SCAN_CHUNK ? 1 : 0;
    }
    BHIP(b, launch_batch_iteration(b->dsd, b->did, b->plan, a, true, b->grid, b->work));
    const int K = b->cfg.iters_per_launch;
    bool graph = b->cfg.use_graph != 0;
    if (graph && (!b->gexec || std::memcmp(&b->gargs, &a, sizeof(a)) != 0 || b->g_iters != K)) {
        if (b->gexec) {
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        BHIP(b, hipStreamBeginCapture(b->work, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int k = 0; k < K && e == hipSuccess; ++k)
            e = launch_batch_iteration(b->dsd, b->did, b->plan, a, false, b->grid, b->work);
        const hipError_t ec = hipStreamEndCapture(b->work, &g);
        if (e != hipSuccess || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(b, CONCORD_EHIP, "capturing the batched iteration failed");
        }
        const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        BHIP(b, ei);
        b->gargs = a;
        b->g_iters = K;
    }
    // bound on the iterations any solve can need (each accepted step or trial batch
    // advances a solve; regrowths restart a step)
    const int64_t cap_iters = max_iter * ((a.total + a.tb - 1) / a.tb) + 8;
    int64_t launched = 0;
    while (max_iter > 0) {
        if (graph) {
            BHIP(b, hipGraphLaunch(b->gexec, b->work));
        } else {
            for (int k = 0; k < K; ++k)
                BHIP(b, launch_batch_iteration(b->dsd, b->did, b->plan, a, false, b->grid, b->work));
        }
        launched += K;
        b->stats.launches += 1;
        BHIP(b, hipMemcpyAsync(b->hstatus, b->plan.status, 4 * sizeof(int), hipMemcpyDeviceToHost,
                               b->work));
        BHIP(b, hipStreamSynchronize(b->work));
        b->stats.host_syncs += 1;
        const int running = b->hstatus[0], grow = b->hstatus[1];
        if (grow > 0 && (rc = regrow(b))) return rc;
        if (running == 0 && grow == 0) break;
        if (launched > cap_iters + 64 * (b->stats.regrows + 1))
            return bfail(b, CONCORD_EHIP, "batched solve did not terminate");
    }
    b->stats.iterations_launched = launched;
    BHIP(b, hipMemcpyAsync(b->hctl.data(), b->dctl, N * sizeof(SolveCtl), hipMemcpyDeviceToHost,
                           b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    b->stats.iterate_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int status = CONCORD_OK;
    for (int s = 0; s < N; ++s) {
        const SolveCtl& c = b->hctl[s];
        int st = max_iter == 0 ? (tol > 0.0 ? CONCORD_WMAXITER : CONCORD_OK) : c.status;
        if (host_iters) host_iters[s] = c.k;
        if (host_F) host_F[s] = c.F;
        if (host_status) host_status[s] = st;
        if (st < 0) { if (status >= 0) status = st; }
        else if (status >= 0 && st > status) status = st;
    }
    if (status < 0) return bfail(b, status, "a solve's line search exhausted max_backtracks");
    return status;
}

int concord_batch_get_omega(concord_batch* b, int32_t instance, int32_t l1_index,
                            int64_t* host_nnz, int64_t* dev_row_ptr, int32_t* dev_col,
                            double* dev_val) {
    if (!b || !host_nnz) return CONCORD_EINVAL;
    if (instance < 0 || instance >= b->count || l1_index < 0 || l1_index >= b->n_l1)
        return bfail(b, CONCORD_EINVAL, "index out of range");
    if (!b->s_ready) return bfail(b, CONCORD_ENODATA, "not solved yet");
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    struct Restore {
        int prev;
        ~Restore() {
            if (prev >= 0) (void)hipSetDevice(prev);
        }
    } restore{prev};
    const int s = instance * b->n_l1 + l1_index;
    const SolveDesc& d = b->hsd[s];
    const Csr& o = d.om[b->hctl[s].cur];
    int64_t nnz = 0;
    BHIP(b, hipMemcpyAsync(&nnz, o.rowptr + d.p, sizeof(int64_t), hipMemcpyDeviceToHost, b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    *host_nnz = nnz;
    if (!dev_row_ptr) return CONCORD_OK;
    if (!dev_col || !dev_val) return bfail(b, CONCORD_EINVAL, "col/val must be given with row_ptr");
    BHIP(b, hipMemcpyAsync(dev_row_ptr, o.rowptr, (d.p + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                           b->work));
    BHIP(b, hipMemcpyAsync(dev_col, o.col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, b->work));
    BHIP(b, hipMemcpyAsync(dev_val, o.val, nnz * sizeof(double), hipMemcpyDeviceToDevice, b->work));
    BHIP(b, hipStreamSynchronize(b->work));
    return CONCORD_OK;
}

}  // extern "C"
