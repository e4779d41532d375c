// Symmetric dense contractions on gfx950 matrix cores.
//
//   syrk :  C = alpha * P P^T              (S = X^T X / n, Algorithm 2, once)
//   syr2k:  C = alpha * (P Q^T + Q P^T)    (Z + Z^T with Z = Y X / n,
//                                           Algorithm 3, gradient step)
//
// Operands are "K-major": P and Q are row-major p x K planes (variable-major
// X^T and Y = Omega X^T), so every product row reads contiguous K.  Only the
// upper-triangle output tiles (I <= J) are computed; each tile writes its
// values to (I, J) and, mirrored, to (J, I), so the result is bitwise
// symmetric and Z^T is never formed separately (the paper's explicit
// transpose becomes a tile-pair store).
//
// Tile: 256 x 256 per workgroup of 8 waves (4 x 2, 64 x 128 each) for the
// BF16-split and FP32 forms, 128 x 128 with 4 waves for FP64; 64 bytes of K
// per plane per stage, double-buffered in LDS with XOR-swizzled rows
// (conflict-free 16-byte fragment reads).  Workgroup ids are remapped so that
// each XCD receives a contiguous run of row-major upper-triangle tiles and
// keeps their shared P/Q rows in its own L2.
//
// Precision forms:
//   GK_F32    v_mfma_f32_32x32x2f32, FP32 in / FP32 accumulate
//   GK_F64    v_mfma_f64_16x16x4f64
//   GK_BF16X3 v_mfma_f32_32x32x16_bf16 three times: hi*hi + hi*lo + lo*hi,
//             where x = hi + lo, hi = bf16(x), lo = bf16(x - hi)
#include <mutex>

#include "internal.h"

namespace concord {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int ROWB = 64;   // bytes of K per row, per stage and plane (4 chunks of 16 B)

__device__ inline uint16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// LDS rows are 64 bytes; the four 16-byte chunks of a row are XOR-swizzled by
// bits 1..2 of the row so that 8 consecutive rows read at the same logical
// chunk hit 8 distinct 16-byte bank groups (conflict-free ds_read_b128).
__device__ inline int swz(int row, int chunk) { return row * ROWB + ((chunk ^ ((row >> 1) & 3)) << 4); }

__device__ inline void tile_of(int w, int ntiles, int T, int& I, int& J) {
    // XCD-aware remap: hardware places workgroup w on XCD w % 8.  Give XCD x
    // the contiguous range [start_x, start_x + count_x) of the tile order below,
    // so the ~32 tiles resident on one XCD are consecutive in that order.
    const int nx = 8;
    const int x = w % nx, r = w / nx;
    const int base = ntiles / nx, rem = ntiles % nx;
    int t = x * base + (x < rem ? x : rem) + r;
    // Tile order over the upper triangle (I <= J): bands of G tile-rows; inside a
    // band, column by column.  G consecutive tiles share one B slab (rows J)
    // and every tile of the band shares the band's G A slabs (rows I), so a run
    // of 32 tiles touches G + 32/G slabs instead of 33.
    constexpr int G = 8;
    int i0 = 0;
    for (;;) {
        const int h = T - i0 < G ? T - i0 : G;
        const int cnt = h * (h + 1) / 2 + h * (T - i0 - h);
        if (t < cnt || i0 + h >= T) break;
        t -= cnt;
        i0 += G;
    }
    const int h = T - i0 < G ? T - i0 : G;
    const int tri = h * (h + 1) / 2;
    if (t < tri) {
        int jj = 0;
        while (t >= jj + 1) { t -= jj + 1; ++jj; }
        I = i0 + t;
        J = i0 + jj;
    } else {
        t -= tri;
        J = i0 + h + t / h;
        I = i0 + t % h;
    }
}

// ---- per-form fragment math ------------------------------------------------
// stage(): consume one 64-byte K stage from LDS.  As/Bs point at the first
// plane of the A (rows I) and B (rows J) sides; `plane` is the byte distance
// between the hi and lo planes.  ra0/rb0: the wave's first row on each side.

template <int KIND> struct Form;

template <> struct Form<GK_BF16X3> {
    static constexpr int NPLANE = 2;
    static constexpr int ELEM = 2;
    static constexpr int BS = 32;   // 32 x 32 result blocks
    typedef f32x16_t acc_t;
    static constexpr int NREG = 16;
    template <int MB, int NB>
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int plane,
                                 int ra0, int rb0, int lane) {
        const int r32 = lane & 31, hk = lane >> 5;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int c = 2 * kk + hk;
            bf16x8_t ah[MB], al[MB], bh[NB], bl[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int o = swz(ra0 + i * 32 + r32, c);
                ah[i] = *(const bf16x8_t*)(As + o);
                al[i] = *(const bf16x8_t*)(As + plane + o);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int o = swz(rb0 + j * 32 + r32, c);
                bh[j] = *(const bf16x8_t*)(Bs + o);
                bl[j] = *(const bf16x8_t*)(Bs + plane + o);
            }
            // term-major order: MB*NB independent accumulators between two
            // MFMAs that depend on each other
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    // v_mfma_f32_32x32*: register r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32
    __device__ static void coord(int r, int lane, int& row, int& col) {
        row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        col = lane & 31;
    }
    __device__ static double get(const acc_t& a, int r) { return (double)a[r]; }
};

template <> struct Form<GK_F32> {
    static constexpr int NPLANE = 1;
    static constexpr int ELEM = 4;
    static constexpr int BS = 32;
    typedef f32x16_t acc_t;
    static constexpr int NREG = 16;
    // 64 bytes = 16 floats of K; lane half hk reads chunk 2*kk+hk, one float per MFMA
    template <int MB, int NB>
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int,
                                 int ra0, int rb0, int lane) {
        const int r32 = lane & 31, hk = lane >> 5;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int c = 2 * kk + hk;
            f32x4_t a[MB], b[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) a[i] = *(const f32x4_t*)(As + swz(ra0 + i * 32 + r32, c));
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = *(const f32x4_t*)(Bs + swz(rb0 + j * 32 + r32, c));
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][m], b[j][m], acc[i][j], 0, 0, 0);
        }
    }
    __device__ static void coord(int r, int lane, int& row, int& col) {
        row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        col = lane & 31;
    }
    __device__ static double get(const acc_t& a, int r) { return (double)a[r]; }
};

template <> struct Form<GK_F64> {
    static constexpr int NPLANE = 1;
    static constexpr int ELEM = 8;
    static constexpr int BS = 16;   // 16 x 16 result blocks
    typedef f64x4_t acc_t;
    static constexpr int NREG = 4;
    // 64 bytes = 8 doubles of K; lane quarter q = l/16 reads chunk q (2 doubles)
    template <int MB, int NB>
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int,
                                 int ra0, int rb0, int lane) {
        const int r16 = lane & 15, q = lane >> 4;
        double2 a[MB], b[NB];
#pragma unroll
        for (int i = 0; i < MB; ++i) a[i] = *(const double2*)(As + swz(ra0 + i * 16 + r16, q));
#pragma unroll
        for (int j = 0; j < NB; ++j) b[j] = *(const double2*)(Bs + swz(rb0 + j * 16 + r16, q));
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc[i][j], 0, 0, 0);
            }
    }
    // v_mfma_f64_16x16x4f64 result: register r of lane l holds row 4r + l/16, column l%16
    __device__ static void coord(int r, int lane, int& row, int& col) {
        row = 4 * r + (lane >> 4);
        col = lane & 15;
    }
    __device__ static double get(const acc_t& a, int r) { return a[r]; }
};

__device__ inline void store_val(void* C, int store, int64_t idx, double v) {
    if (store == ST_F64) ((double*)C)[idx] = v;
    else if (store == ST_F32) ((float*)C)[idx] = (float)v;
    else {
        float x = (float)v;
        uint16_t h = f2bf_rne(x);
        float hv = __uint_as_float(((uint32_t)h) << 16);
        uint16_t l = f2bf_rne(x - hv);
        ((uint32_t*)C)[idx] = (uint32_t)h | ((uint32_t)l << 16);
    }
}

// Tile configuration: BT x BT output tile, WM x WN waves.
template <int KIND> struct Cfg;
template <> struct Cfg<GK_BF16X3> { static constexpr int BT = 256, WM = 4, WN = 2; };
template <> struct Cfg<GK_F32> { static constexpr int BT = 256, WM = 4, WN = 2; };
template <> struct Cfg<GK_F64> { static constexpr int BT = 128, WM = 2, WN = 2; };

template <int KIND>
__global__ void __launch_bounds__(Cfg<KIND>::WM * Cfg<KIND>::WN * 64)
gemm_sym_kernel(const char* __restrict__ P0, const char* __restrict__ P1,
                const char* __restrict__ Q0, const char* __restrict__ Q1, int64_t ldk_bytes,
                int nk, int syr2k, int p, int T, int ntiles, double alpha, void* __restrict__ C,
                int out_store, int64_t ldc) {
    typedef Form<KIND> F;
    constexpr int BT = Cfg<KIND>::BT, WM = Cfg<KIND>::WM, WN = Cfg<KIND>::WN;
    constexpr int NT = WM * WN * 64;
    constexpr int NP = F::NPLANE;
    constexpr int PLANE = BT * ROWB;          // bytes of one plane of one side
    constexpr int STAGE = 2 * NP * PLANE;     // A planes then B planes
    constexpr int CPT = BT * 4 / NT;          // 16-byte chunks per thread per plane and side
    constexpr int WR = BT / WM, WC = BT / WN; // wave tile
    constexpr int MB = WR / F::BS, NB = WC / F::BS;
    extern __shared__ __attribute__((aligned(16))) char smem[];

    int I, J;
    tile_of(blockIdx.x, ntiles, T, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t rowI0 = (int64_t)I * BT, rowJ0 = (int64_t)J * BT;
    const int nk_total = syr2k ? 2 * nk : nk;

    u32x4_t ra[NP][CPT], rb[NP][CPT];

    auto gload = [&](int kt) {
        const bool second = kt >= nk;
        const int64_t kb = (int64_t)(second ? kt - nk : kt) * ROWB;
        // phase 1: A = P rows I, B = Q rows J; phase 2: A = Q rows I, B = P rows J
        const char* a0 = second ? Q0 : P0;
        const char* a1 = second ? Q1 : P1;
        const char* b0 = syr2k ? (second ? P0 : Q0) : P0;
        const char* b1 = syr2k ? (second ? P1 : Q1) : P1;
#pragma unroll
        for (int h = 0; h < CPT; ++h) {
            const int ci = tid + h * NT;
            const int row = ci >> 2, ch = ci & 3;
            const int64_t oa = (rowI0 + row) * ldk_bytes + kb + ch * 16;
            const int64_t ob = (rowJ0 + row) * ldk_bytes + kb + ch * 16;
            ra[0][h] = *(const u32x4_t*)(a0 + oa);
            rb[0][h] = *(const u32x4_t*)(b0 + ob);
            if (NP == 2) {
                ra[NP - 1][h] = *(const u32x4_t*)(a1 + oa);
                rb[NP - 1][h] = *(const u32x4_t*)(b1 + ob);
            }
        }
    };
    auto lstore = [&](int buf) {
        char* base = smem + buf * STAGE;
#pragma unroll
        for (int h = 0; h < CPT; ++h) {
            const int ci = tid + h * NT;
            const int o = swz(ci >> 2, ci & 3);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) {
                *(u32x4_t*)(base + pl * PLANE + o) = ra[pl][h];
                *(u32x4_t*)(base + NP * PLANE + pl * PLANE + o) = rb[pl][h];
            }
        }
    };

    typename F::acc_t acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < F::NREG; ++r) acc[i][j][r] = 0;

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk_total; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk_total) gload(kt + 1);
        const char* base = smem + cur * STAGE;
        F::template stage<MB, NB>(acc, base, base + NP * PLANE, PLANE, wm * WR, wn * WC, lane);
        if (kt + 1 < nk_total) lstore(cur ^ 1);
        __syncthreads();
    }

    // epilogue: symmetric store
    const int64_t r0 = rowI0 + wm * WR, c0 = rowJ0 + wn * WC;
    if (F::BS == 32 && I != J && out_store != ST_F64) {
        // Off-diagonal tile, 4-byte elements.  Direct store: consecutive lanes
        // hold consecutive columns.  Mirrored store: registers 4g..4g+3 of a
        // lane hold 4 consecutive rows, i.e. 16 contiguous bytes of the
        // transposed row, written as one vector.
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int64_t gj = c0 + j * 32 + (lane & 31);
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t gi0 = r0 + i * 32 + 8 * g + 4 * (lane >> 5);
                    uint32_t w[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double v = alpha * F::get(acc[i][j], 4 * g + t);
                        if (out_store == ST_F32) {
                            const float x = (float)v;
                            w[t] = __float_as_uint(x);
                        } else {
                            const float x = (float)v;
                            const uint16_t h = f2bf_rne(x);
                            const uint16_t l = f2bf_rne(x - __uint_as_float(((uint32_t)h) << 16));
                            w[t] = (uint32_t)h | ((uint32_t)l << 16);
                        }
                        if (gj < p && gi0 + t < p) ((uint32_t*)C)[(gi0 + t) * ldc + gj] = w[t];
                    }
                    if (gj < p) {
                        if (gi0 + 3 < p) {
                            *(u32x4_t*)((uint32_t*)C + gj * ldc + gi0) = u32x4_t{w[0], w[1], w[2], w[3]};
                        } else {
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                if (gi0 + t < p) ((uint32_t*)C)[gj * ldc + gi0 + t] = w[t];
                        }
                    }
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < F::NREG; ++r) {
                int rr, cc;
                F::coord(r, lane, rr, cc);
                const int64_t gi = r0 + i * F::BS + rr, gj = c0 + j * F::BS + cc;
                if (gi >= p || gj >= p) continue;
                if (I == J && gi > gj) continue;
                const double v = alpha * F::get(acc[i][j], r);
                store_val(C, out_store, gi * ldc + gj, v);
                if (gi != gj) store_val(C, out_store, gj * ldc + gi, v);
            }
}

template <int KIND>
hipError_t launch_kind(bool syr2k, const void* P0, const void* P1, const void* Q0,
                       const void* Q1, int64_t ldk, int64_t p, double alpha, void* C,
                       int out_store, int64_t ldc, hipStream_t stream) {
    typedef Form<KIND> F;
    constexpr int BT = Cfg<KIND>::BT;
    constexpr int NT = Cfg<KIND>::WM * Cfg<KIND>::WN * 64;
    const int64_t ldk_bytes = ldk * F::ELEM;
    if (ldk_bytes % ROWB) return hipErrorInvalidValue;
    const int nk = (int)(ldk_bytes / ROWB);
    const int T = (int)((p + BT - 1) / BT);
    const int ntiles = T * (T + 1) / 2;
    const size_t lds = 2 * (2 * F::NPLANE * BT * ROWB);
    static std::once_flag attr_once;   // handles on several host threads may launch concurrently
    std::call_once(attr_once, [&] {
        (void)hipFuncSetAttribute((const void*)gemm_sym_kernel<KIND>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    if (ntiles == 0 || nk == 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_sym_kernel<KIND>, dim3(ntiles), dim3(NT), lds, stream,
                       (const char*)P0, (const char*)P1, (const char*)(syr2k ? Q0 : P0),
                       (const char*)(syr2k ? Q1 : P1), ldk_bytes, nk, syr2k ? 1 : 0, (int)p, T,
                       ntiles, alpha, C, out_store, ldc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_sym(int kind, bool syr2k, const void* P0, const void* P1,
                           const void* Q0, const void* Q1, int64_t ldk, int64_t p,
                           double alpha, void* C, int out_store, int64_t ldc,
                           hipStream_t stream) {
    switch (kind) {
        case GK_F64:
            return launch_kind<GK_F64>(syr2k, P0, P1, Q0, Q1, ldk, p, alpha, C, out_store, ldc, stream);
        case GK_F32:
            return launch_kind<GK_F32>(syr2k, P0, P1, Q0, Q1, ldk, p, alpha, C, out_store, ldc, stream);
        case GK_BF16X3:
            return launch_kind<GK_BF16X3>(syr2k, P0, P1, Q0, Q1, ldk, p, alpha, C, out_store, ldc, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace concord
