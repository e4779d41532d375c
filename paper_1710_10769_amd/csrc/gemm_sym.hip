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
// Tile: 128 x 128 per workgroup of 4 waves (2 x 2, 64 x 64 each), 64 bytes of
// K per plane per stage, double-buffered in LDS with rows padded to 80 bytes
// (conflict-free 16-byte fragment reads).  Workgroup ids are remapped so that
// each XCD receives a contiguous run of row-major upper-triangle tiles and
// keeps their shared P/Q rows in its own L2.
//
// Precision forms:
//   GK_F32    v_mfma_f32_32x32x2f32, FP32 in / FP32 accumulate
//   GK_F64    v_mfma_f64_16x16x4f64
//   GK_BF16X3 v_mfma_f32_32x32x16_bf16 three times: hi*hi + hi*lo + lo*hi,
//             where x = hi + lo, hi = bf16(x), lo = bf16(x - hi)
#include "internal.h"

namespace concord {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int BM = GEMM_BM;      // 128
constexpr int ROWB = 64;         // bytes of K per row per stage and plane
constexpr int ROWS = 80;         // padded LDS row stride in bytes
constexpr int PLANE = BM * ROWS; // bytes of one plane of one side in LDS
constexpr int NT = 256;

__device__ inline uint16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline void tile_of(int w, int ntiles, int T, int& I, int& J) {
    // XCD-aware remap: hardware places workgroup w on XCD w % 8.  Give XCD x
    // the contiguous tile range [start_x, start_x + count_x).
    const int nx = 8;
    int x = w % nx, r = w / nx;
    int base = ntiles / nx, rem = ntiles % nx;
    int t = x * base + (x < rem ? x : rem) + r;
    // row-major upper triangle: row I holds T - I tiles
    double tt = (double)t;
    double b = 2.0 * T + 1.0;
    int i = (int)((b - sqrt(b * b - 8.0 * tt)) * 0.5);
    if (i < 0) i = 0;
    while (i > 0 && (long)i * T - (long)i * (i - 1) / 2 > t) --i;
    while ((long)(i + 1) * T - (long)(i + 1) * i / 2 <= t) ++i;
    int start = i * T - i * (i - 1) / 2;
    I = i;
    J = i + (t - start);
}

// ---- per-form fragment math ------------------------------------------------

template <int KIND> struct Form;

template <> struct Form<GK_BF16X3> {
    static constexpr int NPLANE = 2;
    static constexpr int ELEM = 2;
    typedef f32x16_t acc_t;
    static constexpr int MB = 2, NB = 2;   // 32x32 blocks per wave (64 x 64)
    __device__ static void zero(acc_t (&a)[MB][NB]) {
        for (int i = 0; i < MB; ++i)
            for (int j = 0; j < NB; ++j)
                for (int r = 0; r < 16; ++r) a[i][j][r] = 0.f;
    }
    // one stage: 64 bytes = 32 bf16 of K = two k16 steps
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int wm,
                                 int wn, int lane) {
        const int r32 = lane & 31, hk = lane >> 5;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int off = (2 * kk + hk) * 16;
            bf16x8_t ah[MB], al[MB], bh[NB], bl[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int row = wm * 64 + i * 32 + r32;
                ah[i] = *(const bf16x8_t*)(As + row * ROWS + off);
                al[i] = *(const bf16x8_t*)(As + PLANE + row * ROWS + off);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int row = wn * 64 + j * 32 + r32;
                bh[j] = *(const bf16x8_t*)(Bs + row * ROWS + off);
                bl[j] = *(const bf16x8_t*)(Bs + PLANE + row * ROWS + off);
            }
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
    }
    // element (block i,j, register r) -> (row, col) inside the wave tile
    __device__ static void coord(int i, int j, int r, int lane, int& row, int& col) {
        row = i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        col = j * 32 + (lane & 31);
    }
    static constexpr int NREG = 16;
    __device__ static double get(const acc_t& a, int r) { return (double)a[r]; }
};

template <> struct Form<GK_F32> {
    static constexpr int NPLANE = 1;
    static constexpr int ELEM = 4;
    typedef f32x16_t acc_t;
    static constexpr int MB = 2, NB = 2;
    __device__ static void zero(acc_t (&a)[MB][NB]) {
        for (int i = 0; i < MB; ++i)
            for (int j = 0; j < NB; ++j)
                for (int r = 0; r < 16; ++r) a[i][j][r] = 0.f;
    }
    // one stage: 64 bytes = 16 floats of K; lane half hk reads chunk 2*kk+hk
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int wm,
                                 int wn, int lane) {
        const int r32 = lane & 31, hk = lane >> 5;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int off = (2 * kk + hk) * 16;
            f32x4_t a[MB], b[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i)
                a[i] = *(const f32x4_t*)(As + (wm * 64 + i * 32 + r32) * ROWS + off);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                b[j] = *(const f32x4_t*)(Bs + (wn * 64 + j * 32 + r32) * ROWS + off);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][m], b[j][m], acc[i][j], 0, 0, 0);
        }
    }
    __device__ static void coord(int i, int j, int r, int lane, int& row, int& col) {
        row = i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        col = j * 32 + (lane & 31);
    }
    static constexpr int NREG = 16;
    __device__ static double get(const acc_t& a, int r) { return (double)a[r]; }
};

template <> struct Form<GK_F64> {
    static constexpr int NPLANE = 1;
    static constexpr int ELEM = 8;
    typedef f64x4_t acc_t;
    static constexpr int MB = 4, NB = 4;   // 16x16 blocks per wave (64 x 64)
    __device__ static void zero(acc_t (&a)[MB][NB]) {
        for (int i = 0; i < MB; ++i)
            for (int j = 0; j < NB; ++j)
                for (int r = 0; r < 4; ++r) a[i][j][r] = 0.0;
    }
    // one stage: 64 bytes = 8 doubles of K; lane quarter reads chunk lane/16
    __device__ static void stage(acc_t (&acc)[MB][NB], const char* As, const char* Bs, int wm,
                                 int wn, int lane) {
        const int r16 = lane & 15, q = lane >> 4;
        const int off = q * 16;
        double2 a[MB], b[NB];
#pragma unroll
        for (int i = 0; i < MB; ++i)
            a[i] = *(const double2*)(As + (wm * 64 + i * 16 + r16) * ROWS + off);
#pragma unroll
        for (int j = 0; j < NB; ++j)
            b[j] = *(const double2*)(Bs + (wn * 64 + j * 16 + r16) * ROWS + off);
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc[i][j], 0, 0, 0);
            }
    }
    // v_mfma_f64_16x16x4f64 result: register r of lane l holds row 4r + l/16, column l%16
    __device__ static void coord(int i, int j, int r, int lane, int& row, int& col) {
        row = i * 16 + 4 * r + (lane >> 4);
        col = j * 16 + (lane & 15);
    }
    static constexpr int NREG = 4;
    __device__ static double get(const acc_t& a, int r) { return a[r]; }
};

template <typename T> __device__ inline void store_val(void* C, int store, int64_t idx, double v) {
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

template <int KIND>
__global__ void __launch_bounds__(NT)
gemm_sym_kernel(const char* __restrict__ P0, const char* __restrict__ P1,
                const char* __restrict__ Q0, const char* __restrict__ Q1, int64_t ldk_bytes,
                int nk, int syr2k, int p, int T, int ntiles, double alpha, void* __restrict__ C,
                int out_store, int64_t ldc) {
    typedef Form<KIND> F;
    constexpr int NP = F::NPLANE;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // stage s: [A planes][B planes]
    char* const S0 = smem;
    const int stage_bytes = 2 * NP * PLANE;

    int I, J;
    tile_of(blockIdx.x, ntiles, T, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // global chunk assignment: 512 chunks per plane per side, 2 per thread
    const int crow = tid >> 2, cch = tid & 3;
    const int64_t rowI0 = (int64_t)I * BM, rowJ0 = (int64_t)J * BM;

    u32x4_t ra[NP][2], rb[NP][2];
    const int nk_total = syr2k ? 2 * nk : nk;

    auto gload = [&](int kt) {
        const bool second = kt >= nk;
        const int64_t kb = (int64_t)(second ? kt - nk : kt) * ROWB + cch * 16;
        // phase 1: A = P rows I, B = Q rows J; phase 2: A = Q rows I, B = P rows J
        const char* a0 = second ? Q0 : P0;
        const char* a1 = second ? Q1 : P1;
        const char* b0 = syr2k ? (second ? P0 : Q0) : P0;
        const char* b1 = syr2k ? (second ? P1 : Q1) : P1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t ra_off = (rowI0 + crow + 64 * h) * ldk_bytes + kb;
            const int64_t rb_off = (rowJ0 + crow + 64 * h) * ldk_bytes + kb;
            ra[0][h] = *(const u32x4_t*)(a0 + ra_off);
            rb[0][h] = *(const u32x4_t*)(b0 + rb_off);
            if (NP == 2) {
                ra[NP - 1][h] = *(const u32x4_t*)(a1 + ra_off);
                rb[NP - 1][h] = *(const u32x4_t*)(b1 + rb_off);
            }
        }
    };
    auto lstore = [&](int buf) {
        char* base = S0 + buf * stage_bytes;
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int off = (crow + 64 * h) * ROWS + cch * 16;
                *(u32x4_t*)(base + pl * PLANE + off) = ra[pl][h];
                *(u32x4_t*)(base + NP * PLANE + pl * PLANE + off) = rb[pl][h];
            }
    };

    typename F::acc_t acc[F::MB][F::NB];
    F::zero(acc);

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk_total; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk_total) gload(kt + 1);
        const char* base = S0 + cur * stage_bytes;
        F::stage(acc, base, base + NP * PLANE, wm, wn, lane);
        if (kt + 1 < nk_total) lstore(cur ^ 1);
        __syncthreads();
    }

    // epilogue: symmetric store
    const int64_t r0 = rowI0 + wm * 64, c0 = rowJ0 + wn * 64;
#pragma unroll
    for (int i = 0; i < F::MB; ++i)
#pragma unroll
        for (int j = 0; j < F::NB; ++j)
#pragma unroll
            for (int r = 0; r < F::NREG; ++r) {
                int rr, cc;
                F::coord(i, j, r, lane, rr, cc);
                const int64_t gi = r0 + rr, gj = c0 + cc;
                if (gi >= p || gj >= p) continue;
                if (I == J && gi > gj) continue;
                const double v = alpha * F::get(acc[i][j], r);
                store_val<float>(C, out_store, gi * ldc + gj, v);
                if (gi != gj) store_val<float>(C, out_store, gj * ldc + gi, v);
            }
}

template <int KIND>
hipError_t launch_kind(bool syr2k, const void* P0, const void* P1, const void* Q0,
                       const void* Q1, int64_t ldk, int64_t p, double alpha, void* C,
                       int out_store, int64_t ldc, hipStream_t stream) {
    typedef Form<KIND> F;
    const int64_t ldk_bytes = ldk * F::ELEM;
    if (ldk_bytes % ROWB) return hipErrorInvalidValue;
    const int nk = (int)(ldk_bytes / ROWB);
    const int T = (int)((p + BM - 1) / BM);
    const int ntiles = T * (T + 1) / 2;
    const size_t lds = 2 * (2 * F::NPLANE * PLANE);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void*)gemm_sym_kernel<KIND>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
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
