// Sparse and streaming kernels of the proximal-gradient iteration.
//
// Layouts (all device memory):
//   Omega      CSR: rowptr int64[p+1], col int32 (sorted per row, both
//              triangles, diagonal always stored), val double.
//   dense      row-major, rows padded with zeros; a "chunk" is 16 bytes:
//              2 doubles (ST_F64), 4 floats (ST_F32) or 4 packed bf16 hi/lo
//              pairs (ST_B16P, value = hi + lo in FP32).
//   candidates CSR-like (rowptr, col, omega, grad) of the set A that can be
//              nonzero after this iteration's prox step.
//
// One 64-wide wavefront owns one row in every row kernel; compaction is by
// wavefront ballot + popcount prefix, so every emitted row stays sorted.
// Every FP64 reduction is done in a fixed order (lane-local sequential sums,
// then a fixed xor-butterfly, then fixed-order column sums), so results are
// bitwise reproducible run to run.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "../../include/concord.h"
#include "internal.h"

namespace concord {
namespace {

constexpr int NT = 256;
constexpr int WPB = NT / 64;   // waves (rows) per block

__device__ inline int64_t uni(int64_t x) {
    return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(x & 0xffffffff)));
}
__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}
__device__ inline uint16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint32_t h16) { return __uint_as_float(h16 << 16); }

// ---- chunk loaders ----------------------------------------------------------
template <int S> struct Chunk;
template <> struct Chunk<ST_F64> {
    static constexpr int V = 2;
    typedef double T;
    __device__ static void load(const void* b, int64_t idx, T (&v)[V]) {
        double2 d = *(const double2*)((const double*)b + idx);
        v[0] = d.x; v[1] = d.y;
    }
    __device__ static T one(const void* b, int64_t idx) { return ((const double*)b)[idx]; }
};
template <> struct Chunk<ST_F32> {
    static constexpr int V = 4;
    typedef float T;
    __device__ static void load(const void* b, int64_t idx, T (&v)[V]) {
        float4 d = *(const float4*)((const float*)b + idx);
        v[0] = d.x; v[1] = d.y; v[2] = d.z; v[3] = d.w;
    }
    __device__ static T one(const void* b, int64_t idx) { return ((const float*)b)[idx]; }
};
template <> struct Chunk<ST_B16P> {
    static constexpr int V = 4;
    typedef float T;
    __device__ static T cv(uint32_t u) { return bf2f(u & 0xffffu) + bf2f(u >> 16); }
    __device__ static void load(const void* b, int64_t idx, T (&v)[V]) {
        uint4 d = *(const uint4*)((const uint32_t*)b + idx);
        v[0] = cv(d.x); v[1] = cv(d.y); v[2] = cv(d.z); v[3] = cv(d.w);
    }
    __device__ static T one(const void* b, int64_t idx) { return cv(((const uint32_t*)b)[idx]); }
};

template <int S> __device__ inline double load_one_d(const void* b, int64_t idx) {
    return (double)Chunk<S>::one(b, idx);
}

// Element c of the row starting at element `row` (a wave-uniform offset): the row's
// base address stays scalar and the lane offset is a 32-bit vector register.
template <int BS> __device__ inline double load_row_d(const void* b, int64_t row, uint32_t c) {
    typedef typename std::conditional<BS == ST_F64, double, uint32_t>::type U;
    // the row's address goes through readfirstlane, so it is formed in scalar registers
    // and the load takes the scalar-base + 32-bit vector-offset form
    typedef const __attribute__((address_space(1))) char GC;   // global memory
    GC* r = (GC*)uni((int64_t)((const U*)b + row));
    const U x = *(const __attribute__((address_space(1))) U*)(r + (uint32_t)(c * (uint32_t)sizeof(U)));
    if (BS == ST_F64) return (double)x;
    if (BS == ST_F32) return (double)__uint_as_float((uint32_t)x);
    return (double)Chunk<ST_B16P>::cv((uint32_t)x);
}

// Cov form: stored type of M = (W + W^T) / 2 for S stored as BS
template <int BS> struct MType { typedef float T; };
template <> struct MType<ST_F64> { typedef double T; };

// One entry M_ij = (W_ij + W_ji) / 2 of the Cov gradient, W = Omega S, from the CSR
// rows i and j of Omega.  With S exactly symmetric, W_ji = sum_{k in supp_j} omega_jk
// S[i][k].  The arithmetic is that of cov_refresh_kernel (each half is a chain of FMAs
// over its row's nonzeros in CSR order in the accumulation type, both halves are
// rounded to M's type, then added and halved), so the value is bitwise the one the
// refresh tests against lambda1.  Loads are issued four at a time ahead of their FMAs.
// fma_chain: sum over entries k in [s, e) of val[k] * S[base + col[k] * stride].
template <int BS>
__device__ inline typename Chunk<BS>::T fma_chain(const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, int64_t s,
                                                  int64_t e, const void* __restrict__ S,
                                                  int64_t base, int64_t stride) {
    typedef typename Chunk<BS>::T A;
    A acc = (A)0;
    int64_t k = s;
    for (; k + 4 <= e; k += 4) {
        const A x0 = (A)load_one_d<BS>(S, base + (int64_t)col[k] * stride);
        const A x1 = (A)load_one_d<BS>(S, base + (int64_t)col[k + 1] * stride);
        const A x2 = (A)load_one_d<BS>(S, base + (int64_t)col[k + 2] * stride);
        const A x3 = (A)load_one_d<BS>(S, base + (int64_t)col[k + 3] * stride);
        acc = fma((A)val[k], x0, acc);
        acc = fma((A)val[k + 1], x1, acc);
        acc = fma((A)val[k + 2], x2, acc);
        acc = fma((A)val[k + 3], x3, acc);
    }
    for (; k < e; ++k)
        acc = fma((A)val[k], (A)load_one_d<BS>(S, base + (int64_t)col[k] * stride), acc);
    return acc;
}

template <int BS>
__device__ inline double m_entry(const int64_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                 const void* __restrict__ S, int64_t lds, int64_t i, int64_t j) {
    typedef typename MType<BS>::T E;
    // W_ij: S[k][j] over k in supp_i;  W_ji: S[i][k] over k in supp_j
    const E wij = (E)fma_chain<BS>(col, val, rowptr[i], rowptr[i + 1], S, j, lds);
    const E wji = (E)fma_chain<BS>(col, val, rowptr[j], rowptr[j + 1], S, i * lds, 1);
    return (double)((E)0.5 * (wij + wji));
}

// ---- SpMM: C = Omega B ------------------------------------------------------
// grid: x = ceil(p / 4) row blocks, y = column chunks of 64*V (chunk-major
// dispatch keeps one column slab of B hot in L2/MALL across all rows).
template <int BS, int CS>
__global__ void __launch_bounds__(NT)
spmm_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
            const double* __restrict__ val, int64_t p, const void* __restrict__ B, int64_t ldb,
            int64_t ncols, void* __restrict__ C, int64_t ldc, uint16_t* __restrict__ hi,
            uint16_t* __restrict__ lo, int64_t kbs, double* __restrict__ sq_part, const int* gate) {
    if (gate && *gate == 0) return;
    typedef Chunk<BS> Ch;
    typedef typename Ch::T T;
    constexpr int V = Ch::V;
    const int64_t row = uni((int64_t)blockIdx.x * WPB + (threadIdx.x >> 6));
    if (row >= p) return;
    const int lane = lane_id();
    const int64_t c0 = (int64_t)blockIdx.y * 64 * V + lane * V;
    const bool active = c0 < ncols;
    T acc[V];
#pragma unroll
    for (int t = 0; t < V; ++t) acc[t] = 0;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    // a last chunk that ncols cuts (ncols not a multiple of V; never with the library's
    // padded layouts): element loads, nothing read past ncols, the FMA order unchanged
    const int nv = active ? (ncols - c0 < V ? (int)(ncols - c0) : V) : 0;
    if (active && nv < V) {
        for (int64_t k = s; k < e; ++k) {
            const T v0 = (T)val[k];
            const int64_t jb = (int64_t)col[k] * ldb + c0;
#pragma unroll
            for (int t = 0; t < V; ++t)
                if (t < nv) acc[t] = fma(v0, Ch::one(B, jb + t), acc[t]);
        }
    } else if (active) {
        int64_t k = s;
        for (; k + 4 <= e; k += 4) {
            T b0[V], b1[V], b2[V], b3[V];
            const int64_t j0 = col[k], j1 = col[k + 1], j2 = col[k + 2], j3 = col[k + 3];
            Ch::load(B, j0 * ldb + c0, b0);
            Ch::load(B, j1 * ldb + c0, b1);
            Ch::load(B, j2 * ldb + c0, b2);
            Ch::load(B, j3 * ldb + c0, b3);
            const T v0 = (T)val[k], v1 = (T)val[k + 1], v2 = (T)val[k + 2], v3 = (T)val[k + 3];
#pragma unroll
            for (int t = 0; t < V; ++t) {
                acc[t] = fma(v0, b0[t], acc[t]);
                acc[t] = fma(v1, b1[t], acc[t]);
                acc[t] = fma(v2, b2[t], acc[t]);
                acc[t] = fma(v3, b3[t], acc[t]);
            }
        }
        for (; k < e; ++k) {
            T b0[V];
            Ch::load(B, (int64_t)col[k] * ldb + c0, b0);
            const T v0 = (T)val[k];
#pragma unroll
            for (int t = 0; t < V; ++t) acc[t] = fma(v0, b0[t], acc[t]);
        }
    }
    double sq = 0.0;
    if (active) {
        if (C) {
            if (CS == ST_F64) {
                double* o = (double*)C + row * ldc + c0;
                if (nv == V) {
#pragma unroll
                    for (int t = 0; t < V; ++t) o[t] = (double)acc[t];
                } else {
                    for (int t = 0; t < nv; ++t) o[t] = (double)acc[t];
                }
            } else {
                float* o = (float*)C + row * ldc + c0;
                if (nv == V) {
#pragma unroll
                    for (int t = 0; t < V; ++t) o[t] = (float)acc[t];
                } else {
                    for (int t = 0; t < nv; ++t) o[t] = (float)acc[t];
                }
            }
        }
        if (hi) {
            uint16_t h[V], l[V];
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const float x = (float)acc[t];
                h[t] = f2bf_rne(x);
                l[t] = f2bf_rne(x - bf2f(h[t]));
            }
            // V consecutive columns (c0 % V == 0) stay inside one K block
            const int64_t o = kblk_index(row, c0, kbs);
            if (V == 4) {
                *(uint2*)(hi + o) =
                    make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
                *(uint2*)(lo + o) =
                    make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16), (uint32_t)l[2] | ((uint32_t)l[3] << 16));
            } else {
#pragma unroll
                for (int t = 0; t < V; ++t) { hi[o + t] = h[t]; lo[o + t] = l[t]; }
            }
        }
#pragma unroll
        for (int t = 0; t < V; ++t) sq += (double)acc[t] * (double)acc[t];
    }
    if (sq_part) {
        sq = wave_sum(sq);
        if (lane == 0) sq_part[(int64_t)blockIdx.y * p + row] = sq;
    }
}

// ---- candidate set ----------------------------------------------------------
// Per wave: an LDS bitmap of supp(Omega_i) (p bits).
template <int MS>
__device__ inline void cand_load_group(const void* M, int64_t base, int64_t c, int64_t p,
                                       double (&m)[Chunk<MS>::V]) {
    typedef Chunk<MS> Ch;
    constexpr int V = Ch::V;
    typename Ch::T v[V];
    if (c < p) {
        // dense rows are padded to a multiple of 64 columns; chunks never straddle
        Ch::load(M, base + c, v);
#pragma unroll
        for (int t = 0; t < V; ++t) m[t] = (double)v[t];
    } else {
#pragma unroll
        for (int t = 0; t < V; ++t) m[t] = 0.0;
    }
}

__device__ inline void build_supp_bits(uint32_t* bits, int64_t nw32, const int32_t* col, int64_t s,
                                       int64_t e) {
    const int lane = lane_id();
    for (int64_t w = lane; w < nw32; w += 64) bits[w] = 0u;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int64_t k = s + lane; k < e; k += 64) {
        const int32_t c = col[k];
        atomicOr(&bits[c >> 5], 1u << (c & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// in-bit for lane's V columns starting at c (c multiple of V)
template <int V>
__device__ inline uint32_t supp_nibble(const uint32_t* bits, int64_t c) {
    const uint32_t w = bits[c >> 5];
    return (w >> (c & 31)) & ((1u << V) - 1u);
}

template <int MS>
__global__ void __launch_bounds__(NT)
cand_count_kernel(const void* __restrict__ M, int64_t ldm, const int64_t* __restrict__ rowptr,
                  const int32_t* __restrict__ col, int64_t p, double lam1,
                  uint64_t* __restrict__ bitmap, int64_t nwords, int64_t* __restrict__ cnt) {
    typedef Chunk<MS> Ch;
    constexpr int V = Ch::V;
    constexpr int LPW = 64 / V;   // lanes per 64-bit word
    extern __shared__ uint32_t sbits[];
    const int64_t nw32 = nwords * 2;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni((int64_t)blockIdx.x * WPB + wave);
    if (row >= p) return;
    uint32_t* bits = sbits + wave * nw32;
    build_supp_bits(bits, nw32, col, rowptr[row], rowptr[row + 1]);
    const int64_t base = row * ldm;
    int64_t total = 0;
    const int64_t step = 64 * V;
    for (int64_t g = 0; g < p; g += step) {
        const int64_t c = g + lane * V;
        double m[V];
        cand_load_group<MS>(M, base, c, p, m);
        uint32_t nib = c < p ? supp_nibble<V>(bits, c) : 0u;
#pragma unroll
        for (int t = 0; t < V; ++t) {
            const int64_t j = c + t;
            if (j < p && (j == row || fabs(m[t]) > lam1)) nib |= 1u << t;
        }
        // assemble 64-bit words: lane l contributes V bits at V*(l % LPW)
        uint64_t w = (uint64_t)nib << (V * (lane % LPW));
#pragma unroll
        for (int o = LPW / 2; o >= 1; o >>= 1) w |= __shfl_xor(w, o, 64);
        if ((lane % LPW) == 0) {
            const int64_t wi = g / 64 + lane / LPW;
            if (wi < nwords) bitmap[row * nwords + wi] = w;
        }
        total += __popc(nib);
    }
    // total over lanes
    double tt = (double)total;
    tt = wave_sum(tt);
    if (lane == 0) cnt[row] = (int64_t)tt;
}

template <int MS>
__device__ __forceinline__ void cand_fill_body(int64_t bx_, const void* __restrict__ M, int64_t ldm, const int64_t* __restrict__ rowptr,
                 const int32_t* __restrict__ col, const double* __restrict__ val, int64_t p,
                 double lam2, const uint64_t* __restrict__ bitmap, int64_t nwords,
                 const int64_t* __restrict__ arow, int32_t* __restrict__ acol,
                 double* __restrict__ aom, double* __restrict__ agr, const int* overflow,
                 const uint64_t* __restrict__ tmask, bool m_upper = false) {
    if (*overflow) return;
    typedef typename Chunk<MS>::T E;
    extern __shared__ uint64_t swords[];   // with a tile mask: the row's words holding support
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    int64_t out = arow[row];
    const E* Mrow = M ? (const E*)M + row * ldm : nullptr;
    // With a tile mask (screened Cov refresh), a word can be nonzero only if its tile pair
    // was kept or the support of the row has an entry in it: only those words are read.
    const int64_t TW = (nwords + 63) / 64;
    const uint64_t* mrow = tmask ? tmask + (row >> 6) * TW : nullptr;
    uint64_t* sw = swords + wave * TW;   // bit w: the support has an entry in word w
    if (mrow) {
        for (int64_t t = lane; t < TW; t += 64) sw[t] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int64_t k = s + lane; k < e; k += 64) {
            const int64_t ww = col[k] >> 6;
            atomicOr((unsigned long long*)&sw[ww >> 6], 1ull << (ww & 63));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // A row of at most 64 stored entries is copied to LDS once, so the per-candidate
    // search for omega_ij reads LDS instead of making dependent global loads.
    __shared__ int32_t ccol[WPB][64];
    __shared__ double cval[WPB][64];
    const int64_t nrow = e - s;
    const bool cached = nrow <= 64;
    if (cached) {
        if (lane < nrow) {
            ccol[wave][lane] = col[s + lane];
            cval[wave][lane] = val[s + lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // 64 bitmap words (4096 columns) per step, one per lane; an exclusive prefix of
    // their popcounts places each lane's candidates, so the row stays sorted
    for (int64_t w0 = 0; w0 < nwords; w0 += 64) {
        const int64_t w = w0 + lane;
        bool need = w < nwords;
        if (mrow) {
            const uint64_t mk = mrow[w0 >> 6] | sw[w0 >> 6];
            if (__builtin_amdgcn_readfirstlane((int)(mk != 0ull)) == 0) continue;   // empty block
            need = need && ((mk >> lane) & 1ull);
        }
        uint64_t word = need ? bitmap[row * nwords + w] : 0ull;
        const int pc = __popcll(word);
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int up = __shfl_up(incl, o, 64);
            if (lane >= o) incl += up;
        }
        const int total = __shfl(incl, 63, 64);
        int64_t pos = out + (incl - pc);
        while (word) {
            const int b = __builtin_ctzll(word);
            word &= word - 1ull;
            const int64_t j = w * 64 + b;
            // omega_ij: binary search of the sorted CSR row
            double om = 0.0;
            if (cached) {
                int lo_ = 0, hi_ = (int)nrow;
                while (lo_ < hi_) {
                    const int mid = (lo_ + hi_) >> 1;
                    if (ccol[wave][mid] < j) lo_ = mid + 1; else hi_ = mid;
                }
                if (lo_ < nrow && ccol[wave][lo_] == j) om = cval[wave][lo_];
            } else {
                int64_t lo_ = s, hi_ = e;
                while (lo_ < hi_) {
                    const int64_t mid = (lo_ + hi_) >> 1;
                    if (col[mid] < j) lo_ = mid + 1; else hi_ = mid;
                }
                if (lo_ < e && col[lo_] == j) om = val[lo_];
            }
            acol[pos] = (int32_t)j;
            aom[pos] = om;
            if (M) {
                const E mij = m_upper && j < row ? ((const E*)M)[j * ldm + row] : Mrow[j];
                double gval = (double)mij + lam2 * om;
                if (j == row) gval -= 1.0 / om;
                agr[pos] = gval;
            }
            ++pos;
        }
        out += total;
    }
}

template <int MS>
__global__ void __launch_bounds__(NT)
cand_fill_kernel(const void* __restrict__ M, int64_t ldm, const int64_t* __restrict__ rowptr,
                 const int32_t* __restrict__ col, const double* __restrict__ val, int64_t p,
                 double lam2, const uint64_t* __restrict__ bitmap, int64_t nwords,
                 const int64_t* __restrict__ arow, int32_t* __restrict__ acol,
                 double* __restrict__ aom, double* __restrict__ agr, const int* overflow,
                 const uint64_t* __restrict__ tmask, bool m_upper) {
    cand_fill_body<MS>(blockIdx.x, M, ldm, rowptr, col, val, p, lam2, bitmap, nwords, arow, acol, aom, agr, overflow, tmask, m_upper);
}

// Cov form: the gradient on the candidates, G_ij = M_ij + lam2 omega_ij - [i == j] / omega_ii,
// with M_ij gathered from S by m_entry (no dense M).  Wave per row, lanes over the row's
// candidates; the row-i half of every entry walks the same nonzeros in every lane.
template <int BS>
__device__ __forceinline__ void cand_grad_cov_body(int64_t bx_, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                     const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                     int64_t lds, double lam2, const int64_t* __restrict__ arow,
                     const int32_t* __restrict__ acol, const double* __restrict__ aom,
                     double* __restrict__ agr, const int* overflow) {
    if (*overflow) return;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = arow[row], e = arow[row + 1];
    for (int64_t k0 = s; k0 < e; k0 += 64) {
        const int64_t k = k0 + lane;
        const bool act = k < e;
        const int64_t j = act ? acol[k] : row;
        const double m = m_entry<BS>(rowptr, col, val, S, lds, row, j);
        if (act) {
            const double om = aom[k];
            double g = m + lam2 * om;
            if (j == row) g -= 1.0 / om;
            agr[k] = g;
        }
    }
}

template <int BS>
__global__ void __launch_bounds__(NT)
cand_grad_cov_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                     const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                     int64_t lds, double lam2, const int64_t* __restrict__ arow,
                     const int32_t* __restrict__ acol, const double* __restrict__ aom,
                     double* __restrict__ agr, const int* overflow) {
    cand_grad_cov_body<BS>(blockIdx.x, rowptr, col, val, p, S, lds, lam2, arow, acol, aom, agr, overflow);
}

// ---- scan ---------------------------------------------------------------------
// Two-kernel exclusive scan: chunk sums, then each chunk adds the sums before it and
// scans itself.  Integer sums, so the result does not depend on the split.

__device__ inline int64_t block_sum_i64(int64_t v, int64_t* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0) red[wave] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < WPB; ++w) t += red[w];
    return t;
}

__device__ __forceinline__ void scan_part_body(int64_t bx_, const int64_t* __restrict__ cnt, int64_t p, int64_t* __restrict__ part) {
    __shared__ int64_t red[WPB];
    const int64_t base = bx_ * SCAN_CHUNK;
    int64_t s = 0;
#pragma unroll
    for (int e = 0; e < SCAN_CHUNK / NT; ++e) {
        const int64_t i = base + e * NT + threadIdx.x;
        if (i < p) s += cnt[i];
    }
    s = block_sum_i64(s, red);
    if (threadIdx.x == 0) part[bx_] = s;
}

__global__ void __launch_bounds__(NT)
scan_part_kernel(const int64_t* __restrict__ cnt, int64_t p, int64_t* __restrict__ part) {
    scan_part_body(blockIdx.x, cnt, p, part);
}

__device__ __forceinline__ void scan_apply_body(int64_t bx_, int64_t nb_, const int64_t* __restrict__ cnt, int64_t p, const int64_t* __restrict__ part,
                  int64_t* __restrict__ out, int64_t cap, int* overflow, int64_t* total_out) {
    __shared__ int64_t red[WPB];
    __shared__ int64_t wtot[WPB];
    const int64_t b = bx_;
    int64_t o = 0;
    for (int64_t k = threadIdx.x; k < b; k += NT) o += part[k];
    const int64_t off = block_sum_i64(o, red);
    constexpr int PER = SCAN_CHUNK / NT;
    const int64_t i0 = b * SCAN_CHUNK + (int64_t)threadIdx.x * PER;
    int64_t v[PER];
    int64_t ts = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        v[e] = i0 + e < p ? cnt[i0 + e] : 0;
        ts += v[e];
    }
    // exclusive scan of the thread sums: within the wave, then over the waves
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t incl = ts;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t up = __shfl_up(incl, d, 64);
        if (lane >= d) incl += up;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int64_t before = 0, btotal = 0;
#pragma unroll
    for (int w = 0; w < WPB; ++w) {
        before += w < wave ? wtot[w] : 0;
        btotal += wtot[w];
    }
    int64_t run = off + before + incl - ts;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        if (i0 + e < p) out[i0 + e] = run;
        run += v[e];
    }
    if (b == nb_ - 1 && threadIdx.x == 0) {
        const int64_t total = off + btotal;
        out[p] = total;
        if (overflow) *overflow = total > cap ? 1 : 0;
        if (total_out) *total_out = total;
    }
}

__global__ void __launch_bounds__(NT)
scan_apply_kernel(const int64_t* __restrict__ cnt, int64_t p, const int64_t* __restrict__ part,
                  int64_t* __restrict__ out, int64_t cap, int* overflow, int64_t* total_out) {
    scan_apply_body(blockIdx.x, gridDim.x, cnt, p, part, out, cap, overflow, total_out);
}

// ---- trial evaluation ---------------------------------------------------------
constexpr int MAXQ = 8;

__device__ inline double prox_one(double om, double g, double tau, double thr, bool diag) {
    const double z = om - tau * g;
    if (diag) return z;
    return z > thr ? z - thr : (z < -thr ? z + thr : 0.0);
}

// Cov trials, the quadratic term of one candidate b of row `row`: squad[q] += Delta_a(q)
// S[j_a][j_b] Delta_b(q) over the row's candidates a in order s .. e - 1.  The entries of
// four candidates a, then their four S values, are loaded before any of their arithmetic
// (a row's candidates are a chain of dependent loads otherwise); the products and their
// order are those of one candidate at a time.
template <int BS>
__device__ __forceinline__ void cov_quad_b(const int32_t* __restrict__ acol,
                                           const double* __restrict__ aom,
                                           const double* __restrict__ agr, int64_t s, int64_t e,
                                           int64_t row, int64_t jb, const void* __restrict__ B,
                                           int64_t ldb, double tau0, double shrink, double lam1,
                                           int m, const double (&db)[MAXQ], double (&squad)[MAXQ]) {
    auto one = [&](int64_t ja, double oma, double ga, double sab) {
        const bool diaga = ja == row;
        double tau = tau0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            if (q < m) {
                const double da = prox_one(oma, ga, tau, tau * lam1, diaga) - oma;
                squad[q] += da * sab * db[q];
            }
            tau *= shrink;
        }
    };
    int64_t ka = s;
    for (; ka + 4 <= e; ka += 4) {
        int64_t ja[4];
        double oma[4], ga[4], sab[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ja[u] = acol[ka + u];
            oma[u] = aom[ka + u];
            ga[u] = agr[ka + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) sab[u] = load_one_d<BS>(B, ja[u] * ldb + jb);
#pragma unroll
        for (int u = 0; u < 4; ++u) one(ja[u], oma[u], ga[u], sab[u]);
    }
    for (; ka < e; ++ka) {
        const int64_t ja = acol[ka];
        one(ja, aom[ka], agr[ka], load_one_d<BS>(B, ja * ldb + jb));
    }
}

template <int BS, bool OBS>
__device__ __forceinline__ void trial_body(int64_t bx_, int split, int nsplit, const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
             const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
             double tau0, double shrink, int m, double lam1, const void* __restrict__ B,
             int64_t ldb, int64_t ncols, const double* __restrict__ xn2, double* __restrict__ part,
             const DevState* st) {
    if (st->overflow || st->accepted_q >= 0) return;   // capacity exceeded or already decided
    typedef Chunk<BS> Ch;
    typedef typename Ch::T T;
    constexpr int V = Ch::V;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = arow[row], e = arow[row + 1];
    // blockIdx.y = column split of the Obs quadratic term; split 0 also does the
    // elementwise terms.  Partials land in part[((q*4 + t) * nsplit + split) * p + row].
    double slog[MAXQ], sdd[MAXQ], squad[MAXQ], snp[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) { slog[q] = 0; sdd[q] = 0; squad[q] = 0; snp[q] = 0; }

    // elementwise terms (lanes over entries)
    for (int64_t k = s + lane; split == 0 && k < e; k += 64) {
        const int64_t j = acol[k];
        const double om = aom[k], g = agr[k];
        const bool diag = j == row;
        double tau = tau0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            if (q < m) {
                const double wp = prox_one(om, g, tau, tau * lam1, diag);
                const double d = wp - om;
                sdd[q] += d * d;
                if (diag) {
                    if (wp <= 0.0) snp[q] += 1.0;
                    else {
                        const double x = d / om;
                        slog[q] += x - log1p(x);
                    }
                }
            }
            tau *= shrink;
        }
    }
    // quadratic term
    if (OBS && e > s && e - s <= 4) {
        // A row of at most 4 candidates (the common case): the same sums as the general
        // loop below, with the next column chunk's row loads issued before the current
        // chunk's FMAs.  The Delta values do not depend on the column and are formed once.
        const int cnt = (int)(e - s);
        T dq[4][MAXQ];
        int64_t rb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = s + (u < cnt ? u : 0);
            rb[u] = (int64_t)acol[k] * ldb;
            const double om = aom[k], g = agr[k];
            const bool diag = acol[k] == row;
            double tau = tau0;
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                dq[u][q] = (T)(prox_one(om, g, tau, tau * lam1, diag) - om);
                tau *= shrink;
            }
        }
        const int64_t cstep = (int64_t)nsplit * 64 * V;
        if (cnt == 1 && xn2) {
            // one candidate (i, j): Delta_i X^T = delta X^T_j, so the row's term is
            // delta^2 ||X^T_j||^2, from the row norms of X^T (no pass over X^T)
            if (split == 0 && lane == 0) {
                const double nj = xn2[acol[s]];
#pragma unroll
                for (int q = 0; q < MAXQ; ++q) {
                    const double d = (double)dq[0][q];
                    if (q < m) squad[q] = d * d * nj;
                }
            }
        } else if (cnt == 1) {
            // one candidate (a row whose only candidate is the diagonal): one row of B,
            // read PD chunks ahead (the two-chunk pipeline below keeps too few bytes in
            // flight for a single row); the same products and sums in the same order
            constexpr int PD = 8;
            T b1[PD][V];
            const int64_t c00 = (int64_t)split * 64 * V;
#pragma unroll
            for (int d = 0; d < PD; ++d) {
                const int64_t c = c00 + d * cstep + lane * V;
                if (c < ncols) Ch::load(B, rb[0] + c, b1[d]);
                else {
#pragma unroll
                    for (int t = 0; t < V; ++t) b1[d][t] = 0;
                }
            }
            for (int64_t c0 = c00; c0 < ncols; c0 += PD * cstep) {
#pragma unroll
                for (int d = 0; d < PD; ++d) {
                    if (c0 + d * cstep >= ncols) break;
#pragma unroll
                    for (int q = 0; q < MAXQ; ++q) {
                        if (q < m) {
#pragma unroll
                            for (int t = 0; t < V; ++t) {
                                const T a = fma(dq[0][q], b1[d][t], (T)0);
                                squad[q] += (double)a * (double)a;
                            }
                        }
                    }
                    const int64_t c = c0 + (d + PD) * cstep + lane * V;
                    if (c < ncols) Ch::load(B, rb[0] + c, b1[d]);
                }
            }
        } else {
        auto fetch = [&](int64_t c0, T (&b)[4][V]) {
            const int64_t c = c0 + lane * V;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < cnt && c < ncols) Ch::load(B, rb[u] + c, b[u]);
                else {
#pragma unroll
                    for (int t = 0; t < V; ++t) b[u][t] = 0;
                }
            }
        };
        T bc[4][V], bn[4][V];
        int64_t c0 = (int64_t)split * 64 * V;
        if (c0 < ncols) fetch(c0, bc);
        for (; c0 < ncols; c0 += cstep) {
            if (c0 + cstep < ncols) fetch(c0 + cstep, bn);
            T acc[MAXQ][V];
#pragma unroll
            for (int q = 0; q < MAXQ; ++q)
#pragma unroll
                for (int t = 0; t < V; ++t) acc[q][t] = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u >= cnt) break;
#pragma unroll
                for (int q = 0; q < MAXQ; ++q) {
                    if (q < m) {
#pragma unroll
                        for (int t = 0; t < V; ++t) acc[q][t] = fma(dq[u][q], bc[u][t], acc[q][t]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                if (q < m) {
#pragma unroll
                    for (int t = 0; t < V; ++t) squad[q] += (double)acc[q][t] * (double)acc[q][t];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < V; ++t) bc[u][t] = bn[u][t];
        }
        }
    } else if (OBS) {
        // ||Delta_i X^T||^2 over n columns: lanes over columns, loop over entries
        for (int64_t c0 = (int64_t)split * 64 * V; c0 < ncols; c0 += (int64_t)nsplit * 64 * V) {
            const int64_t c = c0 + lane * V;
            const bool act = c < ncols;
            T acc[MAXQ][V];
#pragma unroll
            for (int q = 0; q < MAXQ; ++q)
#pragma unroll
                for (int t = 0; t < V; ++t) acc[q][t] = 0;
            // entries in groups of 4: the group's row loads are issued before its FMAs
            // (one memory latency per group instead of per entry); same FMA order
            constexpr int EG = 4;
            for (int64_t k0 = s; k0 < e; k0 += EG) {
                T b[EG][V];
#pragma unroll
                for (int u = 0; u < EG; ++u) {
                    const int64_t k = k0 + u;
                    if (act && k < e) Ch::load(B, (int64_t)acol[k] * ldb + c, b[u]);
                    else {
#pragma unroll
                        for (int t = 0; t < V; ++t) b[u][t] = 0;
                    }
                }
#pragma unroll
                for (int u = 0; u < EG; ++u) {
                    const int64_t k = k0 + u;
                    if (k >= e) break;
                    const double om = aom[k], g = agr[k];
                    const bool diag = acol[k] == row;
                    double tau = tau0;
#pragma unroll
                    for (int q = 0; q < MAXQ; ++q) {
                        if (q < m) {
                            const T d = (T)(prox_one(om, g, tau, tau * lam1, diag) - om);
#pragma unroll
                            for (int t = 0; t < V; ++t) acc[q][t] = fma(d, b[u][t], acc[q][t]);
                        }
                        tau *= shrink;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                if (q < m) {
#pragma unroll
                    for (int t = 0; t < V; ++t) squad[q] += (double)acc[q][t] * (double)acc[q][t];
                }
            }
        }
    } else {
        // sum_{a,b in A_i} Delta_a S[j_a, j_b] Delta_b : lanes over b, loop over a
        for (int64_t kb = s + lane; kb < e; kb += 64) {
            const int64_t jb = acol[kb];
            const double omb = aom[kb], gb = agr[kb];
            const bool diagb = jb == row;
            double db[MAXQ];
            {
                double tau = tau0;
#pragma unroll
                for (int q = 0; q < MAXQ; ++q) {
                    db[q] = q < m ? prox_one(omb, gb, tau, tau * lam1, diagb) - omb : 0.0;
                    tau *= shrink;
                }
            }
            cov_quad_b<BS>(acol, aom, agr, s, e, row, jb, B, ldb, tau0, shrink, lam1, m, db, squad);
        }
    }
    // The 4 * MAXQ = 32 lane partials (value k = 4q + t) summed over the wave by a
    // reduce-scatter butterfly: each step keeps half of the values and adds the partner
    // lane's copy of them (16 + 8 + 4 + 2 + 1 shuffles), leaving value lane >> 1 summed
    // over the 32 lanes that share bit 0, and a last exchange adds the other 32.  Fixed
    // order, so the sums are reproducible.
    double v[4 * MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        v[4 * q + 0] = slog[q];
        v[4 * q + 1] = sdd[q];
        v[4 * q + 2] = squad[q];
        v[4 * q + 3] = snp[q];
    }
#pragma unroll
    for (int n = 4 * MAXQ, o = 32; n > 1; n >>= 1, o >>= 1) {
        const bool upper = (lane & o) != 0;   // keep the upper half of the n values
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            const double send = upper ? v[i] : v[i + n / 2];
            const double keep = upper ? v[i + n / 2] : v[i];
            v[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    const double tot = v[0] + __shfl_xor(v[0], 1, 64);
    const int k = lane >> 1, q = k >> 2, t = k & 3;
    if ((lane & 1) == 0 && q < m) part[((int64_t)(q * 4 + t) * nsplit + split) * p + row] = tot;
}

template <int BS, bool OBS>
__global__ void __launch_bounds__(NT)
trial_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
             const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
             double tau0, double shrink, int m, double lam1, const void* __restrict__ B,
             int64_t ldb, int64_t ncols, const double* __restrict__ xn2,
             double* __restrict__ part, const DevState* st) {
    trial_body<BS, OBS>(blockIdx.x, blockIdx.y, gridDim.y, arow, acol, aom, agr, p, tau0, shrink,
                        m, lam1, B, ldb, ncols, xn2, part, st);
}

// Squared norms of the rows of X^T (||X^T_j||^2 = n S_jj) in FP64: one wave per row,
// lane l adds the squares of its chunks of columns in column order, then a butterfly over
// the wave (every lane ends with the same sum).  Read by the Obs trials for rows with a
// single candidate.
template <int BS>
__global__ void __launch_bounds__(NT)
row_norm2_kernel(const void* __restrict__ B, int64_t ldb, int64_t ncols, int64_t p,
                 double* __restrict__ out) {
    typedef Chunk<BS> Ch;
    typedef typename Ch::T T;
    constexpr int V = Ch::V;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni((int64_t)blockIdx.x * WPB + wave);
    if (row >= p) return;
    double sum = 0.0;
    for (int64_t c = (int64_t)lane * V; c < ncols; c += 64 * V) {
        T v[V];
        Ch::load(B, row * ldb + c, v);
#pragma unroll
        for (int t = 0; t < V; ++t) sum += (double)v[t] * (double)v[t];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane == 0) out[row] = sum;
}

// Cov trials with 8 lanes per row (8 rows per wave): a Cov candidate row holds a few
// entries, so a whole wave per row would leave most lanes idle.  Same terms as
// trial_kernel's Cov path; the 32 partials are reduced over the row's 8 lanes by a
// reduce-scatter (16 + 8 + 4 shuffles), after which lane g of the group holds the four
// sums of step size q = g.
constexpr int TG = 8;
constexpr int64_t COV_GROUP_MIN_P = COV_TRIAL_GROUP_MIN_P;
template <int BS>
__device__ __forceinline__ void trial_cov_body(int64_t bx_, const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                 const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                 double tau0, double shrink, int m, double lam1, const void* __restrict__ B,
                 int64_t ldb, double* __restrict__ part, const DevState* st) {
    if (st->overflow || st->accepted_q >= 0) return;   // capacity exceeded or already decided
    const int lane = lane_id(), g = lane & (TG - 1);
    const int64_t row = (bx_ * WPB + (threadIdx.x >> 6)) * (64 / TG) + (lane / TG);
    const bool act = row < p;
    const int64_t s = act ? arow[row] : 0, e = act ? arow[row + 1] : 0;
    double slog[MAXQ], sdd[MAXQ], squad[MAXQ], snp[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) { slog[q] = 0; sdd[q] = 0; squad[q] = 0; snp[q] = 0; }
    for (int64_t k = s + g; k < e; k += TG) {
        const int64_t j = acol[k];
        const double om = aom[k], gr = agr[k];
        const bool diag = j == row;
        double tau = tau0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            if (q < m) {
                const double wp = prox_one(om, gr, tau, tau * lam1, diag);
                const double d = wp - om;
                sdd[q] += d * d;
                if (diag) {
                    if (wp <= 0.0) snp[q] += 1.0;
                    else {
                        const double x = d / om;
                        slog[q] += x - log1p(x);
                    }
                }
            }
            tau *= shrink;
        }
    }
    // sum_{a,b in A_i} Delta_a S[j_a, j_b] Delta_b : the group's lanes over b, loop over a
    for (int64_t kb = s + g; kb < e; kb += TG) {
        const int64_t jb = acol[kb];
        const double omb = aom[kb], gb = agr[kb];
        const bool diagb = jb == row;
        double db[MAXQ];
        {
            double tau = tau0;
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                db[q] = q < m ? prox_one(omb, gb, tau, tau * lam1, diagb) - omb : 0.0;
                tau *= shrink;
            }
        }
        cov_quad_b<BS>(acol, aom, agr, s, e, row, jb, B, ldb, tau0, shrink, lam1, m, db, squad);
    }
    double v[4 * MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        v[4 * q + 0] = slog[q];
        v[4 * q + 1] = sdd[q];
        v[4 * q + 2] = squad[q];
        v[4 * q + 3] = snp[q];
    }
#pragma unroll
    for (int n = 4 * MAXQ, o = TG / 2; n > 4; n >>= 1, o >>= 1) {
        const bool upper = (g & o) != 0;   // keep the upper half of the n values
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            const double send = upper ? v[i] : v[i + n / 2];
            const double keep = upper ? v[i + n / 2] : v[i];
            v[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    // lane g now holds values 4g .. 4g + 3: the four sums of step size q = g
    if (act && g < m) {
#pragma unroll
        for (int t = 0; t < 4; ++t) part[(int64_t)(g * 4 + t) * p + row] = v[t];
    }
}

template <int BS>
__global__ void __launch_bounds__(NT)
trial_cov_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                 const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                 double tau0, double shrink, int m, double lam1, const void* __restrict__ B,
                 int64_t ldb, double* __restrict__ part, const DevState* st) {
    trial_cov_body<BS>(blockIdx.x, arow, acol, aom, agr, p, tau0, shrink, m, lam1, B, ldb, part, st);
}

// ---- decision ----------------------------------------------------------------
__device__ void decide_one(const double* __restrict__ sums, int m, double tau0, double shrink,
                           int q_base, double lam2, double inv_n, int forced_q, DevState* st) {
    if (st->overflow || st->accepted_q >= 0) return;   // capacity exceeded / decided earlier
    double tau = tau0;
    for (int q = 0; q < m; ++q) {
        const double slog = sums[q * 4 + 0], dd = sums[q * 4 + 1], quad = sums[q * 4 + 2],
                     np = sums[q * 4 + 3];
        const double lhs = slog + 0.5 * quad * inv_n + 0.5 * lam2 * dd;
        const double rhs = dd / (2.0 * tau);
        for (int t = 0; t < 4; ++t) st->sums[q * 4 + t] = sums[q * 4 + t];
        bool ok;
        if (forced_q >= 0) {
            ok = (q_base + q) == forced_q;
            if (ok && np > 0.0) st->nonpos = 1;
        } else {
            ok = np == 0.0 && lhs <= rhs;
        }
        if (ok) {
            st->accepted = st->nonpos ? 0 : 1;
            st->accepted_q = q_base + q;
            st->tau = tau;
            st->lhs = lhs;
            st->rhs = rhs;
            st->dd = dd;
            return;
        }
        tau *= shrink;
    }
}

// objective sums (log-diagonal, squares, off-diagonal |.|, sum W o Omega) and the nysq
// ||Y||^2 chunk sums into the state, when gated on
__device__ void obj_finish_one(const double* __restrict__ sums, int nysq, DevState* st,
                               const int* gate) {
    if (gate && *gate == 0) return;
    st->obj[0] = sums[0];
    st->obj[1] = sums[1];
    st->obj[2] = sums[2];
    st->obj[3] = sums[3];
    double y = 0.0;
    for (int i = 0; i < nysq; ++i) y += sums[4 + i];
    st->obj[4] = y;
}

struct FinArgs {
    int m, q_base, forced_q, nysq;
    double tau0, shrink, lam2, inv_n;
    const int* gate;
};
enum { FIN_DECIDE = 0, FIN_OBJ = 1 };

// ---- column sums ---------------------------------------------------------------
// Column sums with the step that consumes them in the same launch, in two fixed-order
// stages.  Block (c, b) sums segment b of column c (thread-strided, then an LDS tree)
// into ws[c * nseg + b], then takes a ticket (device-scope atomic after a device-scope
// release fence); the
// block that takes the last ticket adds each column's segment sums in segment order,
// returns the ticket counter to 0 for the next launch and runs the decision (FIN_DECIDE)
// or the objective copy (FIN_OBJ).  No block waits for another, so the kernel always
// completes; the association of every sum depends only on (rows, nseg).
template <int FIN>
__device__ __forceinline__ void colsum_finish_body(int c_, int b_, int ncol_, int nseg_, const double* __restrict__ in, int64_t rows, int64_t seg,
                     double* __restrict__ ws, double* __restrict__ out, unsigned* ticket,
                     FinArgs fa, DevState* st) {
    __shared__ double red[NT];
    __shared__ int last;
    const int c = c_, b = b_, t = threadIdx.x;
    const int ncol = ncol_, nseg = nseg_;
    const double* a = in + (int64_t)c * rows;
    const int64_t lo = (int64_t)b * seg, hi = lo + seg < rows ? lo + seg : rows;
    double s = 0.0;
    for (int64_t i = lo + t; i < hi; i += NT) s += a[i];
    red[t] = s;
    __syncthreads();
    for (int o = NT / 2; o >= 1; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) {
        ws[(int64_t)c * nseg + b] = red[0];
        __threadfence();
        last = atomicAdd(ticket, 1u) == (unsigned)(ncol * nseg - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int k = t; k < ncol; k += NT) {
        double v = ws[(int64_t)k * nseg];
        for (int j = 1; j < nseg; ++j) v += ws[(int64_t)k * nseg + j];
        out[k] = v;
    }
    __syncthreads();
    if (t == 0) {
        *ticket = 0u;
        if (FIN == FIN_DECIDE)
            decide_one(out, fa.m, fa.tau0, fa.shrink, fa.q_base, fa.lam2, fa.inv_n, fa.forced_q, st);
        else
            obj_finish_one(out, fa.nysq, st, fa.gate);
    }
}

template <int FIN>
__global__ void __launch_bounds__(NT)
colsum_finish_kernel(const double* __restrict__ in, int64_t rows, int64_t seg,
                     double* __restrict__ ws, double* __restrict__ out, unsigned* ticket,
                     FinArgs fa, DevState* st) {
    colsum_finish_body<FIN>(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y, in, rows, seg, ws, out, ticket, fa, st);
}

// ---- emission ----------------------------------------------------------------
__device__ __forceinline__ void emit_count_body(int64_t bx_, const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                  const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                  double lam1, const DevState* st, int64_t* __restrict__ cnt) {
    if (st->accepted_q < 0 || st->nonpos) return;
    const double tau = st->tau;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = arow[row], e = arow[row + 1];
    int c = 0;
    for (int64_t k = s + lane; k < e; k += 64) {
        const bool diag = acol[k] == row;
        const double wp = prox_one(aom[k], agr[k], tau, tau * lam1, diag);
        c += (wp != 0.0 || diag) ? 1 : 0;
    }
    double t = wave_sum((double)c);
    if (lane == 0) cnt[row] = (int64_t)t;
}

__global__ void __launch_bounds__(NT)
emit_count_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                  const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                  double lam1, const DevState* st, int64_t* __restrict__ cnt) {
    emit_count_body(blockIdx.x, arow, acol, aom, agr, p, lam1, st, cnt);
}

__device__ __forceinline__ void emit_fill_body(int64_t bx_, const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                 const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                 double lam1, const DevState* st, const int64_t* __restrict__ orow,
                 int32_t* __restrict__ ocol, double* __restrict__ oval) {
    if (st->accepted_q < 0 || st->nonpos) return;
    const double tau = st->tau;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = arow[row], e = arow[row + 1];
    int64_t out = orow[row];
    for (int64_t k0 = s; k0 < e; k0 += 64) {
        const int64_t k = k0 + lane;
        bool keep = false;
        double wp = 0.0;
        int32_t j = 0;
        if (k < e) {
            j = acol[k];
            const bool diag = j == row;
            wp = prox_one(aom[k], agr[k], tau, tau * lam1, diag);
            keep = wp != 0.0 || diag;
        }
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const int64_t pos = out + __popcll(mask & lanemask_lt());
            ocol[pos] = j;
            oval[pos] = wp;
        }
        out += __popcll(mask);
    }
}

__global__ void __launch_bounds__(NT)
emit_fill_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                 const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                 double lam1, const DevState* st, const int64_t* __restrict__ orow,
                 int32_t* __restrict__ ocol, double* __restrict__ oval) {
    emit_fill_body(blockIdx.x, arow, acol, aom, agr, p, lam1, st, orow, ocol, oval);
}

// ---- objective partials --------------------------------------------------------
template <int WS>
__global__ void __launch_bounds__(NT)
obj_parts_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ val, int64_t p, const void* __restrict__ W,
                 int64_t ldw, double* __restrict__ part, const int* gate) {
    if (gate && *gate == 0) return;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni((int64_t)blockIdx.x * WPB + wave);
    if (row >= p) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    double lg = 0, sq = 0, l1 = 0, wv = 0;
    for (int64_t k = s + lane; k < e; k += 64) {
        const int64_t j = col[k];
        const double v = val[k];
        sq += v * v;
        if (j == row) lg += log(v);
        else l1 += fabs(v);
        if (W) wv += load_one_d<WS>(W, row * ldw + j) * v;
    }
    lg = wave_sum(lg); sq = wave_sum(sq); l1 = wave_sum(l1); wv = wave_sum(wv);
    if (lane == 0) {
        part[0 * p + row] = lg;
        part[1 * p + row] = sq;
        part[2 * p + row] = l1;
        part[3 * p + row] = wv;
    }
}

// Cov form: the same four partials, the last as sum_j M_ij omega_ij with M_ij gathered
// from S (m_entry) on the support.
template <int BS>
__device__ __forceinline__ void obj_parts_cov_body(int64_t bx_, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                     const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                     int64_t lds, double* __restrict__ part, const int* gate) {
    if (gate && *gate == 0) return;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    double lg = 0, sq = 0, l1 = 0, wv = 0;
    for (int64_t k0 = s; k0 < e; k0 += 64) {
        const int64_t k = k0 + lane;
        const bool act = k < e;
        const int64_t j = act ? col[k] : row;
        const double m = m_entry<BS>(rowptr, col, val, S, lds, row, j);
        if (act) {
            const double v = val[k];
            sq += v * v;
            if (j == row) lg += log(v);
            else l1 += fabs(v);
            wv = fma(m, v, wv);
        }
    }
    lg = wave_sum(lg); sq = wave_sum(sq); l1 = wave_sum(l1); wv = wave_sum(wv);
    if (lane == 0) {
        part[0 * p + row] = lg;
        part[1 * p + row] = sq;
        part[2 * p + row] = l1;
        part[3 * p + row] = wv;
    }
}

template <int BS>
__global__ void __launch_bounds__(NT)
obj_parts_cov_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                     const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                     int64_t lds, double* __restrict__ part, const int* gate) {
    obj_parts_cov_body<BS>(blockIdx.x, rowptr, col, val, p, S, lds, part, gate);
}

__global__ void smooth_finish_kernel(const DevState* st, double dn, double lam2, double* f) {
    if (threadIdx.x == 0) {
        double F;
        objective_value(st->obj, true, dn, 0.0, lam2, f, &F);
    }
}

__global__ void identity_kernel(int64_t* rowptr, int32_t* col, double* val, int64_t p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p) { rowptr[i] = i; col[i] = (int32_t)i; val[i] = 1.0; }
    if (i == p) rowptr[p] = p;
}

// ---- Cov refresh: M = (W + W^T) / 2 with W = Omega S, one pass -------------------
// Tile-pair order: bands of RG = 8 tile-rows, each walked column block by column block,
// so the 8 tiles of one column block share the S rows of their band's supports.
// Workgroup w runs on XCD w % 8 (one L2 per XCD); in every run of 64 workgroups, XCD x
// is given the 8 tiles of column block 8a + x, so one XCD's L2 serves a column block
// while the 8 XCDs work on 8 neighbouring blocks of the same band (sharing the MALL).
// The mapping is closed-form (a square root per workgroup): a walk over the bands costs
// T / RG scalar steps before the first load, which dominated the kernel at p ~ 10^5.
constexpr int RG = 8;
__device__ inline int2 refresh_tile(int w, int T, int ntiles) {
    int64_t t = w;
    if (w < ntiles / 64 * 64) {
        const int a = w >> 6, b = (w >> 3) & 7, x = w & 7;
        t = 64 * a + 8 * x + b;
    }
    // full bands b' < b hold P(b) = b (G(G+1)/2 + G(T-G)) - G^2 b(b-1)/2 tiles
    constexpr int64_t G = RG;
    const int64_t nfull = T / G, c1 = G * (G + 1) / 2 + G * (T - G);
    auto P = [&](int64_t b) { return b * c1 - G * G * b * (b - 1) / 2; };
    const double q = (double)c1 + 0.5 * G * G;
    const double disc = q * q - 2.0 * G * G * (double)t;
    int64_t b = (int64_t)((q - sqrt(disc > 0.0 ? disc : 0.0)) / (double)(G * G));
    b = b < 0 ? 0 : (b > nfull ? nfull : b);
    while (b > 0 && P(b) > t) --b;
    while (b < nfull && P(b + 1) <= t) ++b;
    t -= P(b);
    const int64_t i0 = b * G, h = T - i0 < G ? T - i0 : G;
    const int64_t tri = h * (h + 1) / 2;
    if (t < tri) {
        // column jj of the band's triangle holds jj + 1 tiles
        int64_t jj = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (jj > 0 && jj * (jj + 1) / 2 > t) --jj;
        while ((jj + 1) * (jj + 2) / 2 <= t) ++jj;
        return make_int2((int)(i0 + t - jj * (jj + 1) / 2), (int)(i0 + jj));
    }
    t -= tri;
    return make_int2((int)(i0 + t % h), (int)(i0 + h + t / h));
}

// FP32 test threshold: |m| > lam1 holds for an FP32 m exactly when |m| > lam1 rounded down.
template <typename E> __device__ inline E test_threshold(double lam1) {
    E thr = (E)lam1;
    if (sizeof(E) == 4 && (double)thr > lam1) thr = __int_as_float(__float_as_int((float)thr) - 1);
    return thr;
}

// One tile pair (I, J) of the refresh; every branch is uniform in the workgroup.
template <int BS>
__device__ __forceinline__ void refresh_pair(const int I, const int J,
                                             const int64_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ col,
                                             const double* __restrict__ val, int64_t p,
                                             const void* __restrict__ S, int64_t lds,
                                             const double* __restrict__ smax, int T, double lam1,
                                             uint64_t* __restrict__ tbits, int64_t nwords,
                                             unsigned long long* __restrict__ active) {
    typedef typename Chunk<BS>::T A;                          // accumulation type
    typedef typename MType<BS>::T E;                          // type of M
    __shared__ E wt[64][65];   // W_JI, then M_IJ read transposed for the rows of J
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = (int64_t)I * 64, j0 = (int64_t)J * 64;

    // W_IJ[i][j] = sum_{k in supp_i} omega_ik S[k][j] for this wave's 16 rows of tile I and
    // W_JI[j][i] = sum_{k in supp_j} omega_jk S[k][i] for the same 16 rows of tile J (on a
    // diagonal pair the same rows twice); M_IJ = (W_IJ + W_JI^T) / 2.  Every row's nonzeros
    // are uniform in the wave, so each load reads 64 consecutive columns of one S row.
    // Lane h < 16 holds the CSR range of I-row h and lane 16 + h that of J-row h, fetched
    // up front; each step fetches all 32 rows' next entries with one vector load and
    // broadcasts them by readlane.  With 4-byte accumulators both halves' 32 S loads are
    // issued before the first FMA; with 8-byte ones the halves run one after the other
    // (register budget).  Rows past their last nonzero (or past p, where they start at
    // entry 0) re-read a valid entry and keep their sum.
    constexpr bool PAIR = sizeof(A) == 4;
    const int hl = lane & 31;
    const int64_t myrow = (hl < 16 ? i0 : j0) + wave * 16 + (hl & 15);
    int64_t my_s0 = 0;
    int my_cnt = 0;
    if (myrow < p) {
        my_s0 = rowptr[myrow];
        my_cnt = (int)(rowptr[myrow + 1] - my_s0);
    }
    // Exact screening of the pair: |W_ij| <= bw(i) = sum_{k in supp_i} |omega_ik| smax[k/64][J]
    // with smax the largest |S| of each 64 x 64 tile, and likewise bv(j) for W_JI, so
    // |M_ij| <= (max_i bw(i) + max_j bv(j)) / 2.  If that bound (widened by the FMA
    // chains' rounding) is at most the threshold, no test in the pair passes and the
    // S loads are skipped.  Diagonal pairs (which hold the j == i bits) always run.
    double rbound = 0.0;
    const bool screen = smax != nullptr;
    if (I != J && screen) {
        // four entries' loads, then their tile maxima, before the sums (same order)
        const int64_t other = hl < 16 ? J : I;
        int m = 0;
        for (; m + 4 <= my_cnt; m += 4) {
            int32_t c[4];
            double v[4], sm[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = col[my_s0 + m + u];
                v[u] = val[my_s0 + m + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) sm[u] = smax[(int64_t)(c[u] >> 6) * T + other];
#pragma unroll
            for (int u = 0; u < 4; ++u) rbound += fabs(v[u]) * sm[u];
        }
        for (; m < my_cnt; ++m)
            rbound += fabs(val[my_s0 + m]) * smax[(int64_t)(col[my_s0 + m] >> 6) * T + other];
    }
    int mx = my_cnt;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) {
        const int other = __shfl_xor(mx, o, 64);
        mx = other > mx ? other : mx;
        const double ob = __shfl_xor(rbound, o, 64);
        rbound = ob > rbound ? ob : rbound;
    }
    const int maxI = __builtin_amdgcn_readlane(mx, 0), maxJ = __builtin_amdgcn_readlane(mx, 16);
    const E thr = test_threshold<E>(lam1);
    const int64_t gj = j0 + lane;
    __shared__ uint32_t cms[4][64];
    if (I != J && screen) {
        __shared__ double bnd[4][2];
        if (lane == 0) bnd[wave][0] = rbound;
        if (lane == 16) bnd[wave][1] = rbound;
        int cmax = maxI > maxJ ? maxI : maxJ;
        if (lane == 0) cms[wave][0] = (uint32_t)cmax;
        __syncthreads();
        double bw = 0.0, bvv = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            bw = bnd[v][0] > bw ? bnd[v][0] : bw;
            bvv = bnd[v][1] > bvv ? bnd[v][1] : bvv;
            cmax = (int)cms[v][0] > cmax ? (int)cms[v][0] : cmax;
        }
        // relative rounding of an FP32 chain of c FMAs (and of omega's conversion) is
        // below (c + 2) 2^-24; 1% on top
        const double widen = 1.01 + (double)(cmax + 2) * 0x1p-23;
        if (0.5 * (bw + bvv) * widen <= (double)thr) {
            const int64_t mine = i0 + wave * 16 + lane;
            if (lane < 16 && mine < p) tbits[mine * nwords + J] = 0ull;
            if (wave == 0 && gj < p) tbits[gj * nwords + I] = 0ull;
            return;
        }
        __syncthreads();   // cms is reused below
    }
    if (active && threadIdx.x == 0) atomicAdd(active, 1ull);   // pairs that load S
    const uint32_t ci = (uint32_t)(i0 + lane), cj = (uint32_t)(j0 + lane);
    A w[16], wj[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) { w[q] = (A)0; wj[q] = (A)0; }

    // step m's entries of the 32 rows (value already converted to A)
    auto fetch = [&](int m, int& cl, A& v) {
        const int64_t k = my_s0 + (m < my_cnt ? m : 0);
        cl = col[k];
        v = (A)val[k];
    };
    auto bcast = [&](A x, int q) -> A {
        if (sizeof(A) == 4)
            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int((float)x), q));
        const int64_t b = __double_as_longlong((double)x);
        return (A)__longlong_as_double(
            ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(b >> 32), q) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((int)b, q));
    };
    // the 16 rows at lanes base .. base + 15 against columns c0 + lane
    auto issue = [&](int cl, int base, uint32_t c0, A (&x)[16]) {
        uint32_t off = c0;
        asm volatile("" : "+v"(off));   // a fresh 32-bit offset each step (scalar-base loads)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t cq = __builtin_amdgcn_readlane(cl, base + q);
            x[q] = (A)load_row_d<BS>(S, cq * lds, off);
        }
    };
    auto accum = [&](int m, int base, A v, const A (&x)[16], A (&acc)[16]) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const A f = fma(bcast(v, base + q), x[q], acc[q]);
            const int cnt_q = __builtin_amdgcn_readlane(my_cnt, base + q);
            acc[q] = m < cnt_q ? f : acc[q];
        }
    };
    // each step's entries are fetched while the previous step's S loads are in flight, so
    // a step waits for one round trip (its S loads), not two
    if (PAIR) {
        const int steps = maxI > maxJ ? maxI : maxJ;
        int cl = 0, cn = 0;
        A v = (A)0, vn = (A)0;
        if (steps > 0) fetch(0, cl, v);
        for (int m = 0; m < steps; ++m) {
            A x[16], xj[16];
            issue(cl, 0, cj, x);
            issue(cl, 16, ci, xj);
            if (m + 1 < steps) fetch(m + 1, cn, vn);
            __builtin_amdgcn_sched_barrier(0);   // keep the 32 loads ahead of their uses
            accum(m, 0, v, x, w);
            accum(m, 16, v, xj, wj);
            cl = cn;
            v = vn;
        }
    } else {
        int cl = 0, cn = 0;
        A v = (A)0, vn = (A)0;
        if (maxJ > 0) fetch(0, cl, v);
        for (int m = 0; m < maxJ; ++m) {
            A x[16];
            issue(cl, 16, ci, x);
            if (m + 1 < maxJ) fetch(m + 1, cn, vn);
            __builtin_amdgcn_sched_barrier(0);   // keep the 16 loads ahead of their uses
            accum(m, 16, v, x, wj);
            cl = cn;
            v = vn;
        }
        if (maxI > 0) fetch(0, cl, v);
        for (int m = 0; m < maxI; ++m) {
            A x[16];
            issue(cl, 0, cj, x);
            if (m + 1 < maxI) fetch(m + 1, cn, vn);
            __builtin_amdgcn_sched_barrier(0);
            accum(m, 0, v, x, w);
            cl = cn;
            v = vn;
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) wt[wave * 16 + q][lane] = (E)wj[q];   // W_JI (W_II if I == J)
    __syncthreads();
    // Threshold words of the next candidate set: word J of row i holds j == i or
    // |M_ij| > lam1 for the 64 columns of tile J, and by symmetry word I of row j the
    // same tests with i and j exchanged.  M itself is not stored: the gradient is needed
    // only on the candidates, where m_entry recomputes it bitwise.  The test is FP64's
    // |M_ij| > lam1 taken in M's type: for FP32, |m| > lam1 holds exactly when
    // |m| > lam1 rounded down to FP32.
    uint64_t wdir = 0;   // lane q < 16: the direct word of row i0 + 16 * wave + q
    uint32_t cm = 0;     // bit q: the test at (row i0 + 16 * wave + q, column gj)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = wave * 16 + q;
        const int64_t gi = i0 + r;
        const E m = (E)0.5 * ((E)w[q] + wt[lane][r]);
        const bool b = gi < p && gj < p && (gj == gi || (m < (E)0 ? -m : m) > thr);
        cm |= (uint32_t)b << q;
        const uint64_t word = __ballot(b);
        wdir = lane == q ? word : wdir;
    }
    const int64_t mine = i0 + wave * 16 + lane;
    if (lane < 16 && mine < p) tbits[mine * nwords + J] = wdir;
    if (I == J) return;
    // mirrored words: row gj, bits over the 64 rows of tile I (16 from each wave)
    cms[wave][lane] = cm;
    __syncthreads();
    if (wave == 0 && gj < p) {
        const uint64_t word = (uint64_t)cms[0][lane] | ((uint64_t)cms[1][lane] << 16) |
                              ((uint64_t)cms[2][lane] << 32) | ((uint64_t)cms[3][lane] << 48);
        tbits[gj * nwords + I] = word;
    }
}

// The refresh proper: workgroup w takes entry w of the list of tile pairs that passed
// the pair screening (screen_pairs_kernel); the grid covers every pair and the
// workgroups past the list's length exit at once.  (A persistent grid walking the list
// needs 107 instead of 75 VGPRs for FP32: the loop around the pair costs occupancy.)
template <int BS>
__global__ void __launch_bounds__(NT)
cov_refresh_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                   const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                   int64_t lds, const double* __restrict__ smax, int T, double lam1,
                   uint64_t* __restrict__ tbits, int64_t nwords, const int* gate,
                   unsigned long long* __restrict__ active, const int* __restrict__ plist,
                   const int* __restrict__ pcount) {
    if (gate && *gate == 0) return;
    int t = blockIdx.x;   // without a list: every pair in the refresh's order
    if (plist) {
        const int n = __builtin_amdgcn_readfirstlane(*pcount);
        if (t >= n) return;
        t = plist[t];
    }
    const int2 ij = refresh_tile(t, T, T * (T + 1) / 2);
    const int I = __builtin_amdgcn_readfirstlane(ij.x);
    const int J = __builtin_amdgcn_readfirstlane(ij.y);
    refresh_pair<BS>(I, J, rowptr, col, val, p, S, lds, smax, T, lam1, tbits, nwords, active);
}

// Pair screening, first part: for every row tile I, the column tiles K its rows' nonzeros
// fall in, with weight w(I, K) = max_{i in I} sum_{k in supp_i, k/64 = K} |omega_ik|, and
// the largest row count.  More than SCREEN_L tiles marks I as unscreened (count > L).
constexpr int SCREEN_L = 64;
__device__ __forceinline__ void screen_rows_body(int I_, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                   const double* __restrict__ val, int64_t p, int T, int* __restrict__ lcnt,
                   int* __restrict__ lK, double* __restrict__ lW, int* __restrict__ lcmax,
                   int* __restrict__ pcount, uint64_t* __restrict__ tmask, const int* gate) {
    if (gate && *gate == 0) return;
    extern __shared__ unsigned long long wk[];   // T weights (bits of non-negative doubles)
    const int I = I_, lane = threadIdx.x;
    if (I == 0 && lane == 0) *pcount = 0;   // the pair kernel (next launch) appends from 0
    const int TW = (T + 63) / 64;
    for (int k = lane; k < TW; k += 64) tmask[(int64_t)I * TW + k] = 0ull;   // kept-tile bits
    for (int k = lane; k < T; k += 64) wk[k] = 0ull;
    __syncthreads();
    const int64_t row = (int64_t)I * 64 + lane;
    int cnt = 0;
    if (row < p) {
        const int64_t s = rowptr[row], e = rowptr[row + 1];
        cnt = (int)(e - s);
        int cur = -1;
        double acc = 0.0;
        for (int64_t k = s; k < e; ++k) {
            const int K = col[k] >> 6;
            if (K != cur) {   // columns are sorted: one run per tile
                if (cur >= 0) atomicMax(&wk[cur], (unsigned long long)__double_as_longlong(acc));
                cur = K;
                acc = 0.0;
            }
            acc += fabs(val[k]);
        }
        if (cur >= 0) atomicMax(&wk[cur], (unsigned long long)__double_as_longlong(acc));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int x = __shfl_xor(cnt, o, 64);
        cnt = x > cnt ? x : cnt;
    }
    __syncthreads();
    int base = 0;
    for (int k0 = 0; k0 < T; k0 += 64) {
        const int k = k0 + lane;
        const unsigned long long v = k < T ? wk[k] : 0ull;
        const uint64_t m = __ballot(v != 0ull);
        const int pos = base + __popcll(m & lanemask_lt());
        if (v != 0ull && pos < SCREEN_L) {
            lK[(int64_t)I * SCREEN_L + pos] = k;
            lW[(int64_t)I * SCREEN_L + pos] = __longlong_as_double((long long)v);
        }
        base += __popcll(m);
    }
    if (lane == 0) {
        lcnt[I] = base;
        lcmax[I] = cnt;
    }
}

__global__ void __launch_bounds__(64)
screen_rows_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                   const double* __restrict__ val, int64_t p, int T, int* __restrict__ lcnt,
                   int* __restrict__ lK, double* __restrict__ lW, int* __restrict__ lcmax,
                   int* __restrict__ pcount, uint64_t* __restrict__ tmask, const int* gate) {
    screen_rows_body(blockIdx.x, rowptr, col, val, p, T, lcnt, lK, lW, lcmax, pcount, tmask, gate);
}

// Pair screening, second part: one thread per tile pair t (the refresh's order).  The
// pair is kept if it is diagonal, if a tile is unscreened, or if
//   (sum_K w(I, K) smax[K][J] + sum_K w(J, K) smax[K][I]) / 2,
// a bound on |M_ij| over the pair no smaller than the refresh's own, exceeds the test
// threshold after the same widening.  Kept pairs are appended to plist (one atomic per
// block; the order of blocks is free, the refresh's result does not depend on it).
template <typename E>
__device__ __forceinline__ void screen_pairs_body(int bx_, int T, const int* __restrict__ lcnt, const int* __restrict__ lK,
                    const double* __restrict__ lW, const int* __restrict__ lcmax,
                    const double* __restrict__ smax, double lam1, int* __restrict__ plist,
                    int* __restrict__ pcount, uint64_t* __restrict__ tmask, const int* gate, int* __restrict__ ulist = nullptr, int* __restrict__ ucount = nullptr,
    uint32_t* __restrict__ ubits = nullptr) {
    if (gate && *gate == 0) return;
    __shared__ int wsum[WPB];
    __shared__ int bbase;
    const int nt = T * (T + 1) / 2;
    const int t = bx_ * NT + threadIdx.x;
    bool keep = false;
    if (t < nt) {
        const int2 ij = refresh_tile(t, T, nt);
        const int I = ij.x, J = ij.y;
        const int cI = lcnt[I], cJ = lcnt[J];
        if (I == J || cI > SCREEN_L || cJ > SCREEN_L) {
            keep = true;
        } else {
            double bw = 0.0, bv = 0.0;
            for (int q = 0; q < cI; ++q)
                bw += lW[(int64_t)I * SCREEN_L + q] * smax[(int64_t)lK[(int64_t)I * SCREEN_L + q] * T + J];
            for (int q = 0; q < cJ; ++q)
                bv += lW[(int64_t)J * SCREEN_L + q] * smax[(int64_t)lK[(int64_t)J * SCREEN_L + q] * T + I];
            const int cm = lcmax[I] > lcmax[J] ? lcmax[I] : lcmax[J];
            const double widen = 1.01 + (double)(cm + 2) * 0x1p-23;
            keep = 0.5 * (bw + bv) * widen > (double)test_threshold<E>(lam1);
        }
    }
    const uint64_t m = __ballot(keep);
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int v = 0; v < WPB; ++v) tot += wsum[v];
        bbase = tot ? atomicAdd(pcount, tot) : 0;
    }
    __syncthreads();
    int before = 0;
    for (int v = 0; v < wave; ++v) before += wsum[v];
    if (keep) {
        plist[bbase + before + __popcll(m & lanemask_lt())] = t;
        // kept-tile bits of both row tiles (the words the refresh writes for this pair)
        const int2 ij = refresh_tile(t, T, nt);
        const int TW = (T + 63) / 64;
        atomicOr((unsigned long long*)&tmask[(int64_t)ij.x * TW + (ij.y >> 6)], 1ull << (ij.y & 63));
        if (ij.x != ij.y)
            atomicOr((unsigned long long*)&tmask[(int64_t)ij.y * TW + (ij.x >> 6)], 1ull << (ij.x & 63));
        // batched solves: the pair joins its instance's list once for all of its solves
        if (ulist) {
            const uint32_t bit = 1u << (t & 31);
            if (!(atomicOr(&ubits[t >> 5], bit) & bit)) ulist[atomicAdd(ucount, 1)] = t;
        }
    }
}

template <typename E>
__global__ void __launch_bounds__(NT)
screen_pairs_kernel(int T, const int* __restrict__ lcnt, const int* __restrict__ lK,
                    const double* __restrict__ lW, const int* __restrict__ lcmax,
                    const double* __restrict__ smax, double lam1, int* __restrict__ plist,
                    int* __restrict__ pcount, uint64_t* __restrict__ tmask, const int* gate) {
    screen_pairs_body<E>(blockIdx.x, T, lcnt, lK, lW, lcmax, smax, lam1, plist, pcount, tmask, gate);
}

// Largest |S| of every 64 x 64 tile (as the refresh reads S), for its screening.
template <int BS>
__global__ void __launch_bounds__(NT)
tile_max_kernel(const void* __restrict__ S, int64_t p, int64_t lds, int T, double* __restrict__ out) {
    __shared__ double red[WPB];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    double m = 0.0;
    for (int r = wave; r < 64; r += WPB) {
        const int64_t gi = i0 + r, gj = j0 + lane;
        if (gi < p && gj < p) {
            const double x = fabs(load_one_d<BS>(S, gi * lds + gj));
            m = x > m ? x : m;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double x = __shfl_xor(m, o, 64);
        m = x > m ? x : m;
    }
    if (lane == 0) red[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int v = 1; v < WPB; ++v) t = red[v] > t ? red[v] : t;
        out[(int64_t)blockIdx.y * T + blockIdx.x] = t;
    }
}

// ---- candidate set from the refresh's threshold bits -------------------------------
// Row i's words already hold {j : j == i or |M_ij| > lam1}; OR in supp(Omega_i) and
// count: the same bitmap and counts as cand_count_kernel, reading p/8 bytes per row
// instead of the row of M.
__device__ __forceinline__ void cand_merge_body(int64_t bx_, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, int64_t p,
                  uint64_t* __restrict__ bitmap, int64_t nwords, int64_t* __restrict__ cnt,
                  const uint64_t* __restrict__ tmask) {
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni(bx_ * WPB + wave);
    if (row >= p) return;
    uint64_t* rw = bitmap + row * nwords;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    // With a tile mask (screened Cov refresh), only the words of kept tile pairs were
    // written this time; a support word outside them may hold an older refresh's bits,
    // so it is cleared first (all writers store 0), then the support bits go in.
    const int64_t TW = (nwords + 63) / 64;
    const uint64_t* mrow = tmask ? tmask + (row >> 6) * TW : nullptr;
    auto kept = [&](int64_t w) { return (mrow[w >> 6] >> (w & 63)) & 1ull; };
    int64_t extra = 0;   // support entries in words outside the kept tiles
    if (mrow) {
        for (int64_t k = s + lane; k < e; k += 64) {
            const int64_t w = col[k] >> 6;
            if (!kept(w)) {
                rw[w] = 0ull;
                ++extra;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    // the support bits go in by atomic OR on the few words they touch (the row's other
    // words are only read); the count reads after every OR has completed, with loads that
    // bypass the CU's L1 (another wave may have pulled a line shared with a neighbouring
    // row into it before the ORs reached L2)
    for (int64_t k = s + lane; k < e; k += 64) {
        const int32_t c = col[k];
        atomicOr((unsigned long long*)&rw[c >> 6], 1ull << (c & 63));
    }
    __builtin_amdgcn_s_waitcnt(0);
    auto word = [&](int64_t w) {
        return __hip_atomic_load(&rw[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    int64_t total = extra;   // each such entry is one bit of a word counted nowhere else
    if (mrow) {
        // only the 64-word blocks whose mask word is nonzero: the mask row is read 64
        // words at a time, one per lane, and its nonzero words are walked by ballot
        for (int64_t m0 = 0; m0 < TW; m0 += 64) {
            const uint64_t mw = m0 + lane < TW ? mrow[m0 + lane] : 0ull;
            uint64_t nz = __ballot(mw != 0ull);
            while (nz) {
                const int t = __builtin_ctzll(nz);
                nz &= nz - 1ull;
                const uint64_t mk = __shfl(mw, t, 64);
                const int64_t w = (m0 + t) * 64 + lane;
                if (w < nwords && ((mk >> lane) & 1ull)) total += __popcll(word(w));
            }
        }
    } else {
        for (int64_t w = lane; w < nwords; w += 64) total += __popcll(word(w));
    }
    double tt = (double)total;
    tt = wave_sum(tt);
    if (lane == 0) cnt[row] = (int64_t)tt;
}

__global__ void __launch_bounds__(NT)
cand_merge_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, int64_t p,
                  uint64_t* __restrict__ bitmap, int64_t nwords, int64_t* __restrict__ cnt,
                  const uint64_t* __restrict__ tmask) {
    cand_merge_body(blockIdx.x, rowptr, col, p, bitmap, nwords, cnt, tmask);
}

// ---- Cov per-row kernels with 8 lanes per row (8 rows per wave) --------------------
// For Cov problems of at least COV_TRIAL_GROUP_MIN_P rows (the trials make the same
// choice): a Cov row holds a few entries, so a wave per row leaves most lanes idle and,
// with many rows, the kernels run latency bound with too few rows in flight.  The
// gradient on the candidates and the emission give the same results as their
// wave-per-row forms (integer work; per-entry values formed by one lane as before); the
// objective partials are sums over the row's 8 lanes (lane g takes entries g, g + 8, ...)
// and a fixed butterfly, so they are reproducible but not bitwise those of the
// wave-per-row form, which is why the choice is made by the problem size alone.  (The
// candidate merge stays a wave per row: its count walks the row's kept bitmap words,
// 64 at a time across the wave, which 8 lanes would walk in long serial chains.)
__device__ inline int64_t group_row(int64_t bx) {
    return (bx * WPB + (threadIdx.x >> 6)) * (64 / TG) + (lane_id() / TG);
}
// sum over the 8 lanes of a row group (butterfly within the group)
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int o = TG / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int BS>
__device__ __forceinline__ void cand_grad_cov_g_body(int64_t bx, const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, int64_t p,
                                                     const void* __restrict__ S, int64_t lds,
                                                     double lam2, const int64_t* __restrict__ arow,
                                                     const int32_t* __restrict__ acol,
                                                     const double* __restrict__ aom,
                                                     double* __restrict__ agr, const int* overflow) {
    if (*overflow) return;
    const int g = lane_id() & (TG - 1);
    const int64_t row = group_row(bx);
    if (row >= p) return;
    const int64_t s = arow[row], e = arow[row + 1];
    for (int64_t k = s + g; k < e; k += TG) {
        const int64_t j = acol[k];
        const double m = m_entry<BS>(rowptr, col, val, S, lds, row, j);
        const double om = aom[k];
        double gr = m + lam2 * om;
        if (j == row) gr -= 1.0 / om;
        agr[k] = gr;
    }
}

__device__ __forceinline__ void emit_count_g_body(int64_t bx, const int64_t* __restrict__ arow,
                                                  const int32_t* __restrict__ acol,
                                                  const double* __restrict__ aom,
                                                  const double* __restrict__ agr, int64_t p,
                                                  double lam1, const DevState* st,
                                                  int64_t* __restrict__ cnt) {
    if (st->accepted_q < 0 || st->nonpos) return;
    const double tau = st->tau;
    const int g = lane_id() & (TG - 1);
    const int64_t row = group_row(bx);
    const bool act = row < p;
    int c = 0;
    if (act) {
        const int64_t s = arow[row], e = arow[row + 1];
        for (int64_t k = s + g; k < e; k += TG) {
            const bool diag = acol[k] == row;
            const double wp = prox_one(aom[k], agr[k], tau, tau * lam1, diag);
            c += (wp != 0.0 || diag) ? 1 : 0;
        }
    }
#pragma unroll
    for (int o = TG / 2; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if (act && g == 0) cnt[row] = c;
}

__device__ __forceinline__ void emit_fill_g_body(int64_t bx, const int64_t* __restrict__ arow,
                                                 const int32_t* __restrict__ acol,
                                                 const double* __restrict__ aom,
                                                 const double* __restrict__ agr, int64_t p,
                                                 double lam1, const DevState* st,
                                                 const int64_t* __restrict__ orow,
                                                 int32_t* __restrict__ ocol,
                                                 double* __restrict__ oval) {
    if (st->accepted_q < 0 || st->nonpos) return;
    const double tau = st->tau;
    const int lane = lane_id(), g = lane & (TG - 1), grp = lane / TG;
    const int64_t row = group_row(bx);
    const bool act = row < p;
    const int64_t s = act ? arow[row] : 0, e = act ? arow[row + 1] : 0;
    int64_t out = act ? orow[row] : 0;
    // every lane runs the wave's longest row (the ballot needs the whole wave)
    int len = (int)(e - s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int x = __shfl_xor(len, o, 64);
        len = x > len ? x : len;
    }
    for (int k0 = 0; k0 < len; k0 += TG) {
        const int64_t k = s + k0 + g;
        bool keep = false;
        double wp = 0.0;
        int32_t j = 0;
        if (k < e) {
            j = acol[k];
            const bool diag = j == row;
            wp = prox_one(aom[k], agr[k], tau, tau * lam1, diag);
            keep = wp != 0.0 || diag;
        }
        const uint32_t gm = (uint32_t)(__ballot(keep) >> (grp * TG)) & ((1u << TG) - 1u);
        if (keep) {
            const int64_t pos = out + __popc(gm & ((1u << g) - 1u));
            ocol[pos] = j;
            oval[pos] = wp;
        }
        out += __popc(gm);
    }
}

template <int BS>
__device__ __forceinline__ void obj_parts_cov_g_body(int64_t bx, const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, int64_t p,
                                                     const void* __restrict__ S, int64_t lds,
                                                     double* __restrict__ part, const int* gate) {
    if (gate && *gate == 0) return;
    const int g = lane_id() & (TG - 1);
    const int64_t row = group_row(bx);
    const bool act = row < p;
    double lg = 0, sq = 0, l1 = 0, wv = 0;
    if (act) {
        const int64_t s = rowptr[row], e = rowptr[row + 1];
        for (int64_t k = s + g; k < e; k += TG) {
            const int64_t j = col[k];
            const double m = m_entry<BS>(rowptr, col, val, S, lds, row, j);
            const double v = val[k];
            sq += v * v;
            if (j == row) lg += log(v);
            else l1 += fabs(v);
            wv = fma(m, v, wv);
        }
    }
    lg = group_sum(lg); sq = group_sum(sq); l1 = group_sum(l1); wv = group_sum(wv);
    if (act && g == 0) {
        part[0 * p + row] = lg;
        part[1 * p + row] = sq;
        part[2 * p + row] = l1;
        part[3 * p + row] = wv;
    }
}

template <int BS>
__global__ void __launch_bounds__(NT)
cand_grad_cov_g_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                       int64_t lds, double lam2, const int64_t* __restrict__ arow,
                       const int32_t* __restrict__ acol, const double* __restrict__ aom,
                       double* __restrict__ agr, const int* overflow) {
    cand_grad_cov_g_body<BS>(blockIdx.x, rowptr, col, val, p, S, lds, lam2, arow, acol, aom, agr,
                             overflow);
}
__global__ void __launch_bounds__(NT)
emit_count_g_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                    const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                    double lam1, const DevState* st, int64_t* __restrict__ cnt) {
    emit_count_g_body(blockIdx.x, arow, acol, aom, agr, p, lam1, st, cnt);
}
__global__ void __launch_bounds__(NT)
emit_fill_g_kernel(const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                   const double* __restrict__ aom, const double* __restrict__ agr, int64_t p,
                   double lam1, const DevState* st, const int64_t* __restrict__ orow,
                   int32_t* __restrict__ ocol, double* __restrict__ oval) {
    emit_fill_g_body(blockIdx.x, arow, acol, aom, agr, p, lam1, st, orow, ocol, oval);
}
template <int BS>
__global__ void __launch_bounds__(NT)
obj_parts_cov_g_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, int64_t p, const void* __restrict__ S,
                       int64_t lds, double* __restrict__ part, const int* gate) {
    obj_parts_cov_g_body<BS>(blockIdx.x, rowptr, col, val, p, S, lds, part, gate);
}

// ---- ingest ----------------------------------------------------------------------
// X (rows x cols, ld) -> Xt (cols x ldo), one 64 x 64 tile per block through LDS, and
// *flag = 1 if any entry read is NaN or Inf.  V4 (F32 in and out, X and ld 16-byte
// aligned): each lane reads 4 consecutive columns of an X row and writes 4 consecutive
// entries of an Xt row (16-byte accesses); entries of Xt past `rows` in a written
// group of 4 are the zero padding (ldo is a multiple of 4, at least rows).
template <typename In, typename Out, bool V4>
__global__ void __launch_bounds__(NT)
transpose_in_kernel(const In* __restrict__ X, int64_t rows, int64_t cols, int64_t ld,
                    Out* __restrict__ Xt, int64_t ldo, uint16_t* __restrict__ hi,
                    uint16_t* __restrict__ lo, int64_t kbs, int* __restrict__ flag) {
    __shared__ Out tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    bool bad = false;
    if (V4) {
        const int q = threadIdx.x & 15, rr = threadIdx.x >> 4;   // 16 lanes per row
        for (int r = rr; r < 64; r += NT / 16) {
            const int64_t gr = r0 + r, gc = c0 + 4 * q;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gr < rows) {
                const In* src = X + gr * ld + gc;
                if (gc + 3 < cols) {
                    const float4 w = *(const float4*)src;
                    v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (gc + t < cols) v[t] = (float)src[t];
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                bad |= !isfinite(v[t]);
                tile[r][4 * q + t] = (Out)v[t];
            }
        }
        __syncthreads();
        for (int c = rr; c < 64; c += NT / 16) {
            const int64_t oc = c0 + c, orr = r0 + 4 * q;   // output row = input col
            if (oc < cols && orr < rows) {
                float w[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) w[t] = (float)tile[4 * q + t][c];
                *(float4*)((float*)Xt + oc * ldo + orr) = make_float4(w[0], w[1], w[2], w[3]);
                if (hi) {
                    uint16_t h[4], l[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        h[t] = f2bf_rne(w[t]);
                        l[t] = f2bf_rne(w[t] - bf2f(h[t]));
                    }
                    // 4 consecutive K entries (orr % 4 == 0) stay inside one K block
                    const int64_t o = kblk_index(oc, orr, kbs);
                    *(uint2*)(hi + o) = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                   (uint32_t)h[2] | ((uint32_t)h[3] << 16));
                    *(uint2*)(lo + o) = make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16),
                                                   (uint32_t)l[2] | ((uint32_t)l[3] << 16));
                }
            }
        }
    } else {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        for (int r = ty; r < 64; r += 4) {
            const int64_t gr = r0 + r, gc = c0 + tx;
            const In x = (gr < rows && gc < cols) ? X[gr * ld + gc] : (In)0;
            bad |= !isfinite((double)x);
            tile[r][tx] = (Out)x;
        }
        __syncthreads();
        for (int r = ty; r < 64; r += 4) {
            const int64_t oc = c0 + r, orr = r0 + tx;   // output row = input col
            if (oc < cols && orr < rows) {
                const Out v = tile[tx][r];
                Xt[oc * ldo + orr] = v;
                if (hi) {
                    const float x = (float)v;
                    const uint16_t h = f2bf_rne(x);
                    const int64_t o = kblk_index(oc, orr, kbs);
                    hi[o] = h;
                    lo[o] = f2bf_rne(x - bf2f(h));
                }
            }
        }
    }
    if (bad) *flag = 1;
}

// (S + S^T) / 2 into `store` layout, one 64 x 64 tile per block: tile (bj, bi) is staged
// transposed in LDS so both reads are row-wise.  out_ij and out_ji are the same FP64
// expression 0.5 s_ij + 0.5 s_ji (the halvings are exact, the sum commutes) rounded
// once to the store type, so the stored matrix is exactly symmetric; an S that already
// is symmetric is copied unchanged.
template <typename In>
__global__ void __launch_bounds__(NT)
sym_copy_kernel(const In* __restrict__ S, int64_t p, int64_t ld, void* out, int store,
                int64_t ldo) {
    __shared__ double t[64][65];
    const int64_t bi = (int64_t)blockIdx.y * 64, bj = (int64_t)blockIdx.x * 64;
    const int c = threadIdx.x & 63;
    for (int r = threadIdx.x >> 6; r < 64; r += NT / 64) {
        const int64_t gi = bj + r, gj = bi + c;
        t[c][r] = gi < p && gj < p ? (double)S[gi * ld + gj] : 0.0;   // S[bj + r][bi + c]
    }
    __syncthreads();
    for (int r = threadIdx.x >> 6; r < 64; r += NT / 64) {
        const int64_t gi = bi + r, gj = bj + c;
        if (gi >= p || gj >= p) continue;
        const double v = __dadd_rn(__dmul_rn(0.5, (double)S[gi * ld + gj]), __dmul_rn(0.5, t[r][c]));
        if (store == ST_F64) ((double*)out)[gi * ldo + gj] = v;
        else if (store == ST_F32) ((float*)out)[gi * ldo + gj] = (float)v;
        else {
            const float x = (float)v;
            const uint16_t h = f2bf_rne(x);
            const uint16_t l = f2bf_rne(x - bf2f(h));
            ((uint32_t*)out)[gi * ldo + gj] = (uint32_t)h | ((uint32_t)l << 16);
        }
    }
}

template <typename In>
__global__ void __launch_bounds__(NT)
check_finite_kernel(const In* __restrict__ A, int64_t rows, int64_t cols, int64_t ld,
                    int* flag) {
    bool bad = false;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
        for (int64_t c = threadIdx.x; c < cols; c += NT)
            if (!isfinite((double)A[r * ld + c])) bad = true;
    if (bad) *flag = 1;
}

// ---- differentiation form ------------------------------------------------------
// Masked gradient and Omega Y in one pass over the rows.  With d_ij = <Y_j, Xt_i>
// (= n (S Omega)_ij) for every stored entry (i, j),
//   G_ij = (d_ij + d_ji) / (2n) + lam2 w_ij - [i == j] / w_ii,
// since (Omega S)_ij = <Y_i, Xt_j> / n = d_ji / n.  Wave i gathers each row Y_j of its
// entries once, for row i of Omega Y (d f / d X^T = Omega Y / n; FMA order of
// spmm_kernel, so the row equals that kernel's bitwise) and for d_ij against its own row
// Xt_i, and writes d_ij to D at the entry.  grad_combine_kernel then finds d_ji at the
// mirror entry (j, i) (the pattern is symmetric), so G_ij and G_ji are the same FP64 sum
// and bitwise equal; the mirror search runs there, over independent entries, rather
// than in this kernel's dependent chain before each row's gathers.  Columns are taken
// in blocks of RC chunks of 64 V; with more than one block the per-block partial sums go
// to D at block offset cb * nnz (summed in block order by the combine).  The wave sums
// of 8 entries share one reduce-scatter (4 + 2 + 1 shuffles, then 3 for the whole wave).
constexpr int GRAD_GROUP = 8;
constexpr int GRAD_RC = 4;
template <int S, int RC, int EG>
__global__ void __launch_bounds__(NT, 3)
grad_rows_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ val, int64_t p, const void* __restrict__ Y,
                 const void* __restrict__ Xt, int64_t ld, int64_t n, int64_t nnz,
                 double* __restrict__ D, void* __restrict__ oy) {
    typedef Chunk<S> Ch;
    typedef typename Ch::T T;
    constexpr int V = Ch::V;
    const int lane = lane_id();
    const int64_t row = uni((int64_t)blockIdx.x * WPB + (threadIdx.x >> 6));
    if (row >= p) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    const int nch = (int)((n + 64 * V - 1) / (64 * V));
    const int ncb = (nch + RC - 1) / RC;
    double v[GRAD_GROUP];
    int m = 0;
    int64_t first = s;   // the entry of slot 0 of the pending group
    // the wave sums of the m pending entries first .. first + m - 1 go to D
    auto flush = [&](int64_t boff) {
#pragma unroll
        for (int w = GRAD_GROUP, o = 32; w > 1; w >>= 1, o >>= 1) {
            const bool upper = (lane & o) != 0;   // keep the upper half of the w values
#pragma unroll
            for (int i = 0; i < w / 2; ++i) {
                const double send = upper ? v[i] : v[i + w / 2];
                const double keep = upper ? v[i + w / 2] : v[i];
                v[i] = keep + __shfl_xor(send, o, 64);
            }
        }
        // v[0]: slot (lane >> 3) & 7 summed over the 8 lanes sharing bits 0..2
        double tot = v[0];
#pragma unroll
        for (int o = 4; o >= 1; o >>= 1) tot += __shfl_xor(tot, o, 64);
        const int g = (lane >> 3) & 7;
        if ((lane & 7) == 0 && g < m) D[boff + first + g] = tot;
#pragma unroll
        for (int i = 0; i < GRAD_GROUP; ++i) v[i] = 0.0;
        first += m;
        m = 0;
    };
#pragma unroll
    for (int i = 0; i < GRAD_GROUP; ++i) v[i] = 0.0;
    for (int cb = 0; cb < ncb; ++cb) {
        const int64_t boff = (int64_t)cb * nnz;
        first = s;
        T acc[RC][V], xi[RC][V];   // this block of row i of Omega Y, and of Xt_i
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int64_t c = (int64_t)(cb * RC + q) * 64 * V + lane * V;
#pragma unroll
            for (int t = 0; t < V; ++t) { acc[q][t] = 0; xi[q][t] = 0; }
            if (c < n) Ch::load(Xt, row * ld + c, xi[q]);
        }
        for (int64_t b = s; b < e; b += 64) {
            const int cnt = (int)(e - b < 64 ? e - b : 64);
            const int jl = lane < cnt ? col[b + lane] : 0;
            for (int t0 = 0; t0 < cnt; t0 += EG) {
                // the rows Y_j of up to EG entries, their loads issued before any FMA
                T yj[EG][RC][V];
#pragma unroll
                for (int u = 0; u < EG; ++u) {
                    const int64_t j = (int64_t)__shfl(jl, t0 + u < cnt ? t0 + u : t0, 64);
#pragma unroll
                    for (int q = 0; q < RC; ++q) {
                        const int64_t c = (int64_t)(cb * RC + q) * 64 * V + lane * V;
                        if (t0 + u < cnt && c < n) Ch::load(Y, j * ld + c, yj[u][q]);
                    }
                }
#pragma unroll
                for (int u = 0; u < EG; ++u) {
                    if (t0 + u >= cnt) break;
                    const T wv = (T)val[b + t0 + u];
                    double a2 = 0.0;
#pragma unroll
                    for (int q = 0; q < RC; ++q) {
                        const int64_t c = (int64_t)(cb * RC + q) * 64 * V + lane * V;
                        if (c < n) {
                            T a = 0;
#pragma unroll
                            for (int w = 0; w < V; ++w) {
                                acc[q][w] = fma(wv, yj[u][q][w], acc[q][w]);
                                a += yj[u][q][w] * xi[q][w];
                            }
                            a2 += (double)a;
                        }
                    }
#pragma unroll
                    for (int g = 0; g < GRAD_GROUP; ++g) v[g] = g == m ? a2 : v[g];
                    if (++m == GRAD_GROUP) flush(boff);
                }
            }
        }
        if (m > 0) flush(boff);
        if (oy) {
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int64_t c = (int64_t)(cb * RC + q) * 64 * V + lane * V;
                if (c < n) {
                    if (S == ST_F64) {
                        double* o = (double*)oy + row * ld + c;
#pragma unroll
                        for (int u = 0; u < V; ++u) o[u] = (double)acc[q][u];
                    } else {
                        float* o = (float*)oy + row * ld + c;
#pragma unroll
                        for (int u = 0; u < V; ++u) o[u] = (float)acc[q][u];
                    }
                }
            }
        }
    }
}

// G on the stored entries: G_ij = (sum_cb D_ij + sum_cb D_ji) / (2n) + lam2 w_ij
// - [i == j] / w_ii (blocks in order), D_ji found by binary search of row j for column i.
__global__ void __launch_bounds__(NT)
grad_combine_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                    const double* __restrict__ val, int64_t p, int64_t nnz, int ncb,
                    const double* __restrict__ D, double inv2n, double lam2, void* out,
                    int out_f64) {
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row = uni((int64_t)blockIdx.x * WPB + wave);
    if (row >= p) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    for (int64_t k = s + lane; k < e; k += 64) {
        const int32_t j = col[k];
        int64_t mk = k;
        if (j != row) {
            const int64_t je = rowptr[j + 1];
            int64_t lo_ = rowptr[j], hi_ = je;
            while (lo_ < hi_) {
                const int64_t mid = (lo_ + hi_) >> 1;
                if (col[mid] < row) lo_ = mid + 1; else hi_ = mid;
            }
            // stored in a symmetric pattern; otherwise the entry's own half stands in
            if (lo_ < je && col[lo_] == row) mk = lo_;
        }
        double dsum = D[k], esum = D[mk];
        for (int cb = 1; cb < ncb; ++cb) {
            dsum += D[(int64_t)cb * nnz + k];
            esum += D[(int64_t)cb * nnz + mk];
        }
        const double wv = val[k];
        double gr = (dsum + esum) * inv2n + lam2 * wv;
        if (j == row) gr -= 1.0 / wv;
        if (out_f64) ((double*)out)[k] = gr;
        else ((float*)out)[k] = (float)gr;
    }
}

template <int S>
__global__ void __launch_bounds__(NT)
dense_grad_kernel(const void* __restrict__ M, int64_t ldm, const int64_t* __restrict__ rowptr,
                  const int32_t* __restrict__ col, const double* __restrict__ val, int64_t p,
                  double lam2, void* out, int out_f64) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p * p) return;
    const int64_t i = idx / p, j = idx % p;
    double g = load_one_d<S>(M, i * ldm + j);
    // add lam2 * omega_ij and the diagonal term
    const int64_t s = rowptr[i], e = rowptr[i + 1];
    int64_t lo_ = s, hi_ = e;
    while (lo_ < hi_) {
        const int64_t mid = (lo_ + hi_) >> 1;
        if (col[mid] < j) lo_ = mid + 1; else hi_ = mid;
    }
    if (lo_ < e && col[lo_] == j) {
        const double v = val[lo_];
        g += lam2 * v;
        if (i == j) g -= 1.0 / v;
    }
    if (out_f64) ((double*)out)[idx] = g;
    else ((float*)out)[idx] = (float)g;
}

// A (p x n, ld) -> out (n x p), each entry times `scale` (in FP64, then rounded to the
// output type).  V4 (F32 in and out, 16-byte aligned rows): 16-byte loads of 4
// consecutive columns of an A row and 16-byte stores of 4 consecutive out entries.
template <typename E, bool V4>
__global__ void __launch_bounds__(NT)
transpose_out_kernel(const E* __restrict__ A, int64_t p, int64_t n, int64_t ld, double scale,
                     void* out, int out_f64) {
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    if (V4) {
        __shared__ float tf[64][65];
        const int q = threadIdx.x & 15, rr = threadIdx.x >> 4;
        for (int r = rr; r < 64; r += NT / 16) {
            const int64_t gr = r0 + r, gc = c0 + 4 * q;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gr < p) {
                const E* src = A + gr * ld + gc;
                if (gc + 3 < n) {
                    const float4 w = *(const float4*)src;
                    v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (gc + t < n) v[t] = (float)src[t];
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) tf[r][4 * q + t] = (float)((double)v[t] * scale);
        }
        __syncthreads();
        for (int c = rr; c < 64; c += NT / 16) {
            const int64_t orow = c0 + c, ocol = r0 + 4 * q;
            if (orow >= n || ocol >= p) continue;
            float* dst = (float*)out + orow * p + ocol;
            if (ocol + 3 < p) {
                *(float4*)dst = make_float4(tf[4 * q][c], tf[4 * q + 1][c], tf[4 * q + 2][c],
                                            tf[4 * q + 3][c]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (ocol + t < p) dst[t] = tf[4 * q + t][c];
            }
        }
        return;
    }
    __shared__ double tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t gr = r0 + r, gc = c0 + tx;
        tile[r][tx] = (gr < p && gc < n) ? (double)A[gr * ld + gc] * scale : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t orow = c0 + r, ocol = r0 + tx;
        if (orow < n && ocol < p) {
            if (out_f64) ((double*)out)[orow * p + ocol] = tile[tx][r];
            else ((float*)out)[orow * p + ocol] = (float)tile[tx][r];
        }
    }
}

// flags[0]: structural error, flags[1]: non-positive diagonal, flags[2]: non-finite
template <typename VT>
__global__ void csr_validate_kernel(const int64_t* rowptr, const int32_t* col, const VT* val,
                                    int64_t p, int64_t nnz, int* flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    const int64_t s = rowptr[i], e = rowptr[i + 1];
    if (i == 0 && s != 0) flags[0] = 1;
    if (i == p - 1 && e != nnz) flags[0] = 1;
    if (s < 0 || e < s || e > nnz) { flags[0] = 1; return; }
    bool has_diag = false;
    for (int64_t k = s; k < e; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= p || (k > s && col[k - 1] >= c)) flags[0] = 1;
        const double v = (double)val[k];
        if (!isfinite(v)) flags[2] = 1;
        if (c == i) { has_diag = true; if (!(v > 0.0)) flags[1] = 1; }
    }
    if (!has_diag) flags[0] = 1;
}

template <typename VT>
__global__ void csr_import_kernel(const int32_t* col, const VT* val, int64_t nnz, int32_t* co,
                                  double* vo) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) { co[k] = col[k]; vo[k] = (double)val[k]; }
}

__global__ void csr_export_kernel(const double* val, int64_t nnz, void* out, int out_f64) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) {
        if (out_f64) ((double*)out)[k] = val[k];
        else ((float*)out)[k] = (float)val[k];
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ================================ launchers ======================================

int spmm_nchunks(int bstore, int64_t ncols) {
    const int V = bstore == ST_F64 ? 2 : 4;
    return (int)((ncols + 64 * V - 1) / (64 * V));
}

hipError_t launch_spmm(const Csr& A, int64_t p, const void* B, int bstore, int64_t ldb,
                       int64_t ncols, void* C, int cstore, int64_t ldc, uint16_t* hi,
                       uint16_t* lo, int64_t kbs, double* sq_part, const int* gate,
                       hipStream_t stream) {
    if (p == 0) return hipSuccess;
    const int nch = spmm_nchunks(bstore, ncols);
    dim3 grid(blocks_for(p, WPB), nch);
#define SPMM(BS, CS)                                                                     \
    hipLaunchKernelGGL((spmm_kernel<BS, CS>), grid, dim3(NT), 0, stream, A.rowptr, A.col, \
                       A.val, p, B, ldb, ncols, C, ldc, hi, lo, kbs, sq_part, gate)
    if (bstore == ST_F64) SPMM(ST_F64, ST_F64);
    else if (bstore == ST_F32) {
        if (cstore == ST_F64) SPMM(ST_F32, ST_F64); else SPMM(ST_F32, ST_F32);
    } else SPMM(ST_B16P, ST_F32);
#undef SPMM
    return hipGetLastError();
}

hipError_t launch_cand_count(const void* M, int mstore, int64_t ldm, const Csr& om, int64_t p,
                             double lam1, uint64_t* bitmap, int64_t nwords, int64_t* cnt,
                             hipStream_t stream) {
    if (p == 0) return hipSuccess;
    const size_t lds = (size_t)WPB * nwords * 8;
    if (mstore == ST_F64)
        hipLaunchKernelGGL(cand_count_kernel<ST_F64>, dim3(blocks_for(p, WPB)), dim3(NT), lds,
                           stream, M, ldm, om.rowptr, om.col, p, lam1, bitmap, nwords, cnt);
    else
        hipLaunchKernelGGL(cand_count_kernel<ST_F32>, dim3(blocks_for(p, WPB)), dim3(NT), lds,
                           stream, M, ldm, om.rowptr, om.col, p, lam1, bitmap, nwords, cnt);
    return hipGetLastError();
}

hipError_t launch_cand_merge(const Csr& om, int64_t p, uint64_t* bitmap, int64_t nwords,
                             int64_t* cnt, hipStream_t stream, const uint64_t* tmask) {
    if (p == 0) return hipSuccess;
    hipLaunchKernelGGL(cand_merge_kernel, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                       om.rowptr, om.col, p, bitmap, nwords, cnt, tmask);
    return hipGetLastError();
}

hipError_t launch_cand_fill(const void* M, int mstore, int64_t ldm, const Csr& om, int64_t p,
                            double lam2, const uint64_t* bitmap, int64_t nwords,
                            const Cand& A, int64_t cap, const int* overflow,
                            hipStream_t stream, const uint64_t* tmask, bool m_upper) {
    (void)cap;
    if (p == 0) return hipSuccess;
    const size_t lds = tmask ? (size_t)WPB * ((nwords + 63) / 64) * 8 : 0;
    if (mstore == ST_F64)
        hipLaunchKernelGGL(cand_fill_kernel<ST_F64>, dim3(blocks_for(p, WPB)), dim3(NT), lds,
                           stream, M, ldm, om.rowptr, om.col, om.val, p, lam2, bitmap, nwords,
                           A.rowptr, A.col, A.omega, A.grad, overflow, tmask, m_upper);
    else
        hipLaunchKernelGGL(cand_fill_kernel<ST_F32>, dim3(blocks_for(p, WPB)), dim3(NT), lds,
                           stream, M, ldm, om.rowptr, om.col, om.val, p, lam2, bitmap, nwords,
                           A.rowptr, A.col, A.omega, A.grad, overflow, tmask, m_upper);
    return hipGetLastError();
}

hipError_t launch_scan(const int64_t* cnt, int64_t p, int64_t* out, int64_t cap, int* overflow,
                       int64_t* ws, hipStream_t stream, int64_t* total_out) {
    if (p == 0) return hipErrorInvalidValue;   // every handle has p >= 1
    const unsigned nb = (unsigned)((p + SCAN_CHUNK - 1) / SCAN_CHUNK);
    if (nb > 1)   // one chunk needs no chunk sums
        hipLaunchKernelGGL(scan_part_kernel, dim3(nb), dim3(NT), 0, stream, cnt, p, ws);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(NT), 0, stream, cnt, p, ws, out, cap,
                       overflow, total_out);
    return hipGetLastError();
}

int64_t scan_ws_len(int64_t p) { return (p + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

// Splitting the Obs column loop over blocks was measured slower than one wave per
// row at the benchmark shape (many tiny waves), so one split is used.
int trial_splits(int variant, int bstore, int64_t ncols) {
    (void)variant;
    (void)bstore;
    (void)ncols;
    return 1;
}

hipError_t launch_trial(const Cand& A, int64_t p, double tau0, double shrink, int m, double lam1,
                        int variant, const void* B, int bstore, int64_t ldb, int64_t ncols,
                        const double* xn2, double* part, const DevState* st, hipStream_t stream) {
    if (p == 0) return hipSuccess;
    if (m < 1 || m > MAXQ) return hipErrorInvalidValue;
    dim3 grid(blocks_for(p, WPB), trial_splits(variant, bstore, ncols));
#define TRIAL(BS, OBS)                                                                       \
    hipLaunchKernelGGL((trial_kernel<BS, OBS>), grid, dim3(NT), 0, stream, A.rowptr, A.col,   \
                       A.omega, A.grad, p, tau0, shrink, m, lam1, B, ldb, ncols,              \
                       obs ? xn2 : nullptr, part, st)
    const bool obs = variant == 1;
    // Cov rows hold a few candidates each.  Below COV_GROUP_MIN_P rows the wave-per-row
    // kernel's p waves fit on the chip at once and the step is latency bound, so packing
    // rows into fewer waves only lengthens each wave's serial loop (p = 200: 17% slower
    // solves); above it, 8 rows per wave leave far fewer lanes idle (p = 16,384: 20%
    // faster solves; in a batch, where many solves' rows share the chip, 6 times faster
    // per row).
    if (!obs && p >= COV_GROUP_MIN_P) {   // Cov: 8 lanes per row
        static_assert(MAXQ == TG, "lane g of a row group holds step size q = g");
        dim3 cg(blocks_for(p, WPB * (64 / TG)));
#define TRIALC(BS)                                                                           \
        hipLaunchKernelGGL((trial_cov_kernel<BS>), cg, dim3(NT), 0, stream, A.rowptr, A.col, \
                           A.omega, A.grad, p, tau0, shrink, m, lam1, B, ldb, part, st)
        if (bstore == ST_F64) TRIALC(ST_F64);
        else if (bstore == ST_F32) TRIALC(ST_F32);
        else TRIALC(ST_B16P);
#undef TRIALC
        return hipGetLastError();
    }
    if (bstore == ST_F64) { if (obs) TRIAL(ST_F64, true); else TRIAL(ST_F64, false); }
    else if (bstore == ST_F32) { if (obs) TRIAL(ST_F32, true); else TRIAL(ST_F32, false); }
    else { if (obs) return hipErrorInvalidValue; TRIAL(ST_B16P, false); }
#undef TRIAL
    return hipGetLastError();
}

hipError_t launch_row_norm2(const void* B, int bstore, int64_t ldb, int64_t ncols, int64_t p,
                            double* out, hipStream_t stream) {
    if (p == 0) return hipSuccess;
    if (ldb % 4 || ncols % 4 || ncols > ldb) return hipErrorInvalidValue;   // whole chunks
    if (bstore == ST_F64)
        hipLaunchKernelGGL(row_norm2_kernel<ST_F64>, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                           B, ldb, ncols, p, out);
    else if (bstore == ST_F32)
        hipLaunchKernelGGL(row_norm2_kernel<ST_F32>, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                           B, ldb, ncols, p, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

namespace {
// segments of at most 8192 rows per column, at most COLSUM_MAXSEG of them
__host__ __device__ void colsum_shape(int64_t rows, int* nseg, int64_t* seg) {
    const int64_t seg0 = 8192;
    int ns = (int)((rows + seg0 - 1) / seg0);
    if (ns < 1) ns = 1;
    if (ns > COLSUM_MAXSEG) ns = COLSUM_MAXSEG;
    const int64_t sg = (rows + ns - 1) / ns;
    *nseg = ns;
    *seg = sg < 1 ? 1 : sg;
}
}  // namespace

hipError_t launch_colsum_decide(const double* in, int64_t rows, int ncol, double* out,
                                double* ws, int m, double tau0, double shrink, int q_base,
                                double lam2, double inv_n, int forced_q, DevState* st,
                                hipStream_t stream) {
    if (ncol <= 0 || ncol > 4 * MAXQ || m < 1 || 4 * m != ncol) return hipErrorInvalidValue;
    int nseg;
    int64_t seg;
    colsum_shape(rows, &nseg, &seg);
    FinArgs fa{m, q_base, forced_q, 0, tau0, shrink, lam2, inv_n, nullptr};
    hipLaunchKernelGGL((colsum_finish_kernel<FIN_DECIDE>), dim3(ncol, nseg), dim3(NT), 0, stream,
                       in, rows, seg, ws, out, &st->ticket, fa, st);
    return hipGetLastError();
}

hipError_t launch_colsum_obj(const double* in, int64_t rows, int ncol, double* out, double* ws,
                             int nysq, const int* gate, DevState* st, hipStream_t stream) {
    if (ncol < 4 || nysq != ncol - 4) return hipErrorInvalidValue;
    int nseg;
    int64_t seg;
    colsum_shape(rows, &nseg, &seg);
    FinArgs fa{0, 0, -1, nysq, 0.0, 0.5, 0.0, 0.0, gate};
    hipLaunchKernelGGL((colsum_finish_kernel<FIN_OBJ>), dim3(ncol, nseg), dim3(NT), 0, stream,
                       in, rows, seg, ws, out, &st->ticket, fa, st);
    return hipGetLastError();
}

hipError_t launch_emit_count(const Cand& A, int64_t p, double lam1, const DevState* st,
                             int64_t* cnt, hipStream_t stream, bool grouped) {
    if (p == 0) return hipSuccess;
    if (grouped) {
        hipLaunchKernelGGL(emit_count_g_kernel, dim3(blocks_for(p, WPB * (64 / TG))), dim3(NT), 0,
                           stream, A.rowptr, A.col, A.omega, A.grad, p, lam1, st, cnt);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(emit_count_kernel, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                       A.rowptr, A.col, A.omega, A.grad, p, lam1, st, cnt);
    return hipGetLastError();
}

hipError_t launch_emit_fill(const Cand& A, int64_t p, double lam1, const DevState* st,
                            const Csr& out, hipStream_t stream, bool grouped) {
    if (p == 0) return hipSuccess;
    if (grouped) {
        hipLaunchKernelGGL(emit_fill_g_kernel, dim3(blocks_for(p, WPB * (64 / TG))), dim3(NT), 0,
                           stream, A.rowptr, A.col, A.omega, A.grad, p, lam1, st, out.rowptr,
                           out.col, out.val);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(emit_fill_kernel, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                       A.rowptr, A.col, A.omega, A.grad, p, lam1, st, out.rowptr, out.col,
                       out.val);
    return hipGetLastError();
}

hipError_t launch_obj_parts(const Csr& om, int64_t p, const void* W, int wstore, int64_t ldw,
                            double* part, const int* gate, hipStream_t stream) {
    if (p == 0) return hipSuccess;
    dim3 grid(blocks_for(p, WPB));
    if (wstore == ST_F64)
        hipLaunchKernelGGL(obj_parts_kernel<ST_F64>, grid, dim3(NT), 0, stream, om.rowptr, om.col,
                           om.val, p, W, ldw, part, gate);
    else
        hipLaunchKernelGGL(obj_parts_kernel<ST_F32>, grid, dim3(NT), 0, stream, om.rowptr, om.col,
                           om.val, p, W, ldw, part, gate);
    return hipGetLastError();
}

hipError_t launch_obj_parts_cov(const Csr& om, int64_t p, const void* S, int sstore, int64_t lds,
                                double* part, const int* gate, hipStream_t stream) {
    if (p == 0) return hipSuccess;
    if (p >= COV_TRIAL_GROUP_MIN_P) {
        dim3 gg(blocks_for(p, WPB * (64 / TG)));
#define OBJG(BS)                                                                               \
        hipLaunchKernelGGL(obj_parts_cov_g_kernel<BS>, gg, dim3(NT), 0, stream, om.rowptr, om.col, \
                           om.val, p, S, lds, part, gate)
        if (sstore == ST_F64) OBJG(ST_F64);
        else if (sstore == ST_F32) OBJG(ST_F32);
        else if (sstore == ST_B16P) OBJG(ST_B16P);
        else return hipErrorInvalidValue;
#undef OBJG
        return hipGetLastError();
    }
    dim3 grid(blocks_for(p, WPB));
    if (sstore == ST_F64)
        hipLaunchKernelGGL(obj_parts_cov_kernel<ST_F64>, grid, dim3(NT), 0, stream, om.rowptr,
                           om.col, om.val, p, S, lds, part, gate);
    else if (sstore == ST_F32)
        hipLaunchKernelGGL(obj_parts_cov_kernel<ST_F32>, grid, dim3(NT), 0, stream, om.rowptr,
                           om.col, om.val, p, S, lds, part, gate);
    else if (sstore == ST_B16P)
        hipLaunchKernelGGL(obj_parts_cov_kernel<ST_B16P>, grid, dim3(NT), 0, stream, om.rowptr,
                           om.col, om.val, p, S, lds, part, gate);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cand_grad_cov(const Csr& om, int64_t p, const void* S, int sstore, int64_t lds,
                                double lam2, const Cand& A, const int* overflow,
                                hipStream_t stream) {
    if (p == 0) return hipSuccess;
    if (p >= COV_TRIAL_GROUP_MIN_P) {
        dim3 gg(blocks_for(p, WPB * (64 / TG)));
#define CGRADG(BS)                                                                            \
        hipLaunchKernelGGL(cand_grad_cov_g_kernel<BS>, gg, dim3(NT), 0, stream, om.rowptr,      \
                           om.col, om.val, p, S, lds, lam2, A.rowptr, A.col, A.omega, A.grad,  \
                           overflow)
        if (sstore == ST_F64) CGRADG(ST_F64);
        else if (sstore == ST_F32) CGRADG(ST_F32);
        else if (sstore == ST_B16P) CGRADG(ST_B16P);
        else return hipErrorInvalidValue;
#undef CGRADG
        return hipGetLastError();
    }
    dim3 grid(blocks_for(p, WPB));
#define CGRAD(BS)                                                                         \
    hipLaunchKernelGGL(cand_grad_cov_kernel<BS>, grid, dim3(NT), 0, stream, om.rowptr, om.col, \
                       om.val, p, S, lds, lam2, A.rowptr, A.col, A.omega, A.grad, overflow)
    if (sstore == ST_F64) CGRAD(ST_F64);
    else if (sstore == ST_F32) CGRAD(ST_F32);
    else if (sstore == ST_B16P) CGRAD(ST_B16P);
    else return hipErrorInvalidValue;
#undef CGRAD
    return hipGetLastError();
}

hipError_t launch_smooth_finish(const DevState* st, int64_t n, double lam2, double* f,
                                hipStream_t stream) {
    hipLaunchKernelGGL(smooth_finish_kernel, dim3(1), dim3(64), 0, stream, st, (double)n, lam2, f);
    return hipGetLastError();
}

hipError_t launch_identity(const Csr& om, int64_t p, hipStream_t stream) {
    hipLaunchKernelGGL(identity_kernel, dim3(blocks_for(p + 1, NT)), dim3(NT), 0, stream,
                       om.rowptr, om.col, om.val, p);
    return hipGetLastError();
}

hipError_t launch_cov_screen(const Csr& A, int64_t p, int sstore, const double* smax,
                             double lam1, uint64_t* tbits, int64_t nwords, const RefreshWs& ws,
                             const int* gate, hipStream_t stream, bool screen) {
    if (!tbits || !smax || nwords != (p + 63) / 64) return hipErrorInvalidValue;
    if (!ws.lcnt || !ws.lK || !ws.lW || !ws.lcmax || !ws.plist || !ws.pcount)
        return hipErrorInvalidValue;
    const int T = (int)((p + 63) / 64);
    const int64_t nt = (int64_t)T * (T + 1) / 2;
    if (nt == 0) return hipSuccess;
    if (nt > INT32_MAX || (size_t)T * 8 > 64 * 1024) return hipErrorInvalidValue;
    if (!screen) return hipSuccess;   // the refresh then runs every pair without a list
    hipLaunchKernelGGL(screen_rows_kernel, dim3(T), dim3(64), (size_t)T * 8, stream, A.rowptr,
                       A.col, A.val, p, T, ws.lcnt, ws.lK, ws.lW, ws.lcmax, ws.pcount, ws.tmask,
                       gate);
    const unsigned pb = (unsigned)((nt + NT - 1) / NT);
    if (sstore == ST_F64)
        hipLaunchKernelGGL(screen_pairs_kernel<double>, dim3(pb), dim3(NT), 0, stream, T, ws.lcnt,
                           ws.lK, ws.lW, ws.lcmax, smax, lam1, ws.plist, ws.pcount, ws.tmask, gate);
    else
        hipLaunchKernelGGL(screen_pairs_kernel<float>, dim3(pb), dim3(NT), 0, stream, T, ws.lcnt,
                           ws.lK, ws.lW, ws.lcmax, smax, lam1, ws.plist, ws.pcount, ws.tmask, gate);
    // the screened-out pairs' words are not cleared: the candidate merge and fill read only
    // the words of kept tiles (ws.tmask) and the row's support words
    return hipGetLastError();
}

hipError_t launch_cov_refresh_pairs(const Csr& A, int64_t p, const void* S, int sstore,
                                    int64_t lds, const double* smax, double lam1,
                                    uint64_t* tbits, int64_t nwords, const RefreshWs& ws,
                                    const int* gate, hipStream_t stream,
                                    unsigned long long* active) {
    if (!tbits || nwords != (p + 63) / 64 || lds < nwords * 64 || !ws.plist || !ws.pcount)
        return hipErrorInvalidValue;
    const int T = (int)((p + 63) / 64);
    const int64_t nt = (int64_t)T * (T + 1) / 2;
    if (nt == 0) return hipSuccess;
    if (nt > INT32_MAX) return hipErrorInvalidValue;
    const unsigned g = (unsigned)nt;
    // smax null: no screening, every pair in order without the list
    const int* pl = smax ? ws.plist : nullptr;
#define REFRESH(BS)                                                                      \
    hipLaunchKernelGGL((cov_refresh_kernel<BS>), dim3(g), dim3(NT), 0, stream, A.rowptr,   \
                       A.col, A.val, p, S, lds, smax, T, lam1, tbits, nwords, gate, active, \
                       pl, ws.pcount)
    if (sstore == ST_F64) REFRESH(ST_F64);
    else if (sstore == ST_F32) REFRESH(ST_F32);
    else if (sstore == ST_B16P) REFRESH(ST_B16P);
    else return hipErrorInvalidValue;
#undef REFRESH
    return hipGetLastError();
}

hipError_t launch_cov_refresh(const Csr& A, int64_t p, const void* S, int sstore, int64_t lds,
                              const double* smax, double lam1, uint64_t* tbits, int64_t nwords,
                              const RefreshWs& ws, const int* gate, hipStream_t stream,
                              unsigned long long* active, bool screen) {
    hipError_t e = launch_cov_screen(A, p, sstore, smax, lam1, tbits, nwords, ws, gate, stream,
                                     screen);
    if (e != hipSuccess) return e;
    return launch_cov_refresh_pairs(A, p, S, sstore, lds, screen ? smax : nullptr, lam1, tbits,
                                    nwords, ws, gate, stream, active);
}

hipError_t launch_tile_max(const void* S, int sstore, int64_t p, int64_t lds, double* out,
                           hipStream_t stream) {
    if (p == 0) return hipSuccess;
    const unsigned T = (unsigned)((p + 63) / 64);
    if (T > 65535u) return hipErrorInvalidValue;
    dim3 grid(T, T);
    if (sstore == ST_F64)
        hipLaunchKernelGGL(tile_max_kernel<ST_F64>, grid, dim3(NT), 0, stream, S, p, lds, (int)T, out);
    else if (sstore == ST_F32)
        hipLaunchKernelGGL(tile_max_kernel<ST_F32>, grid, dim3(NT), 0, stream, S, p, lds, (int)T, out);
    else if (sstore == ST_B16P)
        hipLaunchKernelGGL(tile_max_kernel<ST_B16P>, grid, dim3(NT), 0, stream, S, p, lds, (int)T, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_transpose_in(const void* X, int x_is_f64, int64_t rows, int64_t cols,
                               int64_t ld, void* Xt, int store, int64_t ldo, uint16_t* hi,
                               uint16_t* lo, int64_t kbs, int* flag, hipStream_t stream) {
    if (rows == 0 || cols == 0) return hipSuccess;
    dim3 grid(blocks_for(cols, 64), blocks_for(rows, 64));
    if (grid.y > 65535u) return hipErrorInvalidValue;
    if (x_is_f64) {
        if (store == ST_F64)
            hipLaunchKernelGGL((transpose_in_kernel<double, double, false>), grid, dim3(NT), 0,
                               stream, (const double*)X, rows, cols, ld, (double*)Xt, ldo, hi, lo,
                               kbs, flag);
        else
            hipLaunchKernelGGL((transpose_in_kernel<double, float, false>), grid, dim3(NT), 0,
                               stream, (const double*)X, rows, cols, ld, (float*)Xt, ldo, hi, lo,
                               kbs, flag);
    } else {
        const bool v4 = store != ST_F64 && ((uintptr_t)X & 15) == 0 && ld % 4 == 0 &&
                        ldo % 4 == 0 && ((uintptr_t)Xt & 15) == 0;
        if (store == ST_F64)
            hipLaunchKernelGGL((transpose_in_kernel<float, double, false>), grid, dim3(NT), 0,
                               stream, (const float*)X, rows, cols, ld, (double*)Xt, ldo, hi, lo,
                               kbs, flag);
        else if (v4)
            hipLaunchKernelGGL((transpose_in_kernel<float, float, true>), grid, dim3(NT), 0,
                               stream, (const float*)X, rows, cols, ld, (float*)Xt, ldo, hi, lo,
                               kbs, flag);
        else
            hipLaunchKernelGGL((transpose_in_kernel<float, float, false>), grid, dim3(NT), 0,
                               stream, (const float*)X, rows, cols, ld, (float*)Xt, ldo, hi, lo,
                               kbs, flag);
    }
    return hipGetLastError();
}

hipError_t launch_sym_copy(const void* S, int s_is_f64, int64_t p, int64_t ld, void* out,
                           int store, int64_t ldo, hipStream_t stream) {
    if (p == 0) return hipSuccess;
    const unsigned T = (unsigned)((p + 63) / 64);
    if (T > 65535u) return hipErrorInvalidValue;
    if (s_is_f64)
        hipLaunchKernelGGL(sym_copy_kernel<double>, dim3(T, T), dim3(NT), 0, stream,
                           (const double*)S, p, ld, out, store, ldo);
    else
        hipLaunchKernelGGL(sym_copy_kernel<float>, dim3(T, T), dim3(NT), 0, stream,
                           (const float*)S, p, ld, out, store, ldo);
    return hipGetLastError();
}

hipError_t launch_check_finite(const void* A, int is_f64, int64_t rows, int64_t cols,
                               int64_t ld, int* flag, hipStream_t stream) {
    if (rows == 0 || cols == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<int64_t>(rows, 8192);
    if (is_f64)
        hipLaunchKernelGGL(check_finite_kernel<double>, dim3(nb), dim3(NT), 0, stream,
                           (const double*)A, rows, cols, ld, flag);
    else
        hipLaunchKernelGGL(check_finite_kernel<float>, dim3(nb), dim3(NT), 0, stream,
                           (const float*)A, rows, cols, ld, flag);
    return hipGetLastError();
}

// column blocks of the masked-gradient row pass: GRAD_RC chunks of 64 V columns each
int grad_col_blocks(int store, int64_t n) {
    const int64_t w = GRAD_RC * 64 * (store == ST_F64 ? Chunk<ST_F64>::V : Chunk<ST_F32>::V);
    return (int)((n + w - 1) / w);
}

hipError_t launch_grad_rows(const Csr& om, int64_t p, int64_t nnz, const void* Y, const void* Xt,
                            int store, int64_t ld, int64_t n, double* D, void* oy,
                            hipStream_t stream) {
    if (p == 0) return hipSuccess;
    dim3 grid(blocks_for(p, WPB));
    if (store == ST_F64)
        hipLaunchKernelGGL((grad_rows_kernel<ST_F64, GRAD_RC, 2>), grid, dim3(NT), 0, stream,
                           om.rowptr, om.col, om.val, p, Y, Xt, ld, n, nnz, D, oy);
    else
        hipLaunchKernelGGL((grad_rows_kernel<ST_F32, GRAD_RC, 2>), grid, dim3(NT), 0, stream,
                           om.rowptr, om.col, om.val, p, Y, Xt, ld, n, nnz, D, oy);
    return hipGetLastError();
}

hipError_t launch_grad_combine(const Csr& om, int64_t p, int64_t nnz, int ncb, const double* D,
                               int64_t n, double lam2, void* out, int out_f64,
                               hipStream_t stream) {
    if (p == 0) return hipSuccess;
    hipLaunchKernelGGL(grad_combine_kernel, dim3(blocks_for(p, WPB)), dim3(NT), 0, stream,
                       om.rowptr, om.col, om.val, p, nnz, ncb, D, 1.0 / (2.0 * (double)n), lam2,
                       out, out_f64);
    return hipGetLastError();
}

hipError_t launch_gather_dense_grad(const void* M, int mstore, int64_t ldm, const Csr& om,
                                    int64_t p, double lam2, void* out, int out_f64,
                                    hipStream_t stream) {
    const unsigned nb = blocks_for(p * p, NT);
    if (mstore == ST_F64)
        hipLaunchKernelGGL(dense_grad_kernel<ST_F64>, dim3(nb), dim3(NT), 0, stream, M, ldm,
                           om.rowptr, om.col, om.val, p, lam2, out, out_f64);
    else
        hipLaunchKernelGGL(dense_grad_kernel<ST_F32>, dim3(nb), dim3(NT), 0, stream, M, ldm,
                           om.rowptr, om.col, om.val, p, lam2, out, out_f64);
    return hipGetLastError();
}

hipError_t launch_transpose_out(const void* Yt, int store, int64_t p, int64_t n, int64_t ld,
                                double scale, void* out, int out_f64, hipStream_t stream) {
    if (p == 0 || n == 0) return hipSuccess;
    dim3 grid(blocks_for(n, 64), blocks_for(p, 64));
    if (grid.y > 65535u) return hipErrorInvalidValue;
    const bool v4 = store == ST_F32 && !out_f64 && ld % 4 == 0 && p % 4 == 0 &&
                    ((uintptr_t)Yt & 15) == 0 && ((uintptr_t)out & 15) == 0;
    if (store == ST_F64)
        hipLaunchKernelGGL((transpose_out_kernel<double, false>), grid, dim3(NT), 0, stream,
                           (const double*)Yt, p, n, ld, scale, out, out_f64);
    else if (v4)
        hipLaunchKernelGGL((transpose_out_kernel<float, true>), grid, dim3(NT), 0, stream,
                           (const float*)Yt, p, n, ld, scale, out, out_f64);
    else
        hipLaunchKernelGGL((transpose_out_kernel<float, false>), grid, dim3(NT), 0, stream,
                           (const float*)Yt, p, n, ld, scale, out, out_f64);
    return hipGetLastError();
}

hipError_t launch_csr_validate(const int64_t* rowptr, const int32_t* col, const void* val,
                               int val_f64, int64_t p, int64_t nnz, int* flags,
                               hipStream_t stream) {
    if (val_f64)
        hipLaunchKernelGGL(csr_validate_kernel<double>, dim3(blocks_for(p, NT)), dim3(NT), 0, stream,
                           rowptr, col, (const double*)val, p, nnz, flags);
    else
        hipLaunchKernelGGL(csr_validate_kernel<float>, dim3(blocks_for(p, NT)), dim3(NT), 0, stream,
                           rowptr, col, (const float*)val, p, nnz, flags);
    return hipGetLastError();
}

hipError_t launch_csr_import(const int32_t* col, const void* val, int val_f64, int64_t nnz,
                             int32_t* col_out, double* val_out, hipStream_t stream) {
    if (nnz == 0) return hipSuccess;
    if (val_f64)
        hipLaunchKernelGGL(csr_import_kernel<double>, dim3(blocks_for(nnz, NT)), dim3(NT), 0, stream,
                           col, (const double*)val, nnz, col_out, val_out);
    else
        hipLaunchKernelGGL(csr_import_kernel<float>, dim3(blocks_for(nnz, NT)), dim3(NT), 0, stream,
                           col, (const float*)val, nnz, col_out, val_out);
    return hipGetLastError();
}

hipError_t launch_csr_export(const double* val, int64_t nnz, void* out, int out_f64,
                             hipStream_t stream) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(csr_export_kernel, dim3(blocks_for(nnz, NT)), dim3(NT), 0, stream, val, nnz,
                       out, out_f64);
    return hipGetLastError();
}

// ================================ batched solves ==================================
// Phase kernels over many Cov solves at once (see BatchPlan in internal.h).  Each one
// runs the single solver's kernel body on work items (solve, local block) taken from the
// iteration's tables by a fixed grid whose blocks loop over the items, so a solve's
// arithmetic is exactly the single solver's.
namespace {

constexpr int SCAN_BLOCK = 1024;   // threads of the plan kernels

// active index a with off[a] <= it < off[a + 1]
__device__ inline int find_item(const int* __restrict__ off, int nact, int it) {
    int lo = 0, hi = nact;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= it) lo = mid; else hi = mid;
    }
    return lo;
}

// f(solve, local block) for every item of phase ph; a block barrier after each item
// keeps the block-wide LDS of one item from being overwritten by the next
template <class F>
__device__ __forceinline__ void for_items(const BatchPlan& pl, int nsolve, int ph, F&& f) {
    const int nact = __builtin_amdgcn_readfirstlane(pl.status[2]);
    const int* off = pl.off + ph * (nsolve + 1);
    const int total = __builtin_amdgcn_readfirstlane(off[nact]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int a = __builtin_amdgcn_readfirstlane(find_item(off, nact, it));
        const int si = __builtin_amdgcn_readfirstlane(pl.act[a]);
        f(si, (int64_t)(it - off[a]));
        __syncthreads();
    }
}

__device__ inline bool in_accept(const SolveDesc& d, bool init) {
    return init || d.st->accepted != 0;
}

// trial step size of the batch starting at q_base: tau0 * shrink^q_base, formed by
// q_base successive multiplications as the single solver forms it
__device__ inline double batch_tau(const BatchArgs& a, int q_base) {
    double t = a.tau0;
    for (int i = 0; i < q_base; ++i) t *= a.shrink;
    return t;
}

// Block-wide exclusive scan of BP_N counters per thread (blockDim.x == SCAN_BLOCK).
__device__ void block_scan_counts(int (&v)[BP_N], int (&tot)[BP_N]) {
    __shared__ int ws[SCAN_BLOCK / 64][BP_N];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
    for (int ph = 0; ph < BP_N; ++ph) {
        int x = v[ph];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int up = __shfl_up(x, o, 64);
            if (lane >= o) x += up;
        }
        if (lane == 63) ws[wave][ph] = x;
        v[ph] = x - v[ph];   // exclusive within the wave
    }
    __syncthreads();
#pragma unroll
    for (int ph = 0; ph < BP_N; ++ph) {
        int before = 0, all = 0;
        for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
            before += w < wave ? ws[w][ph] : 0;
            all += ws[w][ph];
        }
        v[ph] += before;
        tot[ph] = all;
    }
    __syncthreads();
}

// Start of an iteration: the running solves, their work counts per phase and the reset
// of their search state; one block.
__global__ void __launch_bounds__(SCAN_BLOCK)
batch_plan_kernel(const SolveDesc* __restrict__ sd, const InstDesc* __restrict__ idesc,
                  BatchPlan pl, BatchArgs a, int init) {
    const int N = a.nsolve;
    int carry[BP_N];
#pragma unroll
    for (int ph = 0; ph < BP_N; ++ph) carry[ph] = 0;
    int grow = 0;
    for (int base = 0; base < N; base += SCAN_BLOCK) {
        const int si = base + threadIdx.x;
        int cnt[BP_N];
#pragma unroll
        for (int ph = 0; ph < BP_N; ++ph) cnt[ph] = 0;
        int run = 0;
        if (si < N) {
            const SolveDesc& d = sd[si];
            SolveCtl* c = d.ctl;
            if (c->grow) ++grow;
            if (c->phase != BPH_DONE && !c->grow) {
                run = 1;
                const int64_t p = d.p;
                const int m = a.tb < a.total - c->q_base ? a.tb : a.total - c->q_base;
                int nseg;
                int64_t seg;
                colsum_shape(p, &nseg, &seg);
                cnt[BP_ROW] = (int)((p + WPB - 1) / WPB);
                cnt[BP_ROWU] = d.grouped ? 0 : cnt[BP_ROW];
                cnt[BP_ROWG] = d.grouped ? (int)((p + WPB * (64 / TG) - 1) / (WPB * (64 / TG))) : 0;
                cnt[BP_SCAN] = (int)((p + SCAN_CHUNK - 1) / SCAN_CHUNK);
                cnt[BP_COLT] = 4 * m * nseg;
                cnt[BP_COLO] = 4 * nseg;
                const int64_t nt = (int64_t)d.T * (d.T + 1) / 2;
                cnt[BP_SROWS] = d.screen ? d.T : 0;
                cnt[BP_SPAIRS] = d.screen ? (int)((nt + NT - 1) / NT) : 0;
                cnt[BP_SOLVE] = 1;
                if (!init) {
                    DevState* st = d.st;
                    st->accepted_q = -1;
                    st->accepted = 0;
                    st->nonpos = 0;
                    if (c->phase == BPH_CAND) st->overflow = 0;
                }
            }
        }
        // a running solve has one BP_SOLVE item, so that scan is its active index
        int v[BP_N], tot[BP_N];
#pragma unroll
        for (int ph = 0; ph < BP_N; ++ph) v[ph] = cnt[ph];
        block_scan_counts(v, tot);
        if (run) {
            const int ai = carry[BP_SOLVE] + v[BP_SOLVE];
            pl.act[ai] = si;
#pragma unroll
            for (int ph = 0; ph < BP_N; ++ph) pl.off[ph * (N + 1) + ai] = carry[ph] + v[ph];
        }
#pragma unroll
        for (int ph = 0; ph < BP_N; ++ph) carry[ph] += tot[ph];
    }
    // every running solve has exactly one item of BP_SOLVE: carry[BP_SOLVE] = nact
    if (threadIdx.x == 0) {
        const int nact = carry[BP_SOLVE];
#pragma unroll
        for (int ph = 0; ph < BP_N; ++ph) pl.off[ph * (N + 1) + nact] = carry[ph];
        pl.status[2] = nact;
        pl.status[0] = 0;
    }
    // solves waiting for more candidate capacity (counted once: sums over threads)
    __shared__ int gsum;
    if (threadIdx.x == 0) gsum = 0;
    __syncthreads();
    if (grow) atomicAdd(&gsum, grow);
    __syncthreads();
    if (threadIdx.x == 0) pl.status[1] = gsum;
    for (int i = threadIdx.x; i < a.ninst; i += SCAN_BLOCK) *idesc[i].ucount = 0;
}

// Omega = I for every solve (the start of Algorithm 1)
__global__ void __launch_bounds__(NT)
batch_identity_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve) {
    for_items(pl, nsolve, BP_ROW, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        const Csr& o = d.om[d.ctl->cur];
        const int64_t i = lb * WPB + (threadIdx.x >> 6);
        if (i < d.p && lane_id() == 0) {
            o.rowptr[i] = i;
            o.col[i] = (int32_t)i;
            o.val[i] = 1.0;
            if (i == d.p - 1) o.rowptr[d.p] = d.p;
        }
    });
}

// ---- candidates: merge of the threshold words, scan, fill, gradient ----
__global__ void __launch_bounds__(NT)
batch_merge_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve) {
    for_items(pl, nsolve, BP_ROW, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.ctl->phase != BPH_CAND) return;
        const Csr& o = d.om[d.ctl->cur];
        cand_merge_body(lb, o.rowptr, o.col, d.p, d.bitmap, d.nwords, d.cnt,
                        d.screen ? d.rws.tmask : nullptr);
    });
}

// scan of cnt into A.rowptr (cands) or into the next iterate's rowptr (emission)
template <bool EMIT>
__global__ void __launch_bounds__(NT)
batch_scan_part_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_SCAN, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (EMIT ? !in_accept(d, init) : d.ctl->phase != BPH_CAND) return;
        scan_part_body(lb, d.cnt, d.p, d.scanws);
    });
}

template <bool EMIT>
__global__ void __launch_bounds__(NT)
batch_scan_apply_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_SCAN, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (EMIT ? !in_accept(d, init) : d.ctl->phase != BPH_CAND) return;
        const int64_t nb = (d.p + SCAN_CHUNK - 1) / SCAN_CHUNK;
        if (EMIT)
            scan_apply_body(lb, nb, d.cnt, d.p, d.scanws, d.om[d.ctl->cur ^ 1].rowptr, d.a_cap,
                            nullptr, &d.st->nnz_next);
        else
            scan_apply_body(lb, nb, d.cnt, d.p, d.scanws, d.A.rowptr, d.a_cap, &d.st->overflow,
                            &d.st->n_cand);
    });
}

__global__ void __launch_bounds__(NT)
batch_fill_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve) {
    for_items(pl, nsolve, BP_ROW, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.ctl->phase != BPH_CAND) return;
        const Csr& o = d.om[d.ctl->cur];
        cand_fill_body<ST_F32>(lb, nullptr, 0, o.rowptr, o.col, o.val, d.p, 0.0, d.bitmap,
                               d.nwords, d.A.rowptr, d.A.col, d.A.omega, d.A.grad,
                               &d.st->overflow, d.screen ? d.rws.tmask : nullptr);
    });
}

template <int BS>
__global__ void __launch_bounds__(NT)
batch_grad_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, BatchArgs a) {
    for_items(pl, a.nsolve, BP_ROWU, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.ctl->phase != BPH_CAND || d.grouped) return;
        const Csr& o = d.om[d.ctl->cur];
        cand_grad_cov_body<BS>(lb, o.rowptr, o.col, o.val, d.p, d.S, d.lds, a.lam2, d.A.rowptr,
                               d.A.col, d.A.omega, d.A.grad, &d.st->overflow);
    });
    for_items(pl, a.nsolve, BP_ROWG, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.ctl->phase != BPH_CAND || !d.grouped) return;
        const Csr& o = d.om[d.ctl->cur];
        cand_grad_cov_g_body<BS>(lb, o.rowptr, o.col, o.val, d.p, d.S, d.lds, a.lam2, d.A.rowptr,
                                 d.A.col, d.A.omega, d.A.grad, &d.st->overflow);
    });
}

// ---- trials and the decision ----
template <int BS>
__global__ void __launch_bounds__(NT)
batch_trial_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, BatchArgs a) {
    for_items(pl, a.nsolve, BP_ROWU, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.grouped) return;
        const int q = d.ctl->q_base;
        const int m = a.tb < a.total - q ? a.tb : a.total - q;
        trial_body<BS, false>(lb, 0, 1, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p,
                              batch_tau(a, q), a.shrink, m, d.lam1, d.S, d.lds, 0, nullptr, d.part,
                              d.st);
    });
}

template <int BS>
__global__ void __launch_bounds__(NT)
batch_trial_grouped_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, BatchArgs a) {
    for_items(pl, a.nsolve, BP_ROWG, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!d.grouped) return;
        const int q = d.ctl->q_base;
        const int m = a.tb < a.total - q ? a.tb : a.total - q;
        trial_cov_body<BS>(lb, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p, batch_tau(a, q),
                           a.shrink, m, d.lam1, d.S, d.lds, d.part, d.st);
    });
}

__global__ void __launch_bounds__(NT)
batch_decide_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, BatchArgs a) {
    for_items(pl, a.nsolve, BP_COLT, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        const int q = d.ctl->q_base;
        const int m = a.tb < a.total - q ? a.tb : a.total - q;
        int nseg;
        int64_t seg;
        colsum_shape(d.p, &nseg, &seg);
        FinArgs fa{m, q, -1, 0, batch_tau(a, q), a.shrink, a.lam2, 1.0, nullptr};
        colsum_finish_body<FIN_DECIDE>((int)(lb % (4 * m)), (int)(lb / (4 * m)), 4 * m, nseg,
                                       d.part, d.p, seg, d.colws, d.tsums, &d.st->ticket, fa,
                                       d.st);
    });
}

// ---- emission of the accepted iterates ----
__global__ void __launch_bounds__(NT)
batch_emit_count_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve) {
    for_items(pl, nsolve, BP_ROWU, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.grouped) return;
        emit_count_body(lb, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p, d.lam1, d.st, d.cnt);
    });
    for_items(pl, nsolve, BP_ROWG, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!d.grouped) return;
        emit_count_g_body(lb, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p, d.lam1, d.st, d.cnt);
    });
}

__global__ void __launch_bounds__(NT)
batch_emit_fill_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve) {
    for_items(pl, nsolve, BP_ROWU, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (d.grouped) return;
        const Csr& o = d.om[d.ctl->cur ^ 1];
        emit_fill_body(lb, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p, d.lam1, d.st, o.rowptr,
                       o.col, o.val);
    });
    for_items(pl, nsolve, BP_ROWG, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!d.grouped) return;
        const Csr& o = d.om[d.ctl->cur ^ 1];
        emit_fill_g_body(lb, d.A.rowptr, d.A.col, d.A.omega, d.A.grad, d.p, d.lam1, d.st, o.rowptr,
                         o.col, o.val);
    });
}

// ---- products at the accepted iterates (or at the start, init) ----
__device__ inline const Csr& prod_csr(const SolveDesc& d, bool init) {
    return d.om[init ? d.ctl->cur : d.ctl->cur ^ 1];
}

__global__ void __launch_bounds__(64)
batch_screen_rows_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_SROWS, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!in_accept(d, init)) return;
        const Csr& o = prod_csr(d, init);
        screen_rows_body((int)lb, o.rowptr, o.col, o.val, d.p, d.T, d.rws.lcnt, d.rws.lK,
                         d.rws.lW, d.rws.lcmax, d.rws.pcount, d.rws.tmask, nullptr);
    });
}

template <typename E>
__global__ void __launch_bounds__(NT)
batch_screen_pairs_kernel(const SolveDesc* __restrict__ sd, const InstDesc* __restrict__ idesc,
                          BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_SPAIRS, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!in_accept(d, init)) return;
        const InstDesc& id = idesc[d.inst];
        screen_pairs_body<E>((int)lb, d.T, d.rws.lcnt, d.rws.lK, d.rws.lW, d.rws.lcmax, d.smax,
                             d.lam1, d.rws.plist, d.rws.pcount, d.rws.tmask, nullptr, id.ulist,
                             id.ucount, id.ubits);
    });
}

// per instance: how many tile pairs its refresh walks (its list, or every pair when the
// instance is not screened and one of its solves refreshes)
__global__ void __launch_bounds__(SCAN_BLOCK)
batch_refresh_plan_kernel(const SolveDesc* __restrict__ sd, const InstDesc* __restrict__ idesc,
                          BatchPlan pl, int ninst, int init) {
    int carry = 0;
    for (int base = 0; base < ninst; base += SCAN_BLOCK) {
        const int i = base + threadIdx.x;
        int v[BP_N], tot[BP_N];
#pragma unroll
        for (int ph = 0; ph < BP_N; ++ph) v[ph] = 0;
        if (i < ninst) {
            const InstDesc& id = idesc[i];
            if (id.screen) {
                v[0] = *id.ucount;
            } else {
                bool any = false;
                for (int l = 0; l < id.nsolve; ++l) {
                    const SolveDesc& d = sd[id.first + l];
                    any = any || (d.ctl->phase != BPH_DONE && !d.ctl->grow && in_accept(d, init));
                }
                v[0] = any ? id.T * (id.T + 1) / 2 : 0;
            }
        }
        block_scan_counts(v, tot);
        if (i < ninst) pl.roff[i] = carry + v[0];
        carry += tot[0];
    }
    if (threadIdx.x == 0) pl.roff[ninst] = carry;
}

// The refresh of Algorithm 2's product at the accepted iterates, lambda-stacked: one work
// item per (instance, listed tile pair) refreshes the pair for every solve of the
// instance that kept it, one after the other in the same workgroup, so the S tiles the
// pair reads are fetched once and served from the cache for the other lambda1 values.
template <int BS>
__global__ void __launch_bounds__(NT)
batch_refresh_kernel(const SolveDesc* __restrict__ sd, const InstDesc* __restrict__ idesc,
                     BatchPlan pl, int ninst, int init) {
    const int total = __builtin_amdgcn_readfirstlane(pl.roff[ninst]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(find_item(pl.roff, ninst, it));
        const InstDesc& id = idesc[i];
        const int t0 = it - pl.roff[i];
        const int T = id.T, nt = T * (T + 1) / 2;
        const int t = __builtin_amdgcn_readfirstlane(id.screen ? id.ulist[t0] : t0);
        if (id.screen && threadIdx.x == 0) atomicAnd(&id.ubits[t >> 5], ~(1u << (t & 31)));
        const int2 ij = refresh_tile(t, T, nt);
        const int I = __builtin_amdgcn_readfirstlane(ij.x), J = __builtin_amdgcn_readfirstlane(ij.y);
        const int TW = (T + 63) / 64;
        for (int l = 0; l < id.nsolve; ++l) {
            const SolveDesc& d = sd[id.first + l];
            const SolveCtl* c = d.ctl;
            if (c->phase == BPH_DONE || c->grow || !in_accept(d, init)) continue;
            if (id.screen && !((d.rws.tmask[(int64_t)I * TW + (J >> 6)] >> (J & 63)) & 1ull)) continue;
            const Csr& o = prod_csr(d, init);
            refresh_pair<BS>(I, J, o.rowptr, o.col, o.val, d.p, d.S, d.lds,
                             id.screen ? d.smax : nullptr, T, d.lam1, d.bitmap, d.nwords, nullptr);
            __syncthreads();   // the pair's LDS is reused by the next solve
        }
    }
}

template <int BS>
__global__ void __launch_bounds__(NT)
batch_obj_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_ROWU, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!in_accept(d, init) || d.grouped) return;
        const Csr& o = prod_csr(d, init);
        obj_parts_cov_body<BS>(lb, o.rowptr, o.col, o.val, d.p, d.S, d.lds,
                               d.part + 4 * MAXQ * d.p, nullptr);
    });
    for_items(pl, nsolve, BP_ROWG, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!in_accept(d, init) || !d.grouped) return;
        const Csr& o = prod_csr(d, init);
        obj_parts_cov_g_body<BS>(lb, o.rowptr, o.col, o.val, d.p, d.S, d.lds,
                                 d.part + 4 * MAXQ * d.p, nullptr);
    });
}

__global__ void __launch_bounds__(NT)
batch_obj_sum_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, int nsolve, int init) {
    for_items(pl, nsolve, BP_COLO, [&](int si, int64_t lb) {
        const SolveDesc& d = sd[si];
        if (!in_accept(d, init)) return;
        int nseg;
        int64_t seg;
        colsum_shape(d.p, &nseg, &seg);
        FinArgs fa{0, 0, -1, 0, 0.0, 0.5, 0.0, 0.0, nullptr};
        colsum_finish_body<FIN_OBJ>((int)(lb % 4), (int)(lb / 4), 4, nseg,
                                    d.part + 4 * MAXQ * d.p, d.p, seg, d.colws, d.osums,
                                    &d.st->ticket, fa, d.st);
    });
}

// End of an iteration: accept (the iterate is the emitted one), the stopping test of
// concord_solve, or the next trial batch; counts the solves still running.
__global__ void __launch_bounds__(NT)
batch_finish_kernel(const SolveDesc* __restrict__ sd, BatchPlan pl, BatchArgs a, int init) {
    for_items(pl, a.nsolve, BP_SOLVE, [&](int si, int64_t) {
        if (threadIdx.x != 0) return;
        const SolveDesc& d = sd[si];
        SolveCtl* c = d.ctl;
        DevState* st = d.st;
        double f, F;
        if (init) {
            objective_value(st->obj, false, 1.0, d.lam1, a.lam2, &f, &F);
            c->F = F;
            atomicAdd(&pl.status[0], 1);
            return;
        }
        if (st->overflow) {   // the host grows the candidate arrays, then the step restarts
            c->grow = 1;
            c->phase = BPH_CAND;
            atomicAdd(&pl.status[1], 1);
            return;
        }
        const int m = a.tb < a.total - c->q_base ? a.tb : a.total - c->q_base;
        if (st->accepted_q < 0) {   // every step size of the batch failed the test
            c->q_base += m;
            if (c->q_base >= a.total) {
                c->status = CONCORD_ELINESEARCH;
                c->phase = BPH_DONE;
            } else {
                c->phase = BPH_TRIAL;
                atomicAdd(&pl.status[0], 1);
            }
            return;
        }
        c->cur ^= 1;
        c->k += 1;
        c->q_base = 0;
        objective_value(st->obj, false, 1.0, d.lam1, a.lam2, &f, &F);
        const double F_old = c->F;
        c->F = F;
        if (a.tol > 0.0 && fabs(F - F_old) < a.tol * fabs(F_old)) {
            c->status = CONCORD_OK;
            c->phase = BPH_DONE;
        } else if (c->k >= a.max_iter) {
            c->status = a.tol > 0.0 ? CONCORD_WMAXITER : CONCORD_OK;
            c->phase = BPH_DONE;
        } else {
            c->phase = BPH_CAND;
            atomicAdd(&pl.status[0], 1);
        }
    });
}

}  // namespace

hipError_t launch_batch_iteration(const SolveDesc* sd, const InstDesc* idesc, const BatchPlan& pl,
                                  const BatchArgs& a, bool init, int grid, hipStream_t stream) {
    const int N = a.nsolve, ini = init ? 1 : 0;
    const dim3 g(grid), b(NT);
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(SCAN_BLOCK), 0, stream, sd, idesc, pl, a, ini);
    if (init) {
        hipLaunchKernelGGL(batch_identity_kernel, g, b, 0, stream, sd, pl, N);
    } else {
        hipLaunchKernelGGL(batch_merge_kernel, g, b, 0, stream, sd, pl, N);
        // chunk sums: none needed while every solve fits one scan chunk (the apply of
        // chunk 0 reads none)
        if (a.any_multichunk)
            hipLaunchKernelGGL(batch_scan_part_kernel<false>, g, b, 0, stream, sd, pl, N, 0);
        hipLaunchKernelGGL(batch_scan_apply_kernel<false>, g, b, 0, stream, sd, pl, N, 0);
        hipLaunchKernelGGL(batch_fill_kernel, g, b, (size_t)WPB * ((a.maxT + 63) / 64) * 8, stream,
                           sd, pl, N);
#define BCAND(BS)                                                                            \
        hipLaunchKernelGGL(batch_grad_kernel<BS>, g, b, 0, stream, sd, pl, a);                \
        if (a.any_rowu) hipLaunchKernelGGL(batch_trial_kernel<BS>, g, b, 0, stream, sd, pl, a); \
        if (a.any_rowg)                                                                       \
            hipLaunchKernelGGL(batch_trial_grouped_kernel<BS>, g, b, 0, stream, sd, pl, a)
        if (a.bstore == ST_F64) { BCAND(ST_F64); }
        else if (a.bstore == ST_F32) { BCAND(ST_F32); }
        else { BCAND(ST_B16P); }
#undef BCAND
        hipLaunchKernelGGL(batch_decide_kernel, g, b, 0, stream, sd, pl, a);
        hipLaunchKernelGGL(batch_emit_count_kernel, g, b, 0, stream, sd, pl, N);
        if (a.any_multichunk)
            hipLaunchKernelGGL(batch_scan_part_kernel<true>, g, b, 0, stream, sd, pl, N, 0);
        hipLaunchKernelGGL(batch_scan_apply_kernel<true>, g, b, 0, stream, sd, pl, N, 0);
        hipLaunchKernelGGL(batch_emit_fill_kernel, g, b, 0, stream, sd, pl, N);
    }
    if (a.any_screen) {
        hipLaunchKernelGGL(batch_screen_rows_kernel, dim3(grid * WPB), dim3(64),
                           (size_t)8 * a.maxT, stream, sd, pl, N, ini);
        if (a.bstore == ST_F64)
            hipLaunchKernelGGL(batch_screen_pairs_kernel<double>, g, b, 0, stream, sd, idesc, pl,
                               N, ini);
        else
            hipLaunchKernelGGL(batch_screen_pairs_kernel<float>, g, b, 0, stream, sd, idesc, pl,
                               N, ini);
    }
    hipLaunchKernelGGL(batch_refresh_plan_kernel, dim3(1), dim3(SCAN_BLOCK), 0, stream, sd, idesc,
                       pl, a.ninst, ini);
#define BREF(BS)                                                                              \
    hipLaunchKernelGGL(batch_refresh_kernel<BS>, g, b, 0, stream, sd, idesc, pl, a.ninst, ini);  \
    hipLaunchKernelGGL(batch_obj_kernel<BS>, g, b, 0, stream, sd, pl, N, ini)
    if (a.bstore == ST_F64) { BREF(ST_F64); }
    else if (a.bstore == ST_F32) { BREF(ST_F32); }
    else { BREF(ST_B16P); }
#undef BREF
    hipLaunchKernelGGL(batch_obj_sum_kernel, g, b, 0, stream, sd, pl, N, ini);
    hipLaunchKernelGGL(batch_finish_kernel, g, b, 0, stream, sd, pl, a, ini);
    return hipGetLastError();
}

}  // namespace concord
