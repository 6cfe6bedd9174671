// Exact K-nearest-neighbour search for the A-tSNE similarity path on gfx950.
//
// The neighbour sets of Sec. 3.1 (Eq. 8) under the squared Euclidean
// distance of Eq. 3, found by brute force: the paper notes that no exact
// method beats a linear scan in high dimension (Sec. 4.2), and on MI355X the
// scan is a dense contraction that belongs on the matrix cores.
//
// Pipeline (all on the caller's stream, no host synchronisation):
//   knn_prep       padded copy of X in the contraction's element type
//                  (FP32 / BF16 RNE / FP8 e4m3 with per-row absmax scales /
//                  FP32X3: BF16 hi and lo parts of each FP32 value), row
//                  norms n_i = ||x_i||^2 and their prefix maximum.
//   knn_tile       S = X_q X_k^T on MFMA, d'_ij = n_j - 2 S_ij (n_i is a row
//                  constant and irrelevant to the ranking), self and padding
//                  masked; operands staged by direct global -> LDS loads; a
//                  running per-(query, split) threshold filters candidates
//                  into a buffer that is cut back (to between k_cand and
//                  k_cand + slack keys, new threshold) whenever it fills, and
//                  shrunk exactly to the best k_cand at the end.
//   knn_select     per query, the best k_cand keys (d', j) over all splits,
//                  exact FP32 direct-difference distances for those that can
//                  reach the (k+1)-th place (on the exact contractions the
//                  contraction's error bound rules the others out), sorted
//                  by (d, j); rows whose k-th/(k+1)-th gap is under FP32
//                  resolution are re-ranked in FP64.  On the exact
//                  contractions (FP32, FP32X3) the same bound certifies that
//                  no non-candidate can beat the k-th neighbour; rows it
//                  cannot certify are queued for knn_scan.
//   knn_scan       exact FP32 linear scan for the queued rows (rare); a
//                  scanned row ends exactly as a certified row would.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <memory>
#include <type_traits>

#include "knn_internal.h"
#include "wave.h"

namespace atsne {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Workgroup geometry: every contraction type runs 8 waves (256 queries x 256
// keys), two waves per SIMD, so one wave's epilogue (filter, appends) and LDS
// waits hide behind the other's MFMAs.  For FP8 this costs a few spilled
// registers per lane and still beats one wave per SIMD by a third.  The
// small geometry (FP32/BF16, 4 waves, 128 queries x 128 keys, two
// workgroups per CU) gives small problems four times as many workgroups.
template <int P, bool SMALL = false>
struct TileGeom {
    static constexpr int WAVES = SMALL ? 4 : 8;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int QB = 32 * WAVES;  // queries per workgroup
    static constexpr int KT = SMALL ? 128 : 256;  // keys per tile
    static constexpr int NKB = KT / 32;          // MFMA key blocks per tile
    static constexpr int WPE = 2;
};
constexpr int KNN_XCDS = 8;  // accelerator complex dies; workgroups go round-robin over them
__host__ __device__ constexpr int qb_of(int) { return 256; }
constexpr int KT = KNN_KT;      // keys per tile (8 MFMA blocks of 32)
constexpr int CHUNK_UNITS = 8;  // 16-byte units per row per D-chunk (128 bytes)

// LDS tile layout: rows of CHUNK_UNITS unpadded 16-byte units, unit u of row r
// in slot u ^ lds_swz(r).  For a fixed unit, any 8 consecutive rows, and the
// 8 even or the 8 odd rows of any 16 consecutive rows aligned to 16, land in
// distinct 16-byte bank groups, so the MFMA fragment reads (one unit of each
// of 32 consecutive rows per half-wave) are free of bank conflicts with 32 or
// with 64 banks.
__device__ __forceinline__ int lds_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// Direct global -> LDS loads (no register staging): lane i of the wave writes
// its 16 (or 4) bytes to lds + 16 i (or 4 i); `lds` must be wave-uniform.
__device__ __forceinline__ void lds_dma16(const uint4* src, uint4* lds) {
    __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma4(const float* src, float* lds) {
    __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

// Elements per 128-byte chunk for each precision.
__host__ __device__ constexpr int chunk_elems(int prec) {
    return (prec == ATSNE_PREC_FP32 || prec == ATSNE_PREC_FP32X3) ? 32 : (prec == ATSNE_PREC_BF16 ? 64 : 128);
}
__host__ __device__ constexpr int elem_bytes(int prec) {
    // (FP32X3: a BF16 hi and a BF16 lo per element)
    return (prec == ATSNE_PREC_FP32 || prec == ATSNE_PREC_FP32X3) ? 4 : (prec == ATSNE_PREC_BF16 ? 2 : 1);
}

// ---------------------------------------------------------------------------
// Element conversions (written from the format definitions).
// ---------------------------------------------------------------------------

// FP32 -> BF16 with round-to-nearest-even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> OCP FP8 E4M3 (bias 7, 3 mantissa bits, max 448, no infinities),
// round-to-nearest-even, saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3_rne(float v) {
    uint8_t sign = (__float_as_uint(v) >> 24) & 0x80u;
    float a = fabsf(v);
    if (!(a < 448.0f)) return sign | 0x7eu;
    if (a < 0.015625f) {  // below 2^-6: subnormal, step 2^-9
        int m = (int)rintf(a * 512.0f);  // 0..8; 8 rounds up into the first normal
        return sign | (uint8_t)m;
    }
    int e;
    frexpf(a, &e);  // a = f * 2^e, f in [0.5, 1)  => unbiased exponent e-1
    int ex = e - 1;
    int m = (int)rintf(ldexpf(a, 3 - ex));  // in [8, 16]
    if (m == 16) { m = 8; ++ex; }
    int be = ex + 7;
    if (be > 15 || (be == 15 && m - 8 > 6)) return sign | 0x7eu;
    return sign | (uint8_t)((be << 3) | (m - 8));
}
__device__ __forceinline__ float e4m3_to_f32(uint8_t b) {
    int e = (b >> 3) & 15, m = b & 7;
    float a = e == 0 ? ldexpf((float)m, -9) : ldexpf((float)(8 + m), e - 10);
    return (b & 0x80u) ? -a : a;
}

// ---------------------------------------------------------------------------
// knn_prep: one wave per row of [r0, r1); rows >= n_live are zero padding.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void knn_prep(const float* __restrict__ X, int64_t ld, int32_t D, int32_t Dp,
                                                int64_t r0, int64_t r1, int64_t n_live, void* __restrict__ Xp,
                                                float* __restrict__ norms, float* __restrict__ scales) {
    const int l = lane_id();
    const int64_t row = r0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= r1) return;
    const bool live = row < n_live;
    const float* x = X + row * ld;
    float s = 1.0f;
    if (P == ATSNE_PREC_FP8_E4M3) {
        float amax = 0.0f;
        if (live)
            for (int d = l; d < D; d += WAVE) amax = fmaxf(amax, fabsf(x[d]));
        amax = wave_max(amax);
        // smallest power of two s with amax / s <= 448: the MFMA applies it
        // exactly through its E8M0 scale operand
        s = 1.0f;
        if (amax > 0.0f) {
            int e;
            frexpf(amax / 448.0f, &e);  // amax/448 = f 2^e, f in [0.5, 1)
            s = ldexpf(1.0f, e);
            if (ldexpf(1.0f, e - 1) >= amax / 448.0f) s = ldexpf(1.0f, e - 1);
        }
    }
    float acc = 0.0f;
    for (int d = l; d < Dp; d += WAVE) {
        float v = (live && d < D) ? x[d] : 0.0f;
        if (P == ATSNE_PREC_FP32) {
            static_cast<float*>(Xp)[row * Dp + d] = v;
            acc = fmaf(v, v, acc);
        } else if (P == ATSNE_PREC_BF16) {
            uint16_t h = f32_to_bf16_rne(v);
            static_cast<uint16_t*>(Xp)[row * Dp + d] = h;
            float r = bf16_to_f32(h);
            acc = fmaf(r, r, acc);
        } else if (P == ATSNE_PREC_FP32X3) {
            // per 32-element chunk: 64 bytes of hi parts, then 64 bytes of lo
            // parts of the same elements; the norm is that of the FP32 row
            const uint16_t h = f32_to_bf16_rne(v);
            const uint16_t lo = f32_to_bf16_rne(v - bf16_to_f32(h));
            uint16_t* chunk = static_cast<uint16_t*>(Xp) + row * 2 * (int64_t)Dp + (d >> 5) * 64;
            chunk[d & 31] = h;
            chunk[32 + (d & 31)] = lo;
            acc = fmaf(v, v, acc);
        } else {
            uint8_t q = f32_to_e4m3_rne(v / s);
            static_cast<uint8_t*>(Xp)[row * Dp + d] = q;
            float r = e4m3_to_f32(q);
            acc = fmaf(r, r, acc);
        }
    }
    acc = wave_sum(acc);
    if (P == ATSNE_PREC_FP8_E4M3) acc *= s * s;
    if (l == 0) {
        norms[row] = live ? acc : 0.0f;
        scales[row] = s;
    }
}

// Prefix maximum of the norms over [r0, r1), continuing from pmax[r0 - 1].
// One workgroup walks the range in chunks of 1024 rows.
// Prefix max of the row norms over rows [r0, r1), continuing pmax[r0 - 1]:
// (1) each workgroup the prefix within its PMAX_CHUNK rows and the chunk's
// maximum, (2) one workgroup the exclusive prefix of the chunk maxima (the
// carry into each chunk), (3) every row its chunk's carry.
constexpr int PMAX_CHUNK = 4096;

__global__ __launch_bounds__(1024) void knn_pmax_local(const float* __restrict__ norms, float* __restrict__ pmax,
                                                       int64_t r0, int64_t r1, float* __restrict__ blk) {
    __shared__ float wmax[16];
    __shared__ float carry_s;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t c0 = r0 + (int64_t)blockIdx.x * PMAX_CHUNK;
    if (t == 0) carry_s = 0.0f;  // norms are non-negative
    __syncthreads();
    for (int s = 0; s < PMAX_CHUNK / 1024; ++s) {
        const int64_t i = c0 + 1024 * s + t;
        float v = i < r1 ? norms[i] : 0.0f;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const float u = __shfl_up(v, o, WAVE);
            if (l >= o) v = fmaxf(v, u);
        }
        if (l == WAVE - 1) wmax[w] = v;
        __syncthreads();
        float pre = carry_s;
        for (int j = 0; j < w; ++j) pre = fmaxf(pre, wmax[j]);
        v = fmaxf(v, pre);
        if (i < r1) pmax[i] = v;
        __syncthreads();
        if (t == 1023) carry_s = v;
        __syncthreads();
    }
    if (t == 0) blk[blockIdx.x] = carry_s;
}

__global__ __launch_bounds__(1024) void knn_pmax_carry(float* __restrict__ blk, int64_t nb,
                                                       const float* __restrict__ pmax, int64_t r0) {
    __shared__ float wmax[16];
    __shared__ float carry_s;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    if (t == 0) carry_s = r0 > 0 ? pmax[r0 - 1] : 0.0f;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t b = base + t;
        const float x = b < nb ? blk[b] : 0.0f;
        float v = x;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const float u = __shfl_up(v, o, WAVE);
            if (l >= o) v = fmaxf(v, u);
        }
        if (l == WAVE - 1) wmax[w] = v;
        __syncthreads();
        float pre = carry_s;
        for (int j = 0; j < w; ++j) pre = fmaxf(pre, wmax[j]);
        // exclusive: the carry before this chunk is the inclusive prefix of
        // the chunks before it
        const float up = __shfl_up(v, 1, WAVE);
        const float excl = l > 0 ? fmaxf(pre, up) : pre;
        v = fmaxf(v, pre);
        __syncthreads();
        if (b < nb) blk[b] = excl;
        if (t == 1023) carry_s = v;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void knn_pmax_apply(float* __restrict__ pmax, int64_t r0, int64_t r1,
                                                      const float* __restrict__ blk) {
    const int64_t i = r0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < r1) pmax[i] = fmaxf(pmax[i], blk[(i - r0) / PMAX_CHUNK]);
}

// Rigorous bound on |d'_qj + n_q - ||x_q - x_j||^2| for the FP32 contraction:
// with gam = (Dp + 2) u for sums of Dp products,
// |fl(n_j) - n_j| + 2|fl(S_qj) - S_qj| + |fl(n_q) - n_q| <= gam (sqrt(n_q) + sqrt(n_j))^2,
// plus the rounding of forming d' and adding n_q back.
__device__ __forceinline__ float fp32_contraction_bound(int32_t Dp, float nq, float nmax, float dprime) {
    const float u = 5.9604645e-8f;
    const float gam = 1.05f * (float)(Dp + 2) * u;
    const float sq = sqrtf(nq) + sqrtf(nmax);
    return gam * (sq * sq) + 2.0f * u * (fabsf(dprime) + nq);
}

// The same bound for the FP32X3 contraction.  With x = h + l + r (h = bf16(x),
// l = bf16(x - h)): |x - h| <= 2^-9 |x|, |r| <= 2^-18 |x|, so the dropped
// terms l l' + h r' + r h' + ... of x x' sum to at most 3.01 * 2^-18 |x x'|.
// Each 32-element chunk's 96 exact BF16 products are summed in FP32 into a
// fresh partial, and the Dp / 32 partials are added to the running sum one
// by one; counting 2u per rounding (which also covers truncating adds inside
// the matrix core), |fl(S) - S| <= (2 (96 + Dp / 32 + 1) u + 3.01 * 2^-18)
// * 1.01 * sum |x_i x'_i|.  The norms are FP32 sums as on the FP32 path.  A
// tiny absolute term covers flushed subnormal lo parts.
__device__ __forceinline__ float x3_contraction_bound(int32_t Dp, float nq, float nmax, float dprime) {
    const float u = 5.9604645e-8f;
    const float gam_s = 1.01f * (2.0f * (float)(96 + Dp / 32 + 1) * u + 3.01f * 3.8146973e-6f);
    const float gam_n = 1.05f * (float)(Dp + 2) * u;
    const float gam = fmaxf(gam_s, gam_n);
    const float sq = sqrtf(nq) + sqrtf(nmax);
    return gam * (sq * sq) + 2.0f * u * (fabsf(dprime) + nq) + (float)(3 * Dp + 2) * 1e-36f;
}

__device__ __forceinline__ int64_t load_qid(const int32_t* qids, int64_t m0, int64_t m) {
    return qids ? (int64_t)qids[m] : (m0 + m);
}

// ---------------------------------------------------------------------------
// MFMA over one 128-byte chunk.  Lane l supplies, for its row (l % 32), the
// 16-byte units chunk_unit(l, i) of the chunk; A (keys) and B (queries) use
// the same unit map, so every contraction index pairs the same dimension.
// ---------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ int chunk_unit(int l, int i) {
    if (P == ATSNE_PREC_FP8_E4M3) return 4 * (i >> 1) + 2 * (l >> 5) + (i & 1);
    return 2 * i + (l >> 5);
}

// Two key blocks against one query block over one chunk, their MFMAs
// interleaved so consecutive instructions use different accumulators.  For
// FP8 the per-row power-of-two scales enter as E8M0 scale operands (sa0, sa1
// for the key rows of each block, sb for the query column).
template <int P, bool FIRST>
__device__ __forceinline__ void mfma_pair(f32x16& acc0, f32x16& acc1, const uint4 (&a0)[4], const uint4 (&a1)[4],
                                          const uint4 (&b)[4], int sa0, int sa1, int sb) {
    const f32x16 zero = {};
    f32x16 c0 = FIRST ? zero : acc0;
    f32x16 c1 = FIRST ? zero : acc1;
    if constexpr (P == ATSNE_PREC_FP32) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[i].x), __uint_as_float(b[i].x), c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[i].x), __uint_as_float(b[i].x), c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[i].y), __uint_as_float(b[i].y), c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[i].y), __uint_as_float(b[i].y), c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[i].z), __uint_as_float(b[i].z), c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[i].z), __uint_as_float(b[i].z), c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[i].w), __uint_as_float(b[i].w), c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[i].w), __uint_as_float(b[i].w), c1, 0, 0, 0);
        }
    } else if constexpr (P == ATSNE_PREC_BF16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bf16x8 vb = __builtin_bit_cast(bf16x8, b[i]);
            c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0[i]), vb, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1[i]), vb, c1, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            const i32x8 vb = {(int)b[i].x, (int)b[i].y, (int)b[i].z, (int)b[i].w,
                              (int)b[i + 1].x, (int)b[i + 1].y, (int)b[i + 1].z, (int)b[i + 1].w};
            const i32x8 va0 = {(int)a0[i].x, (int)a0[i].y, (int)a0[i].z, (int)a0[i].w,
                               (int)a0[i + 1].x, (int)a0[i + 1].y, (int)a0[i + 1].z, (int)a0[i + 1].w};
            const i32x8 va1 = {(int)a1[i].x, (int)a1[i].y, (int)a1[i].z, (int)a1[i].w,
                               (int)a1[i + 1].x, (int)a1[i + 1].y, (int)a1[i + 1].z, (int)a1[i + 1].w};
            // operand format 0 = FP8 E4M3 for A and B
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va0, vb, c0, 0, 0, 0, sa0, 0, sb);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va1, vb, c1, 0, 0, 0, sa1, 0, sb);
        }
    }
    acc0 = c0;
    acc1 = c1;
}

// One FP8 key block against the query block over one chunk (two scaled
// MFMAs, K = 64 each).
template <bool FIRST>
__device__ __forceinline__ void mfma_fp8_block(f32x16& acc, const uint4 (&a)[4], const uint4 (&b)[4], int sa, int sb) {
    const f32x16 zero = {};
    f32x16 c = FIRST ? zero : acc;
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
        const i32x8 vb = {(int)b[i].x, (int)b[i].y, (int)b[i].z, (int)b[i].w,
                          (int)b[i + 1].x, (int)b[i + 1].y, (int)b[i + 1].z, (int)b[i + 1].w};
        const i32x8 va = {(int)a[i].x, (int)a[i].y, (int)a[i].z, (int)a[i].w,
                          (int)a[i + 1].x, (int)a[i + 1].y, (int)a[i + 1].z, (int)a[i + 1].w};
        // operand format 0 = FP8 E4M3 for A and B
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, c, 0, 0, 0, sa, 0, sb);
    }
    acc = c;
}

// One FP32X3 key block against the query block over one chunk.  Fragments
// i = 0, 1 hold the hi parts of the chunk's elements 0-15 and 16-31, i = 2, 3
// their lo parts.  The chunk's 96 exact BF16 products (per K-step lo*hi +
// hi*lo + hi*hi) go into a fresh partial, which one FP32 add folds into the
// running sum: the contraction's rounding error then grows with the number of
// chunks, not of products.
template <bool FIRST>
__device__ __forceinline__ void mfma_x3_block(f32x16& acc, const uint4 (&a)[4], const uint4 (&b)[4]) {
    f32x16 t = {};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const bf16x8 bh = __builtin_bit_cast(bf16x8, b[i]), bl = __builtin_bit_cast(bf16x8, b[i + 2]);
        const bf16x8 ah = __builtin_bit_cast(bf16x8, a[i]), al = __builtin_bit_cast(bf16x8, a[i + 2]);
        t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, t, 0, 0, 0);
    }
    acc = FIRST ? t : acc + t;
}

// E8M0 encoding of a power-of-two float scale: its biased exponent.
__device__ __forceinline__ int e8m0_of(float s) { return (int)((__float_as_uint(s) >> 23) & 0xffu); }

// Shrink one candidate slot to its best `kc` keys (wave-wide). Returns the
// key of rank kc, which becomes the slot's threshold.  With deletion stamps
// (death != null), keys of rows deleted before the query's view are dropped
// first; when no more than kc visible keys remain they are all kept and the
// returned key has distance +inf (no threshold).  Also returns the new count.
struct Shrunk {
    uint64_t kstar;
    int n;
};
__device__ Shrunk shrink_slot(uint64_t* slot, int cnt, int kc, uint32_t* hist, const int32_t* death, int32_t view) {
    const int l = lane_id();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (death) {
        int base = 0;
        for (int i0 = 0; i0 < cnt; i0 += WAVE) {
            const int i = i0 + l;
            const uint64_t k = i < cnt ? slot[i] : ~0ull;
            const bool keep = i < cnt && death[key_index(k)] >= view;
            const uint64_t m = ballot(keep);
            if (keep) slot[base + __popcll(m & lanemask_lt())] = k;
            base += __popcll(m);
        }
        cnt = base;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (cnt <= kc) return Shrunk{pack_key(INFINITY, -1), cnt};
    }
    uint64_t kstar = wave_select(
        [&](auto f) {
            for (int i = l; i < cnt; i += WAVE) f(slot[i]);
        },
        (uint32_t)kc, hist);
    int base = 0;
    for (int i0 = 0; i0 < cnt; i0 += WAVE) {
        int i = i0 + l;
        uint64_t k = i < cnt ? slot[i] : ~0ull;
        bool keep = i < cnt && k <= kstar;
        uint64_t m = ballot(keep);
        if (keep) slot[base + __popcll(m & lanemask_lt())] = k;
        base += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    return Shrunk{kstar, kc};
}

// Make room in a candidate slot while streaming: keep every key whose
// distance code (the order-preserving 32-bit image of the distance) is at
// most a threshold t chosen so that between kc and kc + allow keys remain,
// and return t as the slot's new pass threshold.  Any superset of the kc best
// keys is a valid slot state; the exact cut to kc is left to the final
// shrink.  The keys are read once into registers; t is searched on the codes
// between the smallest live code and the largest, each probe one counting
// pass (ballots and scalar popcounts): regula falsi on the count (Illinois
// variant), bisection if it has not converged after a few probes.  With deletion stamps (death !=
// null), keys deleted before the query's view are dropped first.  Slots
// beyond WAVE * MR_KEYS keys, or ties too wide for the window, take the exact
// shrink.
constexpr int MR_KEYS = 12;  // keys per lane held in registers (slots up to 768 keys)
struct Roomed {
    float tau;
    int n;
};
// NR registers of keys per lane: the loops are fully unrolled and
// branch-free (a single instantiation keeps the tile kernel's code small).
template <int NR>
__device__ Roomed make_room_nr(uint64_t* slot, int cnt, int kc, int allow, uint32_t* hist, const int32_t* death,
                               int32_t view) {
    const int l = lane_id();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    // all loads first, then their uses: one memory latency.  code[i] is the
    // key's distance code, 0xffffffff for an empty register (above every
    // live code, and never probed)
    uint64_t k[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int idx = l + WAVE * i;
        k[i] = idx < cnt ? slot[idx] : ~0ull;
    }
    if (death) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (k[i] != ~0ull && death[key_index(k[i])] < view) k[i] = ~0ull;
    }
    // a key's distance code is its upper word; an empty register (~0) has
    // code 0xffffffff, above every distance's code (at most that of +inf)
    int live = 0;
    uint32_t lo = 0xffffffffu, hi = 0u;  // smallest / largest live code of this lane
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const uint32_t code = (uint32_t)(k[i] >> 32);
        const bool ok = code != 0xffffffffu;
        live += __popcll(ballot(ok));
        lo = min(lo, code);
        hi = max(hi, ok ? code : 0u);
    }
    // number of live keys with code <= v (v < 0xffffffff)
    auto count_le = [&](uint32_t v) {
        int c = 0;
#pragma unroll
        for (int i = 0; i < NR; ++i) c += __popcll(ballot((uint32_t)(k[i] >> 32) <= v));
        return c;
    };
    uint32_t thr = 0xff800000u;  // ordered +inf: keep every live key
    if (live > kc) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, WAVE));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, WAVE));
        }
        // bracket: count_le(a) = ca < kc <= cb = count_le(b); the answer is
        // in (a, b].  Regula falsi on the count, with the Illinois halving of
        // a stale end's excess, falling back to bisection after 8 probes.
        uint32_t a = lo - 1, b = hi;  // (live codes are >= 1)
        int ca = 0, cb = live;
        float wa = 1.0f, wb = 1.0f;
        int side = 0;
        const float target = (float)kc + 0.5f * (float)allow;
        bool found = false;
        for (int it = 0; it < 48; ++it) {
            if (cb <= kc + allow) {
                thr = b;
                found = true;
                break;
            }
            if (b - a <= 1) break;  // more than `allow` keys share code b
            uint32_t g;
            if (it < 8) {
                const float fa = wa * ((float)ca - target), fb = wb * ((float)cb - target);
                g = a + (uint32_t)((float)(b - a) * (-fa / (fb - fa)));
            } else {
                g = a + (b - a) / 2;
            }
            g = g <= a ? a + 1 : (g >= b ? b - 1 : g);
            const int cg = count_le(g);
            if (cg < kc) {
                a = g;
                ca = cg;
                wb = side == -1 ? 0.5f * wb : 1.0f;
                wa = 1.0f;
                side = -1;
            } else {
                b = g;
                cb = cg;
                wa = side == 1 ? 0.5f * wa : 1.0f;
                wb = 1.0f;
                side = 1;
            }
        }
        if (!found) {
            const Shrunk sh = shrink_slot(slot, cnt, kc, hist, death, view);
            return Roomed{key_dist(sh.kstar), sh.n};
        }
        thr = min(thr, 0xff800000u);
    }
    int base = 0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const bool keep = (uint32_t)(k[i] >> 32) <= thr;
        const uint64_t m = ballot(keep);
        if (keep) slot[base + __popcll(m & lanemask_lt())] = k[i];
        base += __popcll(m);
    }
    // (readers of the slot fence before reading it)
    return Roomed{live > kc ? ord2f(thr) : INFINITY, base};
}
__device__ __noinline__ Roomed make_room(uint64_t* slot, int cnt, int kc, int allow, uint32_t* hist, const int32_t* death,
                                        int32_t view) {
    if (cnt <= MR_KEYS * WAVE) return make_room_nr<MR_KEYS>(slot, cnt, kc, allow, hist, death, view);
    const Shrunk sh = shrink_slot(slot, cnt, kc, hist, death, view);
    return Roomed{key_dist(sh.kstar), sh.n};
}

// Balanced schedule: workgroup p of P covers units [floor(p W / P),
// floor((p + 1) W / P)) of the W = MB T (query block, key tile) units.
// owner(u) is the workgroup covering unit u; stream_segments lists the
// (query block, split, first tile, end tile) segments of workgroup p (at
// most max_seg; returns their number).  Host and device use this same code.
constexpr int STREAM_MAX_SEG = 32;
__host__ __device__ inline int stream_owner(int64_t u, int64_t W, int P) {
    int p = (int)((u * P) / W);
    while (p + 1 < P && ((int64_t)(p + 1) * W) / P <= u) ++p;
    while (p > 0 && ((int64_t)p * W) / P > u) --p;
    return p;
}
__host__ __device__ inline int stream_segments(int p, int MB, int T, int P, int4* out, int max_seg) {
    const int64_t W = (int64_t)MB * T;
    int64_t u = ((int64_t)p * W) / P;
    const int64_t u1 = ((int64_t)(p + 1) * W) / P;
    int n = 0;
    while (u < u1 && n < max_seg) {
        const int qb = (int)(u / T);
        const int tb = (int)(u - (int64_t)qb * T);
        const int te = (int)((u1 - u < (int64_t)(T - tb)) ? tb + (u1 - u) : T);
        out[n++] = make_int4(qb, p - stream_owner((int64_t)qb * T, W, P), tb, te);
        u += te - tb;
    }
    if (u < u1) return -1;
    // Run the segments by first tile (longer first on a tie), not in unit
    // order: every workgroup then starts at key tile 0 and, since all ranges
    // have the same length (to one unit), the workgroups of an XCD walk the
    // key tiles nearly in step, in at most two groups a fixed number of tiles
    // apart, so most key chunks come from memory once per group and from the
    // XCD's L2 for the other workgroups.  The order of a workgroup's segments
    // does not change any slot.
    for (int i = 1; i < n; ++i) {
        const int4 x = out[i];
        int j = i;
        while (j > 0 && (out[j - 1].z > x.z || (out[j - 1].z == x.z && out[j - 1].w - out[j - 1].z < x.w - x.z))) {
            out[j] = out[j - 1];
            --j;
        }
        out[j] = x;
    }
    return n;
}

// One thread per workgroup of the balanced schedule writes its segment list.
__global__ void knn_stream_segments(int MB, int T, int P, int4* __restrict__ segs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int4* o = segs + (size_t)p * (STREAM_MAX_SEG + 1);
    const int n = stream_segments(p, MB, T, P, o, STREAM_MAX_SEG);
    o[n < 0 ? 0 : n] = make_int4(-1, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// knn_tile: grid = MB query blocks x S key splits.  blockIdx.x -> (split,
// query block) with the query block fastest, so the workgroups that share an
// XCD (dispatched round-robin) stream the same key tiles through its L2.
// ---------------------------------------------------------------------------
struct TileArgs {
    const uint4* Xp;
    int64_t row_units;
    int n_chunks;
    int32_t Dp;
    const float* norms;
    const float* scales;
    const float* pmax;
    int64_t M;
    const int32_t* qids;
    int64_t m0;
    const int32_t* nlims;
    int64_t nlim;
    int64_t key_lo;
    const int32_t* kcs;
    int kc;
    const float* tau0;
    int64_t tau0_stride;
    const float* tau_seed;
    const int32_t* death;
    const int32_t* views;
    int32_t view;
    int MB, S, tiles_per_split, tile_lo, tile_hi, cap;
    // balanced schedule (segs != null): one workgroup per resident slot, each
    // taking an equal contiguous range of the MB x (tile_hi - tile_lo)
    // (query block, key tile) units; segs[p] lists workgroup p's segments as
    // (query block, split, first tile, end tile) with split = the index of
    // the workgroup among those covering the query block, -1 after the last
    const int4* segs;
    // the final shrink runs for slots above max(kc, final_keep): a split of a
    // single tile hands all its keys to the select, whose union threshold is
    // one parallel pass per row instead of a serial shrink per query here
    int final_keep;
    // tile lists (restricted search): block b holds rows [blk_q[b], blk_q[b+1])
    // and searches the key tiles tl_idx[blk_t[b] .. blk_t[b+1])
    const int32_t* blk_q;
    const int32_t* blk_t;
    const int32_t* tl_idx;
    uint64_t* slots;
    int32_t* counts;
};

// Instantiations of the tile kernel: the plain search, the search over a
// corpus with deletion stamps (serving), and the search restricted to
// per-block tile lists.  Separate instantiations keep the extra logic out of
// the plain search's registers.
enum TileMode { TILE_PLAIN = 0, TILE_VIS = 1, TILE_LIST = 2 };

// Deletion visibility: key j exists for a request with view v iff it was not
// deleted by one of the first v commits.
__device__ __forceinline__ bool key_visible(const int32_t* death, int64_t j, int32_t view) {
    return !death || death[j] >= view;
}

template <int P, int MODE, bool SMALL>
__global__ __launch_bounds__((TileGeom<P, SMALL>::THREADS)) __attribute__((amdgpu_waves_per_eu(TileGeom<P, SMALL>::WPE, TileGeom<P, SMALL>::WPE))) void knn_tile(TileArgs a) {
    using G = TileGeom<P, SMALL>;
    constexpr int QB = G::QB;
    constexpr int KT = G::KT;
    constexpr int NKB = G::NKB;
    constexpr int TILE_WAVES = G::WAVES;
    constexpr int TT = G::THREADS;
    constexpr int RSTEP = TT / 8;  // rows between one thread's staged units
    // double-buffered tiles, filled by direct global -> LDS loads: one barrier
    // per chunk, the next chunk's loads in flight while this chunk's MFMAs
    // run.  The two buffers are separate arrays so the compiler can tell the
    // one being filled from the one being read (it would otherwise wait for
    // the loads in flight before every fragment read).
    __shared__ uint4 Ks0[KT * CHUNK_UNITS];
    __shared__ uint4 Ks1[KT * CHUNK_UNITS];
    __shared__ uint4 Qs0[QB * CHUNK_UNITS];
    __shared__ uint4 Qs1[QB * CHUNK_UNITS];
    // per-tile norms/scales: three buffers, because a tile's epilogue runs
    // after the barrier that lets faster waves stage the following tiles
    __shared__ float Kn[3][KT];
    __shared__ float Ksc[3][P == ATSNE_PREC_FP8_E4M3 ? KT : 1];
    __shared__ uint32_t hist_all[TILE_WAVES][256];

    const int t = threadIdx.x;
    const int l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: LDS bases go to M0
    constexpr bool VIS = MODE == TILE_VIS;
    constexpr bool LIST = MODE == TILE_LIST;
    // XCD-aware order: workgroup b is dispatched to XCD b % 8.  Task grid:
    // each XCD gets a contiguous run of (query block, split) tasks with the
    // split fastest, so the workgroups resident on one XCD share a few query
    // blocks and the same key tiles through its L2.  Balanced schedule: each
    // XCD gets a contiguous eighth of the units.
    const int xcd = (int)(blockIdx.x % KNN_XCDS), jx = (int)(blockIdx.x / KNN_XCDS);
    const int4* my_segs = a.segs ? a.segs + (size_t)(xcd * ((int)gridDim.x / KNN_XCDS) + jx) * (STREAM_MAX_SEG + 1) : nullptr;
    // corpus tile at sequence position p
    auto tile_id = [&](int p) __attribute__((always_inline)) {
        if constexpr (LIST)
            return a.tl_idx[p];
        else
            return p;
    };
    uint32_t* hist = hist_all[w];
    const int64_t row_units = a.row_units;
    const int n_chunks = a.n_chunks;
    // A workgroup runs one segment (query block, split, tile range), or in the
    // balanced schedule the up to three segments its unit range crosses.
    // A workgroup runs one segment (query block, split, tile range), or in the
    // balanced schedule the segments its unit range crosses, one after the
    // other inside the single chunk loop below.
    int seg = 0;
    int qb = 0, split = 0;
    int64_t qbase = 0, qend = 0;
    int tile_begin = 0, tile_end = 0;
    bool qb_done = false;  // this segment ends its query block (balanced schedule)
    auto load_segment = [&](int sidx) __attribute__((always_inline)) {
        if (my_segs) {
            const int4 sg = my_segs[sidx];
            if (sg.x < 0) return false;
            qb = sg.x;
            split = sg.y;
            qbase = (int64_t)qb * QB;
            qend = a.M;
            tile_begin = a.tile_lo + sg.z;
            tile_end = a.tile_lo + sg.w;
            qb_done = sg.w == a.tile_hi - a.tile_lo;
            return true;
        }
        if (sidx > 0) return false;
        const int n_tasks = a.MB * a.S;
        const int task = xcd * (n_tasks / KNN_XCDS) + min(xcd, n_tasks % KNN_XCDS) + jx;
        qb = task / a.S;
        split = task % a.S;
        // this block's query rows and this split's positions in its tile sequence
        if constexpr (LIST) {
            qbase = a.blk_q[qb];
            qend = a.blk_q[qb + 1];
            const int l0 = a.blk_t[qb], l1 = a.blk_t[qb + 1];
            const int tps = (l1 - l0 + a.S - 1) / a.S;
            tile_begin = min(l1, l0 + split * tps);
            tile_end = min(l1, tile_begin + tps);
        } else {
            qbase = (int64_t)qb * QB;
            qend = a.M;
            tile_begin = a.tile_lo + split * a.tiles_per_split;
            tile_end = min(a.tile_hi, tile_begin + a.tiles_per_split);
        }
        return true;
    };

    // Staging map: load instruction j of wave w fills rows 8 (w + WAVES j) ..
    // + 7 of a tile (1 KiB of LDS), lane l row (t >> 3) + RSTEP j and slot
    // l & 7, which holds global unit ulane (the swizzle of that row; WAVES is
    // even, so the row's bit 3 is w & 1).
    static_assert(TILE_WAVES % 2 == 0 && RSTEP == 8 * TILE_WAVES, "staging map");
    const int ulane = (l & 7) ^ (l >> 3) ^ (w & 1);
    // Per-segment query state.  Corpus rows of the 4 query-tile rows this
    // lane loads (kept as 32-bit row numbers; the 64-bit unit offsets are
    // formed per chunk); lanes l and l+32 share query 32w + l%32.
    const int qloc = 32 * w + (l & 31);
    const int32_t* death = VIS ? a.death : nullptr;
    uint32_t qr0 = 0, qr1 = 0, qr2 = 0, qr3 = 0;
    int64_t mq = 0;
    bool qvalid = false;
    // corpus rows and keys are int32 (row counts are checked on the host)
    int32_t self = -1, nl = 0;
    int kcq = 0, sq_e8 = 127, nl_min = 0, count = 0;
    float tau = -INFINITY;
    auto init_query = [&]() __attribute__((always_inline)) {
        auto qrow_of = [&](int i) {
            const int64_t m = qbase + (t >> 3) + RSTEP * i;
            return (uint32_t)(m < qend ? load_qid(a.qids, a.m0, m) : 0);
        };
        qr0 = qrow_of(0);
        qr1 = qrow_of(1);
        qr2 = qrow_of(2);
        qr3 = qrow_of(3);
        mq = qbase + qloc;
        qvalid = mq < qend;
        self = qvalid ? (int32_t)load_qid(a.qids, a.m0, mq) : -1;
        nl = qvalid ? (int32_t)(a.nlims ? (int64_t)a.nlims[mq] : a.nlim) : 0;
        kcq = qvalid ? (a.kcs ? a.kcs[mq] : a.kc) : 0;
        sq_e8 = (P == ATSNE_PREC_FP8_E4M3 && qvalid) ? e8m0_of(a.scales[self]) : 127;
        tau = -INFINITY;
        if (qvalid && key_visible(death, self, a.views ? a.views[mq] : a.view)) {
            // keys with d' <= the seed pass; nextafter keeps the seed's own
            // value, as the filter below is strict
            tau = a.tau_seed ? nextafterf(a.tau_seed[self], INFINITY) : INFINITY;
            if (a.tau0) {
                // reverse mode: only keys that may beat the row's farthest
                // neighbour; d' = d - n_q, widened by the contraction bound
                const float nq = a.norms[self];
                const float nmax = nl > 0 ? a.pmax[nl - 1] : 0.0f;
                const float dmax = a.tau0[mq * a.tau0_stride];
                const float E = P == ATSNE_PREC_FP32X3 ? x3_contraction_bound(a.Dp, nq, nmax, dmax)
                                                       : fp32_contraction_bound(a.Dp, nq, nmax, dmax);
                tau = dmax > -INFINITY ? dmax - nq + E * 2.0f + 1e-30f
                                       : -INFINITY;  // a row with no neighbour left takes none
            }
        }
        // smallest key bound of the wave's queries: tiles below it need no range checks
        nl_min = qvalid ? nl : 0x7fffffff;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) nl_min = min(nl_min, __shfl_xor(nl_min, o, WAVE));
        count = 0;
    };

    // Direct global -> LDS staging of one chunk into buffer PB: KT / RSTEP key
    // rows and 4 query rows per lane, and at a tile's first chunk the tile's
    // norms (and FP8 scales), one dword per lane of the first KT / 64 waves.
    const uint32_t krow_ = (uint32_t)((t >> 3) * row_units) + ulane;  // < KT row_units
    const int64_t kstep_ = RSTEP * row_units;
    auto issue = [&](auto par_tag, int pos, int c) __attribute__((always_inline)) {
        constexpr bool PB = decltype(par_tag)::value;
        uint4* ks = PB ? Ks1 : Ks0;
        uint4* qs = PB ? Qs1 : Qs0;
        const int64_t tile_row = (int64_t)tile_id(pos) * KT;
        const int64_t co = (int64_t)c * CHUNK_UNITS;
        const uint4* kb = a.Xp + tile_row * row_units + co + krow_;
        // every address before the first load goes out
        const uint4* qb = a.Xp + co + ulane;
        const uint4* qa0 = qb + (uint64_t)qr0 * (uint64_t)row_units;
        const uint4* qa1 = qb + (uint64_t)qr1 * (uint64_t)row_units;
        const uint4* qa2 = qb + (uint64_t)qr2 * (uint64_t)row_units;
        const uint4* qa3 = qb + (uint64_t)qr3 * (uint64_t)row_units;
        // single-chunk rows: the query chunk is the same for every tile of a
        // segment, so only its first two tiles (one per buffer) load it
        if (n_chunks > 1 || pos < tile_begin + 2) {
            lds_dma16(qa0, qs + 64 * w);
            lds_dma16(qa1, qs + 64 * (w + TILE_WAVES));
            lds_dma16(qa2, qs + 64 * (w + 2 * TILE_WAVES));
            lds_dma16(qa3, qs + 64 * (w + 3 * TILE_WAVES));
        }
#pragma unroll
        for (int j = 0; j < KT / RSTEP; ++j) lds_dma16(kb + j * kstep_, ks + 64 * (w + TILE_WAVES * j));
        if (c == 0 && w < KT / 64) {
            lds_dma4(a.norms + tile_row + 64 * w + l, &Kn[pos % 3][64 * w]);
            if constexpr (P == ATSNE_PREC_FP8_E4M3) lds_dma4(a.scales + tile_row + 64 * w + l, &Ksc[pos % 3][64 * w]);
        }
    };
    // fragment slot of this lane's rows (32 b + l % 32 and 32 w + l % 32)
    const int sw = lds_swz(l & 31);

    f32x16 acc[NKB];
    int ksc_e8[NKB];
    // One chunk of the contraction from LDS buffer PB: key blocks in pairs,
    // the next pair's fragments read while the current pair's MFMAs run.
    auto compute = [&](auto par_tag) __attribute__((always_inline)) {
        constexpr bool PB = decltype(par_tag)::value;
        constexpr bool FIRST = false;  // accumulators are cleared at each tile's start
        const uint4* K = PB ? Ks1 : Ks0;
        const uint4* Q = PB ? Qs1 : Qs0;
        uint4 bq[4], ca0[4], ca1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bq[i] = Q[qloc * CHUNK_UNITS + (chunk_unit<P>(l, i) ^ sw)];
        if constexpr (P == ATSNE_PREC_FP32X3) {
#pragma unroll
            for (int b = 0; b < NKB; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ca0[i] = K[(32 * b + (l & 31)) * CHUNK_UNITS + (chunk_unit<P>(l, i) ^ sw)];
                mfma_x3_block<FIRST>(acc[b], ca0, bq);
            }
        } else if constexpr (P == ATSNE_PREC_FP8_E4M3) {
#pragma unroll
            for (int b = 0; b < NKB; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ca0[i] = K[(32 * b + (l & 31)) * CHUNK_UNITS + (chunk_unit<P>(l, i) ^ sw)];
                mfma_fp8_block<FIRST>(acc[b], ca0, bq, ksc_e8[b], sq_e8);
                // keep the next block's operand reads from being hoisted over
                // these MFMAs (register budget at two waves per SIMD)
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int pr = 0; pr < NKB / 2; ++pr) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ca0[i] = K[(64 * pr + (l & 31)) * CHUNK_UNITS + (chunk_unit<P>(l, i) ^ sw)];
                    ca1[i] = K[(64 * pr + 32 + (l & 31)) * CHUNK_UNITS + (chunk_unit<P>(l, i) ^ sw)];
                }
                mfma_pair<P, FIRST>(acc[2 * pr], acc[2 * pr + 1], ca0, ca1, bq, 127, 127, 127);
            }
        }
    };

    auto epilogue = [&](int pos) __attribute__((always_inline)) {
        const int key0 = tile_id(pos) * KT;
        // tiles inside every query's key range, and not holding the query
        // itself, skip the per-key checks
        const bool edge = key0 < a.key_lo || key0 + KT > nl_min;
        const bool has_self = ballot(self >= key0 && self < key0 + KT) != 0;
        const float* kn = Kn[pos % 3];
        // A lane holds 16 values of each key block for its query; lane l and
        // l + 32 share query l % 32 and append their passing keys to its slot
        // side by side (lane l first), so no wave-wide compaction is needed.
#pragma unroll
        for (int b = 0; b < NKB; ++b) {
            float dv[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 nj = *reinterpret_cast<const float4*>(&kn[32 * b + 8 * g + 4 * (l >> 5)]);
                dv[4 * g + 0] = fmaf(-2.0f, acc[b][4 * g + 0], nj.x);
                dv[4 * g + 1] = fmaf(-2.0f, acc[b][4 * g + 1], nj.y);
                dv[4 * g + 2] = fmaf(-2.0f, acc[b][4 * g + 2], nj.z);
                dv[4 * g + 3] = fmaf(-2.0f, acc[b][4 * g + 3], nj.w);
            }
            // block-level test first: almost always nothing passes once the
            // threshold has settled
            float dmin = dv[0];
#pragma unroll
            for (int v = 1; v < 16; ++v) dmin = fminf(dmin, dv[v]);
            if (!ballot(dmin < tau)) continue;
            const int kb = key0 + 32 * b + 4 * (l >> 5);  // key of value v: kb + 8 (v / 4) + v % 4
            uint32_t mask = 0;
#pragma unroll
            for (int v = 0; v < 16; ++v) mask |= (dv[v] < tau ? 1u : 0u) << v;
            if (edge || has_self) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int key = kb + 8 * (v >> 2) + (v & 3);
                    if (key < a.key_lo || key >= nl || key == self) mask &= ~(1u << v);
                }
            }
            const int n_me = __popc(mask);
            const int n_other = __shfl_xor(n_me, 32, WAVE);
            if (n_me) {
                // the slot pointer is formed here, not held across the chunk loop
                uint64_t* dst = a.slots + ((size_t)mq * a.S + split) * (size_t)a.cap + count + ((l >> 5) ? n_other : 0);
                if (MODE == TILE_PLAIN && mask == 0xffffu && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                    // every value passes (a slot's first tiles): two keys per
                    // 16-byte store, half the store instructions (plain mode
                    // only: with stamps or tile lists it doubles the spills)
#pragma unroll
                    for (int v = 0; v < 16; v += 2)
                        *reinterpret_cast<ulonglong2*>(dst + v) =
                            make_ulonglong2(pack_key(dv[v], kb + 8 * (v >> 2) + (v & 3)),
                                            pack_key(dv[v + 1], kb + 8 * ((v + 1) >> 2) + ((v + 1) & 3)));
                } else {
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        if (mask & (1u << v)) *dst++ = pack_key(dv[v], kb + 8 * (v >> 2) + (v & 3));
                    }
                }
            }
            count += n_me + n_other;
        }
        // make room for the next tile (the accumulators are dead here, so the
        // shrink has the registers to itself)
        uint64_t need = ballot(count > a.cap - KT) & 0xffffffffull;
        while (need) {
            const int q = __ffsll((unsigned long long)need) - 1;
            need &= need - 1;
            const int cnt_q = __shfl(count, q, WAVE);
            const int kc_q = __shfl(kcq, q, WAVE);
            uint64_t* sq = a.slots + ((size_t)(qbase + 32 * w + q) * a.S + split) * (size_t)a.cap;
            const int32_t v_q = a.views ? a.views[qbase + 32 * w + q] : a.view;
            // the kept count may exceed k' by an eighth of the slack: a
            // tighter threshold than a quarter (fewer appends: BF16 tile
            // -3%, FP32 and FP32X3 unchanged) for a few more probes
            const Roomed r = make_room(sq, cnt_q, kc_q, (a.cap - KT - kc_q) / 8, hist, death, v_q);
            if ((l & 31) == q) {
                count = r.n;
                tau = fminf(tau, r.tau);
            }
        }
    };

    // Final shrink so each slot hands at most max(kc, final_keep) candidates
    // to the next stage; then the slot's count (and, in the balanced
    // schedule, the query block's last workgroup clears the splits nobody
    // covers).
    auto finish_segment = [&]() __attribute__((always_inline)) {
        uint64_t need = ballot(count > max(kcq, a.final_keep)) & 0xffffffffull;
        while (need) {
            int q = __ffsll((unsigned long long)need) - 1;
            need &= need - 1;
            int cnt_q = __shfl(count, q, WAVE);
            int kc_q = __shfl(kcq, q, WAVE);
            uint64_t* sq = a.slots + ((size_t)(qbase + 32 * w + q) * a.S + split) * (size_t)a.cap;
            const int32_t v_q = a.views ? a.views[qbase + 32 * w + q] : a.view;
            const Shrunk sh = shrink_slot(sq, cnt_q, kc_q, hist, death, v_q);
            if ((l & 31) == q) count = sh.n;
        }
        if (qvalid && l < 32) {
            a.counts[mq * a.S + split] = count;
            if (qb_done)
                for (int s2 = split + 1; s2 < a.S; ++s2) a.counts[mq * a.S + s2] = 0;
        }
    };
    // per-tile setup: clear the accumulators, fetch the FP8 key scales
    auto tile_start = [&](int tile) __attribute__((always_inline)) {
        if constexpr (P == ATSNE_PREC_FP8_E4M3) {
#pragma unroll
            for (int b = 0; b < NKB; ++b) ksc_e8[b] = e8m0_of(Ksc[tile % 3][32 * b + (l & 31)]);
        } else {
#pragma unroll
            for (int b = 0; b < NKB; ++b) ksc_e8[b] = 127;
        }
#pragma unroll
        for (int b = 0; b < NKB; ++b) acc[b] = f32x16{};
    };
    // Open segments until one has tiles (the first chunk of its first tile
    // goes to buffer PB); false when the workgroup has no segment left.
    int tile = 0, c = 0;
    auto open_segment = [&](auto par_tag) __attribute__((always_inline)) {
        while (load_segment(seg)) {
            init_query();
            if (tile_begin < tile_end) {
                // earlier epilogues may still read the tile norms the first
                // loads overwrite
                if (seg > 0) __syncthreads();
                issue(par_tag, tile_begin, 0);
                __syncthreads();
                tile = tile_begin;
                c = 0;
                tile_start(tile);
                return true;
            }
            finish_segment();  // no tiles: count 0
            ++seg;
        }
        return false;
    };
    // One chunk from buffer PB: start the loads of the segment's next chunk
    // into the other buffer (read by every wave before the previous
    // barrier), run this chunk's MFMAs, then one barrier, which also waits
    // for those loads.
    auto step = [&](auto par_tag) __attribute__((always_inline)) {
        constexpr bool PB = decltype(par_tag)::value;
        const bool last = c + 1 == n_chunks;
        if (!last || tile + 1 < tile_end)
            issue(std::integral_constant<bool, !PB>{}, last ? tile + 1 : tile, last ? 0 : c + 1);
        compute(par_tag);
        __syncthreads();
    };
    // After a step whose successor reads buffer NB: the tile's epilogue at its
    // last chunk, the segment's end at its last tile.  Returns false when the
    // workgroup is done.
    auto advance = [&](auto nb_tag) __attribute__((always_inline)) {
        if (++c < n_chunks) return true;
        epilogue(tile);
        c = 0;
        if (++tile < tile_end) {
            tile_start(tile);
            return true;
        }
        finish_segment();
        ++seg;
        return open_segment(nb_tag);
    };
    // The chunk sequence runs across tiles (and segments) with the buffers
    // alternating, two chunks per iteration so each step's buffer is fixed at
    // compile time (a runtime choice between two instantiations makes the
    // register allocator copy the accumulators).
    if (open_segment(std::false_type{})) {
        for (;;) {
            step(std::false_type{});
            if (!advance(std::true_type{})) break;
            step(std::true_type{});
            if (!advance(std::false_type{})) break;
        }
    }
}

// ---------------------------------------------------------------------------
// Row finalisation shared by knn_select and knn_scan: sort the n candidates
// held in LDS (index cj, FP32 distance cd) by (d, j), FP64 re-rank when the
// k-th/(k+1)-th gap is below FP32 resolution, write the row.
// ---------------------------------------------------------------------------
constexpr float TIE_REL = 8e-6f;  // > worst-case relative error of the FP32 direct difference used here

// Sort the n candidates (cj, cd) by the key (d, j) into sorted[0, n) by
// counting ranks (keys are distinct); cdl (may be null) is the distances'
// residuals, moved along into sorted_lo.  Each lane ranks up to four
// candidates in one pass over the keys, eight keys per step, so the LDS
// latency is paid once per eight keys.  `tmp` is scratch for n keys.
__device__ void rank_sort(int n, const int32_t* cj, const float* cd, const float* cdl, uint64_t* tmp, uint64_t* sorted,
                          float* sorted_lo) {
    const int l = lane_id();
    for (int c = l; c < n; c += WAVE) tmp[c] = pack_key(cd[c], cj[c]);
    wave_sync();
    for (int c0 = 0; c0 < n; c0 += 4 * WAVE) {
        uint64_t kc[4];
        int r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + l + WAVE * u;
            kc[u] = c < n ? tmp[c] : ~0ull;
            r[u] = 0;
        }
        int o = 0;
        for (; o + 8 <= n; o += 8) {
            uint64_t ko[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) ko[e] = tmp[o + e];
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int u = 0; u < 4; ++u) r[u] += ko[e] < kc[u] ? 1 : 0;
        }
        for (; o < n; ++o) {
            const uint64_t ko = tmp[o];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] += ko < kc[u] ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + l + WAVE * u < n) {
                sorted[r[u]] = kc[u];
                if (cdl) sorted_lo[r[u]] = cdl[c0 + l + WAVE * u];
            }
    }
    wave_sync();
}

// Write the row from candidates already sorted by rank_sort: FP64 re-rank
// when the k-th/(k+1)-th gap is below FP32 resolution.  out_d2_lo (may be
// null) receives each distance's residual: sorted_lo's, or the FP64
// distance's remainder after rounding to FP32 on the re-ranked rows.
__device__ void finalize_sorted(const float* __restrict__ X, int64_t ld, int32_t D, const float* __restrict__ xq_g,
                                int n, int k, const uint64_t* sorted, const float* sorted_lo, double* dd,
                                int32_t* __restrict__ out_idx, float* __restrict__ out_d2,
                                float* __restrict__ out_d2_lo, uint8_t* flag_out, uint8_t extra_flags) {
    const int l = lane_id();
    uint8_t fl = extra_flags;
    bool tie = false;
    if (n > k) {
        float dk = key_dist(sorted[k - 1]), dk1 = key_dist(sorted[k]);
        tie = (dk1 - dk) <= TIE_REL * fabsf(dk);
    }
    if (tie) {
        // FP64 direct differences for every candidate, then rank by (d64, j).
        // Eight candidates at a time keep eight row loads in flight; each
        // candidate's sum is the same arithmetic whatever the group size.
        int c = 0;
        for (; c + 8 <= n; c += 8) {
            const float* xr[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xr[e] = X + (int64_t)key_index(sorted[c + e]) * ld;
            double acc[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] = 0.0;
            for (int d = l; d < D; d += WAVE) {
                const double q = (double)xq_g[d];
                float xv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) xv[e] = xr[e][d];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double t = q - (double)xv[e];
                    acc[e] = fma(t, t, acc[e]);
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] = wave_sum(acc[e]);
            if (l == 0) {
#pragma unroll
                for (int e = 0; e < 8; ++e) dd[c + e] = acc[e];
            }
        }
        for (; c < n; ++c) {
            const float* xc = X + (int64_t)key_index(sorted[c]) * ld;
            double acc = 0.0;
            for (int d = l; d < D; d += WAVE) {
                double t = (double)xq_g[d] - (double)xc[d];
                acc = fma(t, t, acc);
            }
            acc = wave_sum(acc);
            if (l == 0) dd[c] = acc;
        }
        wave_sync();
        // rank by (d64, j), four candidates per lane per pass over the keys
        for (int c0 = 0; c0 < n; c0 += 4 * WAVE) {
            double dc[4];
            int32_t jc[4];
            int r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int cc = c0 + l + WAVE * u;
                dc[u] = cc < n ? dd[cc] : 0.0;
                jc[u] = cc < n ? key_index(sorted[cc]) : 0;
                r[u] = 0;
            }
            int o = 0;
            for (; o + 4 <= n; o += 4) {
                double dox[4];
                int32_t jo[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    dox[e] = dd[o + e];
                    jo[e] = key_index(sorted[o + e]);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int u = 0; u < 4; ++u) r[u] += (dox[e] < dc[u]) || (dox[e] == dc[u] && jo[e] < jc[u]);
            }
            for (; o < n; ++o) {
                const double dox = dd[o];
                const int32_t jo = key_index(sorted[o]);
#pragma unroll
                for (int u = 0; u < 4; ++u) r[u] += (dox < dc[u]) || (dox == dc[u] && jo < jc[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (c0 + l + WAVE * u < n && r[u] < k) {
                    const float h = (float)dc[u];
                    out_idx[r[u]] = jc[u];
                    out_d2[r[u]] = h;
                    if (out_d2_lo) out_d2_lo[r[u]] = (float)(dc[u] - (double)h);
                }
            }
        }
        fl |= ATSNE_FLAG_FP64_RERANKED;
    } else {
        for (int r = l; r < k; r += WAVE) {
            out_idx[r] = key_index(sorted[r]);
            out_d2[r] = key_dist(sorted[r]);
            if (out_d2_lo) out_d2_lo[r] = sorted_lo ? sorted_lo[r] : 0.f;
        }
    }
    if (flag_out && l == 0) *flag_out = fl;
}

// Sort the candidates (rank_sort, with dd as its scratch) and write the row.
__device__ void finalize_row(const float* __restrict__ X, int64_t ld, int32_t D, const float* __restrict__ xq_g,
                             int n, int k, int32_t* cj, float* cd, float* cdl, uint64_t* sorted, float* sorted_lo,
                             double* dd, int32_t* __restrict__ out_idx, float* __restrict__ out_d2,
                             float* __restrict__ out_d2_lo, uint8_t* flag_out, uint8_t extra_flags) {
    rank_sort(n, cj, cd, cdl, reinterpret_cast<uint64_t*>(dd), sorted, sorted_lo);
    finalize_sorted(X, ld, D, xq_g, n, k, sorted, sorted_lo, dd, out_idx, out_d2, out_d2_lo, flag_out, extra_flags);
}

// FP32 direct-difference squared distances |x_q - x_j|^2 for G rows at
// once, each as an unevaluated sum hi + lo: hi is the distance rounded to
// FP32 and lo its residual.  Every kernel that reports a distance uses this
// one summation order: lane l accumulates the elements d = l, l + 64, ... in
// increasing order with one fma each (direct_partials), and the 64 lane
// partials are then added pairwise over the lane-index bits 5, 4, ..., 0 by
// TwoSums whose rounding errors are collected apart; hi, lo = Fast2Sum(sum,
// errors).  The six levels of additions of ever larger partials are where a
// plain FP32 sum loses most of its accuracy; with them compensated, hi + lo
// is within a few hundredths of an ulp of the distance on the image-like
// workload, so distance differences are resolved below FP32 resolution,
// which the perplexity calibration needs when a row's distances are close
// together relative to their size.  The G rows' loads are in flight together.
template <int G>
__device__ __forceinline__ void direct_partials(const float* __restrict__ xq, const float* const (&xr)[G], int32_t D,
                                                float (&s)[G]) {
    const int l = lane_id();
#pragma unroll
    for (int e = 0; e < G; ++e) s[e] = 0.f;
    for (int d = l; d < D; d += WAVE) {
        const float q = xq[d];
        float xv[G];
#pragma unroll
        for (int e = 0; e < G; ++e) xv[e] = xr[e][d];
#pragma unroll
        for (int e = 0; e < G; ++e) {
            const float t = q - xv[e];
            s[e] = fmaf(t, t, s[e]);
        }
    }
}

// One pairwise level of the compensated reduction: (s, c) of this lane and
// of lane l ^ o.
__device__ __forceinline__ void comp_level(float& s, float& c, float s2, float c2) {
    float se;
    s = two_sum(s, s2, se);
    c = (c + c2) + se;
}

// Every lane receives the G pairs (hi, lo).
template <int G>
__device__ __forceinline__ void direct_group(const float* __restrict__ xq, const float* const (&xr)[G], int32_t D,
                                             float (&hi)[G], float (&lo)[G]) {
    float s[G], c[G];
    direct_partials<G>(xq, xr, D, s);
#pragma unroll
    for (int e = 0; e < G; ++e) c[e] = 0.f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int e = 0; e < G; ++e) comp_level(s[e], c[e], __shfl_xor(s[e], o, WAVE), __shfl_xor(c[e], o, WAVE));
    }
#pragma unroll
    for (int e = 0; e < G; ++e) {
        hi[e] = s[e] + c[e];
        lo[e] = c[e] - (hi[e] - s[e]);
    }
}

// The same sums for 16 rows, reduce-scattered: at the levels over lane bits
// 5..2 a lane keeps half of its remaining rows and sends the other half to
// its partner, so each level adds exactly the pairs the full reduction adds
// (identical results) at a quarter of its exchanges.  Lane l ends with row
// e(l) = 8 b5 + 4 b4 + 2 b3 + b2 (b_i = bit i of l); returns e(l).
__device__ __forceinline__ int direct_group16_scatter(const float* __restrict__ xq, const float* const (&xr)[16],
                                                      int32_t D, float& hi, float& lo) {
    const int l = lane_id();
    float s[16], c[16];
    direct_partials<16>(xq, xr, D, s);
#pragma unroll
    for (int e = 0; e < 16; ++e) c[e] = 0.f;
#pragma unroll
    for (int h = 8, o = 32; h >= 1; h >>= 1, o >>= 1) {
        const bool upper = (l & o) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const float ks = upper ? s[i + h] : s[i], kc = upper ? c[i + h] : c[i];
            const float ts = upper ? s[i] : s[i + h], tc = upper ? c[i] : c[i + h];
            s[i] = ks;
            c[i] = kc;
            comp_level(s[i], c[i], __shfl_xor(ts, o, WAVE), __shfl_xor(tc, o, WAVE));
        }
    }
#pragma unroll
    for (int o = 2; o >= 1; o >>= 1) comp_level(s[0], c[0], __shfl_xor(s[0], o, WAVE), __shfl_xor(c[0], o, WAVE));
    hi = s[0] + c[0];
    lo = c[0] - (hi - s[0]);
    return 8 * ((l >> 5) & 1) + 4 * ((l >> 4) & 1) + 2 * ((l >> 3) & 1) + ((l >> 2) & 1);
}

// Direct-difference distances from query xq to the n candidates in cj, into
// cd (hi) and cdl (lo, may be null), sixteen candidates at a time (a short
// last group repeats its last candidate and drops the copies).
__device__ void direct_distances(const float* __restrict__ X, int64_t ld, int32_t D, const float* __restrict__ xq,
                                 int n, const int32_t* cj, float* cd, float* cdl) {
    const int l = lane_id();
    for (int c = 0; c < n; c += 16) {
        const float* xr[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) xr[e] = X + (int64_t)cj[min(c + e, n - 1)] * ld;
        float hi, lo;
        const int e = direct_group16_scatter(xq, xr, D, hi, lo);
        if ((l & 3) == 0 && c + e < n) {
            cd[c + e] = hi;
            if (cdl) cdl[c + e] = lo;
        }
    }
    wave_sync();
}

constexpr int MAX_KC = 1024;

struct SelArgs {
    const float* X;
    int64_t ld;
    int32_t D, Dp;
    const float* norms;
    const float* pmax;
    int64_t M;
    const int32_t* qids;
    int64_t m0;
    const int32_t* nlims;
    int64_t nlim;
    int64_t key_lo;
    const int32_t* ks;
    int k;
    const int32_t* kcs;
    int kc;
    int S, cap;
    const int32_t* death;
    const int32_t* views;
    int32_t view;
    const int32_t* row_blk;  // tile lists: block of each row (NULL: whole key range)
    const int32_t* blk_t;
    const int32_t* tl_idx;
    const uint64_t* slots;
    const int32_t* counts;
    int32_t* out_idx;
    float* out_d2;
    float* out_d2_lo;  // may be null
    uint8_t* out_flags;
    int64_t out_stride;
    int32_t* scan_list;
    int32_t* scan_count;
    float* tau_out;  // threshold mode (seeding pass): see Batch
    const int32_t* tau_map;
    const int32_t* sel_order;  // see Batch
};

// Gathers the union of a row's candidate slots; returns the threshold key
// (rank `take`) so that exactly the keys <= it are the candidates.
template <class Each>
__device__ uint64_t union_threshold(Each each, int take, int total, uint32_t* hist) {
    const int l = lane_id();
    if (take < total) return wave_select(each, (uint32_t)take, hist);
    uint64_t mx = 0;
    each([&](uint64_t key) { mx = key > mx ? key : mx; });
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t other = shfl64(mx, l ^ o);
        mx = other > mx ? other : mx;
    }
    return mx;
}

// knn_select: one wave (workgroup of 64) per query row.
constexpr int SEL_RK = 32;     // union keys per lane held in registers (2048 per row)
constexpr int SEL_MAX_S = 64;  // splits whose prefix counts fit the LDS table

// LDS of knn_select for up to kcap candidates (sized at launch).
__host__ __device__ constexpr size_t select_lds_bytes(int kcap) {
    return (256 * 4 + (size_t)kcap * (8 + 8 + 4 + 4 + 4 + 4) + 16 + 15) & ~(size_t)15;
}
constexpr int SEL_ROWS = 4;  // at most this many rows (one wave each) per workgroup
// rows per workgroup for a candidate capacity: keep the dynamic LDS within 64 KiB
static inline int sel_rows(int kcap) {
    return (int)std::max<size_t>(1, std::min<size_t>(SEL_ROWS, 65536 / select_lds_bytes(kcap)));
}

template <int P>
__global__ __launch_bounds__(64 * SEL_ROWS) void knn_select(SelArgs a, int kcap) {
    extern __shared__ __align__(16) unsigned char sel_lds_all[];
    const int w = threadIdx.x >> 6;
    unsigned char* sel_lds = sel_lds_all + (size_t)w * select_lds_bytes(kcap);
    double* dd = reinterpret_cast<double*>(sel_lds);
    uint64_t* sorted = reinterpret_cast<uint64_t*>(dd + kcap);
    uint32_t* hist = reinterpret_cast<uint32_t*>(sorted + kcap);
    int32_t* cj = reinterpret_cast<int32_t*>(hist + 256);
    float* cd = reinterpret_cast<float*>(cj + kcap);
    float* cdl = cd + kcap;
    float* sorted_lo = cdl + kcap;
    int32_t& ncand = *reinterpret_cast<int32_t*>(sorted_lo + kcap);
    const int l = lane_id();
    const int64_t m_lin = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    if (m_lin >= a.M) return;  // waves are independent: no workgroup barrier below
    const int64_t m = a.sel_order ? (int64_t)a.sel_order[m_lin] : m_lin;
    const int64_t q = load_qid(a.qids, a.m0, m);
    const int64_t nl = a.nlims ? (int64_t)a.nlims[m] : a.nlim;
    const int k = a.ks ? a.ks[m] : a.k;
    const int kc = a.kcs ? a.kcs[m] : a.kc;
    const int32_t* cnt = a.counts + m * a.S;
    const uint64_t* base = a.slots + (size_t)m * a.S * (size_t)a.cap;
    int32_t* out_idx = a.out_idx + m * a.out_stride;
    float* out_d2 = a.out_d2 + m * a.out_stride;
    float* out_d2_lo = a.out_d2_lo ? a.out_d2_lo + m * a.out_stride : nullptr;

    // with deletion stamps, slots can still hold keys of rows deleted before
    // the row's view (those appended after the slot's last shrink): skip them
    const int32_t vq = a.views ? a.views[m] : a.view;
    int total = 0;
    if (!a.death) {
        for (int s = 0; s < a.S; ++s) total += cnt[s];
    } else {
        for (int s = 0; s < a.S; ++s) {
            const uint64_t* sl = base + (size_t)s * a.cap;
            for (int i0 = 0; i0 < cnt[s]; i0 += WAVE)
                total += __popcll(ballot(i0 + l < cnt[s] && a.death[key_index(sl[i0 + l])] >= vq));
        }
    }
    const int take = min(kc, total);
    // threshold of the union, then its candidates into cj
    auto select_union = [&](auto each) {
        const uint64_t ks = union_threshold(each, take, total, hist);
        if (l == 0) ncand = 0;
        wave_sync();
        each([&](uint64_t key) {
            if (key <= ks) {
                int p = atomicAdd(&ncand, 1);
                cj[p] = key_index(key);
                cd[p] = key_dist(key);
            }
        });
        wave_sync();
        return ks;
    };
    if (a.tau_out) {
        // threshold mode: the kc-th smallest key of the row's union
        const uint64_t ks = union_threshold(
            [&](auto f) {
                for (int s = 0; s < a.S; ++s) {
                    const uint64_t* sl = base + (size_t)s * a.cap;
                    for (int i = l; i < cnt[s]; i += WAVE) f(sl[i]);
                }
            },
            min(kc, total), total, hist);
        if (l == 0) a.tau_out[a.tau_map ? (int64_t)a.tau_map[q] : q] = total >= kc ? key_dist(ks) : INFINITY;
        return;
    }
    uint64_t kstar;
    if (!a.death && total <= SEL_RK * WAVE) {
        // small unions are read once into registers, every load in flight
        // together, so the radix passes run without memory latency
        __shared__ int32_t spre_all[SEL_ROWS][SEL_MAX_S + 1];
        int32_t* spre = spre_all[w];
        if (a.S <= SEL_MAX_S) {
            int c = l < a.S ? cnt[l] : 0;
            const int incl = (int)wave_incl_scan((uint32_t)c);
            if (l < a.S) spre[l + 1] = incl;
            if (l == 0) spre[0] = 0;
            wave_sync();
        }
        uint64_t rk[SEL_RK];
        int sp = 0;
#pragma unroll
        for (int u = 0; u < SEL_RK; ++u) {
            const int pos = l + WAVE * u;
            rk[u] = ~0ull;
            if (pos < total) {
                if (a.S <= SEL_MAX_S) {
                    while (pos >= spre[sp + 1]) ++sp;
                    rk[u] = base[(size_t)sp * a.cap + (pos - spre[sp])];
                } else {
                    int s = 0, b0 = 0;
                    while (pos >= b0 + cnt[s]) b0 += cnt[s++];
                    rk[u] = base[(size_t)s * a.cap + (pos - b0)];
                }
            }
        }
        kstar = select_union([&](auto f) {
#pragma unroll
            for (int u = 0; u < SEL_RK; ++u)
                if (l + WAVE * u < total) f(rk[u]);
        });
    } else {
        kstar = select_union([&](auto f) {
            for (int s = 0; s < a.S; ++s) {
                const uint64_t* sl = base + (size_t)s * a.cap;
                const int c = cnt[s];
                for (int i = l; i < c; i += WAVE) {
                    const uint64_t key = sl[i];
                    if (!a.death || a.death[key_index(key)] >= vq) f(key);
                }
            }
        });
    }
    const int n = ncand;
    const float* xq = a.X + q * a.ld;
    const float nq = a.norms ? a.norms[q] : 0.0f;
    const float nmax = (a.pmax && nl > 0) ? a.pmax[nl - 1] : 0.0f;
    // ne: the candidates whose exact distance is computed.  On the exact
    // contractions the key code d' bounds each distance within the
    // contraction error E(d') (monotone in d'), so only candidates whose
    // lower bound d' + n_q - E(d') can reach the (k+1)-th exact distance
    // need it: the k+1 smallest d' are computed first, their largest exact
    // distance (times 1 + 4 TIE_REL, which covers the direct-difference
    // error of both orderings) caps the (k+1)-th, and every candidate whose
    // lower bound exceeds the cap is strictly beyond the (k+1)-th under the
    // FP32 and the FP64 ordering alike.  The k + 1 best, the tie test, the
    // FP64 re-rank and the certificate are therefore those of all n.
    int ne = n;
    if ((P == ATSNE_PREC_FP32 || P == ATSNE_PREC_FP32X3) && a.norms && a.pmax && n > k + 1) {
        rank_sort(n, cj, cd, nullptr, reinterpret_cast<uint64_t*>(dd), sorted, nullptr);  // by (d', j)
        for (int c = l; c < n; c += WAVE) cj[c] = key_index(sorted[c]);
        wave_sync();
        direct_distances(a.X, a.ld, a.D, xq, k + 1, cj, cd, cdl);
        float mx = 0.0f;
        for (int c = l; c < k + 1; c += WAVE) mx = fmaxf(mx, cd[c]);
        const float cap = wave_max(mx) * (1.0f + 4.0f * TIE_REL);
        int last = k;
        for (int c0 = k + 1; c0 < n; c0 += WAVE) {
            const int c = c0 + l;
            bool in = false;
            if (c < n) {
                const float dp = key_dist(sorted[c]);
                const float E = P == ATSNE_PREC_FP32X3 ? x3_contraction_bound(a.Dp, nq, nmax, dp)
                                                       : fp32_contraction_bound(a.Dp, nq, nmax, dp);
                in = !(dp + nq - E > cap);
            }
            const uint64_t bm = ballot(in);
            if (bm) last = c0 + 63 - __clzll(bm);
        }
        ne = last + 1;
        direct_distances(a.X, a.ld, a.D, xq, ne - (k + 1), cj + k + 1, cd + k + 1, cdl + k + 1);
    } else {
        direct_distances(a.X, a.ld, a.D, xq, n, cj, cd, cdl);
    }
    if (n < k) {  // fewer keys than requested neighbours (caller error): pad
        for (int r = l; r < k; r += WAVE) {
            out_idx[r] = -1;
            out_d2[r] = INFINITY;
            if (out_d2_lo) out_d2_lo[r] = 0.f;
        }
    }

    uint8_t extra = 0;
    if (n >= k) rank_sort(ne, cj, cd, cdl, reinterpret_cast<uint64_t*>(dd), sorted, sorted_lo);
    const int64_t n_valid = max<int64_t>(0, nl - a.key_lo) - ((q >= a.key_lo && q < nl) ? 1 : 0);
    if ((P == ATSNE_PREC_FP32 || P == ATSNE_PREC_FP32X3) && take < n_valid && n >= k) {
        // Certificate: every non-candidate j has d'_j >= d'(kstar), so its
        // true distance is at least d'(kstar) + n_q - E.  If that exceeds the
        // (k+1)-th exact candidate distance (plus the direct-difference
        // error), the candidates hold the true k+1 nearest and the row's
        // ranking, tie decision included, is that of a full scan.
        const int rk = ne > k ? k : k - 1;
        const float dk = key_dist(sorted[rk]);
        const float dthr = key_dist(kstar);
        const float lb = dthr + nq - (P == ATSNE_PREC_FP32X3 ? x3_contraction_bound(a.Dp, nq, nmax, dthr)
                                                             : fp32_contraction_bound(a.Dp, nq, nmax, dthr));
        if (!(lb > dk * (1.0f + 2.0f * TIE_REL))) {
            extra = ATSNE_FLAG_EXACT_SCAN;
            if (l == 0) {
                int p = atomicAdd(a.scan_count, 1);
                a.scan_list[p] = (int32_t)m;
            }
        }
    }
    if (n >= k)
        finalize_sorted(a.X, a.ld, a.D, xq, ne, k, sorted, sorted_lo, dd, out_idx, out_d2, out_d2_lo,
                        a.out_flags ? a.out_flags + m : nullptr, extra);
}

// knn_scan: exact FP32 linear scan for rows whose candidate margin was not
// certified.  One workgroup (4 waves) per queued row, persistent over the
// queue; every workgroup exits once the queue is drained.  Each wave scans
// the keys j = key_lo + w, +4, ... in increasing order with the same
// direct-difference arithmetic as knn_select, keeps (d, j) keys at or below
// its running threshold in an LDS region and shrinks the region to its best
// `keep` keys when full; keys arrive in increasing j, so after a shrink a
// strict d < tau filter is exact.  The four regions are merged at the end.
constexpr int SCAN_REGION = 1024;
__global__ __launch_bounds__(256) void knn_scan(SelArgs a, int keep_extra, int32_t* __restrict__ cursor) {
    __shared__ uint64_t region[4][SCAN_REGION];
    __shared__ uint32_t hist_all[4][256];
    __shared__ int32_t rcount[4];
    __shared__ int32_t cj[MAX_KC];
    __shared__ float cd[MAX_KC];
    __shared__ float cdl[MAX_KC];
    __shared__ uint64_t sorted[MAX_KC];
    __shared__ float sorted_lo[MAX_KC];
    __shared__ double dd[MAX_KC];
    __shared__ int32_t item;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int nq = *a.scan_count;
    uint64_t* reg = region[w];
    uint32_t* hist = hist_all[w];
    for (;;) {
        __syncthreads();
        if (t == 0) item = atomicAdd(cursor, 1);
        __syncthreads();
        const int it = item;
        if (it >= nq) break;
        const int64_t m = a.scan_list[it];
        const int64_t q = load_qid(a.qids, a.m0, m);
        const int64_t nl = a.nlims ? (int64_t)a.nlims[m] : a.nlim;
        const int k = a.ks ? a.ks[m] : a.k;
        const int32_t vq = a.views ? a.views[m] : a.view;
        const int keep = min(k + keep_extra, SCAN_REGION - 24);
        int32_t* out_idx = a.out_idx + m * a.out_stride;
        float* out_d2 = a.out_d2 + m * a.out_stride;
        float* out_d2_lo = a.out_d2_lo ? a.out_d2_lo + m * a.out_stride : nullptr;
        const float* xq = a.X + q * a.ld;
        // The current k-th exact distance bounds the true k-th from above;
        // widened by the near-tie band, so the keys just past the k-th (which
        // the near-tie test and the FP64 re-rank look at) stay candidates and
        // the row ends exactly as a certified row would.
        float tau = out_d2[k - 1] * (1.0f + 4.0f * TIE_REL);
        bool strict = false;
        int cnt = 0;
        // key ranges: the row's tile list, or [key_lo, nl); ascending either way
        const int32_t* tl = nullptr;
        int n_ranges = 1;
        if (a.row_blk) {
            const int bk = a.row_blk[m];
            tl = a.tl_idx + a.blk_t[bk];
            n_ranges = a.blk_t[bk + 1] - a.blk_t[bk];
        }
        for (int rg = 0; rg < n_ranges; ++rg) {
        const int64_t r_lo = tl ? (int64_t)tl[rg] * KT : a.key_lo;
        const int64_t r_hi = tl ? min<int64_t>(r_lo + KT, nl) : nl;
        for (int64_t j0 = r_lo + w; j0 < r_hi; j0 += 16) {
            // four keys per pass (a key past the range repeats j0; its sum is dropped)
            const float* xr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xr[u] = a.X + (j0 + 4 * u < r_hi ? j0 + 4 * u : j0) * a.ld;
            float dj[4], dj_lo[4];
            direct_group<4>(xq, xr, a.D, dj, dj_lo);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = j0 + 4 * u;
                const bool pass = j < r_hi && j != q && key_visible(a.death, j, vq) &&
                                  (strict ? (dj[u] < tau) : (dj[u] <= tau));
                if (pass) {
                    if (l == 0) reg[cnt] = pack_key(dj[u], (int32_t)j);
                    ++cnt;
                }
            }
            if (cnt > SCAN_REGION - 4) {
                wave_sync();
                const int c0 = cnt;
                uint64_t kstar = wave_select(
                    [&](auto f) {
                        for (int i = l; i < c0; i += WAVE) f(reg[i]);
                    },
                    (uint32_t)keep, hist);
                int base = 0;
                for (int i0 = 0; i0 < c0; i0 += WAVE) {
                    int i = i0 + l;
                    uint64_t kk = i < c0 ? reg[i] : ~0ull;
                    bool kp = i < c0 && kk <= kstar;
                    uint64_t mm = ballot(kp);
                    wave_sync();
                    if (kp) reg[base + __popcll(mm & lanemask_lt())] = kk;
                    base += __popcll(mm);
                    wave_sync();
                }
                cnt = keep;
                tau = key_dist(kstar);
                strict = true;
            }
        }
        }
        if (l == 0) rcount[w] = cnt;
        __syncthreads();
        if (w == 0) {
            const int tot = rcount[0] + rcount[1] + rcount[2] + rcount[3];
            auto each = [&](auto f) {
                for (int r = 0; r < 4; ++r)
                    for (int i = l; i < rcount[r]; i += WAVE) f(region[r][i]);
            };
            const int take = min(keep, tot);
            const uint64_t kstar = union_threshold(each, take, tot, hist);
            int n = 0;
            for (int r = 0; r < 4; ++r) {
                for (int i0 = 0; i0 < rcount[r]; i0 += WAVE) {
                    int i = i0 + l;
                    uint64_t kk = i < rcount[r] ? region[r][i] : ~0ull;
                    bool kp = i < rcount[r] && kk <= kstar;
                    uint64_t mm = ballot(kp);
                    if (kp) {
                        int p = n + __popcll(mm & lanemask_lt());
                        cj[p] = key_index(kk);
                        cd[p] = key_dist(kk);
                    }
                    n += __popcll(mm);
                }
            }
            wave_sync();
            // the residuals of the chosen candidates (their distances are
            // recomputed by the same arithmetic, so hi equals the key's)
            if (out_d2_lo) direct_distances(a.X, a.ld, a.D, xq, n, cj, cd, cdl);
            if (n >= k)
                finalize_row(a.X, a.ld, a.D, xq, n, k, cj, cd, out_d2_lo ? cdl : nullptr, sorted, sorted_lo, dd,
                             out_idx, out_d2, out_d2_lo, a.out_flags ? a.out_flags + m : nullptr,
                             ATSNE_FLAG_EXACT_SCAN);
        }
    }
}

// knn_reverse_merge: one wave per resident row.  Its candidates are new rows
// whose approximate distance may beat the row's farthest neighbour; the exact
// FP32 distance decides (Eq. 13, strict), and the survivors are merged into
// the row's list, keeping its best by (d, j).  A list may hold absent entries
// (index -1, distance +inf) at its tail after deletions (Sec. 5.3): Eq. 13
// then works on the np present entries, whose farthest is d_max and is
// evicted, so a merge never changes the number of present entries.
struct RevArgs {
    SelArgs s;
    int32_t* res_idx;
    float* res_d2;
    float* res_d2_lo;  // may be null
    uint8_t* res_flags;
    int64_t res_stride;
    int32_t* changed;
    int32_t* n_changed;
};

__global__ __launch_bounds__(64) void knn_reverse_merge(RevArgs r) {
    __shared__ uint32_t hist[256];
    __shared__ int32_t cj[MAX_KC];
    __shared__ float cd[MAX_KC];
    __shared__ float cdl[MAX_KC];
    __shared__ uint64_t sorted[MAX_KC];
    __shared__ float sorted_lo[MAX_KC];
    __shared__ double dd[MAX_KC];
    __shared__ int32_t ncand;
    const SelArgs& a = r.s;
    const int l = lane_id();
    const int64_t m = blockIdx.x;
    if (m >= a.M) return;
    const int64_t q = load_qid(a.qids, a.m0, m);
    const int k = a.k;
    if (!key_visible(a.death, q, a.view)) return;
    const int32_t* cnt = a.counts + m * a.S;
    int total = 0;
    for (int s = 0; s < a.S; ++s) total += cnt[s];
    if (total == 0) return;
    const uint64_t* base = a.slots + (size_t)m * a.S * (size_t)a.cap;
    auto each = [&](auto f) {
        for (int s = 0; s < a.S; ++s) {
            const uint64_t* sl = base + (size_t)s * a.cap;
            const int c = cnt[s];
            for (int i = l; i < c; i += WAVE) f(sl[i]);
        }
    };
    const int take = min(total, MAX_KC - k);
    const uint64_t kstar = union_threshold(each, take, total, hist);
    int32_t* ridx = r.res_idx + q * r.res_stride;
    float* rd2 = r.res_d2 + q * r.res_stride;
    float* rd2_lo = r.res_d2_lo ? r.res_d2_lo + q * r.res_stride : nullptr;
    int np = 0;
    for (int i0 = 0; i0 < k; i0 += WAVE) np += __popcll(ballot(i0 + l < k && ridx[i0 + l] >= 0));
    if (np == 0) return;
    if (l == 0) ncand = 0;
    wave_sync();
    each([&](uint64_t key) {
        if (key <= kstar) {
            int p = atomicAdd(&ncand, 1);
            cj[k + p] = key_index(key);
        }
    });
    wave_sync();
    const int nc = ncand;
    const float* xq = a.X + q * a.ld;
    direct_distances(a.X, a.ld, a.D, xq, nc, cj + k, cd + k, cdl + k);
    const float dmax = rd2[np - 1];
    // keep the new keys strictly closer than the farthest present neighbour
    int c = 0;
    for (int i0 = 0; i0 < nc; i0 += WAVE) {
        const int i = i0 + l;
        const bool kp = i < nc && cd[k + i] < dmax;
        int32_t jj = kp ? cj[k + i] : 0;
        float dv = kp ? cd[k + i] : 0.f;
        float dvl = kp ? cdl[k + i] : 0.f;
        const uint64_t mm = ballot(kp);
        wave_sync();
        if (kp) {
            const int p = c + __popcll(mm & lanemask_lt());
            cj[k + p] = jj;
            cd[k + p] = dv;
            cdl[k + p] = dvl;
        }
        c += __popcll(mm);
        wave_sync();
    }
    if (c == 0) return;
    if (np < k) {
        // survivors move down next to the present entries (dst < src, so a
        // chunk never overwrites a later chunk's unread entries)
        for (int i0 = 0; i0 < c; i0 += WAVE) {
            const int i = i0 + l;
            const int32_t jj = i < c ? cj[k + i] : 0;
            const float dv = i < c ? cd[k + i] : 0.f;
            const float dvl = i < c ? cdl[k + i] : 0.f;
            wave_sync();
            if (i < c) {
                cj[np + i] = jj;
                cd[np + i] = dv;
                cdl[np + i] = dvl;
            }
            wave_sync();
        }
    }
    for (int i = l; i < np; i += WAVE) {
        cj[i] = ridx[i];
        cd[i] = rd2[i];
        cdl[i] = rd2_lo ? rd2_lo[i] : 0.f;
    }
    wave_sync();
    finalize_row(a.X, a.ld, a.D, xq, np + c, np, cj, cd, cdl, sorted, sorted_lo, dd, ridx, rd2, rd2_lo,
                 r.res_flags ? r.res_flags + q : nullptr, 0);
    if (l == 0) {
        const int p = atomicAdd(r.n_changed, 1);
        r.changed[p] = (int32_t)q;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int default_kcand(int prec, int k) {
    if (prec == ATSNE_PREC_FP32 || prec == ATSNE_PREC_FP32X3) return k + std::max(32, k / 2);
    return 2 * k;
}

static int pick_splits(int64_t MB, int total_tiles, int slots_avail) {
    int best_s = 1;
    double best_eff = -1.0;
    const int smax = std::max(1, std::min(64, total_tiles));
    for (int s = 1; s <= smax; ++s) {
        double wgs = (double)MB * s;
        double rounds = wgs / slots_avail;
        double eff = rounds / std::ceil(rounds);
        if (wgs >= slots_avail && eff >= 0.92) return s;
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best_s = s;
        }
    }
    return best_s;
}

size_t corpus_bytes(int prec, int64_t rows_cap, int32_t D) {
    const int ce = chunk_elems(prec);
    const int64_t Dp = ceil_div(D, ce) * ce;
    const int64_t rows = ceil_div(std::max<int64_t>(rows_cap, 1), KT) * KT;
    Arena a;
    a.take<char>((size_t)rows * Dp * elem_bytes(prec));
    a.take<float>(rows);
    a.take<float>(rows);
    a.take<float>(rows);
    a.take<float>(rows / PMAX_CHUNK + 1);  // chunk carries of the norms' prefix max
    return a.used;
}

void corpus_bind(Corpus& c, int prec, const float* X, int64_t ld, int32_t D, int64_t rows_cap, void* mem) {
    const int ce = chunk_elems(prec);
    c.prec = prec;
    c.X = X;
    c.ld = ld;
    c.D = D;
    c.Dp = (int32_t)(ceil_div(D, ce) * ce);
    c.n_chunks = c.Dp / ce;
    c.row_units = (int64_t)c.Dp * elem_bytes(prec) / 16;
    c.rows_cap = ceil_div(std::max<int64_t>(rows_cap, 1), KT) * KT;
    Arena a(mem, corpus_bytes(prec, rows_cap, D));
    c.Xp = a.take<char>((size_t)c.rows_cap * c.Dp * elem_bytes(prec));
    c.norms = a.take<float>(c.rows_cap);
    c.scales = a.take<float>(c.rows_cap);
    c.pmax = a.take<float>(c.rows_cap);
    c.pmax_blk = a.take<float>(c.rows_cap / PMAX_CHUNK + 1);
}

atsne_status corpus_prep(const Corpus& c, int64_t r0, int64_t r1, int64_t n_live, hipStream_t st) {
    if (r1 <= r0) return ATSNE_OK;
    ProfScope ps_("knn_prep", st);
    const dim3 grid((unsigned)ceil_div(r1 - r0, 4)), block(256);
    switch (c.prec) {
        case ATSNE_PREC_FP32:
            knn_prep<ATSNE_PREC_FP32><<<grid, block, 0, st>>>(c.X, c.ld, c.D, c.Dp, r0, r1, n_live, c.Xp, c.norms,
                                                              c.scales);
            break;
        case ATSNE_PREC_BF16:
            knn_prep<ATSNE_PREC_BF16><<<grid, block, 0, st>>>(c.X, c.ld, c.D, c.Dp, r0, r1, n_live, c.Xp, c.norms,
                                                              c.scales);
            break;
        case ATSNE_PREC_FP32X3:
            knn_prep<ATSNE_PREC_FP32X3><<<grid, block, 0, st>>>(c.X, c.ld, c.D, c.Dp, r0, r1, n_live, c.Xp, c.norms,
                                                                c.scales);
            break;
        default:
            knn_prep<ATSNE_PREC_FP8_E4M3><<<grid, block, 0, st>>>(c.X, c.ld, c.D, c.Dp, r0, r1, n_live, c.Xp,
                                                                  c.norms, c.scales);
    }
    ATSNE_LAUNCH_CHECK();
    const int64_t nb = ceil_div(r1 - r0, (int64_t)PMAX_CHUNK);
    knn_pmax_local<<<dim3((unsigned)nb), dim3(1024), 0, st>>>(c.norms, c.pmax, r0, r1, c.pmax_blk);
    ATSNE_LAUNCH_CHECK();
    knn_pmax_carry<<<dim3(1), dim3(1024), 0, st>>>(c.pmax_blk, nb, c.pmax, r0);
    ATSNE_LAUNCH_CHECK();
    knn_pmax_apply<<<dim3((unsigned)ceil_div(r1 - r0, (int64_t)256)), dim3(256), 0, st>>>(c.pmax, r0, r1, c.pmax_blk);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

// Workgroups of the balanced schedule: one per CU, a whole number per XCD.
static int stream_wgs() {
    const int cu = device_cu_count();
    return cu / KNN_XCDS * KNN_XCDS;
}

// Splits per query block of the balanced schedule (the most workgroups that
// cover one query block), 0 when a workgroup's range has too many segments.
static int stream_splits(int MB, int T, int P) {
    int S = 1;
    int4 seg[STREAM_MAX_SEG];
    for (int p = 0; p < P; ++p) {
        const int n = stream_segments(p, MB, T, P, seg, STREAM_MAX_SEG);
        if (n < 0) return 0;
        for (int i = 0; i < n; ++i) S = std::max(S, seg[i].y + 1);
    }
    return S;
}

// Keys a slot holds: k' kept plus a tile's appends plus slack, and at least
// what make_room's register path covers (WAVE * MR_KEYS): the slack sets how
// often a slot is cut back, and each cut waits one memory round trip for
// the slot's keys, so the register path's full size is used.
static int slot_cap(int kc_max) {
    return std::max(WAVE * MR_KEYS, (int)align_up((size_t)(kc_max + KT + std::max(kc_max, 128)), 64));
}

SearchPlan plan_search(int prec, int64_t M, int64_t key_lo, int64_t key_hi, int k_max, int kc_max, int s_max,
                       bool allow_small, bool stream) {
    SearchPlan p;
    p.qb = qb_of(prec);
    p.M = M;
    p.k_max = k_max;
    p.kc_max = kc_max;
    // small problems (fewer (query block, key tile) pairs than two per CU in
    // the large geometry) take the 128 x 128 geometry: four times the workgroups
    if (allow_small && prec != ATSNE_PREC_FP8_E4M3 && key_lo % 128 == 0) {
        const int64_t pairs = ceil_div(std::max<int64_t>(M, 1), p.qb) * ceil_div(std::max<int64_t>(key_hi - key_lo, 1), KT);
        if (pairs < 2 * (int64_t)device_cu_count()) {
            p.small = true;
            p.qb = TileGeom<ATSNE_PREC_FP32, true>::QB;
            p.kt = TileGeom<ATSNE_PREC_FP32, true>::KT;
        }
    }
    p.tile_lo = (int)(key_lo / p.kt);
    p.tile_hi = (int)ceil_div(key_hi, p.kt);
    const int total_tiles = std::max(1, p.tile_hi - p.tile_lo);
    p.cap = slot_cap(kc_max);
    p.MB = (int)ceil_div(std::max<int64_t>(M, 1), p.qb);
    int S = pick_splits(p.MB, total_tiles, device_cu_count());
    if (s_max > 0) S = std::min(S, s_max);
    // Balanced schedule when the task grid would run more than one round:
    // one workgroup per CU (the large geometry holds one per CU), no partial
    // last round, and at most a few splits per query block (fewer candidate
    // streams, a smaller select).  It needs its splits to fit under s_max.
    if (stream && !p.small && key_lo % KT == 0) {
        const int P = stream_wgs();
        const int64_t W = (int64_t)p.MB * total_tiles;
        if (P > 0 && W >= 2 * (int64_t)P) {
            const int S_stream = stream_splits(p.MB, total_tiles, P);
            if (S_stream > 0 && (s_max <= 0 || S_stream <= s_max)) {
                p.stream_wgs = P;
                S = S_stream;
            }
        }
    }
    p.tiles_per_split = (int)ceil_div(total_tiles, S);
    p.S = p.stream_wgs ? S : (int)ceil_div(total_tiles, p.tiles_per_split);
    Arena a;
    a.take<uint64_t>((size_t)p.MB * p.qb * p.S * p.cap);
    a.take<int32_t>((size_t)p.MB * p.qb * p.S);
    a.take<int32_t>(64);
    a.take<int32_t>(std::max<int64_t>(M, 1));
    a.take<int4>((size_t)std::max(p.stream_wgs, 1) * (STREAM_MAX_SEG + 1));
    p.ws_bytes = a.used;
    return p;
}

SearchPlan plan_list_search(int64_t M, int64_t n_blocks, int k_max, int kc_max, int S) {
    SearchPlan p;
    p.qb = qb_of(ATSNE_PREC_FP32);
    p.M = M;
    p.k_max = k_max;
    p.kc_max = kc_max;
    p.cap = slot_cap(kc_max);
    p.MB = (int)std::max<int64_t>(n_blocks, 1);
    p.S = std::max(1, S);
    p.tiles_per_split = 1;
    // slots are indexed by batch row; MB * qb >= M since a block holds at most qb rows
    Arena a;
    a.take<uint64_t>((size_t)p.MB * p.qb * p.S * p.cap);
    a.take<int32_t>((size_t)p.MB * p.qb * p.S);
    a.take<int32_t>(64);
    a.take<int32_t>(std::max<int64_t>(M, 1));
    a.take<int4>((size_t)STREAM_MAX_SEG + 1);  // (segment table, unused here)
    p.ws_bytes = a.used;
    return p;
}

struct SearchWs {
    uint64_t* slots;
    int32_t* counts;
    int32_t* misc;
    int32_t* scan_list;
    int4* segs;
};

static SearchWs carve(const SearchPlan& p, void* ws) {
    Arena a(ws, p.ws_bytes);
    SearchWs w;
    w.slots = a.take<uint64_t>((size_t)p.MB * p.qb * p.S * p.cap);
    w.counts = a.take<int32_t>((size_t)p.MB * p.qb * p.S);
    w.misc = a.take<int32_t>(64);
    w.scan_list = a.take<int32_t>(std::max<int64_t>(p.M, 1));
    w.segs = a.take<int4>((size_t)std::max(p.stream_wgs, 1) * (STREAM_MAX_SEG + 1));
    return w;
}

template <int P>
static atsne_status launch_tile(const Corpus& c, const Batch& b, const SearchPlan& p, const SearchWs& w,
                                hipStream_t st) {
    TileArgs t;
    t.Xp = static_cast<const uint4*>(c.Xp);
    t.row_units = c.row_units;
    t.n_chunks = c.n_chunks;
    t.Dp = c.Dp;
    t.norms = c.norms;
    t.scales = c.scales;
    t.pmax = c.pmax;
    t.M = b.M;
    t.qids = b.qids;
    t.m0 = b.m0;
    t.nlims = b.nlims;
    t.nlim = b.nlim;
    t.key_lo = b.key_lo;
    t.kcs = b.kcs;
    t.kc = b.kc;
    t.tau0 = b.tau0;
    t.tau0_stride = b.tau0_stride;
    t.tau_seed = b.tau_seed;
    t.death = c.death;
    t.views = b.views;
    t.view = b.view;
    t.MB = (int)ceil_div(b.M, p.qb);
    t.S = p.S;
    t.tiles_per_split = p.tiles_per_split;
    t.tile_lo = p.tile_lo;
    t.tile_hi = p.tile_hi;
    t.cap = p.cap;
    t.final_keep = (!b.blk_q && !b.tau0 && p.tiles_per_split == 1) ? p.kt : 0;
    // threshold mode: the select cuts each row's union (held in registers
    // while it fits) instead of a serial exact shrink per query in the tile
    if (b.tau_out) t.final_keep = SEL_RK * WAVE / std::max(1, p.S);
    t.blk_q = b.blk_q;
    t.blk_t = b.blk_t;
    t.tl_idx = b.tl_idx;
    if (b.blk_q) t.MB = (int)b.n_blocks;
    t.slots = w.slots;
    t.counts = w.counts;
    t.segs = nullptr;
    unsigned n_wg = (unsigned)(t.MB * p.S);
    // The balanced schedule serves the plain search; a batch whose own
    // segments would need more splits than the plan (a smaller last batch)
    // takes the task grid with the plan's splits.
    if (p.stream_wgs && !p.small && !c.death && !b.blk_q && !b.tau0) {
        const int T = p.tile_hi - p.tile_lo;
        const int S_b = (int64_t)t.MB * T >= 2 * (int64_t)p.stream_wgs ? stream_splits(t.MB, T, p.stream_wgs) : 0;
        if (S_b > 0 && S_b <= p.S) {
            knn_stream_segments<<<dim3((unsigned)ceil_div(p.stream_wgs, 256)), dim3(256), 0, st>>>(t.MB, T, p.stream_wgs,
                                                                                              w.segs);
            ATSNE_LAUNCH_CHECK();
            t.segs = w.segs;
            // slots go to the select unshrunk while the row's union still
            // fits the select's registers (S slots of up to cap keys): its
            // union threshold replaces the serial exact shrink per query
            // (BF16 tile -6%, FP32 -1%, outputs identical)
            t.final_keep = SEL_RK * WAVE / std::max(1, p.S);
            n_wg = (unsigned)p.stream_wgs;
        }
    }
    if (!t.segs && p.stream_wgs) t.tiles_per_split = (int)ceil_div(p.tile_hi - p.tile_lo, p.S);
    ProfScope ps_(b.tau_out ? "seed_tile" : (b.tau0 ? "knn_tile_reverse" : (b.blk_q ? "knn_tile_list" : "knn_tile")),
                  st);
    const dim3 grid(n_wg);
    if (p.small) {
        ATSNE_REQUIRE(!c.death && !b.blk_q && !b.tau0 && P != ATSNE_PREC_FP8_E4M3, ATSNE_E_UNSUPPORTED,
                      "the small geometry serves the plain search only");
        if constexpr (P != ATSNE_PREC_FP8_E4M3)
            knn_tile<P, TILE_PLAIN, true><<<grid, dim3(TileGeom<P, true>::THREADS), 0, st>>>(t);
    } else if constexpr (P == ATSNE_PREC_FP32 || P == ATSNE_PREC_FP32X3) {
        // the exact contractions: deletion stamps (the server's corpus) and
        // tile lists (the approximate search's corpus)
        const dim3 block(TileGeom<P>::THREADS);
        ATSNE_REQUIRE(!(c.death && b.blk_q), ATSNE_E_UNSUPPORTED, "tile lists with deletion stamps");
        if (b.blk_q)
            knn_tile<P, TILE_LIST, false><<<grid, block, 0, st>>>(t);
        else if (c.death)
            knn_tile<P, TILE_VIS, false><<<grid, block, 0, st>>>(t);
        else
            knn_tile<P, TILE_PLAIN, false><<<grid, block, 0, st>>>(t);
    } else {
        ATSNE_REQUIRE(!c.death && (!b.blk_q || P == ATSNE_PREC_FP8_E4M3), ATSNE_E_UNSUPPORTED,
                      "deletion stamps need an exact contraction's corpus, tile lists an exact or the FP8 one");
        if constexpr (P == ATSNE_PREC_FP8_E4M3) {
            if (b.blk_q) {
                // the seeding pass of a large FP8 search
                knn_tile<P, TILE_LIST, false><<<grid, dim3(TileGeom<P>::THREADS), 0, st>>>(t);
                ATSNE_LAUNCH_CHECK();
                return ATSNE_OK;
            }
        }
        knn_tile<P, TILE_PLAIN, false><<<grid, dim3(TileGeom<P>::THREADS), 0, st>>>(t);
    }
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

static atsne_status launch_tile_any(const Corpus& c, const Batch& b, const SearchPlan& p, const SearchWs& w,
                                    hipStream_t st) {
    switch (c.prec) {
        case ATSNE_PREC_FP32:
            return launch_tile<ATSNE_PREC_FP32>(c, b, p, w, st);
        case ATSNE_PREC_BF16:
            return launch_tile<ATSNE_PREC_BF16>(c, b, p, w, st);
        case ATSNE_PREC_FP32X3:
            return launch_tile<ATSNE_PREC_FP32X3>(c, b, p, w, st);
        default:
            return launch_tile<ATSNE_PREC_FP8_E4M3>(c, b, p, w, st);
    }
}

static SelArgs sel_args(const Corpus& c, const Batch& b, const SearchPlan& p, const SearchWs& w) {
    SelArgs s;
    s.X = c.X;
    s.ld = c.ld;
    s.D = c.D;
    s.Dp = c.Dp;
    s.norms = c.norms;
    s.pmax = c.pmax;
    s.M = b.M;
    s.qids = b.qids;
    s.m0 = b.m0;
    s.nlims = b.nlims;
    s.nlim = b.nlim;
    s.key_lo = b.key_lo;
    s.ks = b.ks;
    s.k = b.k;
    s.kcs = b.kcs;
    s.kc = b.kc;
    s.S = p.S;
    s.cap = p.cap;
    s.death = c.death;
    s.views = b.views;
    s.view = b.view;
    s.row_blk = b.row_blk;
    s.blk_t = b.blk_t;
    s.tl_idx = b.tl_idx;
    s.slots = w.slots;
    s.counts = w.counts;
    s.tau_out = b.tau_out;
    s.tau_map = b.tau_map;
    s.sel_order = b.sel_order;
    s.out_idx = b.out_idx;
    s.out_d2 = b.out_d2;
    s.out_d2_lo = b.out_d2_lo;
    s.out_flags = b.out_flags;
    s.out_stride = b.out_stride;
    s.scan_list = w.scan_list;
    s.scan_count = w.misc + 1;
    return s;
}

atsne_status knn_search(const Corpus& c, const Batch& b, const SearchPlan& p, void* ws, hipStream_t st) {
    if (b.M == 0) return ATSNE_OK;
    ATSNE_REQUIRE(b.M <= p.M && b.kc <= p.kc_max && b.k <= p.k_max, ATSNE_E_INVALID_ARG, "batch exceeds its plan");
    const SearchWs w = carve(p, ws);
    ATSNE_HIP(hipMemsetAsync(w.misc, 0, 256, st));
    ATSNE_TRY(launch_tile_any(c, b, p, w, st));
    const SelArgs s = sel_args(c, b, p, w);
    {
        ProfScope ps_(b.tau_out ? "seed_select" : "knn_select", st);
        const int kcap = p.kc_max;
        const int rows = sel_rows(kcap);
        const size_t lds = rows * select_lds_bytes(kcap);
        const dim3 sel_grid((unsigned)ceil_div(b.M, rows));
        switch (c.prec) {
            case ATSNE_PREC_FP32:
                knn_select<ATSNE_PREC_FP32><<<sel_grid, dim3(64 * rows), lds, st>>>(s, kcap);
                break;
            case ATSNE_PREC_BF16:
                knn_select<ATSNE_PREC_BF16><<<sel_grid, dim3(64 * rows), lds, st>>>(s, kcap);
                break;
            case ATSNE_PREC_FP32X3:
                knn_select<ATSNE_PREC_FP32X3><<<sel_grid, dim3(64 * rows), lds, st>>>(s, kcap);
                break;
            default:
                knn_select<ATSNE_PREC_FP8_E4M3><<<sel_grid, dim3(64 * rows), lds, st>>>(s, kcap);
        }
        ATSNE_LAUNCH_CHECK();
    }
    if (c.prec == ATSNE_PREC_FP32 || c.prec == ATSNE_PREC_FP32X3) {
        const int grid = (int)std::min<int64_t>(b.M, 4 * (int64_t)device_cu_count());
        ProfScope ps_("knn_scan", st);
        knn_scan<<<dim3((unsigned)grid), dim3(256), 0, st>>>(s, 32, w.misc + 2);
        ATSNE_LAUNCH_CHECK();
    }
    return ATSNE_OK;
}

atsne_status knn_reverse(const Corpus& c, const Batch& b, const SearchPlan& p, int32_t* res_idx, float* res_d2,
                         float* res_d2_lo, uint8_t* res_flags, int64_t res_stride, int32_t* changed,
                         int32_t* n_changed, void* ws, hipStream_t st) {
    if (b.M == 0) return ATSNE_OK;
    ATSNE_REQUIRE(c.prec == ATSNE_PREC_FP32 || c.prec == ATSNE_PREC_FP32X3, ATSNE_E_UNSUPPORTED,
                  "reverse merge needs an exact contraction (FP32 or FP32X3 corpus)");
    ATSNE_REQUIRE(b.tau0 && b.M <= p.M && b.kc <= p.kc_max, ATSNE_E_INVALID_ARG, "bad reverse batch");
    const SearchWs w = carve(p, ws);
    ATSNE_TRY(launch_tile_any(c, b, p, w, st));
    RevArgs r;
    r.s = sel_args(c, b, p, w);
    r.res_idx = res_idx;
    r.res_d2 = res_d2;
    r.res_d2_lo = res_d2_lo;
    r.res_flags = res_flags;
    r.res_stride = res_stride;
    r.changed = changed;
    r.n_changed = n_changed;
    ProfScope ps_("knn_reverse_merge", st);
    knn_reverse_merge<<<dim3((unsigned)b.M), dim3(64), 0, st>>>(r);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

// ---- C ABI: standalone search over a caller corpus ----
constexpr int64_t KNN_SEED_MIN_N = (int64_t)1 << 18;  // full FP8 searches from this many rows are seeded

struct KnnPlan {
    int prec, k, kc;
    int64_t N, M, Mb;
    int32_t D;
    size_t b_corpus;
    SearchPlan sp;
    size_t total;
};

static atsne_status make_plan(int64_t N, int64_t M, int32_t D, int prec, int k, int k_cand, KnnPlan& p) {
    ATSNE_REQUIRE(prec == ATSNE_PREC_FP32 || prec == ATSNE_PREC_BF16 || prec == ATSNE_PREC_FP8_E4M3 ||
                      prec == ATSNE_PREC_FP32X3,
                  ATSNE_E_INVALID_ARG, "unknown precision %d", prec);
    ATSNE_REQUIRE(N >= 2 && N < (1ll << 31) - KT, ATSNE_E_INVALID_ARG, "N=%lld out of range", (long long)N);
    ATSNE_REQUIRE(M >= 0 && M < (1ll << 31), ATSNE_E_INVALID_ARG, "M=%lld out of range", (long long)M);
    ATSNE_REQUIRE(D >= 1 && D <= 65536, ATSNE_E_INVALID_ARG, "D=%d out of range", D);
    ATSNE_REQUIRE(k >= 1 && k <= N - 1, ATSNE_E_K_RANGE, "k=%d must be in [1, N-1=%lld]", k, (long long)(N - 1));
    ATSNE_REQUIRE(k <= 1000, ATSNE_E_K_RANGE, "k=%d above the supported maximum 1000", k);
    int kc = k_cand > 0 ? k_cand : default_kcand(prec, k);
    kc = (int)std::min<int64_t>(kc, N - 1);
    ATSNE_REQUIRE(kc >= k && kc <= MAX_KC, ATSNE_E_K_RANGE, "k_cand=%d must be in [k=%d, %d]", kc, k, MAX_KC);
    p.prec = prec;
    p.k = k;
    p.kc = kc;
    p.N = N;
    p.M = M;
    p.D = D;
    p.b_corpus = corpus_bytes(prec, N, D);
    // Keep the candidate slots within a sixteenth of the device's memory,
    // between 2 and 16 GiB (16 GiB on a 288 GB MI355X): fewer key splits
    // first, then batches of query rows.  Each batch re-streams the whole
    // corpus, so the larger budget pays at large N (N = 10^6, FP8: four
    // launches in 2 GiB, one in 16 GiB, 9% faster).
    const size_t slot_budget =
        std::min<size_t>((size_t)16 << 30, std::max<size_t>((size_t)2 << 30, device_hbm_bytes() / 16));
    const int64_t Mq = std::max<int64_t>(M, 1);
    SearchPlan full = plan_search(prec, Mq, 0, N, k, kc, 0, true, true);
    if (full.ws_bytes > slot_budget && full.S > 1) {
        const int64_t s_fit = (int64_t)(slot_budget / ((size_t)Mq * full.cap * 8));
        full = plan_search(prec, Mq, 0, N, k, kc, (int)std::max<int64_t>(1, std::min<int64_t>(full.S, s_fit)), true,
                           true);
    }
    const int qb = qb_of(prec);
    const size_t per_row = (size_t)full.S * full.cap * 8;
    int64_t max_rows = (int64_t)(slot_budget / per_row);
    max_rows = std::max<int64_t>(qb, max_rows / qb * qb);
    p.Mb = std::min<int64_t>(Mq, max_rows);
    p.sp = p.Mb < Mq ? plan_search(prec, p.Mb, 0, N, k, kc, full.S, true, true) : full;
    p.total = align_up(p.b_corpus, 256) + p.sp.ws_bytes;
    return ATSNE_OK;
}

static atsne_status knn_impl(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* qids, int64_t M,
                             atsne_precision prec, int32_t k, int32_t k_cand, int32_t* nbr_idx, float* nbr_d2,
                             float* nbr_d2_lo, uint8_t* flags, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    ATSNE_REQUIRE(X && (M == 0 || (nbr_idx && nbr_d2)), ATSNE_E_INVALID_ARG, "null X or output pointer");
    ATSNE_REQUIRE(ld >= D, ATSNE_E_INVALID_ARG, "ld=%lld < D=%d", (long long)ld, D);
    KnnPlan p;
    ATSNE_TRY(make_plan(N, M, D, (int)prec, k, k_cand, p));
    if (M == 0) return ATSNE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // A full FP8 search over many rows first bounds each row's k'-th key
    // code from the keys near it (fp8_seed_thresholds), so its tiles append
    // about k' keys per row instead of every key below a threshold that
    // tightens only as the corpus streams past; the outputs are unchanged.
    // ATSNE_FP8_SEED=0 turns the pass off.
    float* tau_seed = nullptr;
    int32_t* order = nullptr;  // the points in cluster order (the seeding pass's partition)
    std::unique_ptr<float, void (*)(float*)> tau_guard(nullptr, [](float* q) { (void)hipFree(q); });
    std::unique_ptr<int32_t, void (*)(int32_t*)> order_guard(nullptr, [](int32_t* q) { (void)hipFree(q); });
    if (prec == ATSNE_PREC_FP8_E4M3 && !qids && N >= KNN_SEED_MIN_N && ld == D) {
        const char* env = std::getenv("ATSNE_FP8_SEED");
        if (!(env && env[0] == '0')) {
            // the pass is an optimisation: without the memory for it, or
            // where it does not apply (D above the partition's limit, cells
            // too coarse to pay), the search runs unseeded (same results)
            atsne_status s = ATSNE_E_NOMEM;
            if (hipMalloc((void**)&tau_seed, sizeof(float) * N) == hipSuccess) {
                tau_guard.reset(tau_seed);
                if (hipMalloc((void**)&order, sizeof(int32_t) * N) == hipSuccess) {
                    order_guard.reset(order);
                    ProfScope ps_("seed_total", st);
                    ProfQuiet quiet_;  // the pass's own searches report as seed_total only
                    s = fp8_seed_thresholds(X, N, D, ld, p.kc, tau_seed, order, st);
                }
            }
            if (s == ATSNE_E_NOMEM || s == ATSNE_E_UNSUPPORTED) {
                (void)hipGetLastError();  // clear a failed allocation's sticky error
                // a pass that ran but stepped aside shows in the kernel
                // timing as an empty "seed_declined" record
                if (order) ProfScope declined_("seed_declined", st);
                (void)hipStreamSynchronize(st);
                tau_guard.reset();
                order_guard.reset();
                tau_seed = nullptr;
                order = nullptr;
                clear_error();
            } else if (s != ATSNE_OK) {
                return s;
            }
        }
    }
    Scratch scr;
    ATSNE_TRY(scr.acquire(ws, ws_bytes, p.total, st));
    Corpus c;
    corpus_bind(c, (int)prec, X, ld, D, N, scr.ptr);
    ATSNE_TRY(corpus_prep(c, 0, c.rows_cap, N, st));
    void* sws = static_cast<char*>(scr.ptr) + align_up(p.b_corpus, 256);
    for (int64_t m0 = 0; m0 < M; m0 += p.Mb) {
        Batch b;
        b.M = std::min<int64_t>(p.Mb, M - m0);
        b.qids = qids ? qids + m0 : nullptr;
        b.m0 = m0;
        b.nlim = N;
        b.key_lo = 0;
        b.k = k;
        b.kc = p.kc;
        b.out_idx = nbr_idx + m0 * k;
        b.out_d2 = nbr_d2 + m0 * k;
        b.out_d2_lo = nbr_d2_lo ? nbr_d2_lo + m0 * k : nullptr;
        b.out_flags = flags ? flags + m0 : nullptr;
        b.out_stride = k;
        b.tau_seed = tau_seed;
        // one batch of all rows: the select takes them in cluster order
        if (order && b.M == N && m0 == 0) b.sel_order = order;
        ATSNE_TRY(knn_search(c, b, p.sp, sws, st));
    }
    // the thresholds and the order are freed on return: the searches reading them first
    if (tau_seed) ATSNE_HIP(hipStreamSynchronize(st));
    return ATSNE_OK;
}

}  // namespace atsne

extern "C" atsne_status atsne_knn_workspace_size(int64_t N, int64_t M, int32_t D, atsne_precision prec, int32_t k,
                                                 int32_t k_cand, size_t* bytes) {
    atsne::clear_error();
    ATSNE_REQUIRE(bytes, ATSNE_E_INVALID_ARG, "null bytes pointer");
    atsne::KnnPlan p;
    ATSNE_TRY(atsne::make_plan(N, M, D, (int)prec, k, k_cand, p));
    *bytes = p.total;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_knn(const float* X, int64_t N, int32_t D, int64_t ld, atsne_precision prec, int32_t k,
                                  int32_t k_cand, int32_t* nbr_idx, float* nbr_d2, float* nbr_d2_lo, uint8_t* flags,
                                  void* ws, size_t ws_bytes, void* stream) {
    return atsne::knn_impl(X, N, D, ld, nullptr, N, prec, k, k_cand, nbr_idx, nbr_d2, nbr_d2_lo, flags, ws, ws_bytes,
                           stream);
}

extern "C" atsne_status atsne_knn_subset(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* query_ids,
                                         int64_t M, atsne_precision prec, int32_t k, int32_t k_cand, int32_t* nbr_idx,
                                         float* nbr_d2, float* nbr_d2_lo, uint8_t* flags, void* ws, size_t ws_bytes,
                                         void* stream) {
    ATSNE_REQUIRE(query_ids || M == 0, ATSNE_E_INVALID_ARG, "null query_ids");
    return atsne::knn_impl(X, N, D, ld, query_ids, M, prec, k, k_cand, nbr_idx, nbr_d2, nbr_d2_lo, flags, ws,
                           ws_bytes, stream);
}
