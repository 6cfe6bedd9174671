// Exact K-nearest-neighbour search for the A-tSNE similarity path on gfx950.
//
// The neighbour sets of Sec. 3.1 (Eq. 8) under the squared Euclidean
// distance of Eq. 3, found by brute force: the paper notes that no exact
// method beats a linear scan in high dimension (Sec. 4.2), and on MI355X the
// scan is a dense contraction that belongs on the matrix cores.
//
// Pipeline (all on the caller's stream, no host synchronisation):
//   knn_prep       padded copy of X in the contraction's element type
//                  (FP32 / BF16 RNE / FP8 e4m3 with per-row absmax scales),
//                  row norms n_i = ||x_i||^2 and the corpus max norm.
//   knn_tile       S = X_q X_k^T on MFMA, d'_ij = n_j - 2 S_ij (n_i is a row
//                  constant and irrelevant to the ranking), self and padding
//                  masked; a running per-(query, split) threshold filters
//                  candidates into a buffer that a wave-level radix select
//                  shrinks back to the best k_cand whenever it fills.
//   knn_select     per query, the best k_cand keys (d', j) over all splits,
//                  exact FP32 direct-difference distances for them, sorted by
//                  (d, j); rows whose k-th/(k+1)-th gap is under FP32
//                  resolution are re-ranked in FP64.  On the FP32 path a
//                  rigorous error bound of the contraction certifies that no
//                  non-candidate can beat the k-th neighbour; rows it cannot
//                  certify are queued for knn_scan.
//   knn_scan       exact FP32 linear scan for the queued rows (rare).
#include <algorithm>
#include <cmath>

#include "common.h"
#include "wave.h"

namespace atsne {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int QB = 128;         // queries per workgroup (4 waves x 32)
constexpr int KT = 256;         // keys per tile (8 MFMA blocks of 32)
constexpr int NKB = KT / 32;    // key blocks per tile
constexpr int CHUNK_UNITS = 8;  // 16-byte units per row per D-chunk (128 bytes)
constexpr int ROW_UNITS = 9;    // LDS row stride in 16-byte units (one unit of padding)
constexpr int TILE_THREADS = 256;

// Elements per 128-byte chunk for each precision.
__host__ __device__ constexpr int chunk_elems(int prec) {
    return prec == ATSNE_PREC_FP32 ? 32 : (prec == ATSNE_PREC_BF16 ? 64 : 128);
}
__host__ __device__ constexpr int elem_bytes(int prec) {
    return prec == ATSNE_PREC_FP32 ? 4 : (prec == ATSNE_PREC_BF16 ? 2 : 1);
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
// knn_prep: one wave per row.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void knn_prep(const float* __restrict__ X, int64_t N, int32_t D, int64_t ld,
                                                int64_t N_pad, int32_t Dp, void* __restrict__ Xp,
                                                float* __restrict__ norms, float* __restrict__ scales,
                                                uint32_t* __restrict__ nmax_bits) {
    const int l = lane_id();
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N_pad) return;
    const bool live = row < N;
    const float* x = X + row * ld;
    float s = 1.0f;
    if (P == ATSNE_PREC_FP8_E4M3) {
        float amax = 0.0f;
        if (live)
            for (int d = l; d < D; d += WAVE) amax = fmaxf(amax, fabsf(x[d]));
        amax = wave_max(amax);
        s = amax > 0.0f ? amax / 448.0f : 1.0f;
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
        if (live) atomicMax(nmax_bits, __float_as_uint(acc));  // non-negative floats order as uints
    }
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

template <int P>
__device__ __forceinline__ f32x16 mfma_chunk(f32x16 acc, const uint4 (&a)[4], const uint4 (&b)[4]) {
    if constexpr (P == ATSNE_PREC_FP32) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[i].x), __uint_as_float(b[i].x), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[i].y), __uint_as_float(b[i].y), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[i].z), __uint_as_float(b[i].z), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[i].w), __uint_as_float(b[i].w), acc, 0, 0, 0);
        }
    } else if constexpr (P == ATSNE_PREC_BF16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf16x8 va = __builtin_bit_cast(bf16x8, a[i]);
            bf16x8 vb = __builtin_bit_cast(bf16x8, b[i]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va, vb, acc, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            i32x8 va = {(int)a[i].x, (int)a[i].y, (int)a[i].z, (int)a[i].w,
                        (int)a[i + 1].x, (int)a[i + 1].y, (int)a[i + 1].z, (int)a[i + 1].w};
            i32x8 vb = {(int)b[i].x, (int)b[i].y, (int)b[i].z, (int)b[i].w,
                        (int)b[i + 1].x, (int)b[i + 1].y, (int)b[i + 1].z, (int)b[i + 1].w};
            // format 0 = FP8 E4M3 for both operands; E8M0 scale 127 = 2^0
            acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, acc, 0, 0, 0, 127, 0, 127);
        }
    }
    return acc;
}

// Shrink one candidate slot to its best `kc` keys (wave-wide). Returns the
// key of rank kc, which becomes the slot's threshold.
__device__ uint64_t shrink_slot(uint64_t* slot, int cnt, int kc, uint32_t* hist) {
    const int l = lane_id();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
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
    return kstar;
}

// ---------------------------------------------------------------------------
// knn_tile: grid = MB query blocks x S key splits.  blockIdx.x -> (split,
// query block) with the query block fastest, so the workgroups that share an
// XCD (dispatched round-robin) stream the same key tiles through its L2.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(TILE_THREADS) __attribute__((amdgpu_waves_per_eu(1, 1))) void knn_tile(
    const uint4* __restrict__ Xp, int64_t row_units, int n_chunks, const float* __restrict__ norms,
    const float* __restrict__ scales, int64_t N, const int32_t* __restrict__ qids, int64_t m0, int64_t Mb, int MB,
    int S, int tiles_per_split, int total_tiles, int kc, int cap, uint64_t* __restrict__ slots,
    int32_t* __restrict__ counts) {
    __shared__ uint4 Ks[KT * ROW_UNITS];
    __shared__ uint4 Qs[QB * ROW_UNITS];
    __shared__ float Kn[KT];
    __shared__ float Ksc[KT];
    __shared__ uint32_t hist_all[4][256];

    const int t = threadIdx.x;
    const int l = t & 63;
    const int w = t >> 6;
    const int qb = blockIdx.x % MB;
    const int split = blockIdx.x / MB;
    const int tile_begin = split * tiles_per_split;
    const int tile_end = min(total_tiles, tile_begin + tiles_per_split);
    uint32_t* hist = hist_all[w];

    // Rows of the query tile this thread loads (4 rows, unit t & 7).
    int64_t qrow_off[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int r = (t >> 3) + 32 * i;
        int64_t m = (int64_t)qb * QB + r;
        int64_t row = 0;
        if (m < Mb) row = qids ? (int64_t)qids[m0 + m] : (m0 + m);
        qrow_off[i] = row * row_units + (t & 7);
    }

    // Per-lane query state (lanes l and l+32 share query 32w + l%32).
    const int qloc = 32 * w + (l & 31);
    const int64_t mq = (int64_t)qb * QB + qloc;
    const bool qvalid = mq < Mb;
    const int64_t self = qvalid ? (qids ? (int64_t)qids[m0 + mq] : (m0 + mq)) : -1;
    const float qscale = (P == ATSNE_PREC_FP8_E4M3 && qvalid) ? scales[self] : 1.0f;
    uint64_t* myslot = slots + ((size_t)(qvalid ? mq : 0) * S + split) * (size_t)cap;
    float tau = qvalid ? INFINITY : -INFINITY;
    int count = 0;

    uint4 pk[8], pq[4];
    auto load_chunk = [&](int tile, int c) {
        const uint4* kbase = Xp + (int64_t)tile * KT * row_units + (int64_t)c * CHUNK_UNITS;
#pragma unroll
        for (int i = 0; i < 8; ++i) pk[i] = kbase[(int64_t)((t >> 3) + 32 * i) * row_units + (t & 7)];
#pragma unroll
        for (int i = 0; i < 4; ++i) pq[i] = Xp[qrow_off[i] + (int64_t)c * CHUNK_UNITS];
    };

    if (tile_begin < tile_end) load_chunk(tile_begin, 0);
    for (int tile = tile_begin; tile < tile_end; ++tile) {
        f32x16 acc[NKB];
#pragma unroll
        for (int b = 0; b < NKB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

        for (int c = 0; c < n_chunks; ++c) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 8; ++i) Ks[((t >> 3) + 32 * i) * ROW_UNITS + (t & 7)] = pk[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) Qs[((t >> 3) + 32 * i) * ROW_UNITS + (t & 7)] = pq[i];
            if (c == 0) {
                Kn[t] = norms[(int64_t)tile * KT + t];
                if (P == ATSNE_PREC_FP8_E4M3) Ksc[t] = scales[(int64_t)tile * KT + t];
            }
            __syncthreads();
            if (c + 1 < n_chunks)
                load_chunk(tile, c + 1);
            else if (tile + 1 < tile_end)
                load_chunk(tile + 1, 0);

            uint4 bq[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) bq[i] = Qs[qloc * ROW_UNITS + chunk_unit<P>(l, i)];
#pragma unroll
            for (int b = 0; b < NKB; ++b) {
                uint4 ak[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ak[i] = Ks[(32 * b + (l & 31)) * ROW_UNITS + chunk_unit<P>(l, i)];
                acc[b] = mfma_chunk<P>(acc[b], ak, bq);
            }
        }

        // ---- epilogue: make room, then filter this tile's candidates ----
        {
            uint64_t need = ballot(count > cap - KT) & 0xffffffffull;
            while (need) {
                int q = __ffsll((unsigned long long)need) - 1;
                need &= need - 1;
                int cnt_q = __shfl(count, q, WAVE);
                uint64_t* sq = slots + ((size_t)((int64_t)qb * QB + 32 * w + q) * S + split) * (size_t)cap;
                uint64_t kstar = shrink_slot(sq, cnt_q, kc, hist);
                if ((l & 31) == q) {
                    count = kc;
                    tau = key_dist(kstar);
                }
            }
        }
        const int64_t key0 = (int64_t)tile * KT;
#pragma unroll
        for (int b = 0; b < NKB; ++b) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int kl = 32 * b + 8 * g + 4 * (l >> 5);
                float4 nj = *reinterpret_cast<const float4*>(&Kn[kl]);
                float4 sj = make_float4(1.f, 1.f, 1.f, 1.f);
                if (P == ATSNE_PREC_FP8_E4M3) sj = *reinterpret_cast<const float4*>(&Ksc[kl]);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t key = key0 + kl + e;
                    const float nje = e == 0 ? nj.x : e == 1 ? nj.y : e == 2 ? nj.z : nj.w;
                    float s = acc[b][4 * g + e];
                    if (P == ATSNE_PREC_FP8_E4M3) {
                        const float sje = e == 0 ? sj.x : e == 1 ? sj.y : e == 2 ? sj.z : sj.w;
                        s *= qscale * sje;
                    }
                    const float d = fmaf(-2.0f, s, nje);
                    const bool pass = (d < tau) && (key < N) && (key != self);
                    const uint64_t m = ballot(pass);
                    if (m) {
                        const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
                        const int q = l & 31;
                        const int bl = (lo >> q) & 1, bh = (hi >> q) & 1;
                        const int pos = count + ((l >> 5) ? bl : 0);
                        if (pass) myslot[pos] = pack_key(d, (int32_t)key);
                        count += bl + bh;
                    }
                }
            }
        }
    }

    // Final shrink so each slot hands at most kc candidates to knn_select.
    {
        uint64_t need = ballot(count > kc) & 0xffffffffull;
        while (need) {
            int q = __ffsll((unsigned long long)need) - 1;
            need &= need - 1;
            int cnt_q = __shfl(count, q, WAVE);
            uint64_t* sq = slots + ((size_t)((int64_t)qb * QB + 32 * w + q) * S + split) * (size_t)cap;
            (void)shrink_slot(sq, cnt_q, kc, hist);
            if ((l & 31) == q) count = kc;
        }
    }
    if (qvalid && l < 32) counts[mq * S + split] = count;
}

// ---------------------------------------------------------------------------
// Row finalisation shared by knn_select and knn_scan: sort the n candidates
// held in LDS (index cj, FP32 distance cd) by (d, j), FP64 re-rank when the
// k-th/(k+1)-th gap is below FP32 resolution, write the row.
// ---------------------------------------------------------------------------
constexpr float TIE_REL = 8e-6f;  // > worst-case relative error of the FP32 direct difference used here

__device__ void finalize_row(const float* __restrict__ X, int64_t ld, int32_t D, const float* __restrict__ xq_g,
                             int n, int k, int32_t* cj, float* cd, uint64_t* sorted, double* dd,
                             int32_t* __restrict__ out_idx, float* __restrict__ out_d2, uint8_t* flag_out,
                             uint8_t extra_flags) {
    const int l = lane_id();
    // rank by counting on the 64-bit key (d, j); keys are distinct
    for (int c = l; c < n; c += WAVE) {
        uint64_t kc_ = pack_key(cd[c], cj[c]);
        int r = 0;
        for (int o = 0; o < n; ++o) r += pack_key(cd[o], cj[o]) < kc_;
        sorted[r] = kc_;
    }
    wave_sync();
    uint8_t fl = extra_flags;
    bool tie = false;
    if (n > k) {
        float dk = key_dist(sorted[k - 1]), dk1 = key_dist(sorted[k]);
        tie = (dk1 - dk) <= TIE_REL * fabsf(dk);
    }
    if (tie) {
        // FP64 direct differences for every candidate, then rank by (d64, j).
        for (int c = 0; c < n; ++c) {
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
        for (int c = l; c < n; c += WAVE) {
            double dc = dd[c];
            int32_t jc = key_index(sorted[c]);
            int r = 0;
            for (int o = 0; o < n; ++o) {
                double dox = dd[o];
                int32_t jo = key_index(sorted[o]);
                r += (dox < dc) || (dox == dc && jo < jc);
            }
            if (r < k) {
                out_idx[r] = jc;
                out_d2[r] = (float)dc;
            }
        }
        fl |= ATSNE_FLAG_FP64_RERANKED;
    } else {
        for (int r = l; r < k; r += WAVE) {
            out_idx[r] = key_index(sorted[r]);
            out_d2[r] = key_dist(sorted[r]);
        }
    }
    if (flag_out && l == 0) *flag_out = fl;
}

// Exact FP32 direct-difference distances from query q to the n candidates in
// cj (wave-parallel over dimensions, butterfly reduction), into cd.
__device__ void direct_distances(const float* __restrict__ X, int64_t ld, int32_t D, const float* __restrict__ xq,
                                 int n, const int32_t* cj, float* cd) {
    const int l = lane_id();
    int c = 0;
    for (; c + 4 <= n; c += 4) {
        const float* x0 = X + (int64_t)cj[c] * ld;
        const float* x1 = X + (int64_t)cj[c + 1] * ld;
        const float* x2 = X + (int64_t)cj[c + 2] * ld;
        const float* x3 = X + (int64_t)cj[c + 3] * ld;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        for (int d = l; d < D; d += WAVE) {
            float q = xq[d];
            float t0 = q - x0[d], t1 = q - x1[d], t2 = q - x2[d], t3 = q - x3[d];
            a0 = fmaf(t0, t0, a0);
            a1 = fmaf(t1, t1, a1);
            a2 = fmaf(t2, t2, a2);
            a3 = fmaf(t3, t3, a3);
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        a3 = wave_sum(a3);
        if (l == 0) {
            cd[c] = a0;
            cd[c + 1] = a1;
            cd[c + 2] = a2;
            cd[c + 3] = a3;
        }
    }
    for (; c < n; ++c) {
        const float* x0 = X + (int64_t)cj[c] * ld;
        float a0 = 0.f;
        for (int d = l; d < D; d += WAVE) {
            float t0 = xq[d] - x0[d];
            a0 = fmaf(t0, t0, a0);
        }
        a0 = wave_sum(a0);
        if (l == 0) cd[c] = a0;
    }
    wave_sync();
}

constexpr int MAX_KC = 1024;

// knn_select: one wave (workgroup of 64) per query.
template <int P>
__global__ __launch_bounds__(64) void knn_select(
    const float* __restrict__ X, int64_t ld, int32_t D, int64_t N, const int32_t* __restrict__ qids, int64_t m0,
    int64_t Mb, int S, int cap, int kc, int k, const uint64_t* __restrict__ slots, const int32_t* __restrict__ counts,
    const float* __restrict__ norms, const uint32_t* __restrict__ nmax_bits, int32_t Dp,
    int32_t* __restrict__ nbr_idx, float* __restrict__ nbr_d2, uint8_t* __restrict__ flags,
    int32_t* __restrict__ scan_list, int32_t* __restrict__ scan_count) {
    __shared__ uint32_t hist[256];
    __shared__ int32_t cj[MAX_KC];
    __shared__ float cd[MAX_KC];
    __shared__ uint64_t sorted[MAX_KC];
    __shared__ double dd[MAX_KC];
    __shared__ int32_t ncand;
    const int l = lane_id();
    const int64_t m = blockIdx.x;
    if (m >= Mb) return;
    const int64_t q = qids ? (int64_t)qids[m0 + m] : (m0 + m);
    const int32_t* cnt = counts + m * S;
    const uint64_t* base = slots + (size_t)m * S * (size_t)cap;

    int total = 0;
    for (int s = 0; s < S; ++s) total += cnt[s];
    const int take = min(kc, total);
    auto each = [&](auto f) {
        for (int s = 0; s < S; ++s) {
            const uint64_t* sl = base + (size_t)s * cap;
            const int c = cnt[s];
            for (int i = l; i < c; i += WAVE) f(sl[i]);
        }
    };
    uint64_t kstar;
    if (take < total) {
        kstar = wave_select(each, (uint32_t)take, hist);
    } else {
        // every entry is a candidate: the threshold is the largest key held
        uint64_t mx = 0;
        each([&](uint64_t key) { mx = key > mx ? key : mx; });
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            uint64_t other = shfl64(mx, l ^ o);
            mx = other > mx ? other : mx;
        }
        kstar = mx;
    }
    if (l == 0) ncand = 0;
    wave_sync();
    each([&](uint64_t key) {
        if (key <= kstar) {
            int p = atomicAdd(&ncand, 1);
            cj[p] = key_index(key);
        }
    });
    wave_sync();
    const int n = ncand;
    const float* xq = X + q * ld;
    direct_distances(X, ld, D, xq, n, cj, cd);

    uint8_t extra = 0;
    if (P == ATSNE_PREC_FP32 && take < (int)(N - 1)) {
        // Certificate: every non-candidate j has d'_j >= d'(kstar); its true
        // distance is at least d'(kstar) + n_q - E, E bounding the FP32
        // contraction error.  If that exceeds the k-th exact distance (with
        // the direct-difference error), no non-candidate can be a neighbour.
        // |fl(n_j) - n_j| + 2|fl(S_qj) - S_qj| + |fl(n_q) - n_q| <= gam (n_j + 2 sqrt(n_q n_j) + n_q)
        // with gam = (Dp + 2) u for sums of Dp products, n_j <= n_max.
        const float u = 5.9604645e-8f;
        const float nq = norms[q];
        const float nmax = __uint_as_float(*nmax_bits);
        const float gam = 1.05f * (float)(Dp + 2) * u;
        const float sq = sqrtf(nq) + sqrtf(nmax);
        float dk = 0.f;
        // k-th smallest exact distance among the candidates
        for (int c = l; c < n; c += WAVE) {
            uint64_t kc_ = pack_key(cd[c], cj[c]);
            int r = 0;
            for (int o = 0; o < n; ++o) r += pack_key(cd[o], cj[o]) < kc_;
            if (r == k - 1) sorted[0] = kc_;
        }
        wave_sync();
        dk = key_dist(sorted[0]);
        wave_sync();
        const float dthr = key_dist(kstar);
        const float E = gam * (sq * sq) + 2.0f * u * (fabsf(dthr) + nq);
        const float lb = dthr + nq - E;
        if (!(lb > dk * (1.0f + 2.0f * TIE_REL))) {
            extra = ATSNE_FLAG_EXACT_SCAN;
            if (l == 0) {
                int p = atomicAdd(scan_count, 1);
                scan_list[p] = (int32_t)m;
            }
        }
    }
    finalize_row(X, ld, D, xq, n, k, cj, cd, sorted, dd, nbr_idx + m * k, nbr_d2 + m * k,
                 flags ? flags + m : nullptr, extra);
}

// knn_scan: exact FP32 linear scan for rows whose candidate margin was not
// certified.  One workgroup (4 waves) per queued row, persistent over the
// queue; every workgroup exits once the queue is drained.  Each wave scans
// the keys j = w, w+4, ... in increasing order with the same direct-difference
// arithmetic as knn_select, keeps (d, j) keys below its running threshold in
// an LDS region and shrinks the region to its best SCAN_KEEP keys when full;
// keys arrive in increasing j, so after a shrink a strict d < tau filter is
// exact.  The four regions are merged at the end.
constexpr int SCAN_REGION = 1024;
__global__ __launch_bounds__(256) void knn_scan(const float* __restrict__ X, int64_t ld, int32_t D, int64_t N,
                                                const int32_t* __restrict__ qids, int64_t m0, int k, int keep,
                                                const int32_t* __restrict__ scan_list,
                                                const int32_t* __restrict__ scan_count, int32_t* __restrict__ cursor,
                                                int32_t* __restrict__ nbr_idx, float* __restrict__ nbr_d2,
                                                uint8_t* __restrict__ flags) {
    __shared__ uint64_t region[4][SCAN_REGION];
    __shared__ uint32_t hist_all[4][256];
    __shared__ int32_t rcount[4];
    __shared__ int32_t cj[MAX_KC];
    __shared__ float cd[MAX_KC];
    __shared__ uint64_t sorted[MAX_KC];
    __shared__ double dd[MAX_KC];
    __shared__ int32_t item;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int nq = *scan_count;
    uint64_t* reg = region[w];
    uint32_t* hist = hist_all[w];
    for (;;) {
        __syncthreads();
        if (t == 0) item = atomicAdd(cursor, 1);
        __syncthreads();
        const int it = item;
        if (it >= nq) break;
        const int64_t m = scan_list[it];
        const int64_t q = qids ? (int64_t)qids[m0 + m] : (m0 + m);
        const float* xq = X + q * ld;
        // The current k-th exact distance bounds the true k-th from above.
        float tau = nbr_d2[m * k + (k - 1)];
        bool strict = false;
        int cnt = 0;
        for (int64_t j0 = w; j0 < N; j0 += 16) {
            float a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = j0 + 4 * u;
                float acc = 0.f;
                if (j < N) {
                    const float* xj = X + j * ld;
                    for (int d = l; d < D; d += WAVE) {
                        float tt = xq[d] - xj[d];
                        acc = fmaf(tt, tt, acc);
                    }
                }
                a[u] = wave_sum(acc);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = j0 + 4 * u;
                const bool pass = j < N && j != q && (strict ? (a[u] < tau) : (a[u] <= tau));
                if (pass) {
                    if (l == 0) reg[cnt] = pack_key(a[u], (int32_t)j);
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
        if (l == 0) rcount[w] = cnt;
        __syncthreads();
        if (w == 0) {
            const int tot = rcount[0] + rcount[1] + rcount[2] + rcount[3];
            auto each = [&](auto f) {
                for (int r = 0; r < 4; ++r)
                    for (int i = l; i < rcount[r]; i += WAVE) f(region[r][i]);
            };
            const int take = min(keep, tot);
            uint64_t kstar = ~0ull;
            if (take < tot) kstar = wave_select(each, (uint32_t)take, hist);
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
            if (n >= k)
                finalize_row(X, ld, D, xq, n, k, cj, cd, sorted, dd, nbr_idx + m * k, nbr_d2 + m * k,
                             flags ? flags + m : nullptr, ATSNE_FLAG_EXACT_SCAN);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct KnnPlan {
    int prec;
    int64_t N, M, N_pad;
    int32_t D, Dp;
    int k, kc, cap;
    int n_chunks, total_tiles;
    int64_t Mb;  // queries per batch
    int MB, S, tiles_per_split;
    size_t b_xp, b_norm, b_scale, b_misc, b_slots, b_counts, b_list;
    size_t total;
};

static int default_kcand(int prec, int k) {
    if (prec == ATSNE_PREC_FP32) return k + std::max(32, k / 2);
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

static atsne_status make_plan(int64_t N, int64_t M, int32_t D, int prec, int k, int k_cand, KnnPlan& p) {
    ATSNE_REQUIRE(prec == ATSNE_PREC_FP32 || prec == ATSNE_PREC_BF16 || prec == ATSNE_PREC_FP8_E4M3,
                  ATSNE_E_INVALID_ARG, "unknown precision %d", prec);
    ATSNE_REQUIRE(N >= 2 && N < (1ll << 31) - KT, ATSNE_E_INVALID_ARG, "N=%lld out of range", (long long)N);
    ATSNE_REQUIRE(M >= 0 && M < (1ll << 31), ATSNE_E_INVALID_ARG, "M=%lld out of range", (long long)M);
    ATSNE_REQUIRE(D >= 1 && D <= 65536, ATSNE_E_INVALID_ARG, "D=%d out of range", D);
    ATSNE_REQUIRE(k >= 1 && k <= N - 1, ATSNE_E_K_RANGE, "k=%d must be in [1, N-1=%lld]", k, (long long)(N - 1));
    int kc = k_cand > 0 ? k_cand : default_kcand(prec, k);
    kc = (int)std::min<int64_t>(kc, N - 1);
    ATSNE_REQUIRE(kc >= k && kc <= MAX_KC, ATSNE_E_K_RANGE, "k_cand=%d must be in [k=%d, %d]", kc, k, MAX_KC);
    ATSNE_REQUIRE(k <= 1000, ATSNE_E_K_RANGE, "k=%d above the supported maximum 1000", k);
    p.prec = prec;
    p.N = N;
    p.M = M;
    p.D = D;
    p.k = k;
    p.kc = kc;
    const int ce = chunk_elems(prec);
    p.Dp = (int32_t)(ceil_div(D, ce) * ce);
    p.n_chunks = p.Dp / ce;
    p.N_pad = ceil_div(N, KT) * KT;
    p.total_tiles = (int)(p.N_pad / KT);
    p.cap = (int)align_up((size_t)(kc + KT + std::max(kc, 128)), 64);
    // Batch the queries so the candidate slots stay within ~2 GiB.
    const int cu = device_cu_count();
    const int slots_avail = cu;  // one 256-thread tile workgroup per CU
    int64_t MBall = ceil_div(std::max<int64_t>(M, 1), QB);
    int S = pick_splits(MBall, p.total_tiles, slots_avail);
    const size_t slot_bytes = (size_t)p.cap * 8;
    int64_t max_rows = (int64_t)((size_t)2 << 30) / (slot_bytes * S);
    max_rows = std::max<int64_t>(QB, max_rows / QB * QB);
    p.Mb = std::min<int64_t>(std::max<int64_t>(M, 1), max_rows);
    p.MB = (int)ceil_div(p.Mb, QB);
    if (p.Mb < M) S = pick_splits(p.MB, p.total_tiles, slots_avail);
    p.S = S;
    p.tiles_per_split = (int)ceil_div(p.total_tiles, S);
    p.S = (int)ceil_div(p.total_tiles, p.tiles_per_split);
    p.b_xp = (size_t)p.N_pad * p.Dp * elem_bytes(prec);
    p.b_norm = (size_t)p.N_pad * 4;
    p.b_scale = (size_t)p.N_pad * 4;
    p.b_misc = 256;
    p.b_slots = (size_t)p.MB * QB * p.S * slot_bytes;
    p.b_counts = (size_t)p.MB * QB * p.S * 4;
    p.b_list = (size_t)std::max<int64_t>(M, 1) * 4;
    Arena a;
    a.take<char>(p.b_xp);
    a.take<char>(p.b_norm);
    a.take<char>(p.b_scale);
    a.take<char>(p.b_misc);
    a.take<char>(p.b_slots);
    a.take<char>(p.b_counts);
    a.take<char>(p.b_list);
    p.total = a.used;
    return ATSNE_OK;
}

template <int P>
static atsne_status run_knn(const KnnPlan& p, const float* X, int64_t ld, const int32_t* qids, int32_t* nbr_idx,
                            float* nbr_d2, uint8_t* flags, void* wsp, hipStream_t st) {
    Arena a(wsp, p.total);
    void* Xp = a.take<char>(p.b_xp);
    float* norms = a.take<float>(p.N_pad);
    float* scales = a.take<float>(p.N_pad);
    int32_t* misc = a.take<int32_t>(64);
    uint64_t* slots = reinterpret_cast<uint64_t*>(a.take<char>(p.b_slots));
    int32_t* counts = a.take<int32_t>((size_t)p.MB * QB * p.S);
    int32_t* scan_list = a.take<int32_t>(std::max<int64_t>(p.M, 1));
    uint32_t* nmax_bits = reinterpret_cast<uint32_t*>(misc);
    int32_t* scan_count = misc + 1;
    int32_t* cursor = misc + 2;

    ATSNE_HIP(hipMemsetAsync(misc, 0, 256, st));
    {
        ProfScope ps_("knn_prep", st);
        knn_prep<P><<<dim3((unsigned)ceil_div(p.N_pad, 4)), dim3(256), 0, st>>>(
            X, p.N, p.D, ld, p.N_pad, p.Dp, Xp, norms, scales, nmax_bits);
        ATSNE_LAUNCH_CHECK();
    }
    const int64_t row_units = (int64_t)p.Dp * elem_bytes(P) / 16;
    for (int64_t m0 = 0; m0 < p.M; m0 += p.Mb) {
        const int64_t Mb = std::min<int64_t>(p.Mb, p.M - m0);
        const int MB = (int)ceil_div(Mb, QB);
        {
        ProfScope ps_("knn_tile", st);
        knn_tile<P><<<dim3((unsigned)(MB * p.S)), dim3(TILE_THREADS), 0, st>>>(
            reinterpret_cast<const uint4*>(Xp), row_units, p.n_chunks, norms, scales, p.N, qids, m0, Mb, MB, p.S,
            p.tiles_per_split, p.total_tiles, p.kc, p.cap, slots, counts);
        ATSNE_LAUNCH_CHECK();
        }
        {
        ProfScope ps_("knn_select", st);
        knn_select<P><<<dim3((unsigned)Mb), dim3(64), 0, st>>>(
            X, ld, p.D, p.N, qids, m0, Mb, p.S, p.cap, p.kc, p.k, slots, counts, norms, nmax_bits, p.Dp,
            nbr_idx + m0 * p.k, nbr_d2 + m0 * p.k, flags ? flags + m0 : nullptr, scan_list, scan_count);
        ATSNE_LAUNCH_CHECK();
        }
        if (P == ATSNE_PREC_FP32) {
            const int grid = (int)std::min<int64_t>(Mb, 4 * (int64_t)device_cu_count());
            ProfScope ps_("knn_scan", st);
            knn_scan<<<dim3((unsigned)grid), dim3(256), 0, st>>>(X, ld, p.D, p.N, qids, m0, p.k,
                                                                  std::min(p.k + 32, SCAN_REGION - 24), scan_list,
                                                                  scan_count, cursor, nbr_idx + m0 * p.k,
                                                                  nbr_d2 + m0 * p.k, flags ? flags + m0 : nullptr);
            ATSNE_LAUNCH_CHECK();
            if (m0 + p.Mb < p.M) ATSNE_HIP(hipMemsetAsync(misc + 1, 0, 8, st));
        }
    }
    return ATSNE_OK;
}

static atsne_status knn_impl(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* qids, int64_t M,
                             atsne_precision prec, int32_t k, int32_t k_cand, int32_t* nbr_idx, float* nbr_d2,
                             uint8_t* flags, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    ATSNE_REQUIRE(X && nbr_idx && nbr_d2, ATSNE_E_INVALID_ARG, "null X or output pointer");
    ATSNE_REQUIRE(ld >= D, ATSNE_E_INVALID_ARG, "ld=%lld < D=%d", (long long)ld, D);
    KnnPlan p;
    ATSNE_TRY(make_plan(N, M, D, (int)prec, k, k_cand, p));
    if (M == 0) return ATSNE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch scr;
    ATSNE_TRY(scr.acquire(ws, ws_bytes, p.total, st));
    switch (prec) {
        case ATSNE_PREC_FP32:
            return run_knn<ATSNE_PREC_FP32>(p, X, ld, qids, nbr_idx, nbr_d2, flags, scr.ptr, st);
        case ATSNE_PREC_BF16:
            return run_knn<ATSNE_PREC_BF16>(p, X, ld, qids, nbr_idx, nbr_d2, flags, scr.ptr, st);
        case ATSNE_PREC_FP8_E4M3:
            return run_knn<ATSNE_PREC_FP8_E4M3>(p, X, ld, qids, nbr_idx, nbr_d2, flags, scr.ptr, st);
    }
    return ATSNE_E_INVALID_ARG;
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
                                  int32_t k_cand, int32_t* nbr_idx, float* nbr_d2, uint8_t* flags, void* ws,
                                  size_t ws_bytes, void* stream) {
    return atsne::knn_impl(X, N, D, ld, nullptr, N, prec, k, k_cand, nbr_idx, nbr_d2, flags, ws, ws_bytes, stream);
}

extern "C" atsne_status atsne_knn_subset(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* query_ids,
                                         int64_t M, atsne_precision prec, int32_t k, int32_t k_cand, int32_t* nbr_idx,
                                         float* nbr_d2, uint8_t* flags, void* ws, size_t ws_bytes, void* stream) {
    ATSNE_REQUIRE(query_ids || M == 0, ATSNE_E_INVALID_ARG, "null query_ids");
    return atsne::knn_impl(X, N, D, ld, query_ids, M, prec, k, k_cand, nbr_idx, nbr_d2, flags, ws, ws_bytes, stream);
}
