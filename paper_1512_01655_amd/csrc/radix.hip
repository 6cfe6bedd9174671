// Device-wide ascending sort of 64-bit keys, optionally carrying a 32-bit
// value each: the transpose of the conditional pattern in the
// symmetrisation (keys (column, row), values p), the density order of the
// refinement orderings (keys (sigma rank, index)) and the cluster-sorted
// corpus of the approximate search (keys (cluster, index)).
//
// Least-significant-digit radix sort over the caller's bit range
// [begin_bit, end_bit) (keys are equal on the other bits), with digits of up
// to 10 bits chosen so the range takes as few passes as possible.  A pass is
//   radix_hist    per tile of keys, the count of each digit (LDS histogram)
//   radix_scan_d  per digit, exclusive scan of its tiles' counts, in place,
//                 and the digit's total; radix_scan_t then scans the totals
//   radix_move    stable scatter: each tile, chunk by chunk (4096 keys held
//                 in registers, 16 per thread), ranks its keys by wave
//                 multi-split, stages the chunk in LDS in (digit, input)
//                 order, a quarter at a time, and writes it out so that
//                 consecutive lanes store consecutive positions of a digit,
//                 after the keys of smaller digits, of earlier tiles and of
//                 earlier keys of the tile
// Keys are moved, never compared, so the sort is exact and deterministic.
#include <algorithm>

#include "knn_internal.h"
#include "wave.h"

namespace atsne {

constexpr int RADIX_CHUNK = 4096;      // keys per chunk: 256 threads x 16
constexpr int RADIX_PER_THREAD = 16;
constexpr int RADIX_MAX_BINS = 1024;   // digits of up to 10 bits
constexpr int RADIX_MAX_TILES = 4096;  // tiles per sort (a tile is whole chunks)
constexpr int RADIX_STAGE = 1024;      // slots staged in LDS at a time (a quarter chunk)

struct RadixGeom {
    int64_t n;
    int64_t n_tiles, tile;  // tile = keys per tile, a multiple of RADIX_CHUNK
};

static RadixGeom radix_geom(int64_t n) {
    RadixGeom g;
    g.n = n;
    const int64_t chunks = std::max<int64_t>(1, ceil_div(n, RADIX_CHUNK));
    const int64_t per = ceil_div(chunks, RADIX_MAX_TILES);
    g.tile = per * RADIX_CHUNK;
    g.n_tiles = std::max<int64_t>(1, ceil_div(n, g.tile));
    return g;
}

__device__ __forceinline__ uint32_t radix_digit(uint64_t k, int shift, int bits) {
    return (uint32_t)(k >> shift) & ((1u << bits) - 1u);
}

__global__ __launch_bounds__(256) void radix_hist(const uint64_t* __restrict__ in, RadixGeom g, int shift, int bits,
                                                  uint32_t* __restrict__ cnt) {
    __shared__ uint32_t h[RADIX_MAX_BINS];
    const int t = threadIdx.x;
    const int bins = 1 << bits;
    for (int b = t; b < bins; b += 256) h[b] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * g.tile, e1 = std::min(g.n, e0 + g.tile);
    for (int64_t e = e0 + t; e < e1; e += 256) atomicAdd(&h[radix_digit(in[e], shift, bits)], 1u);
    __syncthreads();
    for (int b = t; b < bins; b += 256) cnt[(int64_t)b * g.n_tiles + blockIdx.x] = h[b];
}

// One workgroup per digit: exclusive scan of its n_tiles (<= 4096) counts,
// four per thread, in place; the digit's total to tot.
__global__ __launch_bounds__(1024) void radix_scan_d(uint32_t* __restrict__ cnt, int64_t n_tiles,
                                                    uint32_t* __restrict__ tot) {
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    uint32_t* c = cnt + (int64_t)blockIdx.x * n_tiles;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t x = 4 * (int64_t)t + q;
        v[q] = x < n_tiles ? c[x] : 0u;
        s += v[q];
    }
    const uint32_t incl = wave_incl_scan(s);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t run = incl - s;
    for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t x = 4 * (int64_t)t + q;
        if (x < n_tiles) c[x] = run;
        run += v[q];
    }
    if (t == 1023) tot[blockIdx.x] = run;
}

// Exclusive scan of the bins (<= 1024) digit totals in place, one workgroup.
__global__ __launch_bounds__(1024) void radix_scan_t(uint32_t* __restrict__ tot, int bins) {
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const uint32_t v = t < bins ? tot[t] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t run = incl - v;
    for (int i = 0; i < w; ++i) run += wsum[i];
    if (t < bins) tot[t] = run;
}

__global__ __launch_bounds__(256) void radix_move(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                  uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, RadixGeom g,
                                                  int shift, int bits, const uint32_t* __restrict__ cnt,
                                                  const uint32_t* __restrict__ doff) {
    __shared__ uint32_t start[RADIX_MAX_BINS];    // tile's next output position of each digit
    __shared__ uint32_t wcnt[4][RADIX_MAX_BINS];  // per wave: its count of each digit, then its offset within the digit
    __shared__ uint32_t cofs[RADIX_MAX_BINS];     // per digit: its count in the chunk, then its first staged slot
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t sk[RADIX_STAGE];          // a quarter of the chunk staged in (digit, input) order
    __shared__ uint32_t sv[RADIX_STAGE];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int bins = 1 << bits;
    for (int b = t; b < bins; b += 256) start[b] = doff[b] + cnt[(int64_t)b * g.n_tiles + blockIdx.x];
    const int64_t e0 = (int64_t)blockIdx.x * g.tile, e1 = std::min(g.n, e0 + g.tile);
    for (int64_t c0 = e0; c0 < e1; c0 += RADIX_CHUNK) {
        // wave w takes the chunk's keys [1024 w, 1024 (w + 1)), lane l of round
        // r holding key 1024 w + 64 r + l: waves in order, then rounds, then lanes
        // is the chunk's input order
        const int64_t wb = c0 + 1024 * w;
        uint64_t k[RADIX_PER_THREAD];
        uint32_t v[RADIX_PER_THREAD];
#pragma unroll
        for (int r = 0; r < RADIX_PER_THREAD; ++r) {
            const int64_t e = wb + 64 * r + l;
            k[r] = e < e1 ? kin[e] : 0;
            v[r] = (vin && e < e1) ? vin[e] : 0u;
        }
        for (int b = l; b < bins; b += WAVE) wcnt[w][b] = 0;
        wave_sync();
        // each key's place among the wave's earlier keys of its digit
        uint32_t pos[RADIX_PER_THREAD];
#pragma unroll
        for (int r = 0; r < RADIX_PER_THREAD; ++r) {
            const bool act = wb + 64 * r + l < e1;
            const uint32_t d = radix_digit(k[r], shift, bits);
            uint64_t peers = ballot(act);
            for (int b = 0; b < bits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = ballot(act && bit);
                peers &= bit ? m : ~m;
            }
            const int rank = __popcll(peers & lanemask_lt()), count = __popcll(peers);
            pos[r] = act ? wcnt[w][d] + (uint32_t)rank : 0u;
            wave_sync();
            if (act && rank == count - 1) wcnt[w][d] += (uint32_t)count;
            wave_sync();
        }
        __syncthreads();
        // per digit: the waves' offsets within the digit, and its chunk count
        for (int b = t; b < bins; b += 256) {
            uint32_t a = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t x = wcnt[u][b];
                wcnt[u][b] = a;
                a += x;
            }
            cofs[b] = a;
        }
        __syncthreads();
        // exclusive scan of the chunk counts over the digits (thread t holds
        // digits 4t .. 4t + 3): each digit's first slot in the staged chunk
        uint32_t c4[4], s = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = 4 * t + u;
            c4[u] = b < bins ? cofs[b] : 0u;
            s += c4[u];
        }
        const uint32_t incl = wave_incl_scan(s);
        if (l == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t run = incl - s;
        for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = 4 * t + u;
            if (b < bins) cofs[b] = run;
            run += c4[u];
        }
        __syncthreads();
        // each key's slot in the chunk's (digit, input) order: its stable
        // rank in the chunk, below the chunk's key count
#pragma unroll
        for (int r = 0; r < RADIX_PER_THREAD; ++r) {
            const uint32_t d = radix_digit(k[r], shift, bits);
            pos[r] = wb + 64 * r + l < e1 ? cofs[d] + wcnt[w][d] + pos[r] : (uint32_t)RADIX_CHUNK;
        }
        // a quarter of the slots at a time: stage them in LDS, then write
        // them out so that consecutive slots of a digit go to consecutive
        // positions, after the digit's keys of earlier chunks
        const int n_c = (int)std::min<int64_t>(RADIX_CHUNK, e1 - c0);
        for (int q0 = 0; q0 < n_c; q0 += RADIX_STAGE) {
#pragma unroll
            for (int r = 0; r < RADIX_PER_THREAD; ++r) {
                const uint32_t s = pos[r] - (uint32_t)q0;  // wraps above the quarter when below it
                if (s < (uint32_t)RADIX_STAGE) {
                    sk[s] = k[r];
                    if (vin) sv[s] = v[r];
                }
            }
            __syncthreads();
            const int q1 = std::min(n_c, q0 + RADIX_STAGE);
            for (int q = q0 + t; q < q1; q += 256) {
                const uint64_t key = sk[q - q0];
                const uint32_t d = radix_digit(key, shift, bits);
                const uint32_t p = start[d] + (uint32_t)q - cofs[d];
                if (p < (uint64_t)g.n) {  // always true: the guard keeps every store in bounds
                    kout[p] = key;
                    if (vout) vout[p] = sv[q - q0];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = 4 * t + u;
            if (b < bins) start[b] += c4[u];
        }
        __syncthreads();
    }
}

size_t sort_u64_temp_bytes(int64_t n) {
    const RadixGeom g = radix_geom(n);
    Arena a;
    a.take<uint64_t>(std::max<int64_t>(n, 1));                   // ping-pong keys
    a.take<uint32_t>(std::max<int64_t>(n, 1));                   // ping-pong values
    a.take<uint32_t>((size_t)RADIX_MAX_BINS * g.n_tiles);        // per (digit, tile) counts / offsets
    a.take<uint32_t>(RADIX_MAX_BINS);                            // digit offsets
    return a.used;
}

atsne_status sort_pairs_u64(void* tmp, size_t tmp_bytes, const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                            uint32_t* vout, int64_t n, hipStream_t st, int begin_bit, int end_bit) {
    if (n == 0) return ATSNE_OK;
    ATSNE_REQUIRE(tmp_bytes >= sort_u64_temp_bytes(n), ATSNE_E_NOMEM, "sort scratch too small");
    ATSNE_REQUIRE(0 <= begin_bit && begin_bit < end_bit && end_bit <= 64, ATSNE_E_INVALID_ARG, "bad bit range");
    ATSNE_REQUIRE(n < (int64_t)UINT32_MAX, ATSNE_E_INVALID_ARG, "sort of %lld keys: at most 2^32 - 1",
                  (long long)n);
    ATSNE_REQUIRE((vin == nullptr) == (vout == nullptr), ATSNE_E_INVALID_ARG, "values in and out go together");
    const RadixGeom g = radix_geom(n);
    Arena a(tmp, tmp_bytes);
    uint64_t* kp = a.take<uint64_t>(std::max<int64_t>(n, 1));
    uint32_t* vp = a.take<uint32_t>(std::max<int64_t>(n, 1));
    uint32_t* cnt = a.take<uint32_t>((size_t)RADIX_MAX_BINS * g.n_tiles);
    uint32_t* doff = a.take<uint32_t>(RADIX_MAX_BINS);
    const int total_bits = end_bit - begin_bit;
    const int passes = (total_bits + 9) / 10;
    const int width = (total_bits + passes - 1) / passes;
    // the last pass must land in the output: alternate so that it does
    const uint64_t* ks = kin;
    const uint32_t* vs = vin;
    uint64_t* kb[2] = {passes % 2 ? kout : kp, passes % 2 ? kp : kout};
    uint32_t* vb[2] = {passes % 2 ? vout : (vin ? vp : nullptr), passes % 2 ? (vin ? vp : nullptr) : vout};
    for (int p = 0; p < passes; ++p) {
        const int shift = begin_bit + width * p;
        const int bits = std::min(width, end_bit - shift);
        uint64_t* kd = kb[p % 2];
        uint32_t* vd = vb[p % 2];
        radix_hist<<<dim3((unsigned)g.n_tiles), dim3(256), 0, st>>>(ks, g, shift, bits, cnt);
        ATSNE_LAUNCH_CHECK();
        radix_scan_d<<<dim3(1u << bits), dim3(1024), 0, st>>>(cnt, g.n_tiles, doff);
        ATSNE_LAUNCH_CHECK();
        radix_scan_t<<<dim3(1), dim3(1024), 0, st>>>(doff, 1 << bits);
        ATSNE_LAUNCH_CHECK();
        radix_move<<<dim3((unsigned)g.n_tiles), dim3(256), 0, st>>>(ks, vs, kd, vd, g, shift, bits, cnt, doff);
        ATSNE_LAUNCH_CHECK();
        ks = kd;
        vs = vd;
    }
    return ATSNE_OK;
}

atsne_status sort_u64(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, int64_t n, hipStream_t st,
                      int begin_bit, int end_bit) {
    return sort_pairs_u64(tmp, tmp_bytes, in, nullptr, out, nullptr, n, st, begin_bit, end_bit);
}

}  // namespace atsne
