// Wavefront-level building blocks for gfx950 (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace atsne {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders LDS traffic between the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    uint32_t lo = __shfl((int)(uint32_t)v, src, WAVE);
    uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

// Butterfly sum: every lane ends with the same value, fixed order.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, WAVE);
        if (l >= o) v += t;
    }
    return v;
}

// Error-free sum (Knuth's TwoSum): returns s = fl(a + b) and sets e so that
// s + e = a + b exactly.  Symmetric in a and b.
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// Total order on floats as unsigned integers (negatives included).
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}
// 64-bit key ordering candidates by (distance, index) lexicographically.
__device__ __forceinline__ uint64_t pack_key(float d, int32_t j) {
    return ((uint64_t)f2ord(d) << 32) | (uint32_t)j;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return ord2f((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_index(uint64_t k) { return (int32_t)(uint32_t)k; }

// Stable multi-split of one wave's elements by an 8-bit digit: for each
// active lane, the number of active lanes below it with the same digit
// (rank) and the number of active lanes with that digit (count).  Eight
// ballots narrow the set of peer lanes one digit bit at a time.
__device__ __forceinline__ void wave_digit_rank(bool active, uint32_t digit, int& rank, int& count) {
    uint64_t peers = ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t m = ballot(active && bit);
        peers &= bit ? m : ~m;
    }
    rank = __popcll(peers & lanemask_lt());
    count = __popcll(peers);
}

// Radix selection by one wave: returns the key of 1-based rank `rank` among
// the keys that `for_each` feeds (each lane visits its own share; keys are
// distinct).  8-bit digits from the top; stops as soon as the rank's bucket
// holds a single key.  `hist` is 256 words of LDS private to the wave.
template <class ForEach>
__device__ uint64_t wave_select(ForEach for_each, uint32_t rank, uint32_t* hist) {
    const int l = lane_id();
    uint64_t prefix = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = l; b < 256; b += WAVE) hist[b] = 0;
        wave_sync();
        const uint64_t hi_mask = (shift == 56) ? 0ull : (~0ull << (shift + 8));
        for_each([&](uint64_t k) {
            if ((k & hi_mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
        });
        wave_sync();
        uint32_t h0 = hist[4 * l], h1 = hist[4 * l + 1], h2 = hist[4 * l + 2], h3 = hist[4 * l + 3];
        uint32_t incl = wave_incl_scan(h0 + h1 + h2 + h3);
        uint32_t excl = incl - (h0 + h1 + h2 + h3);
        bool mine = (excl < rank) && (rank <= incl);
        uint32_t bin = 0, before = 0, cnt = 0;
        if (mine) {
            uint32_t a = excl;
            if (rank <= a + h0) { bin = 0; before = a; cnt = h0; }
            else if (rank <= a + h0 + h1) { bin = 1; before = a + h0; cnt = h1; }
            else if (rank <= a + h0 + h1 + h2) { bin = 2; before = a + h0 + h1; cnt = h2; }
            else { bin = 3; before = a + h0 + h1 + h2; cnt = h3; }
            bin += 4 * l;
        }
        int src = __ffsll((unsigned long long)ballot(mine)) - 1;
        bin = __shfl((int)bin, src, WAVE);
        before = __shfl((int)before, src, WAVE);
        cnt = __shfl((int)cnt, src, WAVE);
        prefix |= (uint64_t)bin << shift;
        rank -= before;
        wave_sync();
        if (cnt == 1 && shift > 0) {
            const uint64_t m = ~0ull << shift;
            uint64_t found = 0;
            bool got = false;
            for_each([&](uint64_t k) {
                if ((k & m) == prefix) { found = k; got = true; }
            });
            int s2 = __ffsll((unsigned long long)ballot(got)) - 1;
            return shfl64(found, s2);
        }
    }
    return prefix;
}

}  // namespace atsne
