// Refinement orderings of Sec. 5.1 on gfx950: which points to refine first.
//
//   density: points of sparse regions first, i.e. sigma_i descending
//            (sigma_i = 1/sqrt(2 beta_i), beta from the calibration), ties
//            by index; over all points or a user selection.
//   neighbourhood: the breadth-first visit of the kNN graph (edges i -> j
//            for j in N_i) from a user selection, either by hop count or
//            driven by a priority queue on high-dimensional distance, which
//            is the shortest path length with edge weight ||x_i - x_j||.
//
// The visit is level-synchronous: every round expands one frontier with one
// thread per (frontier point, neighbour slot).  Hop counts are set once by
// compare-and-swap; path lengths are lowered by atomicMin on the IEEE bits
// (non-negative floats order like unsigned integers) and a lowered point
// re-enters the next frontier, so the rounds converge to the least fixed
// point of d_j = min_i fl(d_i + w_ij): the same FP32 values whatever the
// order of the atomics.  The reached points are then sorted by (key, index)
// with a 64-bit radix sort.
#include <climits>


#include "knn_internal.h"
#include "wave.h"

namespace atsne {

constexpr uint32_t ORD_UNREACHED = 0xffffffffu;

// Sort keys are (key code << ib) | index with ib = index_bits(N): only the
// 32 + ib significant bits are sorted (five radix passes at N = 70000 instead
// of seven over the whole word), and the order is that of (code, index).
static int index_bits(int64_t N) {
    int b = 1;
    while (((int64_t)1 << b) < N) ++b;
    return b;
}

__global__ __launch_bounds__(256) void ord_density_keys(const float* __restrict__ beta,
                                                        const int32_t* __restrict__ ids, int64_t M, int64_t N, int ib,
                                                        uint64_t* __restrict__ keys, int32_t* __restrict__ bad) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    const int64_t id = ids ? (int64_t)ids[m] : m;
    if (id < 0 || id >= N) {
        atomicOr(bad, 1);
        keys[m] = ~0ull;
        return;
    }
    keys[m] = ((uint64_t)f2ord(beta[id]) << ib) | (uint64_t)id;
}

__global__ __launch_bounds__(256) void ord_unpack(const uint64_t* __restrict__ keys, int64_t n, int ib,
                                                  int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (int32_t)(keys[i] & (((uint64_t)1 << ib) - 1));
}

__global__ __launch_bounds__(256) void ord_init(int64_t N, uint32_t* __restrict__ dist, int32_t* __restrict__ stamp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < N) {
        dist[i] = ORD_UNREACHED;
        stamp[i] = -1;
    }
}

__global__ __launch_bounds__(256) void ord_seed(const int32_t* __restrict__ seeds, int64_t n_seeds, int64_t N,
                                                uint32_t* __restrict__ dist, int32_t* __restrict__ front,
                                                int32_t* __restrict__ n_front, int32_t* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_seeds) return;
    const int32_t s = seeds[t];
    if (s < 0 || s >= N) {
        atomicOr(bad, 1);
        return;
    }
    if (atomicCAS(&dist[s], ORD_UNREACHED, 0u) == ORD_UNREACHED) front[atomicAdd(n_front, 1)] = s;
}

// One round: thread t handles slot t % k of frontier point t / k.
__global__ __launch_bounds__(256) void ord_expand(const int32_t* __restrict__ front, int64_t n_front,
                                                  const int32_t* __restrict__ nbr_idx,
                                                  const float* __restrict__ nbr_d2, int k, int64_t N, int weighted,
                                                  uint32_t level, uint32_t* __restrict__ dist,
                                                  int32_t* __restrict__ stamp, int32_t round,
                                                  int32_t* __restrict__ next, int32_t* __restrict__ n_next) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_front * k) return;
    const int64_t i = front[t / k];
    const int s = (int)(t % k);
    const int32_t j = nbr_idx[i * k + s];
    if (j < 0 || j >= N) return;  // absent entry: no edge
    if (!weighted) {
        if (atomicCAS(&dist[j], ORD_UNREACHED, level + 1) == ORD_UNREACHED) next[atomicAdd(n_next, 1)] = j;
        return;
    }
    const float di = __uint_as_float(__atomic_load_n(&dist[i], __ATOMIC_RELAXED));
    const float nd = di + sqrtf(nbr_d2[i * k + s]);
    const uint32_t nb = __float_as_uint(nd);
    if (nb < atomicMin(&dist[j], nb) && atomicExch(&stamp[j], round) != round) next[atomicAdd(n_next, 1)] = j;
}

// Keys of the reached points, and the per-point key as a float (+inf: unreached).
__global__ __launch_bounds__(256) void ord_collect(const uint32_t* __restrict__ dist, int64_t N, int weighted, int ib,
                                                   float* __restrict__ key_out, uint64_t* __restrict__ keys,
                                                   int32_t* __restrict__ n_keys) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const uint32_t d = dist[i];
    if (key_out) key_out[i] = d == ORD_UNREACHED ? INFINITY : (weighted ? __uint_as_float(d) : (float)d);
    if (d != ORD_UNREACHED) keys[atomicAdd(n_keys, 1)] = ((uint64_t)d << ib) | (uint64_t)i;
}

static unsigned blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 256)); }

static size_t sort_temp_bytes(int64_t n) { return sort_u64_temp_bytes(n); }

struct OrderWs {
    uint64_t *keys_in, *keys_out;
    uint32_t* dist;
    int32_t *stamp, *front, *next, *counters;
    void* sort_tmp;
    size_t sort_bytes;
};

static size_t order_ws(int64_t N, void* base, OrderWs* w) {
    Arena a(base, base ? ~size_t(0) : 0);
    const int64_t n = std::max<int64_t>(N, 1);
    OrderWs o;
    o.keys_in = a.take<uint64_t>(n);
    o.keys_out = a.take<uint64_t>(n);
    o.dist = a.take<uint32_t>(n);
    o.stamp = a.take<int32_t>(n);
    o.front = a.take<int32_t>(n);
    o.next = a.take<int32_t>(n);
    o.counters = a.take<int32_t>(4);
    o.sort_bytes = std::max<size_t>(sort_temp_bytes(n), 1);
    o.sort_tmp = a.take<char>(o.sort_bytes);
    if (w) *w = o;
    return a.used;
}

static atsne_status sort_and_unpack(OrderWs& w, int64_t n, int ib, int32_t* out, hipStream_t st) {
    if (n == 0) return ATSNE_OK;
    ATSNE_TRY(sort_u64(w.sort_tmp, w.sort_bytes, w.keys_in, w.keys_out, n, st, 0, 32 + ib));
    ord_unpack<<<blocks(n), 256, 0, st>>>(w.keys_out, n, ib, out);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

static atsne_status read_counter(const int32_t* dev, int32_t* host, hipStream_t st) {
    ATSNE_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ATSNE_HIP(hipStreamSynchronize(st));
    return ATSNE_OK;
}

}  // namespace atsne

using namespace atsne;

extern "C" atsne_status atsne_order_workspace_size(int64_t N, size_t* bytes) {
    clear_error();
    ATSNE_REQUIRE(bytes && N >= 0, ATSNE_E_INVALID_ARG, "bad arguments");
    *bytes = order_ws(N, nullptr, nullptr);
    return ATSNE_OK;
}

extern "C" atsne_status atsne_order_density(const float* beta, int64_t N, const int32_t* ids, int64_t M,
                                            int32_t* order_out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    ATSNE_REQUIRE(N >= 0 && M >= 0 && M <= INT32_MAX, ATSNE_E_INVALID_ARG, "bad sizes");
    ATSNE_REQUIRE(ids || M == N, ATSNE_E_INVALID_ARG, "without ids the selection is all N points");
    if (M == 0) return ATSNE_OK;
    ATSNE_REQUIRE(beta && order_out, ATSNE_E_INVALID_ARG, "null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    ATSNE_TRY(sc.acquire(ws, ws_bytes, order_ws(M, nullptr, nullptr), st));
    OrderWs w;
    order_ws(M, sc.ptr, &w);
    ATSNE_HIP(hipMemsetAsync(w.counters, 0, sizeof(int32_t) * 4, st));
    const int ib = index_bits(N);
    ord_density_keys<<<blocks(M), 256, 0, st>>>(beta, ids, M, N, ib, w.keys_in, w.counters);
    ATSNE_LAUNCH_CHECK();
    ATSNE_TRY(sort_and_unpack(w, M, ib, order_out, st));
    if (ids) {
        int32_t bad = 0;
        ATSNE_TRY(read_counter(w.counters, &bad, st));
        ATSNE_REQUIRE(!bad, ATSNE_E_INVALID_ARG, "selection id outside [0, %lld)", (long long)N);
    }
    return ATSNE_OK;
}

extern "C" atsne_status atsne_order_neighbourhood(const int32_t* nbr_idx, const float* nbr_d2, int64_t N, int32_t k,
                                                  const int32_t* seeds, int64_t n_seeds, int32_t weighted,
                                                  int32_t max_depth, float* key_out, int32_t* order_out,
                                                  int64_t* n_reached_host, void* ws, size_t ws_bytes,
                                                  void* stream) {
    clear_error();
    ATSNE_REQUIRE(n_reached_host && N >= 1 && N <= INT32_MAX && k >= 1 && n_seeds >= 0, ATSNE_E_INVALID_ARG,
                  "bad arguments");
    ATSNE_REQUIRE(nbr_idx && order_out && (n_seeds == 0 || seeds) && (!weighted || nbr_d2), ATSNE_E_INVALID_ARG,
                  "null pointer");
    ATSNE_REQUIRE(!weighted || max_depth < 0, ATSNE_E_INVALID_ARG, "max_depth applies to the hop-count visit only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    ATSNE_TRY(sc.acquire(ws, ws_bytes, order_ws(N, nullptr, nullptr), st));
    OrderWs w;
    order_ws(N, sc.ptr, &w);
    // counters: 0 bad seed, 1 frontier size, 2 next size, 3 reached
    ATSNE_HIP(hipMemsetAsync(w.counters, 0, sizeof(int32_t) * 4, st));
    ord_init<<<blocks(N), 256, 0, st>>>(N, w.dist, w.stamp);
    ATSNE_LAUNCH_CHECK();
    if (n_seeds > 0) {
        ord_seed<<<blocks(n_seeds), 256, 0, st>>>(seeds, n_seeds, N, w.dist, w.front, w.counters + 1, w.counters);
        ATSNE_LAUNCH_CHECK();
    }
    int32_t h[2] = {0, 0};
    ATSNE_HIP(hipMemcpyAsync(h, w.counters, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
    ATSNE_HIP(hipStreamSynchronize(st));
    ATSNE_REQUIRE(!h[0], ATSNE_E_INVALID_ARG, "seed outside [0, %lld)", (long long)N);
    int64_t n_front = h[1];
    int32_t* front = w.front;
    int32_t* next = w.next;
    // a point re-enters a frontier only when its key falls, which happens at
    // most once per round of the slowest path: N + 1 rounds always suffice
    for (int32_t round = 0; n_front > 0; ++round) {
        ATSNE_REQUIRE(round <= N + 1, ATSNE_E_HIP, "visit did not converge");
        if (!weighted && max_depth >= 0 && round >= max_depth) break;
        ATSNE_HIP(hipMemsetAsync(w.counters + 2, 0, sizeof(int32_t), st));
        ord_expand<<<blocks(n_front * k), 256, 0, st>>>(front, n_front, nbr_idx, nbr_d2, k, N, weighted,
                                                         (uint32_t)round, w.dist, w.stamp, round, next,
                                                         w.counters + 2);
        ATSNE_LAUNCH_CHECK();
        int32_t nn = 0;
        ATSNE_TRY(read_counter(w.counters + 2, &nn, st));
        std::swap(front, next);
        n_front = nn;
    }
    const int ib = index_bits(N);
    ord_collect<<<blocks(N), 256, 0, st>>>(w.dist, N, weighted, ib, key_out, w.keys_in, w.counters + 3);
    ATSNE_LAUNCH_CHECK();
    int32_t reached = 0;
    ATSNE_TRY(read_counter(w.counters + 3, &reached, st));
    ATSNE_TRY(sort_and_unpack(w, reached, ib, order_out, st));
    *n_reached_host = reached;
    return ATSNE_OK;
}
