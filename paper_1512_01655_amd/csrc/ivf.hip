// Precision-controlled approximate kNN on gfx950: a cluster-pruned
// brute-force search standing in for the paper's randomized kd-forest
// (Sec. 4.2), with its work budget fitted to a requested precision rho
// (Eq. 9) on a sample, as the forest's parameters are in the paper.
//
// Build: k-means (Lloyd) from caller-chosen initial points.  The assignment
// step is the exact FP32 kNN search (k = 1) of the points against the
// centroids; the update is a deterministic per-cluster mean (one workgroup
// per cluster sums its members in index order), so the partition does not
// depend on scheduling.  The corpus is then sorted by (cluster, index) and
// each cluster's probe order is its centroid's exact neighbour list.
//
// Search: every point searches the 256-row tiles of the sorted corpus that
// overlap its cluster's first n_probe probe clusters (extended with further
// probe clusters until those clusters hold at least k + 1 rows).  Query blocks
// never straddle clusters, so a block's tile list is its cluster's, and the
// whole search is one launch of the MFMA tile kernel over per-block tile
// lists, followed by the same exact FP32 re-rank, certificate and exact scan
// (over the same tiles) as the exact path: the result is the exact kNN over
// the point's candidates.
//
// Fit: the smallest n_probe whose precision on the points of a sample of
// clusters reaches rho.  Candidate sets grow with n_probe and the exact kNN
// over a larger set keeps every true neighbour the smaller set had, so the
// precision is non-decreasing in n_probe and a bisection finds it.
#include <algorithm>
#include <climits>
#include <memory>
#include <set>
#include <vector>

#include "knn_internal.h"
#include "wave.h"

struct atsne_ivf {
    int64_t N = 0;
    int32_t D = 0, C = 0;
    float* Xperm = nullptr;  // corpus sorted by (cluster, index)
    void* cmem = nullptr;
    atsne::Corpus corpus;
    int32_t* perm = nullptr;    // sorted row r holds point perm[r]
    int32_t* assign = nullptr;  // cluster of each point (original order)
    float* cent = nullptr;      // C x D centroids
    std::vector<int64_t> start;  // cluster c holds sorted rows [start[c], start[c+1])
    std::vector<int32_t> probe;  // C x C probe order, itself first
};

namespace atsne {
namespace {

constexpr int IVF_TILE = KNN_KT;
constexpr int IVF_MAX_C = 1024;  // the probe order is a (C - 1)-NN search among centroids
// The sorted corpus's contraction: FP32X3 (BF16 hi + lo, three BF16
// matrix-core products per element pair), whose candidate rows and exact
// re-rank equal the FP32 contraction's at about twice the tile speed.  The
// centroid searches of the build stay FP32 (they are tiny).
constexpr int IVF_PREC = ATSNE_PREC_FP32X3;

__global__ __launch_bounds__(256) void ivf_gather(const float* __restrict__ src, const int32_t* __restrict__ ids,
                                                  int64_t n, int32_t D, float* __restrict__ dst) {
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    const float* s = src + (int64_t)ids[r] * D;
    for (int d = threadIdx.x; d < D; d += 256) dst[r * D + d] = s[d];
}

// Deterministic Lloyd update: workgroup c sums the rows of its members in
// increasing index order, one dimension per thread (R dimensions each).
template <int R>
__global__ __launch_bounds__(256) void ivf_update(const float* __restrict__ X, const int32_t* __restrict__ assign,
                                                  int64_t N, int32_t D, float* __restrict__ cent) {
    __shared__ int32_t members[256];
    __shared__ int32_t wcount[4];
    const int c = blockIdx.x;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
    int64_t count = 0;
    for (int64_t i0 = 0; i0 < N; i0 += 256) {
        const int64_t i = i0 + t;
        const bool mine = i < N && assign[i] == c;
        const uint64_t m = ballot(mine);
        if (l == 0) wcount[w] = __popcll(m);
        __syncthreads();
        int base = 0;
        for (int v = 0; v < w; ++v) base += wcount[v];
        const int total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (mine) members[base + __popcll(m & lanemask_lt())] = (int32_t)i;
        __syncthreads();
        for (int e = 0; e < total; ++e) {
            const float* x = X + (int64_t)members[e] * D;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int d = t + 256 * r;
                if (d < D) acc[r] += x[d];
            }
        }
        count += total;
        __syncthreads();
    }
    if (count == 0) return;  // an empty cluster keeps its centroid
    const float inv = 1.0f / (float)count;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int d = t + 256 * r;
        if (d < D) cent[(int64_t)c * D + d] = acc[r] * inv;
    }
}

__global__ __launch_bounds__(256) void ivf_count(const int32_t* __restrict__ assign, int64_t N,
                                                 int32_t* __restrict__ counts, uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int32_t c = assign[i];
    atomicAdd(&counts[c], 1);
    keys[i] = ((uint64_t)(uint32_t)c << 32) | (uint32_t)i;
}

__global__ __launch_bounds__(256) void ivf_unpack(const uint64_t* __restrict__ keys, int64_t n,
                                                  int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (int32_t)(uint32_t)keys[i];
}

// Results of sorted row r go to point perm[r], neighbour ids mapped back.
__global__ __launch_bounds__(256) void ivf_scatter(const int32_t* __restrict__ tidx, const float* __restrict__ td2,
                                                   const uint8_t* __restrict__ tfl, const int32_t* __restrict__ perm,
                                                   int64_t N, int k, int32_t* __restrict__ idx,
                                                   float* __restrict__ d2, uint8_t* __restrict__ flags) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * k) return;
    const int64_t r = e / k, s = e % k;
    const int64_t o = (int64_t)perm[r] * k + s;
    const int32_t j = tidx[e];
    idx[o] = j >= 0 ? perm[j] : -1;
    d2[o] = td2[e];
    if (s == 0 && flags) flags[perm[r]] = tfl[r];
}

// Eq. 9 numerator: for each row, how many approximate neighbours are exact ones.
__global__ __launch_bounds__(64) void ivf_hits(const int32_t* __restrict__ approx, const int32_t* __restrict__ exact,
                                               int64_t M, int k, unsigned long long* __restrict__ hits) {
    const int64_t m = blockIdx.x;
    if (m >= M) return;
    const int l = threadIdx.x;
    int h = 0;
    for (int s = l; s < k; s += 64) {
        const int32_t a = approx[m * k + s];
        if (a < 0) continue;
        for (int u = 0; u < k; ++u) h += exact[m * k + u] == a ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
    if (l == 0) atomicAdd(hits, (unsigned long long)h);
}

unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 256)); }

atsne_status alloc(void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) {
        set_error("device allocation of %zu bytes failed", bytes);
        return ATSNE_E_NOMEM;
    }
    return ATSNE_OK;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    atsne_status get(size_t bytes) { return alloc(&p, bytes); }
};

// Per-cluster candidate tiles.  The candidate clusters are the first n_probe
// probe clusters, extended until their rows number at least k + 1; the
// search covers the tiles of the sorted corpus that overlap their rows, a
// superset of those rows (the tile kernel works on whole tiles), so every
// point's result is the exact kNN over at least its candidate clusters.
std::vector<std::vector<int32_t>> cluster_tiles(const atsne_ivf& ix, int n_probe, int k) {
    const int C = ix.C;
    std::vector<std::vector<int32_t>> out(C);
    for (int c = 0; c < C; ++c) {
        std::set<int32_t> cover;
        int64_t rows = 0;
        int used = 0;
        for (int u = 0; u < C; ++u) {
            if (used >= n_probe && rows >= k + 1) break;
            ++used;
            const int p = ix.probe[(size_t)c * C + u];
            const int64_t lo = ix.start[p], hi = ix.start[p + 1];
            if (hi <= lo) continue;
            rows += hi - lo;
            for (int64_t t = lo / IVF_TILE; t <= (hi - 1) / IVF_TILE; ++t) cover.insert((int32_t)t);
        }
        out[c].assign(cover.begin(), cover.end());
    }
    return out;
}

// Query blocks for the batch rows of the given clusters (rows of a cluster
// are batch rows [row0, row0 + n) in the order given); host arrays.
struct Blocks {
    std::vector<int32_t> blk_q, blk_t, tl, row_blk;
    double cand_rows = 0;  // sum over rows of candidate rows
};

Blocks make_blocks(const atsne_ivf& ix, const std::vector<std::vector<int32_t>>& tiles,
                   const std::vector<int32_t>& clusters) {
    Blocks b;
    b.blk_q.push_back(0);
    b.blk_t.push_back(0);
    int32_t row = 0;
    for (int c : clusters) {
        const int64_t n = ix.start[c + 1] - ix.start[c];
        int64_t rows_in_tiles = 0;
        for (int32_t t : tiles[c]) rows_in_tiles += std::min<int64_t>(ix.N, (int64_t)(t + 1) * IVF_TILE) - (int64_t)t * IVF_TILE;
        for (int64_t q0 = 0; q0 < n; q0 += IVF_TILE) {
            const int32_t cnt = (int32_t)std::min<int64_t>(IVF_TILE, n - q0);
            for (int32_t i = 0; i < cnt; ++i) b.row_blk.push_back((int32_t)(b.blk_q.size() - 1));
            row += cnt;
            b.blk_q.push_back(row);
            b.tl.insert(b.tl.end(), tiles[c].begin(), tiles[c].end());
            b.blk_t.push_back((int32_t)b.tl.size());
        }
        b.cand_rows += (double)n * (double)rows_in_tiles;
    }
    return b;
}

// One restricted search: batch rows are sorted-corpus rows qids[m] (NULL: all
// N in order) grouped by cluster as in `b`; results in batch-row order with
// sorted-corpus neighbour ids.
atsne_status list_search(atsne_ivf& ix, const Blocks& b, const int32_t* qids_dev, int64_t M, int k,
                         int32_t* out_idx, float* out_d2, uint8_t* out_flags, hipStream_t st) {
    const int64_t nb = (int64_t)b.blk_q.size() - 1;
    const int kc = (int)std::min<int64_t>(k + std::max(32, k / 2), ix.N - 1);
    const int S = (int)std::min<int64_t>(8, std::max<int64_t>(1, ceil_div(4 * (int64_t)device_cu_count(), nb)));
    SearchPlan p = plan_list_search(M, nb, k, kc, S);
    Arena a;
    a.take<char>(p.ws_bytes);
    a.take<int32_t>(nb + 1);
    a.take<int32_t>(nb + 1);
    a.take<int32_t>(std::max<size_t>(b.tl.size(), 1));
    a.take<int32_t>(M);
    DevBuf buf;
    ATSNE_TRY(buf.get(a.used));
    Arena c(buf.p, a.used);
    void* ws = c.take<char>(p.ws_bytes);
    int32_t* d_blk_q = c.take<int32_t>(nb + 1);
    int32_t* d_blk_t = c.take<int32_t>(nb + 1);
    int32_t* d_tl = c.take<int32_t>(std::max<size_t>(b.tl.size(), 1));
    int32_t* d_row_blk = c.take<int32_t>(M);
    ATSNE_HIP(hipMemcpyAsync(d_blk_q, b.blk_q.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(d_blk_t, b.blk_t.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st));
    if (!b.tl.empty())
        ATSNE_HIP(hipMemcpyAsync(d_tl, b.tl.data(), sizeof(int32_t) * b.tl.size(), hipMemcpyHostToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(d_row_blk, b.row_blk.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
    Batch bt;
    bt.M = M;
    bt.qids = qids_dev;
    bt.m0 = 0;
    bt.nlim = ix.N;
    bt.key_lo = 0;
    bt.k = k;
    bt.kc = kc;
    bt.n_blocks = nb;
    bt.blk_q = d_blk_q;
    bt.blk_t = d_blk_t;
    bt.tl_idx = d_tl;
    bt.row_blk = d_row_blk;
    bt.out_idx = out_idx;
    bt.out_d2 = out_d2;
    bt.out_flags = out_flags;
    bt.out_stride = k;
    ATSNE_TRY(knn_search(ix.corpus, bt, p, ws, st));
    // host arrays and the device buffer must outlive the queued work
    ATSNE_HIP(hipStreamSynchronize(st));
    return ATSNE_OK;
}

}  // namespace
}  // namespace atsne

using namespace atsne;

extern "C" atsne_status atsne_ivf_build(const float* X, int64_t N, int32_t D, int32_t n_clusters,
                                        const int32_t* init_ids_host, int32_t iters, atsne_ivf** out, void* stream) {
    clear_error();
    ATSNE_REQUIRE(X && init_ids_host && out && N >= 2 && D >= 1 && iters >= 0, ATSNE_E_INVALID_ARG, "bad arguments");
    ATSNE_REQUIRE(n_clusters >= 2 && n_clusters <= N && n_clusters <= IVF_MAX_C && N <= INT32_MAX, ATSNE_E_K_RANGE,
                  "n_clusters %d outside [2, min(N, %d)]", n_clusters, IVF_MAX_C);
    ATSNE_REQUIRE(D <= 256 * 16, ATSNE_E_UNSUPPORTED, "D %d above %d", D, 256 * 16);
    {
        std::vector<int32_t> ids(init_ids_host, init_ids_host + n_clusters);
        std::sort(ids.begin(), ids.end());
        for (int32_t c = 0; c < n_clusters; ++c)
            ATSNE_REQUIRE(ids[c] >= 0 && ids[c] < N && (c == 0 || ids[c] != ids[c - 1]), ATSNE_E_INVALID_ARG,
                          "initial ids must be distinct points");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int C = n_clusters;
    const int64_t Cpad = ceil_div(C, KNN_KT) * KNN_KT;
    const int64_t comb_rows = Cpad + N;
    const int64_t comb_cap = ceil_div(comb_rows, KNN_KT) * KNN_KT;
    const int64_t cap = ceil_div(N, KNN_KT) * KNN_KT;
    auto ix = std::make_unique<atsne_ivf>();
    ix->N = N;
    ix->D = D;
    ix->C = C;
    atsne_status s_;
    auto fail = [&](atsne_status s) {
        (void)hipStreamSynchronize(st);
        if (ix->Xperm) (void)hipFree(ix->Xperm);
        if (ix->cmem) (void)hipFree(ix->cmem);
        if (ix->perm) (void)hipFree(ix->perm);
        if (ix->assign) (void)hipFree(ix->assign);
        if (ix->cent) (void)hipFree(ix->cent);
        return s;
    };
    // working set of the build: [centroids (padded); points] as one corpus
    DevBuf comb, comb_mem, ids_dev, tmp, sws;
    if ((s_ = comb.get(sizeof(float) * comb_cap * D)) != ATSNE_OK) return fail(s_);
    if ((s_ = comb_mem.get(corpus_bytes(ATSNE_PREC_FP32, comb_cap, D))) != ATSNE_OK) return fail(s_);
    if ((s_ = ids_dev.get(sizeof(int32_t) * C)) != ATSNE_OK) return fail(s_);
    float* cX = static_cast<float*>(comb.p);
    float* pts = cX + Cpad * D;
    if (hipMemsetAsync(cX, 0, sizeof(float) * comb_cap * D, st) != hipSuccess ||
        hipMemcpyAsync(pts, X, sizeof(float) * N * D, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ids_dev.p, init_ids_host, sizeof(int32_t) * C, hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("build staging failed");
        return fail(ATSNE_E_HIP);
    }
    ivf_gather<<<C, 256, 0, st>>>(pts, static_cast<const int32_t*>(ids_dev.p), C, D, cX);
    Corpus cc;
    corpus_bind(cc, ATSNE_PREC_FP32, cX, D, D, comb_cap, comb_mem.p);
    if ((s_ = corpus_prep(cc, 0, comb_cap, comb_rows, st)) != ATSNE_OK) return fail(s_);
    // outputs of the build
    if ((s_ = alloc((void**)&ix->assign, sizeof(int32_t) * N)) != ATSNE_OK) return fail(s_);
    if ((s_ = alloc((void**)&ix->perm, sizeof(int32_t) * N)) != ATSNE_OK) return fail(s_);
    if ((s_ = alloc((void**)&ix->cent, sizeof(float) * C * D)) != ATSNE_OK) return fail(s_);
    // assignment: exact nearest centroid (k = 1) of every point
    const int kc1 = std::min(33, C);
    SearchPlan pa = plan_search(ATSNE_PREC_FP32, N, 0, C, 1, kc1);
    const int kcc = C - 1;
    SearchPlan pc = plan_search(ATSNE_PREC_FP32, C, 0, C, kcc, kcc);
    const size_t sort_bytes = sort_u64_temp_bytes(N);
    {
        Arena a;
        a.take<float>(N);
        a.take<uint8_t>(N);
        a.take<int32_t>((size_t)C * kcc);
        a.take<float>((size_t)C * kcc);
        a.take<int32_t>(C);
        a.take<uint64_t>(N);
        a.take<uint64_t>(N);
        a.take<char>(sort_bytes);
        if ((s_ = tmp.get(a.used)) != ATSNE_OK) return fail(s_);
    }
    if ((s_ = sws.get(std::max(pa.ws_bytes, pc.ws_bytes))) != ATSNE_OK) return fail(s_);
    Arena ta(tmp.p, ~size_t(0));
    float* d1 = ta.take<float>(N);
    uint8_t* f1 = ta.take<uint8_t>(N);
    int32_t* cidx = ta.take<int32_t>((size_t)C * kcc);
    float* cd2 = ta.take<float>((size_t)C * kcc);
    int32_t* counts = ta.take<int32_t>(C);
    uint64_t* keys = ta.take<uint64_t>(N);
    uint64_t* keys2 = ta.take<uint64_t>(N);
    void* sort_tmp = ta.take<char>(sort_bytes);
    for (int it = 0;; ++it) {
        Batch b;
        b.M = N;
        b.m0 = Cpad;
        b.nlim = C;
        b.key_lo = 0;
        b.k = 1;
        b.kc = kc1;
        b.out_idx = ix->assign;
        b.out_d2 = d1;
        b.out_flags = f1;
        b.out_stride = 1;
        if ((s_ = knn_search(cc, b, pa, sws.p, st)) != ATSNE_OK) return fail(s_);
        if (it == iters) break;
        const int R = (int)ceil_div(D, 256);
        const dim3 g(C), blk(256);
        if (R <= 1)
            ivf_update<1><<<g, blk, 0, st>>>(pts, ix->assign, N, D, cX);
        else if (R <= 2)
            ivf_update<2><<<g, blk, 0, st>>>(pts, ix->assign, N, D, cX);
        else if (R <= 4)
            ivf_update<4><<<g, blk, 0, st>>>(pts, ix->assign, N, D, cX);
        else if (R <= 8)
            ivf_update<8><<<g, blk, 0, st>>>(pts, ix->assign, N, D, cX);
        else
            ivf_update<16><<<g, blk, 0, st>>>(pts, ix->assign, N, D, cX);
        if (hipGetLastError() != hipSuccess) {
            set_error("update launch failed");
            return fail(ATSNE_E_HIP);
        }
        if ((s_ = corpus_prep(cc, 0, Cpad, comb_rows, st)) != ATSNE_OK) return fail(s_);
    }
    // probe order: each centroid's exact neighbours among the centroids
    {
        Batch b;
        b.M = C;
        b.m0 = 0;
        b.nlim = C;
        b.key_lo = 0;
        b.k = kcc;
        b.kc = kcc;
        b.out_idx = cidx;
        b.out_d2 = cd2;
        b.out_stride = kcc;
        if ((s_ = knn_search(cc, b, pc, sws.p, st)) != ATSNE_OK) return fail(s_);
    }
    // sorted order and cluster ranges
    if (hipMemsetAsync(counts, 0, sizeof(int32_t) * C, st) != hipSuccess) return fail(ATSNE_E_HIP);
    ivf_count<<<blocks_of(N), 256, 0, st>>>(ix->assign, N, counts, keys);
    if ((s_ = sort_u64(sort_tmp, sort_bytes, keys, keys2, N, st)) != ATSNE_OK) return fail(s_);
    ivf_unpack<<<blocks_of(N), 256, 0, st>>>(keys2, N, ix->perm);
    if (hipMemcpyAsync(ix->cent, cX, sizeof(float) * C * D, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ATSNE_E_HIP);
    std::vector<int32_t> h_counts(C), h_cidx((size_t)C * kcc);
    if (hipMemcpyAsync(h_counts.data(), counts, sizeof(int32_t) * C, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(h_cidx.data(), cidx, sizeof(int32_t) * C * kcc, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("build readback failed");
        return fail(ATSNE_E_HIP);
    }
    ix->start.assign(C + 1, 0);
    for (int c = 0; c < C; ++c) ix->start[c + 1] = ix->start[c] + h_counts[c];
    ix->probe.resize((size_t)C * C);
    for (int c = 0; c < C; ++c) {
        ix->probe[(size_t)c * C] = c;
        for (int u = 0; u < kcc; ++u) ix->probe[(size_t)c * C + 1 + u] = h_cidx[(size_t)c * kcc + u];
    }
    // the sorted corpus the searches run on
    if ((s_ = alloc((void**)&ix->Xperm, sizeof(float) * cap * D)) != ATSNE_OK) return fail(s_);
    if ((s_ = alloc(&ix->cmem, corpus_bytes(IVF_PREC, cap, D))) != ATSNE_OK) return fail(s_);
    if (hipMemsetAsync(ix->Xperm + N * D, 0, sizeof(float) * (cap - N) * D, st) != hipSuccess)
        return fail(ATSNE_E_HIP);
    ivf_gather<<<(unsigned)N, 256, 0, st>>>(pts, ix->perm, N, D, ix->Xperm);
    corpus_bind(ix->corpus, IVF_PREC, ix->Xperm, D, D, cap, ix->cmem);
    if ((s_ = corpus_prep(ix->corpus, 0, cap, N, st)) != ATSNE_OK) return fail(s_);
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("build failed");
        return fail(ATSNE_E_HIP);
    }
    *out = ix.release();
    return ATSNE_OK;
}

extern "C" atsne_status atsne_ivf_partition(const atsne_ivf* ix, int32_t* assign, float* centroids,
                                            int64_t* cluster_start_host, int32_t* probe_host, void* stream) {
    clear_error();
    ATSNE_REQUIRE(ix, ATSNE_E_INVALID_ARG, "null index");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (assign) ATSNE_HIP(hipMemcpyAsync(assign, ix->assign, sizeof(int32_t) * ix->N, hipMemcpyDeviceToDevice, st));
    if (centroids)
        ATSNE_HIP(hipMemcpyAsync(centroids, ix->cent, sizeof(float) * ix->C * ix->D, hipMemcpyDeviceToDevice, st));
    if (cluster_start_host) std::copy(ix->start.begin(), ix->start.end(), cluster_start_host);
    if (probe_host) std::copy(ix->probe.begin(), ix->probe.end(), probe_host);
    return ATSNE_OK;
}

extern "C" atsne_status atsne_ivf_knn(atsne_ivf* ix, int32_t k, int32_t n_probe, int32_t* nbr_idx, float* nbr_d2,
                                      uint8_t* flags, double* candidate_fraction_host, void* stream) {
    clear_error();
    ATSNE_REQUIRE(ix && nbr_idx && nbr_d2, ATSNE_E_INVALID_ARG, "bad arguments");
    ATSNE_REQUIRE(k >= 1 && k <= ix->N - 1 && k <= 1024 - std::max(32, k / 2), ATSNE_E_K_RANGE, "k=%d out of range", k);
    ATSNE_REQUIRE(n_probe >= 1, ATSNE_E_INVALID_ARG, "n_probe must be positive");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto tiles = cluster_tiles(*ix, std::min(n_probe, ix->C), k);
    std::vector<int32_t> all(ix->C);
    for (int c = 0; c < ix->C; ++c) all[c] = c;
    const Blocks b = make_blocks(*ix, tiles, all);
    const int64_t N = ix->N;
    DevBuf tmp;
    Arena a;
    a.take<int32_t>(N * k);
    a.take<float>(N * k);
    a.take<uint8_t>(N);
    ATSNE_TRY(tmp.get(a.used));
    Arena c(tmp.p, a.used);
    int32_t* tidx = c.take<int32_t>(N * k);
    float* td2 = c.take<float>(N * k);
    uint8_t* tfl = c.take<uint8_t>(N);
    ATSNE_HIP(hipMemsetAsync(tfl, 0, N, st));
    ATSNE_TRY(list_search(*ix, b, nullptr, N, k, tidx, td2, tfl, st));
    ivf_scatter<<<blocks_of(N * k), 256, 0, st>>>(tidx, td2, tfl, ix->perm, N, k, nbr_idx, nbr_d2, flags);
    ATSNE_LAUNCH_CHECK();
    ATSNE_HIP(hipStreamSynchronize(st));
    if (candidate_fraction_host) *candidate_fraction_host = b.cand_rows / ((double)N * (double)N);
    return ATSNE_OK;
}

extern "C" atsne_status atsne_ivf_fit(atsne_ivf* ix, int32_t k, float rho, const int32_t* sample_clusters_host,
                                      int32_t n_sample, int32_t* n_probe_out, float* rho_sample_out, void* stream) {
    clear_error();
    ATSNE_REQUIRE(ix && sample_clusters_host && n_probe_out && n_sample >= 1, ATSNE_E_INVALID_ARG, "bad arguments");
    ATSNE_REQUIRE(k >= 1 && k <= ix->N - 1 && k <= 1024 - std::max(32, k / 2), ATSNE_E_K_RANGE, "k=%d out of range", k);
    ATSNE_REQUIRE(rho > 0.f && rho <= 1.f, ATSNE_E_INVALID_ARG, "rho must be in (0, 1]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<int32_t> cl(sample_clusters_host, sample_clusters_host + n_sample);
    std::vector<int32_t> qrows;
    for (int32_t c : cl) {
        ATSNE_REQUIRE(c >= 0 && c < ix->C, ATSNE_E_INVALID_ARG, "sample cluster %d outside [0, %d)", c, ix->C);
        for (int64_t r = ix->start[c]; r < ix->start[c + 1]; ++r) qrows.push_back((int32_t)r);
    }
    const int64_t M = (int64_t)qrows.size();
    ATSNE_REQUIRE(M >= 1, ATSNE_E_INVALID_ARG, "the sample clusters are empty");
    DevBuf tmp, ews;
    Arena a;
    a.take<int32_t>(M);
    a.take<int32_t>(M * k);
    a.take<float>(M * k);
    a.take<int32_t>(M * k);
    a.take<float>(M * k);
    a.take<unsigned long long>(1);
    ATSNE_TRY(tmp.get(a.used));
    Arena c(tmp.p, a.used);
    int32_t* d_q = c.take<int32_t>(M);
    int32_t* e_idx = c.take<int32_t>(M * k);
    float* e_d2 = c.take<float>(M * k);
    int32_t* a_idx = c.take<int32_t>(M * k);
    float* a_d2 = c.take<float>(M * k);
    unsigned long long* hits = c.take<unsigned long long>(1);
    ATSNE_HIP(hipMemcpyAsync(d_q, qrows.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
    // exact neighbours of the sample over the whole corpus
    {
        const int kc = (int)std::min<int64_t>(k + std::max(32, k / 2), ix->N - 1);
        SearchPlan p = plan_search(IVF_PREC, M, 0, ix->N, k, kc);
        ATSNE_TRY(ews.get(p.ws_bytes));
        Batch b;
        b.M = M;
        b.qids = d_q;
        b.nlim = ix->N;
        b.k = k;
        b.kc = kc;
        b.out_idx = e_idx;
        b.out_d2 = e_d2;
        b.out_stride = k;
        ATSNE_TRY(knn_search(ix->corpus, b, p, ews.p, st));
    }
    auto precision = [&](int n_probe, float* out) -> atsne_status {
        const auto tiles = cluster_tiles(*ix, n_probe, k);
        const Blocks b = make_blocks(*ix, tiles, cl);
        ATSNE_TRY(list_search(*ix, b, d_q, M, k, a_idx, a_d2, nullptr, st));
        ATSNE_HIP(hipMemsetAsync(hits, 0, sizeof(unsigned long long), st));
        ivf_hits<<<(unsigned)M, 64, 0, st>>>(a_idx, e_idx, M, k, hits);
        ATSNE_LAUNCH_CHECK();
        unsigned long long h = 0;
        ATSNE_HIP(hipMemcpyAsync(&h, hits, sizeof(h), hipMemcpyDeviceToHost, st));
        ATSNE_HIP(hipStreamSynchronize(st));
        *out = (float)((double)h / ((double)M * k));
        return ATSNE_OK;
    };
    int lo = 1, hi = ix->C;
    float p_hi = 1.f;
    ATSNE_TRY(precision(hi, &p_hi));
    float p_best = p_hi;
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        float pm = 0.f;
        ATSNE_TRY(precision(mid, &pm));
        if (pm >= rho) {
            hi = mid;
            p_best = pm;
        } else {
            lo = mid + 1;
        }
    }
    if (hi == ix->C) p_best = p_hi;
    *n_probe_out = hi;
    if (rho_sample_out) *rho_sample_out = p_best;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_ivf_destroy(atsne_ivf* ix) {
    clear_error();
    if (!ix) return ATSNE_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(ix->Xperm);
    (void)hipFree(ix->cmem);
    (void)hipFree(ix->perm);
    (void)hipFree(ix->assign);
    (void)hipFree(ix->cent);
    delete ix;
    return ATSNE_OK;
}

namespace atsne {

// Seeding pass of a large FP8 search.  Any subset of a row's keys has a
// kc-th smallest key code d' at least the row's kc-th smallest over all
// keys, so the search may keep only keys at or below it from its first tile
// on (Batch::tau_seed).  The subset here is the keys near the row: the
// k-means partition of the approximate search (strided initial points, no
// Lloyd step: Voronoi cells of about SEED_CLUSTER_ROWS points), the row's own
// cluster and its nearest ones in probe order, searched in FP8 with the same
// tile kernel, so every d' is bit for bit the one the full search computes.
constexpr int64_t SEED_CLUSTER_ROWS = 1000;
constexpr int SEED_PROBE = 8;               // clusters searched per point (extended to kc + 1 rows)
constexpr int64_t SEED_BATCH_ROWS = 524288;  // rows per seeding launch (bounds the slot memory, ~3.8 GB)

// The tiles of cluster_tiles, listed cluster by cluster in probe order (the
// own cluster first): a row's threshold settles on its nearest keys within
// a few tiles, so the later tiles append few keys.  The order changes no
// result: a row's union still holds its kc smallest over all listed tiles.
static std::vector<std::vector<int32_t>> seed_tiles(const atsne_ivf& ix, int n_probe, int k) {
    const int C = ix.C;
    std::vector<std::vector<int32_t>> out(C);
    for (int c = 0; c < C; ++c) {
        std::set<int32_t> cover;
        int64_t rows = 0;
        int used = 0;
        for (int u = 0; u < C; ++u) {
            if (used >= n_probe && rows >= k + 1) break;
            ++used;
            const int p = ix.probe[(size_t)c * C + u];
            const int64_t lo = ix.start[p], hi = ix.start[p + 1];
            if (hi <= lo) continue;
            rows += hi - lo;
            for (int64_t t = lo / IVF_TILE; t <= (hi - 1) / IVF_TILE; ++t)
                if (cover.insert((int32_t)t).second) out[c].push_back((int32_t)t);
        }
    }
    return out;
}

atsne_status fp8_seed_thresholds(const float* X, int64_t N, int32_t D, int64_t ld, int kc, float* tau,
                                 int32_t* order, hipStream_t st) {
    ATSNE_REQUIRE(ld == D, ATSNE_E_UNSUPPORTED, "seeding needs contiguous rows");
    const int C = (int)std::min<int64_t>(IVF_MAX_C, std::max<int64_t>(2, N / SEED_CLUSTER_ROWS));
    std::vector<int32_t> init(C);
    for (int c = 0; c < C; ++c) init[c] = (int32_t)((int64_t)c * N / C);
    atsne_ivf* ixp = nullptr;
    ATSNE_TRY(atsne_ivf_build(X, N, D, C, init.data(), 0, &ixp, st));
    std::unique_ptr<atsne_ivf, atsne_status (*)(atsne_ivf*)> guard(ixp, atsne_ivf_destroy);
    atsne_ivf& ix = *ixp;
    const auto tiles = seed_tiles(ix, SEED_PROBE, kc);
    // decline when the cells are too coarse to pay (e.g. data in one cell):
    // the lists would cover more than a tenth of all row pairs
    double pairs = 0;
    for (int c = 0; c < C; ++c)
        pairs += (double)(ix.start[c + 1] - ix.start[c]) * (double)tiles[c].size() * IVF_TILE;
    ATSNE_REQUIRE(pairs <= 0.1 * (double)N * (double)N, ATSNE_E_UNSUPPORTED,
                  "seeding lists would cover %.0f%% of the row pairs", 100.0 * pairs / ((double)N * (double)N));
    if (order) ATSNE_HIP(hipMemcpyAsync(order, ix.perm, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, st));
    // FP8 copy of the sorted corpus (per-row scales: the rows' FP8 codes,
    // norms and scales equal those of the same rows in the caller's order)
    const int64_t cap = ceil_div(N, (int64_t)KNN_KT) * KNN_KT;
    DevBuf cm;
    ATSNE_TRY(cm.get(corpus_bytes(ATSNE_PREC_FP8_E4M3, cap, D)));
    Corpus c8;
    corpus_bind(c8, ATSNE_PREC_FP8_E4M3, ix.Xperm, D, D, cap, cm.p);
    ATSNE_TRY(corpus_prep(c8, 0, cap, N, st));
    for (int c0 = 0; c0 < C;) {
        int c1 = c0 + 1;
        while (c1 < C && ix.start[c1 + 1] - ix.start[c0] <= SEED_BATCH_ROWS) ++c1;
        std::vector<int32_t> clusters;
        for (int c = c0; c < c1; ++c) clusters.push_back(c);
        const Blocks b = make_blocks(ix, tiles, clusters);
        const int64_t M = ix.start[c1] - ix.start[c0];
        const int64_t nb = (int64_t)b.blk_q.size() - 1;
        if (M > 0 && nb > 0) {
            const SearchPlan p = plan_list_search(M, nb, kc, kc, 1);
            Arena a;
            a.take<char>(p.ws_bytes);
            a.take<int32_t>(nb + 1);
            a.take<int32_t>(nb + 1);
            a.take<int32_t>(std::max<size_t>(b.tl.size(), 1));
            a.take<int32_t>(M);
            DevBuf buf;
            ATSNE_TRY(buf.get(a.used));
            Arena w(buf.p, a.used);
            void* ws = w.take<char>(p.ws_bytes);
            int32_t* d_blk_q = w.take<int32_t>(nb + 1);
            int32_t* d_blk_t = w.take<int32_t>(nb + 1);
            int32_t* d_tl = w.take<int32_t>(std::max<size_t>(b.tl.size(), 1));
            int32_t* d_row_blk = w.take<int32_t>(M);
            ATSNE_HIP(hipMemcpyAsync(d_blk_q, b.blk_q.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st));
            ATSNE_HIP(hipMemcpyAsync(d_blk_t, b.blk_t.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st));
            if (!b.tl.empty())
                ATSNE_HIP(hipMemcpyAsync(d_tl, b.tl.data(), sizeof(int32_t) * b.tl.size(), hipMemcpyHostToDevice, st));
            ATSNE_HIP(hipMemcpyAsync(d_row_blk, b.row_blk.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
            Batch bt;
            bt.M = M;
            bt.qids = nullptr;
            bt.m0 = ix.start[c0];  // batch row m is sorted row start[c0] + m
            bt.nlim = N;
            bt.key_lo = 0;
            bt.k = kc;
            bt.kc = kc;
            bt.n_blocks = nb;
            bt.blk_q = d_blk_q;
            bt.blk_t = d_blk_t;
            bt.tl_idx = d_tl;
            bt.row_blk = d_row_blk;
            bt.tau_out = tau;
            bt.tau_map = ix.perm;  // sorted row -> the caller's row
            ATSNE_TRY(knn_search(c8, bt, p, ws, st));
            // host arrays and the device buffer must outlive the queued work
            ATSNE_HIP(hipStreamSynchronize(st));
        }
        c0 = c1;
    }
    return ATSNE_OK;
}

}  // namespace atsne
