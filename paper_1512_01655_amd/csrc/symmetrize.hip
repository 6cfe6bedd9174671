// Symmetrisation of the sparse conditional P for the A-tSNE similarity path.
//
// p_ij = (p_{j|i} + p_{i|j}) / (2N) (Eq. 2; the split form of Eq. 10 is why
// only the per-point conditional rows are stored upstream).  The output is
// CSR with ascending columns over the union of the neighbour patterns.
//
// Device pipeline (HBM/atomic bound, one wave per row where rows are walked):
//   sym_count    cnt[i] = |N_i| + in-degree(i)          (atomics on cnt[j])
//   scan         off = exclusive scan of cnt
//   sym_scatter  row i receives (j, p_{j|i}) in place and, mirrored, row j
//                receives (i, p_{j|i}) at an atomic cursor
//   sym_merge    per row: sort by (column, origin), add the at most two
//                entries of each column, divide by 2N; unique count u[i]
//   scan         row_ptr = exclusive scan of u
//   sym_compact  copy the merged rows to their final place
// Each output value is the sum of at most two addends, so the atomics'
// arbitrary order does not change any result bit.
#include <algorithm>

#include "common.h"
#include "wave.h"

namespace atsne {

constexpr int SCAN_BLOCK = 1024;  // elements per scan block (256 threads x 4)

// ---- exclusive scan of int32 counts into int64 offsets (3 phases) ----
__global__ __launch_bounds__(256) void scan_blocks(const int32_t* __restrict__ in, int64_t n,
                                                   int64_t* __restrict__ out, int64_t* __restrict__ block_sums) {
    __shared__ int64_t wsum[4];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + 4 * t;
    int64_t v[4];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    // wave inclusive scan of per-thread sums
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t tv = __shfl_up(incl, o, 64);
        if (l >= o) incl += tv;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    int64_t woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int64_t run = woff + incl - s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (t == 255) block_sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(64) void scan_sums(int64_t* __restrict__ block_sums, int64_t nb, int64_t* __restrict__ total) {
    // one wave, sequential over chunks of 64 (nb is small)
    const int l = lane_id();
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 64) {
        int64_t v = (b0 + l < nb) ? block_sums[b0 + l] : 0;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int64_t tv = __shfl_up(incl, o, 64);
            if (l >= o) incl += tv;
        }
        if (b0 + l < nb) block_sums[b0 + l] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (l == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + 4 * threadIdx.x;
    const int64_t add = block_sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] += add;
}

// out[0..n) = exclusive scan of in, out[n] = total.  block_sums: ceil(n/1024) entries.
static atsne_status exclusive_scan(const int32_t* in, int64_t n, int64_t* out, int64_t* block_sums, hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, ceil_div(n, SCAN_BLOCK));
    scan_blocks<<<dim3((unsigned)nb), dim3(256), 0, st>>>(in, n, out, block_sums);
    ATSNE_LAUNCH_CHECK();
    scan_sums<<<dim3(1), dim3(64), 0, st>>>(block_sums, nb, out + n);
    ATSNE_LAUNCH_CHECK();
    scan_add<<<dim3((unsigned)nb), dim3(256), 0, st>>>(out, n, block_sums);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

// Row extent of the conditional input: CSR (in_ptr) or fixed k.
struct RowsIn {
    const int64_t* ptr;
    int k;
    __device__ __forceinline__ int64_t begin(int64_t i) const { return ptr ? ptr[i] : i * k; }
    __device__ __forceinline__ int64_t end(int64_t i) const { return ptr ? ptr[i + 1] : (i + 1) * k; }
};

__global__ __launch_bounds__(256) void sym_count(RowsIn rin, const int32_t* __restrict__ col, int64_t N,
                                                 int32_t* __restrict__ cnt) {
    const int l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int64_t b = rin.begin(i), e = rin.end(i);
    for (int64_t t = b + l; t < e; t += WAVE) atomicAdd(&cnt[col[t]], 1);
    if (l == 0) atomicAdd(&cnt[i], (int32_t)(e - b));
}

// Entry key: column in the high bits, origin (0 own, 1 mirrored) in bit 0.
__global__ __launch_bounds__(256) void sym_scatter(RowsIn rin, const int32_t* __restrict__ col,
                                                   const float* __restrict__ val, int64_t N,
                                                   const int64_t* __restrict__ off, int32_t* __restrict__ fill,
                                                   int64_t* __restrict__ tkey, float* __restrict__ tval) {
    const int l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int64_t b = rin.begin(i), e = rin.end(i);
    for (int64_t t = b + l; t < e; t += WAVE) {
        const int32_t j = col[t];
        const float p = val[t];
        const int64_t own = off[i] + (t - b);
        tkey[own] = ((int64_t)j << 1);
        tval[own] = p;
        const int64_t lenj = rin.end(j) - rin.begin(j);
        const int64_t mir = off[j] + lenj + atomicAdd(&fill[j], 1);
        tkey[mir] = ((int64_t)i << 1) | 1;
        tval[mir] = p;
    }
}

constexpr int MERGE_LDS = 2048;

__device__ __forceinline__ void row_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// In-place ascending sort of n (key, value) pairs by one wave: bitonic
// network whose comparators all point the same way (a flip step, then
// half-cleaners), so positions >= n act as +inf and are never touched.
// Works on LDS or global memory alike.
__device__ void wave_bitonic_sort(int64_t* key, float* val, int n) {
    const int l = lane_id();
    int P = 1;
    while (P < n) P <<= 1;
    auto cmpswap = [&](int a, int b) {
        if (b < n) {
            int64_t ka = key[a], kb = key[b];
            if (ka > kb) {
                float va = val[a], vb = val[b];
                key[a] = kb;
                key[b] = ka;
                val[a] = vb;
                val[b] = va;
            }
        }
    };
    for (int size = 2; size <= P; size <<= 1) {
        const int half = size >> 1;
        for (int t = l; t < P / 2; t += WAVE) {
            const int blk = t / half, o = t % half;
            cmpswap(blk * size + o, blk * size + size - 1 - o);
        }
        row_sync();
        for (int stride = half >> 1; stride > 0; stride >>= 1) {
            for (int t = l; t < P / 2; t += WAVE) {
                const int a = (t / stride) * (2 * stride) + (t % stride);
                cmpswap(a, a + stride);
            }
            row_sync();
        }
    }
}

// Per row: sort entries by key (column, origin), fold the mirrored half of a
// column into its own entry, write the merged row at off[i] into mcol/mval
// and its length into u[i].  Rows longer than MERGE_LDS (hubs of the kNN
// graph) are sorted in place in the global scratch.
__global__ __launch_bounds__(64) void sym_merge(const int64_t* __restrict__ off, int64_t N,
                                                int64_t* __restrict__ tkey, float* __restrict__ tval,
                                                float inv_norm, int32_t* __restrict__ mcol,
                                                float* __restrict__ mval, int32_t* __restrict__ u) {
    __shared__ int64_t skey[MERGE_LDS];
    __shared__ float sval[MERGE_LDS];
    const int l = lane_id();
    const int64_t i = blockIdx.x;
    if (i >= N) return;
    const int64_t b = off[i];
    const int n = (int)(off[i + 1] - b);
    int64_t* K = tkey + b;
    float* V = tval + b;
    if (n <= MERGE_LDS) {
        for (int t = l; t < n; t += WAVE) {
            skey[t] = K[t];
            sval[t] = V[t];
        }
        row_sync();
        K = skey;
        V = sval;
    }
    wave_bitonic_sort(K, V, n);
    // an entry whose column equals its predecessor's is the mirrored half
    // of that column and is folded into it (own + mirrored, fixed order)
    int uniq = 0;
    for (int r0 = 0; r0 < n; r0 += WAVE) {
        const int r = r0 + l;
        bool head = false;
        int64_t kr = 0;
        if (r < n) {
            kr = K[r];
            head = (r == 0) || ((K[r - 1] >> 1) != (kr >> 1));
        }
        const uint64_t m = ballot(head);
        if (head) {
            float v = V[r];
            if (r + 1 < n && (K[r + 1] >> 1) == (kr >> 1)) v += V[r + 1];
            const int pos = uniq + __popcll(m & lanemask_lt());
            mcol[b + pos] = (int32_t)(kr >> 1);
            mval[b + pos] = v * inv_norm;
        }
        uniq += __popcll(m);
    }
    if (l == 0) u[i] = uniq;
}

__global__ __launch_bounds__(256) void sym_compact(const int64_t* __restrict__ off, const int64_t* __restrict__ row_ptr,
                                                   int64_t N, const int32_t* __restrict__ mcol,
                                                   const float* __restrict__ mval, int32_t* __restrict__ col,
                                                   float* __restrict__ val) {
    const int l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int64_t src = off[i], dst = row_ptr[i], n = row_ptr[i + 1] - dst;
    for (int64_t t = l; t < n; t += WAVE) {
        col[dst + t] = mcol[src + t];
        val[dst + t] = mval[src + t];
    }
}

struct SymPlan {
    int64_t N, nnz_in, nb;
    size_t total;
};

static void sym_plan(int64_t N, int64_t nnz_in, SymPlan& p) {
    p.N = N;
    p.nnz_in = nnz_in;
    p.nb = std::max<int64_t>(1, ceil_div(N, SCAN_BLOCK));
    Arena a;
    a.take<int32_t>(N);            // cnt
    a.take<int32_t>(N);            // fill
    a.take<int32_t>(N);            // u
    a.take<int64_t>(N + 1);        // off
    a.take<int64_t>(p.nb);         // block sums
    a.take<int64_t>(2 * nnz_in);   // tkey
    a.take<float>(2 * nnz_in);     // tval
    a.take<int32_t>(2 * nnz_in);   // mcol
    a.take<float>(2 * nnz_in);     // mval
    p.total = a.used;
}

static atsne_status sym_run(const SymPlan& p, RowsIn rin, const int32_t* in_col, const float* in_val,
                            int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* wsp,
                            hipStream_t st) {
    Arena a(wsp, p.total);
    int32_t* cnt = a.take<int32_t>(p.N);
    int32_t* fill = a.take<int32_t>(p.N);
    int32_t* u = a.take<int32_t>(p.N);
    int64_t* off = a.take<int64_t>(p.N + 1);
    int64_t* bsum = a.take<int64_t>(p.nb);
    int64_t* tkey = a.take<int64_t>(2 * p.nnz_in);
    float* tval = a.take<float>(2 * p.nnz_in);
    int32_t* mcol = a.take<int32_t>(2 * p.nnz_in);
    float* mval = a.take<float>(2 * p.nnz_in);
    const int64_t N = p.N;
    ProfScope ps_("sym_total", st);
    ATSNE_HIP(hipMemsetAsync(cnt, 0, (size_t)N * 4, st));
    ATSNE_HIP(hipMemsetAsync(fill, 0, (size_t)N * 4, st));
    const dim3 g4((unsigned)ceil_div(N, 4)), b256(256);
    sym_count<<<g4, b256, 0, st>>>(rin, in_col, N, cnt);
    ATSNE_LAUNCH_CHECK();
    ATSNE_TRY(exclusive_scan(cnt, N, off, bsum, st));
    sym_scatter<<<g4, b256, 0, st>>>(rin, in_col, in_val, N, off, fill, tkey, tval);
    ATSNE_LAUNCH_CHECK();
    const float inv_norm = (float)(1.0 / (2.0 * (double)N));
    sym_merge<<<dim3((unsigned)N), dim3(64), 0, st>>>(off, N, tkey, tval, inv_norm, mcol, mval, u);
    ATSNE_LAUNCH_CHECK();
    ATSNE_TRY(exclusive_scan(u, N, row_ptr, bsum, st));
    sym_compact<<<g4, b256, 0, st>>>(off, row_ptr, N, mcol, mval, col, val);
    ATSNE_LAUNCH_CHECK();
    ATSNE_HIP(hipMemcpyAsync(nnz_host, row_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ps_.stop();
    ATSNE_HIP(hipStreamSynchronize(st));
    return ATSNE_OK;
}

}  // namespace atsne

extern "C" atsne_status atsne_symmetrize_workspace_size(int64_t N, int64_t nnz_in, size_t* bytes) {
    atsne::clear_error();
    ATSNE_REQUIRE(bytes && N >= 1 && nnz_in >= 0, ATSNE_E_INVALID_ARG, "bad arguments");
    atsne::SymPlan p;
    atsne::sym_plan(N, nnz_in, p);
    *bytes = p.total;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_symmetrize(const int32_t* nbr_idx, const float* P_cond, int64_t N, int32_t k,
                                         int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* ws,
                                         size_t ws_bytes, void* stream) {
    using namespace atsne;
    clear_error();
    ATSNE_REQUIRE(nbr_idx && P_cond && row_ptr && col && val && nnz_host, ATSNE_E_INVALID_ARG, "null pointer");
    ATSNE_REQUIRE(N >= 1 && N < (1ll << 31), ATSNE_E_INVALID_ARG, "N=%lld out of range", (long long)N);
    ATSNE_REQUIRE(k >= 1 && k <= N - 1, ATSNE_E_K_RANGE, "k=%d out of [1, N-1]", k);
    SymPlan p;
    sym_plan(N, N * (int64_t)k, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch scr;
    ATSNE_TRY(scr.acquire(ws, ws_bytes, p.total, st));
    RowsIn rin{nullptr, k};
    return sym_run(p, rin, nbr_idx, P_cond, row_ptr, col, val, nnz_host, scr.ptr, st);
}

extern "C" atsne_status atsne_symmetrize_csr(const int64_t* in_ptr, const int32_t* in_col, const float* in_val,
                                             int64_t N, int64_t nnz_in_host, int64_t* row_ptr, int32_t* col,
                                             float* val, int64_t* nnz_host, void* ws, size_t ws_bytes,
                                             void* stream) {
    using namespace atsne;
    clear_error();
    ATSNE_REQUIRE(in_ptr && in_col && in_val && row_ptr && col && val && nnz_host, ATSNE_E_INVALID_ARG,
                  "null pointer");
    ATSNE_REQUIRE(N >= 1 && N < (1ll << 31) && nnz_in_host >= 0, ATSNE_E_INVALID_ARG, "bad sizes");
    SymPlan p;
    sym_plan(N, nnz_in_host, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch scr;
    ATSNE_TRY(scr.acquire(ws, ws_bytes, p.total, st));
    RowsIn rin{in_ptr, 0};
    return sym_run(p, rin, in_col, in_val, row_ptr, col, val, nnz_host, scr.ptr, st);
}
