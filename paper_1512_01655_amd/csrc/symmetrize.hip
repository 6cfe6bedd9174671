// Symmetrisation of the sparse conditional P for the A-tSNE similarity path.
//
// p_ij = (p_{j|i} + p_{i|j}) / (2N) (Eq. 2; the split form of Eq. 10 is why
// only the per-point conditional rows are stored upstream).  The output is
// CSR with ascending columns over the union of the neighbour patterns.
//
// Device pipeline (HBM bound; one global key sort instead of per-row sorts,
// so hub rows of the kNN graph cost no more than any other entries):
//   sym_keys     each conditional entry (i, j, p_{j|i}) becomes two keys,
//                (row i, column j, own) and (row j, column i, mirrored),
//                both carrying p_{j|i}
//   radix sort   of the 2*nnz (key, value) pairs over the 2b+1 key bits
//                (b bits per index), giving row-major, column-ascending order
//                with the own half of a column before its mirrored half
//   sym_heads    per 1024 sorted entries: number of distinct (row, column)
//   scan         exclusive block offsets (one workgroup)
//   sym_emit     each distinct (row, column) adds its at most two addends,
//                scales by 1/(2N) and lands at its CSR position; the first
//                entry of each row (and every empty row before it) writes
//                row_ptr
// All keys are distinct and each output value is the sum of at most two
// addends, so the result is bit-for-bit deterministic.
#include <algorithm>
#include <mutex>

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "wave.h"

namespace atsne {

constexpr int SYM_BLOCK = 1024;  // sorted entries per sym_heads / sym_emit workgroup (256 threads x 4)
constexpr uint64_t SYM_NONE = ~0ull;  // sentinel key: (SYM_NONE >> 1) equals no real (row, column) pair
// Radix passes at every size above one block's worth: rocPRIM's default
// switches to a merge sort below 2^20 items, which is slower here (18 merge
// launches for the 3.6e5 pairs of N = 2000, k = 90: the whole
// symmetrisation took 0.27 ms that way, 0.125 ms with radix passes).
using SymSortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                 rocprim::default_config, 0>;

// Row extent of the conditional input: CSR (in_ptr) or fixed k.
struct RowsIn {
    const int64_t* ptr;
    int k;
    __device__ __forceinline__ int64_t begin(int64_t i) const { return ptr ? ptr[i] : i * k; }
    __device__ __forceinline__ int64_t end(int64_t i) const { return ptr ? ptr[i + 1] : (i + 1) * k; }
};

// Key layout: row << s | column << 1 | origin (0 own, 1 mirrored), s = b + 1.
__global__ __launch_bounds__(256) void sym_keys(RowsIn rin, const int32_t* __restrict__ col,
                                                const float* __restrict__ val, int64_t N, int s,
                                                ulonglong2* __restrict__ key, float2* __restrict__ kval) {
    const int l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int64_t b = rin.begin(i), e = rin.end(i);
    const uint64_t ui = (uint64_t)i;
    for (int64_t t = b + l; t < e; t += WAVE) {
        const uint64_t j = (uint64_t)(uint32_t)col[t];
        const float p = val[t];
        key[t] = make_ulonglong2((ui << s) | (j << 1), (j << s) | (ui << 1) | 1);
        kval[t] = make_float2(p, p);
    }
}

// Sum of v over a 256-thread workgroup (result valid in every thread).
__device__ __forceinline__ int block_sum256(int v, int* red) {
    const int w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void sym_heads(const uint64_t* __restrict__ key, int64_t n,
                                                 int64_t* __restrict__ block_sums) {
    __shared__ int red[4];
    const int64_t base = (int64_t)blockIdx.x * SYM_BLOCK + 4 * threadIdx.x;
    int c = 0;
    if (base < n) {
        uint64_t prev = base > 0 ? key[base - 1] >> 1 : SYM_NONE;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base + q < n) {
                const uint64_t kq = key[base + q] >> 1;
                c += kq != prev;
                prev = kq;
            }
        }
    }
    const int tot = block_sum256(c, red);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// In-place exclusive scan of nb block counts by one workgroup (each thread
// takes a contiguous run); *total receives the sum.
__global__ __launch_bounds__(1024) void sym_scan_blocks(int64_t* __restrict__ bs, int64_t nb, int64_t* __restrict__ total) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = std::min<int64_t>(nb, t * per), b1 = std::min<int64_t>(nb, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bs[b];
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t tv = __shfl_up(incl, o, 64);
        if (l >= o) incl += tv;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    int64_t woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int64_t run = woff + incl - s;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = bs[b];
        bs[b] = run;
        run += v;
    }
    if (t == 1023) *total = woff + incl;
}

struct EmitArgs {
    const uint64_t* key;
    const float* v;
    int64_t n, N;
    int s;
    uint64_t cmask;  // (1 << b) - 1
    const int64_t* block_off;
    float inv_norm;
    int64_t* row_ptr;
    int32_t* col;
    float* val;
};

__global__ __launch_bounds__(256) void sym_emit(EmitArgs a) {
    __shared__ int64_t wsum[4];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SYM_BLOCK + 4 * t;
    // kk[0] = predecessor, kk[1..4] = own entries, kk[5] = successor
    uint64_t kk[6];
    int c = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int64_t e = base + q - 1;
        kk[q] = (base < a.n && e >= 0 && e < a.n) ? a.key[e] : SYM_NONE;
    }
    bool h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = base + q < a.n && (kk[q + 1] >> 1) != (kk[q] >> 1);
        c += h[q];
    }
    int64_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t tv = __shfl_up(incl, o, 64);
        if (l >= o) incl += tv;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    if (base >= a.n) return;
    int64_t woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    int64_t pos = a.block_off[blockIdx.x] + woff + incl - c;
    int64_t prow = base > 0 ? (int64_t)(kk[0] >> a.s) : -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = base + q;
        if (e < a.n) {
            const uint64_t kq = kk[q + 1];
            const int64_t row = (int64_t)(kq >> a.s);
            // rows (prow, row] start here: row's first entry and the empty rows before it
            for (int64_t r = prow + 1; r <= std::min(row, a.N - 1); ++r) a.row_ptr[r] = pos;
            prow = row;
            if (h[q]) {
                float x = a.v[e];
                if ((kk[q + 2] >> 1) == (kq >> 1)) x += a.v[e + 1];  // own + mirrored
                a.col[pos] = (int32_t)((kq >> 1) & a.cmask);
                a.val[pos] = x * a.inv_norm;
                ++pos;
            }
            if (e == a.n - 1)  // rows after the last stored row are empty
                for (int64_t r = row + 1; r < a.N; ++r) a.row_ptr[r] = pos;
        }
    }
}

__global__ __launch_bounds__(256) void sym_zero_rows(int64_t* __restrict__ row_ptr, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) row_ptr[i] = 0;
}

struct SymPlan {
    int64_t N, nnz_in, n2, nb;
    int b;  // bits per index
    size_t sort_bytes, total;
};

static void sym_plan(int64_t N, int64_t nnz_in, SymPlan& p) {
    p.N = N;
    p.nnz_in = nnz_in;
    p.n2 = 2 * nnz_in;
    p.nb = std::max<int64_t>(1, ceil_div(p.n2, SYM_BLOCK));
    p.b = N > 1 ? 64 - __builtin_clzll((unsigned long long)(N - 1)) : 1;
    p.sort_bytes = 0;
    rocprim::double_buffer<uint64_t> kb(nullptr, nullptr);
    rocprim::double_buffer<float> vb(nullptr, nullptr);
    (void)rocprim::radix_sort_pairs<SymSortConfig>(nullptr, p.sort_bytes, kb, vb, (size_t)std::max<int64_t>(p.n2, 1), 0,
                                    (unsigned)(2 * p.b + 1));
    p.sort_bytes = std::max<size_t>(p.sort_bytes, 1);
    const int64_t n2 = std::max<int64_t>(p.n2, 1);
    Arena a;
    a.take<uint64_t>(n2);        // keys (ping)
    a.take<uint64_t>(n2);        // keys (pong)
    a.take<float>(n2);           // values (ping)
    a.take<float>(n2);           // values (pong)
    a.take<int64_t>(p.nb);       // block offsets
    a.take<char>(p.sort_bytes);  // radix sort temporary storage
    p.total = a.used;
}

static atsne_status sym_run(const SymPlan& p, RowsIn rin, const int32_t* in_col, const float* in_val,
                            int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* wsp,
                            hipStream_t st) {
    Arena a(wsp, p.total);
    const int64_t n2 = std::max<int64_t>(p.n2, 1);
    uint64_t* k0 = a.take<uint64_t>(n2);
    uint64_t* k1 = a.take<uint64_t>(n2);
    float* v0 = a.take<float>(n2);
    float* v1 = a.take<float>(n2);
    int64_t* bsum = a.take<int64_t>(p.nb);
    void* sort_tmp = a.take<char>(p.sort_bytes);
    const int64_t N = p.N;
    ProfScope ps_("sym_total", st);
    if (p.n2 == 0) {
        sym_zero_rows<<<dim3((unsigned)ceil_div(N + 1, 256)), dim3(256), 0, st>>>(row_ptr, N + 1);
        ATSNE_LAUNCH_CHECK();
    } else {
        const int s = p.b + 1;
        sym_keys<<<dim3((unsigned)ceil_div(N, 4)), dim3(256), 0, st>>>(rin, in_col, in_val, N, s,
                                                                       reinterpret_cast<ulonglong2*>(k0),
                                                                       reinterpret_cast<float2*>(v0));
        ATSNE_LAUNCH_CHECK();
        rocprim::double_buffer<uint64_t> kb(k0, k1);
        rocprim::double_buffer<float> vb(v0, v1);
        size_t sort_bytes = p.sort_bytes;
        ATSNE_HIP(rocprim::radix_sort_pairs<SymSortConfig>(sort_tmp, sort_bytes, kb, vb, (size_t)p.n2, 0, (unsigned)(2 * p.b + 1),
                                            st));
        const uint64_t* K = kb.current();
        const float* V = vb.current();
        sym_heads<<<dim3((unsigned)p.nb), dim3(256), 0, st>>>(K, p.n2, bsum);
        ATSNE_LAUNCH_CHECK();
        sym_scan_blocks<<<dim3(1), dim3(1024), 0, st>>>(bsum, p.nb, row_ptr + N);
        ATSNE_LAUNCH_CHECK();
        EmitArgs e{K, V, p.n2, N, s, (1ull << p.b) - 1, bsum, (float)(1.0 / (2.0 * (double)N)), row_ptr, col, val};
        sym_emit<<<dim3((unsigned)p.nb), dim3(256), 0, st>>>(e);
        ATSNE_LAUNCH_CHECK();
    }
    ATSNE_HIP(hipMemcpyAsync(nnz_host, row_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ps_.stop();
    ATSNE_HIP(hipStreamSynchronize(st));
    return ATSNE_OK;
}

// Allocation-free variant: the scratch lives in this file-scope device
// array, one copy per GPU the library runs on, held until the process ends.
// Host code never uses the array's name as a device address: each device's
// copy is looked up once with hipGetSymbolAddress (with that device current)
// and that address is what the kernels receive.  Calls on one GPU share its
// copy, so calls that overlap on one GPU race; every kernel overwrites what
// it reads, so the previous call's contents need no clearing.
constexpr size_t SYM_NOALLOC_SCRATCH = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[SYM_NOALLOC_SCRATCH];

static atsne_status noalloc_scratch(void** out) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static void* addr[MAX_DEV] = {};
    int dev = -1;
    ATSNE_HIP(hipGetDevice(&dev));
    ATSNE_REQUIRE(dev >= 0 && dev < MAX_DEV, ATSNE_E_UNSUPPORTED, "device ordinal %d above %d", dev, MAX_DEV - 1);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        ATSNE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        ATSNE_REQUIRE(p != nullptr, ATSNE_E_HIP, "no device address for the symmetrisation scratch");
        addr[dev] = p;
    }
    *out = addr[dev];
    return ATSNE_OK;
}

}  // namespace atsne

extern "C" atsne_status atsne_symmetrize_noalloc(const int32_t* nbr_idx, const float* P_cond, int64_t N, int32_t k,
                                                 int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host,
                                                 void* stream) {
    using namespace atsne;
    clear_error();
    ATSNE_REQUIRE(nbr_idx && P_cond && row_ptr && col && val && nnz_host, ATSNE_E_INVALID_ARG, "null pointer");
    ATSNE_REQUIRE(N >= 1 && N < (1ll << 31), ATSNE_E_INVALID_ARG, "N=%lld out of range", (long long)N);
    ATSNE_REQUIRE(k >= 1 && k <= N - 1, ATSNE_E_K_RANGE, "k=%d out of [1, N-1]", k);
    SymPlan p;
    sym_plan(N, N * (int64_t)k, p);
    ATSNE_REQUIRE(p.total <= SYM_NOALLOC_SCRATCH, ATSNE_E_NOMEM,
                  "N=%lld, k=%d needs %zu bytes of scratch, above the %zu of the allocation-free symmetrisation "
                  "(use atsne_symmetrize)",
                  (long long)N, k, p.total, SYM_NOALLOC_SCRATCH);
    void* ws = nullptr;
    ATSNE_TRY(noalloc_scratch(&ws));
    RowsIn rin{nullptr, k};
    return sym_run(p, rin, nbr_idx, P_cond, row_ptr, col, val, nnz_host, ws, static_cast<hipStream_t>(stream));
}

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
