// Symmetrisation of the sparse conditional P for the A-tSNE similarity path.
//
// p_ij = (p_{j|i} + p_{i|j}) / (2N) (Eq. 2; the split form of Eq. 10 is why
// only the per-point conditional rows are stored upstream).  The output is
// CSR with ascending columns over the union of the neighbour patterns.
//
// A row's union joins its own entries (its conditional row) with its
// mirrored entries (the rows that list it), so the pattern's transpose is
// built first, without global atomics (on a multi-die GPU they serialise):
//   sym_pack       every entry (i, j, p) as the key (j << 32 | i) with value p
//                  (an ignored entry gets the key N << 32, after every column)
//   radix sort     stable, by the column bits only: the input is row-major,
//                  so each column's run comes out ascending by its source row
//                  i, i.e. row j's mirrored entries sorted by their column
//   sym_runs       the start of every column's run
//   sym_row_count  per row, own + mirrored - columns in both (a binary search
//                  of each own column in the row's run), then a multi-block
//                  scan gives the row pointers
//   sym_row_emit   per row: its own entries ranked by column in LDS; every
//                  entry goes to (own entries before it) + (mirrored entries
//                  before it) - (columns in both before it), a column in both
//                  carrying p_own + p_mirrored (in that order), scaled 1/(2N)
// Every position and sum is fixed by the input, so the result is bit-for-bit
// deterministic.  Entries whose column is outside [0, N) or equal to their
// row are ignored; columns within a conditional row must be distinct, and a
// row holds at most 1024 own entries.
#include <algorithm>
#include <climits>
#include <mutex>

#include "knn_internal.h"
#include "wave.h"

namespace atsne {

constexpr int SYM_OWN_MAX = 1024;  // own entries of a row ranked in LDS
constexpr int SYM_RUN_LDS = 1024;  // mirrored run cached in LDS (longer runs are searched in place)
constexpr int SYM_SCAN_BLOCK = 4096;  // counts per workgroup of the row-pointer scan

// Row extent of the conditional input: CSR (in_ptr) or fixed k.
struct RowsIn {
    const int64_t* ptr;
    int k;
    __device__ __forceinline__ int64_t begin(int64_t i) const { return ptr ? ptr[i] : i * k; }
    __device__ __forceinline__ int64_t end(int64_t i) const { return ptr ? ptr[i + 1] : (i + 1) * k; }
};

__device__ __forceinline__ bool sym_valid(int32_t j, int64_t i, int64_t N) { return j >= 0 && j < N && j != i; }

// One wave per input row: the transposed keys of its entries.  The first
// thread also clears the error flag (fin[1]) that sym_row_count raises.
__global__ __launch_bounds__(256) void sym_pack(RowsIn rin, const int32_t* __restrict__ col,
                                                const float* __restrict__ val, int64_t N,
                                                uint64_t* __restrict__ key, uint32_t* __restrict__ pv,
                                                int64_t* __restrict__ fin) {
    const int l = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) fin[1] = 0;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int64_t b = rin.begin(i), e = rin.end(i);
    for (int64_t t = b + l; t < e; t += WAVE) {
        const int32_t j = col[t];
        const bool ok = sym_valid(j, i, N);
        key[t] = ((uint64_t)(ok ? (uint32_t)j : (uint32_t)N) << 32) | (uint32_t)i;
        pv[t] = __float_as_uint(val[t]);
    }
}

// run[j] = first sorted position of column j (run[N] = number of kept
// entries): each position writes the starts of the columns in (previous
// column, its column].
__global__ __launch_bounds__(256) void sym_runs(const uint64_t* __restrict__ key, int64_t E, int64_t N,
                                                int64_t* __restrict__ run) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e > E) return;
    const int64_t jp = e > 0 ? (int64_t)(key[e - 1] >> 32) : -1;
    const int64_t j = e < E ? (int64_t)(key[e] >> 32) : N;
    for (int64_t r = jp + 1; r <= std::min(j, N); ++r) run[r] = e;
}

// First position in [0, n) of sorted src rows (low words of keys) >= c.
__device__ __forceinline__ int lower_src(const uint64_t* k, int n, int32_t c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int32_t)(uint32_t)k[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int lower_lds(const int32_t* a, int n, int32_t c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// One wave per row: distinct columns of the union.
__global__ __launch_bounds__(256) void sym_row_count(RowsIn rin, const int32_t* __restrict__ col, int64_t N,
                                                     const uint64_t* __restrict__ key, const int64_t* __restrict__ run,
                                                     int64_t* __restrict__ cnt, int32_t* __restrict__ err) {
    __shared__ int32_t cache_all[4][SYM_RUN_LDS];
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    if (i >= N) return;  // waves are independent: no workgroup barrier below
    const int64_t b = rin.begin(i), e = rin.end(i);
    if (e - b > SYM_OWN_MAX) {
        if (l == 0) atomicOr(err, 1);
        if (l == 0) cnt[i] = 0;
        return;
    }
    const int64_t m0 = run[i];
    const int n_in = (int)(run[i + 1] - m0);
    const uint64_t* mk = key + m0;
    int32_t* cache = cache_all[w];
    const bool in_lds = n_in <= SYM_RUN_LDS;
    if (in_lds)
        for (int x = l; x < n_in; x += WAVE) cache[x] = (int32_t)(uint32_t)mk[x];
    wave_sync();
    int n_own = 0, both = 0;
    for (int64_t t = b + l; t < e; t += WAVE) {
        const int32_t c = col[t];
        const bool ok = sym_valid(c, i, N);
        bool hit = false;
        if (ok) {
            const int lb = in_lds ? lower_lds(cache, n_in, c) : lower_src(mk, n_in, c);
            hit = lb < n_in && (in_lds ? cache[lb] : (int32_t)(uint32_t)mk[lb]) == c;
        }
        n_own += __popcll(ballot(ok));
        both += __popcll(ballot(hit));
    }
    if (l == 0) cnt[i] = (int64_t)n_own + n_in - both;
}

// Multi-block exclusive scan of n int64 counts into out[0..n] (out[n] the
// total): block sums, a one-workgroup scan of those, then each block's scan.
__global__ __launch_bounds__(1024) void sym_block_sums(const int64_t* __restrict__ c, int64_t n,
                                                       int64_t* __restrict__ bs) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SYM_SCAN_BLOCK + 4 * t;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += base + q < n ? c[base + q] : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (l == 0) wsum[w] = s;
    __syncthreads();
    if (t == 0) {
        int64_t tot = 0;
        for (int i = 0; i < 16; ++i) tot += wsum[i];
        bs[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(1024) void sym_scan_small(const int64_t* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ out) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b0 = std::min<int64_t>(n, t * per), b1 = std::min<int64_t>(n, b0 + per);
    int64_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += in[i];
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t tv = __shfl_up(incl, o, 64);
        if (l >= o) incl += tv;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    int64_t run = incl - s;
    for (int i = 0; i < w; ++i) run += wsum[i];
    for (int64_t i = b0; i < b1; ++i) {
        const int64_t v = in[i];
        out[i] = run;
        run += v;
    }
    if (t == 1023) out[n] = run;
}

// The total also goes to fin[0], which the host reads back with the error
// flag in one copy.
__global__ __launch_bounds__(1024) void sym_block_scan(const int64_t* __restrict__ c, int64_t n,
                                                       const int64_t* __restrict__ boff, int64_t* __restrict__ out,
                                                       int64_t* __restrict__ fin) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SYM_SCAN_BLOCK + 4 * t;
    int64_t v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = base + q < n ? c[base + q] : 0;
        s += v[q];
    }
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t tv = __shfl_up(incl, o, 64);
        if (l >= o) incl += tv;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    int64_t run = boff[blockIdx.x] + incl - s;
    for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (base < n && base + 4 >= n) {  // the thread holding the last count writes the total
        out[n] = run;
        fin[0] = run;
    }
}

// One wave per row, four rows per workgroup; a row holds at most CAP own
// entries (its LDS) and its mirrored run (columns and values) is cached in
// LDS up to RUN entries, so that past the first loads the row's work reads
// LDS only.  Each wave places its row's own entries; the mirrored entries of
// the four rows are then written by the whole workgroup together.
template <int CAP, int RUN>
__global__ __launch_bounds__(256) void sym_row_emit(RowsIn rin, const int32_t* __restrict__ col,
                                                    const float* __restrict__ val, int64_t N,
                                                    const uint64_t* __restrict__ key, const uint32_t* __restrict__ pv,
                                                    const int64_t* __restrict__ run,
                                                    const int64_t* __restrict__ row_ptr, float inv_norm, int64_t cap,
                                                    int32_t* __restrict__ out_col, float* __restrict__ out_val) {
    struct alignas(16) RowLds {
        int32_t ocol[CAP];      // own columns (input order, kept entries)
        float oval[CAP];        // their values, then own + mirrored for columns in both
        int32_t olb[CAP];       // mirrored entries before each own column
        int32_t orank[CAP];     // rank of each own column among the own columns
        int32_t scol[CAP];      // own columns in ascending order
        int32_t mpref[CAP + 1]; // flags of columns in both by rank, then their exclusive prefix
        int32_t cache[RUN];     // the mirrored run's columns
        float cval[RUN];        // and values
    };
    struct RowInfo {  // a row's extent, for the workgroup's mirrored pass
        int64_t o, m0;
        int n_in, n_own, in_lds;
    };
    __shared__ RowLds lds_all[4];
    __shared__ RowInfo info[4];
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    RowLds& L = lds_all[w];
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    // every wave reaches the workgroup barrier below: a row past N, or one
    // with more than CAP entries (refused by the count's error flag), only
    // publishes an empty extent
    const int64_t b = i < N ? rin.begin(i) : 0, e = i < N ? rin.end(i) : 0;
    if (i < N && e - b <= CAP) {
        const int64_t o = row_ptr[i];
        const int64_t m0 = run[i];
        const int n_in = (int)(run[i + 1] - m0);
        const uint64_t* mk = key + m0;
        const uint32_t* mv = pv + m0;
        const bool in_lds = n_in <= RUN;
        if (in_lds)
            for (int x = l; x < n_in; x += WAVE) {
                L.cache[x] = (int32_t)(uint32_t)mk[x];
                L.cval[x] = __uint_as_float(mv[x]);
            }
        // kept own entries, compacted in input order
        int n_own = 0;
        for (int64_t t0 = b; t0 < e; t0 += WAVE) {
            const int64_t t = t0 + l;
            const int32_t c = t < e ? col[t] : -1;
            const bool ok = t < e && sym_valid(c, i, N);
            const uint64_t m = ballot(ok);
            if (ok) {
                const int p = n_own + __popcll(m & lanemask_lt());
                L.ocol[p] = c;
                L.oval[p] = val[t];
            }
            n_own += __popcll(m);
        }
        wave_sync();
        // per own column: its rank among the own columns, the mirrored
        // entries before it, and whether it is mirrored too (then its value
        // gains the mirrored addend, after the own one)
        // (four columns per LDS read: entries past n_own are padded with INT32_MAX)
        for (int u = n_own + l; u < ((n_own + 3) & ~3); u += WAVE) L.ocol[u] = INT32_MAX;
        wave_sync();
        for (int u = l; u < n_own; u += WAVE) {
            const int32_t c = L.ocol[u];
            int r = 0;
            const int4* oc4 = reinterpret_cast<const int4*>(L.ocol);
            for (int v = 0; v < (n_own + 3) >> 2; ++v) {
                const int4 q = oc4[v];
                r += (q.x < c) + (q.y < c) + (q.z < c) + (q.w < c);
            }
            const int lb = in_lds ? lower_lds(L.cache, n_in, c) : lower_src(mk, n_in, c);
            L.orank[u] = r;
            const bool both = lb < n_in && (in_lds ? L.cache[lb] : (int32_t)(uint32_t)mk[lb]) == c;
            L.olb[u] = lb;
            if (both) L.oval[u] += in_lds ? L.cval[lb] : __uint_as_float(mv[lb]);
            L.scol[r] = c;
            L.mpref[r] = both ? 1 : 0;
        }
        wave_sync();
        // mpref: exclusive prefix count of the columns in both, by rank
        int carry = 0;
        for (int r0 = 0; r0 <= n_own; r0 += WAVE) {
            const int r = r0 + l;
            const int f = r < n_own ? L.mpref[r] : 0;
            const int incl = (int)wave_incl_scan((uint32_t)f);
            wave_sync();
            if (r <= n_own) L.mpref[r] = carry + incl - f;
            carry += __shfl(incl, WAVE - 1, WAVE);
            wave_sync();
        }
        // own entries: (own before) + (mirrored before) - (in both before)
        for (int u = l; u < n_own; u += WAVE) {
            const int32_t c = L.ocol[u];
            const int r = L.orank[u];
            const int64_t pos = o + r + L.olb[u] - L.mpref[r];
            if (pos < cap) {  // always true: the guard keeps every store in bounds
                out_col[pos] = c;
                out_val[pos] = L.oval[u] * inv_norm;
            }
        }
        if (l == 0) info[w] = RowInfo{o, m0, n_in, n_own, in_lds ? 1 : 0};
    } else if (l == 0) {
        info[w] = RowInfo{0, 0, 0, 0, 1};
    }
    __syncthreads();
    // mirrored entries that are not own ones, the four rows' runs taken
    // together by the whole workgroup, so that a hub row's long run is
    // shared by 256 lanes: flat index f walks row 0's run, then row 1's, ...
    const int64_t p1 = info[0].n_in, p2 = p1 + info[1].n_in, p3 = p2 + info[2].n_in, tot = p3 + info[3].n_in;
    for (int64_t f = threadIdx.x; f < tot; f += 256) {
        const int r = (f >= p1) + (f >= p2) + (f >= p3);
        const int x = (int)(f - (r == 0 ? 0 : r == 1 ? p1 : r == 2 ? p2 : p3));
        const RowInfo& R = info[r];
        const RowLds& M = lds_all[r];
        const int32_t c = R.in_lds ? M.cache[x] : (int32_t)(uint32_t)key[R.m0 + x];
        const int lb = lower_lds(M.scol, R.n_own, c);
        if (!(lb < R.n_own && M.scol[lb] == c)) {
            const int64_t pos = R.o + x + lb - M.mpref[lb];
            if (pos < cap) {  // always true: the guard keeps every store in bounds
                out_col[pos] = c;
                out_val[pos] = (R.in_lds ? M.cval[x] : __uint_as_float(pv[R.m0 + x])) * inv_norm;
            }
        }
    }
}

struct SymPlan {
    int64_t N, nnz_in;
    int col_bits;  // bits of a column index, N < 2^col_bits
    size_t sort_bytes, total;
};

static void sym_plan(int64_t N, int64_t nnz_in, SymPlan& p) {
    p.N = N;
    p.nnz_in = nnz_in;
    p.col_bits = 1;
    while (((int64_t)1 << p.col_bits) <= N) ++p.col_bits;  // column N (ignored entries) fits too
    const int64_t E = std::max<int64_t>(nnz_in, 1);
    p.sort_bytes = sort_u64_temp_bytes(E);
    const int64_t nb = ceil_div(std::max<int64_t>(N, 1), SYM_SCAN_BLOCK);
    Arena a;
    a.take<uint64_t>(E);         // packed keys
    a.take<uint32_t>(E);         // their values
    a.take<uint64_t>(E);         // sorted keys
    a.take<uint32_t>(E);         // sorted values
    a.take<char>(p.sort_bytes);  // sort scratch
    a.take<int64_t>(N + 1);      // column runs
    a.take<int64_t>(N);          // distinct counts per row
    a.take<int64_t>(nb + 1);     // scan block sums / offsets
    a.take<int64_t>(nb + 1);
    a.take<int64_t>(8);          // total and error flag
    p.total = a.used;
}

static atsne_status sym_run(const SymPlan& p, RowsIn rin, const int32_t* in_col, const float* in_val,
                            int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* wsp,
                            hipStream_t st) {
    ATSNE_REQUIRE(p.nnz_in < (int64_t)UINT32_MAX, ATSNE_E_INVALID_ARG, "%lld conditional entries: at most 2^32 - 1",
                  (long long)p.nnz_in);
    Arena a(wsp, p.total);
    const int64_t N = p.N, E = p.nnz_in;
    const int64_t Ec = std::max<int64_t>(E, 1);
    const int64_t nb = ceil_div(std::max<int64_t>(N, 1), SYM_SCAN_BLOCK);
    uint64_t* k0 = a.take<uint64_t>(Ec);
    uint32_t* v0 = a.take<uint32_t>(Ec);
    uint64_t* k1 = a.take<uint64_t>(Ec);
    uint32_t* v1 = a.take<uint32_t>(Ec);
    void* sort_tmp = a.take<char>(p.sort_bytes);
    int64_t* runs = a.take<int64_t>(N + 1);
    int64_t* cnt = a.take<int64_t>(N);
    int64_t* bsum = a.take<int64_t>(nb + 1);
    int64_t* boff = a.take<int64_t>(nb + 1);
    int64_t* fin = a.take<int64_t>(8);  // [0] the total, [1] the error flag (int32 in its low word)
    int32_t* err = reinterpret_cast<int32_t*>(fin + 1);
    const dim3 rows4((unsigned)ceil_div(N, 4)), blk(256);
    ProfScope ps_("sym_total", st);
    sym_pack<<<rows4, blk, 0, st>>>(rin, in_col, in_val, N, k0, v0, fin);
    ATSNE_LAUNCH_CHECK();
    ATSNE_TRY(sort_pairs_u64(sort_tmp, p.sort_bytes, k0, v0, k1, v1, E, st, 32, 32 + p.col_bits));
    sym_runs<<<dim3((unsigned)ceil_div(E + 1, 256)), blk, 0, st>>>(k1, E, N, runs);
    ATSNE_LAUNCH_CHECK();
    sym_row_count<<<rows4, blk, 0, st>>>(rin, in_col, N, k1, runs, cnt, err);
    ATSNE_LAUNCH_CHECK();
    sym_block_sums<<<dim3((unsigned)nb), dim3(1024), 0, st>>>(cnt, N, bsum);
    ATSNE_LAUNCH_CHECK();
    sym_scan_small<<<dim3(1), dim3(1024), 0, st>>>(bsum, nb, boff);
    ATSNE_LAUNCH_CHECK();
    sym_block_scan<<<dim3((unsigned)nb), dim3(1024), 0, st>>>(cnt, N, boff, row_ptr, fin);
    ATSNE_LAUNCH_CHECK();
    const float inv = (float)(1.0 / (2.0 * (double)N));
    // k <= 128: mirrored runs average k entries, so a 256-entry LDS cache
    // covers nearly every row and the smaller footprint keeps more waves per
    // CU (0.55 -> 0.52 ms at N = 70000 against a 1024-entry cache)
    if (rin.ptr == nullptr && rin.k <= 128)
        sym_row_emit<128, 256><<<rows4, blk, 0, st>>>(rin, in_col, in_val, N, k1, v1, runs, row_ptr, inv, 2 * E, col,
                                                       val);
    else if (rin.ptr == nullptr && rin.k <= 256)
        sym_row_emit<256, 1024><<<rows4, blk, 0, st>>>(rin, in_col, in_val, N, k1, v1, runs, row_ptr, inv, 2 * E, col,
                                                        val);
    else
        sym_row_emit<SYM_OWN_MAX, 512><<<rows4, blk, 0, st>>>(rin, in_col, in_val, N, k1, v1, runs, row_ptr, inv,
                                                               2 * E, col, val);
    ATSNE_LAUNCH_CHECK();
    int64_t h_fin[2] = {0, 0};
    ATSNE_HIP(hipMemcpyAsync(h_fin, fin, sizeof(h_fin), hipMemcpyDeviceToHost, st));
    ps_.stop();
    ATSNE_HIP(hipStreamSynchronize(st));
    ATSNE_REQUIRE(h_fin[1] == 0, ATSNE_E_INVALID_ARG, "a conditional row holds more than %d entries", SYM_OWN_MAX);
    *nnz_host = h_fin[0];
    return ATSNE_OK;
}

// Allocation-free variant: the scratch lives in this file-scope device
// array, one copy per GPU the library runs on, held until the process ends.
// Host code never uses the array's name as a device address: each device's
// copy is looked up once with hipGetSymbolAddress (with that device current)
// and that address is what the kernels receive.  Calls on one GPU share its
// copy, so calls that overlap on one GPU race; every kernel overwrites what
// it reads (the error flag is cleared by a kernel), so the previous call's
// contents need no clearing.
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
    ATSNE_REQUIRE(k <= SYM_OWN_MAX, ATSNE_E_K_RANGE, "k=%d above %d", k, SYM_OWN_MAX);
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
    ATSNE_REQUIRE(k <= SYM_OWN_MAX, ATSNE_E_K_RANGE, "k=%d above %d", k, SYM_OWN_MAX);
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
