// Device kernels of the serving loop's data manipulation (Sec. 5.3): point
// deletion from the resident neighbour table, the per-row farthest present
// neighbour that Eq. 13 compares against, and the per-row state a snapshot
// reports.  A resident list holds its present entries sorted by (d, j) and
// then absent entries (index -1, distance +inf).
#include <climits>

#include "knn_internal.h"
#include "wave.h"

namespace atsne {

constexpr int PURGE_MAXR = 4;  // resident k <= 256

__global__ __launch_bounds__(256) void serve_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void serve_mark_dead(int32_t* death, const int32_t* ids, int64_t M, int32_t c) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) death[ids[i]] = c;
}

// Commit of the deletion with commit index c over table rows [0, n_rows).
// Rows deleted by this commit are emptied (P = 0, beta = 0).  In every other
// row alive after it, entries whose point was deleted by a commit <= c are
// removed without a replacement; the remaining entries keep their order and
// the list ends in absent entries.  Changed rows are appended to `changed`
// and lose their calibration flags, which the re-calibration sets again.
__global__ __launch_bounds__(256) void serve_purge(int32_t* __restrict__ res_idx, float* __restrict__ res_d2,
                                                   float* __restrict__ res_d2_lo, float* __restrict__ res_P, float* __restrict__ res_beta,
                                                   uint8_t* __restrict__ res_flags, int k, int64_t n_rows,
                                                   const int32_t* __restrict__ death, int32_t c,
                                                   int32_t* __restrict__ changed, int32_t* __restrict__ n_changed) {
    const int l = lane_id();
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int32_t dr = death[row];
    if (dr < c) return;  // emptied by an earlier commit
    int32_t* idx = res_idx + row * k;
    float* d2 = res_d2 + row * k;
    float* d2l = res_d2_lo + row * k;
    if (dr == c) {
        for (int i = l; i < k; i += WAVE) {
            idx[i] = -1;
            d2[i] = INFINITY;
            d2l[i] = 0.f;
            res_P[row * k + i] = 0.f;
        }
        if (l == 0) {
            res_beta[row] = 0.f;
            res_flags[row] = ATSNE_FLAG_DEGENERATE;
        }
        return;
    }
    // the whole row is read before any entry is written
    int32_t ji[PURGE_MAXR];
    float di[PURGE_MAXR], dli[PURGE_MAXR];
    bool keep[PURGE_MAXR];
    int removed = 0;
#pragma unroll
    for (int r = 0; r < PURGE_MAXR; ++r) {
        const int i = l + WAVE * r;
        ji[r] = i < k ? idx[i] : -1;
        di[r] = i < k ? d2[i] : INFINITY;
        dli[r] = i < k ? d2l[i] : 0.f;
        keep[r] = ji[r] >= 0 && death[ji[r]] > c;
        removed += __popcll(ballot(ji[r] >= 0 && !keep[r]));
    }
    if (removed == 0) return;
    int base = 0;
#pragma unroll
    for (int r = 0; r < PURGE_MAXR; ++r) {
        const uint64_t m = ballot(keep[r]);
        if (keep[r]) {
            const int p = base + __popcll(m & lanemask_lt());
            idx[p] = ji[r];
            d2[p] = di[r];
            d2l[p] = dli[r];
        }
        base += __popcll(m);
    }
    for (int i = base + l; i < k; i += WAVE) {
        idx[i] = -1;
        d2[i] = INFINITY;
        d2l[i] = 0.f;
    }
    if (l == 0) {
        res_flags[row] &= (uint8_t)~(ATSNE_FLAG_DEGENERATE | ATSNE_FLAG_NOT_CONVERGED);
        changed[atomicAdd(n_changed, 1)] = (int32_t)row;
    }
}

// Distance to the farthest present neighbour of each row (-inf when none).
__global__ __launch_bounds__(256) void serve_dmax(const int32_t* __restrict__ res_idx, const float* __restrict__ res_d2,
                                                  int k, int64_t n_rows, float* __restrict__ dmax) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n_rows) return;
    float v = -INFINITY;
    for (int i = k - 1; i >= 0; --i)
        if (res_idx[row * k + i] >= 0) {
            v = res_d2[row * k + i];
            break;
        }
    dmax[row] = v;
}

// Per-row state once every commit is applied: precision rho_i (present
// entries / k, which is 1 minus 1/k per removed neighbour) and alive flag.
__global__ __launch_bounds__(256) void serve_row_state(const int32_t* __restrict__ res_idx, int k, int64_t n_rows,
                                                       const int32_t* __restrict__ death, float* __restrict__ rho,
                                                       uint8_t* __restrict__ alive) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n_rows) return;
    int np = 0;
    for (int i = 0; i < k; ++i) np += res_idx[row * k + i] >= 0 ? 1 : 0;
    if (rho) rho[row] = (float)np / (float)k;
    if (alive) alive[row] = death[row] == INT_MAX ? 1 : 0;
}

static unsigned blocks_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, ceil_div(n, per)); }

atsne_status serve_fill_death(int32_t* death, int64_t n, hipStream_t st) {
    serve_fill_i32<<<blocks_of(n, 256), 256, 0, st>>>(death, n, INT_MAX);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

atsne_status serve_mark_deleted(int32_t* death, const int32_t* ids, int64_t M, int32_t c, hipStream_t st) {
    serve_mark_dead<<<blocks_of(M, 256), 256, 0, st>>>(death, ids, M, c);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

atsne_status serve_purge_deleted(int32_t* res_idx, float* res_d2, float* res_d2_lo, float* res_P, float* res_beta,
                                 uint8_t* res_flags, int k, int64_t n_rows, const int32_t* death, int32_t c,
                                 int32_t* changed, int32_t* n_changed, hipStream_t st) {
    ATSNE_REQUIRE(k >= 1 && k <= WAVE * PURGE_MAXR, ATSNE_E_K_RANGE, "resident k=%d above %d", k, WAVE * PURGE_MAXR);
    if (n_rows == 0) return ATSNE_OK;
    ProfScope ps_("serve_purge", st);
    serve_purge<<<blocks_of(n_rows, 4), 256, 0, st>>>(res_idx, res_d2, res_d2_lo, res_P, res_beta, res_flags, k,
                                                      n_rows, death, c, changed, n_changed);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

atsne_status serve_farthest(const int32_t* res_idx, const float* res_d2, int k, int64_t n_rows, float* dmax,
                            hipStream_t st) {
    if (n_rows == 0) return ATSNE_OK;
    serve_dmax<<<blocks_of(n_rows, 256), 256, 0, st>>>(res_idx, res_d2, k, n_rows, dmax);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

atsne_status serve_state(const int32_t* res_idx, int k, int64_t n_rows, const int32_t* death, float* rho,
                         uint8_t* alive, hipStream_t st) {
    if (n_rows == 0 || (!rho && !alive)) return ATSNE_OK;
    serve_row_state<<<blocks_of(n_rows, 256), 256, 0, st>>>(res_idx, k, n_rows, death, rho, alive);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

}  // namespace atsne
