// Attractive forces of the t-SNE gradient over the sparse symmetric P on
// gfx950: the consumer of the similarity path's output.
//
// F_i = m_i * sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2), which is the
// attractive term p_ij q_ij Z (y_i - y_j) of Eq. 7 with q_ij Z from Eq. 5 and
// Eq. 6 (the factor 4 of Eq. 7 is left to the caller).  m_i is the global
// (early) exaggeration times the selective exaggeration of Sec. 4.3: a point
// refined at iteration t_ref starts at tau and decays exponentially to 1
// with time constant `decay` iterations.
//
// Layout: one wave per row, 4 rows per 256-thread workgroup.  The wave
// streams its row's (col, val) entries with coalesced 256-byte loads, four
// entries per lane in flight (a row of the symmetric P of a k = 90 graph,
// ~160 entries, takes one step), and gathers y_j (the embedding, N x dims
// FP32, small enough to stay in L2).  The pass is a chain of three dependent
// loads per row (row pointers, entries, embedding rows): at 16 lanes per row
// it took 94 us at N = 70000, at 32 lanes 73 us, at 64 lanes 64 us.
#include <climits>

#include "common.h"
#include "wave.h"

namespace atsne {

constexpr int ATTR_G = 64;  // lanes per row
constexpr int ATTR_U = 4;   // entries per lane in flight

template <int DIMS>
__global__ __launch_bounds__(256) void attractive_rows(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val, int64_t N, int64_t nnz,
                                                       const float* __restrict__ Y, const int32_t* __restrict__ t_ref,
                                                       float tau, float inv_decay, int32_t t_now, float global,
                                                       float* __restrict__ F) {
    const int g = threadIdx.x & (ATTR_G - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / ATTR_G) + (threadIdx.x / ATTR_G);
    if (i >= N) return;  // whole waves leave together
    float yi[DIMS], acc[DIMS];
#pragma unroll
    for (int d = 0; d < DIMS; ++d) {
        yi[d] = Y[i * DIMS + d];
        acc[d] = 0.f;
    }
    const int64_t e0 = row_ptr[i];
    const int64_t e1 = min(row_ptr[i + 1], nnz);
    // ATTR_U entries per lane per step: their column loads, then their
    // embedding gathers, are all in flight together
    for (int64_t eb = e0 + g; eb < e1; eb += ATTR_G * ATTR_U) {
        int32_t j[ATTR_U];
        float p[ATTR_U];
#pragma unroll
        for (int u = 0; u < ATTR_U; ++u) {
            const int64_t e = eb + (int64_t)ATTR_G * u;
            const bool ok = e < e1;
            j[u] = ok ? col[e] : -1;
            p[u] = ok ? val[e] : 0.f;
        }
        float yj[ATTR_U][DIMS];
#pragma unroll
        for (int u = 0; u < ATTR_U; ++u) {
            const bool ok = (uint64_t)j[u] < (uint64_t)N;  // malformed or padding entry: no force
            if (!ok) p[u] = 0.f;
            const int64_t jj = ok ? (int64_t)j[u] : i;
#pragma unroll
            for (int d = 0; d < DIMS; ++d) yj[u][d] = Y[jj * DIMS + d];
        }
#pragma unroll
        for (int u = 0; u < ATTR_U; ++u) {
            float diff[DIMS];
            float d2 = 0.f;
#pragma unroll
            for (int d = 0; d < DIMS; ++d) {
                diff[d] = yi[d] - yj[u][d];
                d2 = fmaf(diff[d], diff[d], d2);
            }
            const float w = p[u] / (1.0f + d2);
#pragma unroll
            for (int d = 0; d < DIMS; ++d) acc[d] = fmaf(w, diff[d], acc[d]);
        }
    }
#pragma unroll
    for (int d = 0; d < DIMS; ++d) {
#pragma unroll
        for (int o = ATTR_G / 2; o >= 1; o >>= 1) acc[d] += __shfl_xor(acc[d], o, ATTR_G);
    }
    if (g == 0) {
        float m = global;
        if (t_ref) {
            const int32_t tr = t_ref[i];
            if (tr >= 0 && tr <= t_now) m *= 1.0f + (tau - 1.0f) * expf(-(float)(t_now - tr) * inv_decay);
        }
#pragma unroll
        for (int d = 0; d < DIMS; ++d) F[i * DIMS + d] = m * acc[d];
    }
}

}  // namespace atsne

using namespace atsne;

extern "C" atsne_status atsne_attractive_forces(const int64_t* row_ptr, const int32_t* col, const float* val,
                                                int64_t N, int64_t nnz, const float* Y, int32_t dims,
                                                const int32_t* t_ref, float tau, float decay, int32_t t_now,
                                                float global_exaggeration, float* F, void* stream) {
    clear_error();
    ATSNE_REQUIRE(N >= 0 && nnz >= 0, ATSNE_E_INVALID_ARG, "negative sizes");
    if (N == 0) return ATSNE_OK;
    ATSNE_REQUIRE(row_ptr && Y && F && (nnz == 0 || (col && val)), ATSNE_E_INVALID_ARG, "null pointer");
    ATSNE_REQUIRE(dims == 2 || dims == 3, ATSNE_E_UNSUPPORTED, "embedding dimension %d (2 or 3)", dims);
    ATSNE_REQUIRE(!t_ref || decay > 0.f, ATSNE_E_INVALID_ARG, "decay must be positive");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned grid = (unsigned)ceil_div(N, 256 / ATTR_G);
    const float inv_decay = t_ref ? 1.0f / decay : 0.f;
    ProfScope ps_("attractive_rows", st);
    if (dims == 2)
        attractive_rows<2><<<grid, 256, 0, st>>>(row_ptr, col, val, N, nnz, Y, t_ref, tau, inv_decay, t_now,
                                                 global_exaggeration, F);
    else
        attractive_rows<3><<<grid, 256, 0, st>>>(row_ptr, col, val, N, nnz, Y, t_ref, tau, inv_decay, t_now,
                                                 global_exaggeration, F);
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}
