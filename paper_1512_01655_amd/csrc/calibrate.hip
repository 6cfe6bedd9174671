// Perplexity calibration for the A-tSNE similarity path on gfx950.
//
// For every row i, the Gaussian precision beta_i = 1/(2 sigma_i^2) of Eq. 3,
// restricted to the neighbour set of Eq. 8, such that the row's perplexity
// (Eq. 4) equals the target mu.  The entropy is taken in nats (2^{H_2} =
// e^{H_e}) and the row is normalised over its neighbours, so it sums to one.
//
// Distances may come as unevaluated sums hi + lo (the kNN stage's residuals):
// the shift delta_j = d_j - min d then resolves differences below FP32
// resolution of d, which a row of close-together large distances needs for
// its probabilities to be exact to 1e-6.
//
// One wavefront per row: each lane holds ceil(k/64) shifted distances in
// registers; every bisection step costs one exponential per held distance
// and two butterfly reductions (Z and sum w*delta).  H(beta) = ln Z +
// beta * sum p_j delta_j is non-increasing in beta, so bisection on beta
// converges to the unique root whenever m < mu < k (m = multiplicity of the
// minimum distance).  All arithmetic is FP32.
#include <cmath>
#include <vector>

#include "knn_internal.h"
#include "wave.h"

namespace atsne {

constexpr int CAL_MAXR = 16;  // k <= 1024

// Row r of the launch is table row (row_ids ? row_ids[r] : r); rows at or
// beyond *n_rows_dev (when given) are skipped.  Distance and P rows have
// stride `stride`; d2_lo (may be null) holds the distances' residuals.
template <int R>
__global__ __launch_bounds__(256) void calibrate_rows(const float* __restrict__ d2, const float* __restrict__ d2_lo,
                                                      int64_t stride,
                                                      const int32_t* __restrict__ row_ids,
                                                      const int32_t* __restrict__ n_rows_dev, int64_t N, int k,
                                                      float mu, float tol, int max_iter, float* __restrict__ P,
                                                      float* __restrict__ beta_out, float* __restrict__ perp_out,
                                                      uint8_t* __restrict__ flags) {
    const int l = lane_id();
    const int64_t r_ = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r_ >= N || (n_rows_dev && r_ >= *n_rows_dev)) return;
    const int64_t row = row_ids ? (int64_t)row_ids[r_] : r_;
    const float* d = d2 + row * stride;
    const float* dlo = d2_lo ? d2_lo + row * stride : nullptr;
    float dl[R], dlw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int c = l + WAVE * r;
        dl[r] = c < k ? d[c] : INFINITY;
        dlw[r] = (c < k && dlo) ? dlo[c] : 0.f;
    }
    // +inf marks an absent entry (a deleted neighbour): weight 0.  The
    // minimum is taken on (hi, lo) lexicographically; |lo| is at most about
    // half an ulp of hi, so that is the minimum of hi + lo.
    float mn = INFINITY;
#pragma unroll
    for (int r = 0; r < R; ++r) mn = fminf(mn, dl[r]);
    mn = wave_min(mn);
    float mn_lo = INFINITY;
#pragma unroll
    for (int r = 0; r < R; ++r) mn_lo = dl[r] == mn ? fminf(mn_lo, dlw[r]) : mn_lo;
    mn_lo = wave_min(mn_lo);
    float sum = 0.f, zeros = 0.f, live = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (dl[r] < INFINITY) {
            // delta_j >= 0, min 0: Z >= 1, no overflow (hi - mn is exact
            // whenever hi <= 2 mn; the residuals carry what FP32 drops)
            dl[r] = fmaxf(0.f, (dl[r] - mn) + (dlw[r] - mn_lo));
            sum += dl[r];
            zeros += dl[r] == 0.f ? 1.f : 0.f;
            live += 1.f;
        }
    }
    sum = wave_sum(sum);
    zeros = wave_sum(zeros);
    live = wave_sum(live);

    uint8_t fl = 0;
    float b = 0.f;
    float w[R];
    float Z = 0.f;
    if (live == 0.f) {
        // no neighbour left
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = 0.f;
        Z = 1.f;
        fl |= ATSNE_FLAG_DEGENERATE;
    } else if (sum == 0.f || !(mu < live)) {
        // all neighbours equidistant (H = ln live for every beta), or too few
        // left to reach mu: uniform over the present entries
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = dl[r] < INFINITY ? 1.f : 0.f;
        Z = live;
        b = 0.f;
        fl |= ATSNE_FLAG_DEGENERATE;
    } else if (zeros >= mu) {
        // H falls to ln m >= ln mu only as beta -> inf: take the limit
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = dl[r] == 0.f ? 1.f : 0.f;
        Z = zeros;
        b = INFINITY;
        fl |= ATSNE_FLAG_DEGENERATE;
    } else {
        const float target = logf(mu);
        const float htol = tol / mu;  // |e^H - mu| ~ mu |H - ln mu|
        auto entropy = [&](float bb, float& Zo) {
            float z = 0.f, s = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float e = expf(-bb * dl[r]);  // delta = inf (absent or padding) gives 0
                w[r] = e;
                z += e;
                s = fmaf(e, dl[r] < INFINITY ? dl[r] : 0.f, s);
            }
            z = wave_sum(z);
            s = wave_sum(s);
            Zo = z;
            return logf(z) + bb * (s / z);
        };
        float lo = 0.f, hi = live / sum;  // 1 / mean(delta)
        int it = 0;
        float h = entropy(hi, Z);
        while (h > target && it < max_iter) {
            lo = hi;
            hi *= 2.f;
            h = entropy(hi, Z);
            ++it;
        }
        float mid = hi;
        bool done = fabsf(h - target) <= htol;
        bool collapsed = false;
        for (; !done && it < max_iter; ++it) {
            mid = 0.5f * (lo + hi);
            if (!(mid > lo && mid < hi)) {  // bracket collapsed to adjacent floats
                collapsed = true;
                break;
            }
            h = entropy(mid, Z);
            if (fabsf(h - target) <= htol) break;
            if (h > target)
                lo = mid;
            else
                hi = mid;
        }
        if (it >= max_iter)
            fl |= ATSNE_FLAG_NOT_CONVERGED;
        else if (collapsed)
            fl |= ATSNE_FLAG_TOL_LIMITED;  // no FP32 beta meets tol: the entropy's rounding decides
        b = mid;
        h = entropy(b, Z);  // weights of the returned beta
    }
    const float invZ = 1.f / Z;
    float ent = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int c = l + WAVE * r;
        if (c < k) {
            float p = w[r] * invZ;
            P[row * stride + c] = p;
            if (p > 0.f) ent -= p * logf(p);
        }
    }
    ent = wave_sum(ent);
    if (l == 0) {
        beta_out[row] = b;
        if (perp_out) perp_out[row] = expf(ent);
        if (flags) flags[row] |= fl;
    }
}

atsne_status calibrate_table(const float* d2, const float* d2_lo, int64_t stride, const int32_t* row_ids,
                             const int32_t* n_rows_dev, int64_t n_rows, int k, float mu, float tol, int max_iter,
                             float* P, float* beta, float* perp, uint8_t* flags, hipStream_t st) {
    if (n_rows == 0) return ATSNE_OK;
    const dim3 grid((unsigned)ceil_div(n_rows, 4)), block(256);
    const int R = (k + 63) / 64;
    ProfScope ps_("calibrate_rows", st);
#define ATSNE_CAL(RR)                                                                                      \
    calibrate_rows<RR><<<grid, block, 0, st>>>(d2, d2_lo, stride, row_ids, n_rows_dev, n_rows, k, mu, tol, max_iter, P, \
                                               beta, perp, flags)
    if (R <= 1)
        ATSNE_CAL(1);
    else if (R <= 2)
        ATSNE_CAL(2);
    else if (R <= 4)
        ATSNE_CAL(4);
    else if (R <= 8)
        ATSNE_CAL(8);
    else
        ATSNE_CAL(16);
#undef ATSNE_CAL
    ATSNE_LAUNCH_CHECK();
    return ATSNE_OK;
}

}  // namespace atsne

extern "C" atsne_status atsne_calibrate_p(const float* nbr_d2, const float* nbr_d2_lo, int64_t N, int32_t k,
                                          float perplexity, float tol, int32_t max_iter, int32_t strict, float* P_cond,
                                          float* beta, float* perp, uint8_t* flags, void* stream) {
    using namespace atsne;
    clear_error();
    ATSNE_REQUIRE(nbr_d2 && P_cond && beta, ATSNE_E_INVALID_ARG, "null input or output pointer");
    ATSNE_REQUIRE(N >= 0, ATSNE_E_INVALID_ARG, "N=%lld < 0", (long long)N);
    ATSNE_REQUIRE(k >= 1 && k <= 64 * CAL_MAXR, ATSNE_E_K_RANGE, "k=%d out of [1, %d]", k, 64 * CAL_MAXR);
    ATSNE_REQUIRE(perplexity >= 1.0f && perplexity < (float)k, ATSNE_E_K_RANGE,
                  "perplexity %g must be in [1, k=%d)", (double)perplexity, k);
    ATSNE_REQUIRE(!strict || flags, ATSNE_E_INVALID_ARG, "strict calibration needs a flags array");
    if (tol <= 0.f) tol = 1e-5f;
    if (max_iter <= 0) max_iter = 200;
    if (N == 0) return ATSNE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ATSNE_TRY(calibrate_table(nbr_d2, nbr_d2_lo, k, nullptr, nullptr, N, k, perplexity, tol, max_iter, P_cond, beta,
                              perp, flags, st));
    if (strict) {
        std::vector<uint8_t> h((size_t)N);
        ATSNE_HIP(hipMemcpyAsync(h.data(), flags, (size_t)N, hipMemcpyDeviceToHost, st));
        ATSNE_HIP(hipStreamSynchronize(st));
        for (uint8_t f : h)
            if (f & ATSNE_FLAG_NOT_CONVERGED) {
                set_error("calibration did not converge within %d iterations for some row", max_iter);
                return ATSNE_E_NOT_CONVERGED;
            }
    }
    return ATSNE_OK;
}
