/*
 * atsne_oracle.c -- FP64 CPU oracle for the A-tSNE high-dimensional
 * similarity computation (Pezzotti et al., "Approximated and User Steerable
 * tSNE for Progressive Visual Analytics", arXiv:1512.01655).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (all arithmetic in IEEE double, inputs are FP32 upcast
 * exactly):
 *   - atsne_oracle_knn: exact K nearest neighbours by brute force over the
 *     squared Euclidean distance of Eq. 3 (Sec. 3), computed by direct
 *     difference.  Self is excluded by index (the k != i of Eq. 3).  Ties are
 *     broken by the lower index, i.e. rows are ordered by the key (d, j).
 *     K = floor(3*mu) is the neighbourhood size of Sec. 3.1 (Eq. 8).
 *   - atsne_oracle_knn_candidates: the same ranking restricted to a
 *     per-query candidate set (the definition of a candidate-restricted,
 *     approximate search).
 *   - atsne_oracle_calibrate: per row, the Gaussian precision beta = 1/(2
 *     sigma^2) of Eq. 3 restricted to the neighbour set (Eq. 8) such that the
 *     row's perplexity (Eq. 4) equals mu, found by bisection on beta.  The
 *     entropy is taken in nats: 2^{H_2} = e^{H_e}, so Eq. 4 is H_e = ln mu.
 *   - atsne_oracle_symmetrize: the joint p_ij = (p_{j|i} + p_{i|j}) / (2N) of
 *     Eq. 2, equivalently the split form of Eq. 10, as CSR with ascending
 *     columns.
 *   - atsne_oracle_attractive: the attractive term of the gradient (Eq. 7)
 *     over the sparse symmetric P, sum_j p_ij q_ij Z (y_i - y_j) with
 *     q_ij Z = 1/(1 + |y_i - y_j|^2) (Eq. 5, Eq. 6), scaled per point by the
 *     exaggeration of Sec. 4.3.
 *
 * Readings of the paper taken here (the paper is silent or literal-minded):
 *   - Eq. 8 writes the normaliser as a sum over all k != i; the sparse rows
 *     are normalised over the neighbour set only, so each row sums to one.
 *   - The entropy of Eq. 4 is summed over the neighbour set.
 *   - Degenerate rows (the target perplexity is unreachable because m >= mu
 *     neighbours sit at the minimum distance, or all distances are equal) are
 *     flagged and given the limiting distribution.
 *   - Selective exaggeration with exponential decay (Sec. 4.3) gives no
 *     formula: point i refined at iteration t_ref has its attraction scaled
 *     by 1 + (tau - 1) exp(-(t - t_ref)/decay), times the global early
 *     exaggeration factor.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (exact-rational brute force, closed forms, invariants, metamorphic
 * relations); see the test files for the list.
 *
 * Planted mistakes: building with -DORACLE_MUTANT=n (n > 0) plants one
 * deliberate bug so that the tests can show that the pins catch it.  The
 * default build (ORACLE_MUTANT undefined or 0) is the oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

#define FLAG_DEGENERATE 4u
#define FLAG_NOT_CONVERGED 2u

/* ------------------------------------------------------------------------ */
/* Distances and K nearest neighbours                                        */
/* ------------------------------------------------------------------------ */

/* Squared Euclidean distance ||x_a - x_b||^2 of Eq. 3, by direct difference. */
static double sq_dist(const float* a, const float* b, int32_t D) {
    double s = 0.0;
    int32_t d_end = D;
#if ORACLE_MUTANT == 3
    d_end = D - 1; /* planted: drops the last coordinate */
#endif
    for (int32_t d = 0; d < d_end; ++d) {
        double t = (double)a[d] - (double)b[d];
#if ORACLE_MUTANT == 4
        s += fabs(t); /* planted: L1 instead of squared L2 */
#else
        s += t * t;
#endif
    }
    return s;
}

typedef struct {
    double d;
    int32_t j;
} entry_t;

/* Strict total order on (distance, index): the tie rule "lower index wins". */
static int key_less(entry_t a, entry_t b) {
#if ORACLE_MUTANT == 1
    if (a.d != b.d) return a.d < b.d;
    return a.j > b.j; /* planted: higher index wins ties */
#else
    if (a.d != b.d) return a.d < b.d;
    return a.j < b.j;
#endif
}

/* Max-heap (by key_less) of the K+1 smallest keys seen so far. */
static void heap_sift_down(entry_t* h, int n, int i) {
    for (;;) {
        int l = 2 * i + 1, r = l + 1, big = i;
        if (l < n && key_less(h[big], h[l])) big = l;
        if (r < n && key_less(h[big], h[r])) big = r;
        if (big == i) return;
        entry_t t = h[i];
        h[i] = h[big];
        h[big] = t;
        i = big;
    }
}

static void heap_sift_up(entry_t* h, int i) {
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!key_less(h[p], h[i])) return;
        entry_t t = h[i];
        h[i] = h[p];
        h[p] = t;
        i = p;
    }
}

static int cmp_entry(const void* pa, const void* pb) {
    entry_t a = *(const entry_t*)pa, b = *(const entry_t*)pb;
    if (key_less(a, b)) return -1;
    if (key_less(b, a)) return 1;
    return 0;
}

/*
 * Exact kNN.  Queries are the corpus rows query_ids[m] (or row m when
 * query_ids is NULL, M == N); the corpus is rows 0..N-1 of X (row stride ld).
 * For every query, all j != self are ranked by (d, j) and the first K kept,
 * ascending.  d2_next[m] receives the (K+1)-th distance (+inf when the
 * corpus has no K+1 other rows); the set tie rule needs it.
 * Returns 0, or -1 on bad arguments.
 */
int atsne_oracle_knn(const float* X, int64_t N, int32_t D, int64_t ld,
                     const int32_t* query_ids, int64_t M, int32_t K,
                     int32_t* idx, double* d2, double* d2_next, int32_t nthreads) {
    if (!X || !idx || !d2 || N < 1 || D < 1 || ld < D || K < 1 || M < 0) return -1;
    if (K > N - 1) return -1;
    if (!query_ids && M != N) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        entry_t* heap = (entry_t*)malloc(sizeof(entry_t) * (size_t)(K + 1));
        if (!heap) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t m = 0; m < M; ++m) {
            if (!heap) continue;
            int64_t q = query_ids ? query_ids[m] : m;
            if (q < 0 || q >= N) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            const float* xq = X + q * ld;
            int n = 0;
            for (int64_t j = 0; j < N; ++j) {
#if ORACLE_MUTANT == 2
                /* planted: self is not excluded */
#else
                if (j == q) continue;
#endif
                entry_t e;
                e.d = sq_dist(xq, X + j * ld, D);
                e.j = (int32_t)j;
                if (n < K + 1) {
                    heap[n] = e;
                    heap_sift_up(heap, n);
                    ++n;
                } else if (key_less(e, heap[0])) {
                    heap[0] = e;
                    heap_sift_down(heap, n, 0);
                }
            }
            qsort(heap, (size_t)n, sizeof(entry_t), cmp_entry);
            for (int32_t t = 0; t < K; ++t) {
                idx[m * K + t] = heap[t].j;
                d2[m * K + t] = heap[t].d;
            }
            if (d2_next) d2_next[m] = (n > K) ? heap[K].d : INFINITY;
        }
        free(heap);
    }
    return bad ? -1 : 0;
}

/*
 * Exact kNN of each query over its own candidate set: query m (corpus row
 * query_ids[m]) ranks the rows cand_idx[cand_ptr[m] .. cand_ptr[m+1]) other
 * than itself by (d, j) and keeps the first K; when fewer than K remain, the
 * tail is index -1 with distance +inf.  d2_next as for atsne_oracle_knn.
 * This is the definition of a candidate-restricted (approximate) search.
 * Returns 0, or -1 on bad arguments.
 */
int atsne_oracle_knn_candidates(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* query_ids,
                                int64_t M, const int64_t* cand_ptr, const int32_t* cand_idx, int32_t K,
                                int32_t* idx, double* d2, double* d2_next, int32_t nthreads) {
    if (!X || !query_ids || !cand_ptr || !idx || !d2 || N < 1 || D < 1 || ld < D || K < 1 || M < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        entry_t* heap = (entry_t*)malloc(sizeof(entry_t) * (size_t)(K + 1));
        if (!heap) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t m = 0; m < M; ++m) {
            if (!heap) continue;
            const int64_t q = query_ids[m];
            if (q < 0 || q >= N) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            const float* xq = X + q * ld;
            int n = 0;
            for (int64_t e0 = cand_ptr[m]; e0 < cand_ptr[m + 1]; ++e0) {
                const int64_t j = cand_idx[e0];
                if (j < 0 || j >= N) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                if (j == q) continue;
                entry_t e;
                e.d = sq_dist(xq, X + j * ld, D);
                e.j = (int32_t)j;
                if (n < K + 1) {
                    heap[n] = e;
                    heap_sift_up(heap, n);
                    ++n;
                } else if (key_less(e, heap[0])) {
                    heap[0] = e;
                    heap_sift_down(heap, n, 0);
                }
            }
            qsort(heap, (size_t)n, sizeof(entry_t), cmp_entry);
            for (int32_t t = 0; t < K; ++t) {
                idx[m * K + t] = t < n ? heap[t].j : -1;
                d2[m * K + t] = t < n ? heap[t].d : INFINITY;
            }
            if (d2_next) d2_next[m] = (n > K) ? heap[K].d : INFINITY;
        }
        free(heap);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Perplexity calibration                                                    */
/* ------------------------------------------------------------------------ */

/* Entropy in nats of the row p_j(beta) = e^{-beta delta_j} / Z:
 * H = ln Z + beta * sum_j p_j delta_j.  delta >= 0 with min 0, so Z >= 1. */
static double row_entropy(const double* delta, int32_t K, double beta) {
    double Z = 0.0, S = 0.0;
    int32_t k_end = K;
#if ORACLE_MUTANT == 6
    k_end = K - 1; /* planted: normaliser misses the last neighbour */
#endif
    for (int32_t t = 0; t < k_end; ++t) {
#if ORACLE_MUTANT == 5
        double w = exp(-beta * delta[t] * 0.5); /* planted: wrong kernel width (sigma vs 2 sigma^2) */
#else
        double w = exp(-beta * delta[t]);
#endif
        Z += w;
        S += w * delta[t];
    }
    return log(Z) + beta * S / Z;
}

static void row_probs(const double* delta, int32_t K, double beta, double* p) {
    double Z = 0.0;
    for (int32_t t = 0; t < K; ++t) {
#if ORACLE_MUTANT == 5
        p[t] = exp(-beta * delta[t] * 0.5);
#else
        p[t] = exp(-beta * delta[t]);
#endif
        Z += p[t];
    }
#if ORACLE_MUTANT == 6
    Z -= p[K - 1];
#endif
    for (int32_t t = 0; t < K; ++t) p[t] /= Z;
}

/*
 * Calibrate rows of squared neighbour distances d2 (M rows of K) to the
 * target perplexity mu[m] (one per row; mu_scalar when mu is NULL).
 * Outputs P (conditional p_{j|i}, aligned with d2), beta (= 1/(2 sigma^2)),
 * perp (achieved e^{H} recomputed from the returned row) and flags
 * (bit1: bisection hit max_iter, bit2: degenerate row).
 * Returns 0, or -1 on bad arguments (mu must satisfy 1 <= mu < K).
 */
int atsne_oracle_calibrate(const double* d2, int64_t M, int32_t K, const double* mu,
                           double mu_scalar, int32_t max_iter, double* P, double* beta,
                           double* perp, uint8_t* flags, int32_t nthreads) {
    if (!d2 || !P || !beta || !perp || !flags || M < 0 || K < 1) return -1;
    if (max_iter <= 0) max_iter = 2000;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        double* delta = (double*)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(dynamic, 64)
        for (int64_t m = 0; m < M; ++m) {
            if (!delta) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            const double target_mu = mu ? mu[m] : mu_scalar;
            if (!(target_mu >= 1.0) || !(target_mu < (double)K)) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            const double* d = d2 + m * K;
            double* p = P + m * K;
            double dmin = d[0];
            for (int32_t t = 1; t < K; ++t)
                if (d[t] < dmin) dmin = d[t];
            double mean = 0.0;
            int32_t zeros = 0;
            for (int32_t t = 0; t < K; ++t) {
#if ORACLE_MUTANT == 7
                delta[t] = dmin - d[t]; /* planted: wrong sign of the shift */
#else
                delta[t] = d[t] - dmin;
#endif
                mean += delta[t];
                if (delta[t] == 0.0) ++zeros;
            }
            mean /= (double)K;
            uint8_t f = 0;
            double b;
            if (mean == 0.0) {
                /* All neighbours equidistant: H(beta) = ln K for every beta. */
                for (int32_t t = 0; t < K; ++t) p[t] = 1.0 / (double)K;
                b = 0.0;
                f |= FLAG_DEGENERATE;
            } else if ((double)zeros >= target_mu) {
                /* H decreases to ln(zeros) >= ln mu as beta -> inf: take the limit. */
                for (int32_t t = 0; t < K; ++t) p[t] = (delta[t] == 0.0) ? 1.0 / (double)zeros : 0.0;
                b = INFINITY;
                f |= FLAG_DEGENERATE;
            } else {
                const double target = log(target_mu);
                double lo = 0.0, hi = 1.0 / mean;
                int32_t it = 0;
                /* Expand the bracket until H(hi) < ln mu; H is non-increasing. */
                while (row_entropy(delta, K, hi) > target && it < max_iter) {
                    lo = hi;
                    hi *= 2.0;
                    ++it;
                }
                double mid = 0.5 * (lo + hi);
                for (; it < max_iter; ++it) {
                    mid = 0.5 * (lo + hi);
                    double h = row_entropy(delta, K, mid);
                    if (fabs(h - target) <= 1e-13) break;
                    if (h > target)
                        lo = mid;
                    else
                        hi = mid;
                    if (hi - lo <= 1e-15 * hi) {
                        mid = 0.5 * (lo + hi);
                        break;
                    }
                }
                if (it >= max_iter) f |= FLAG_NOT_CONVERGED;
                b = mid;
                row_probs(delta, K, b, p);
            }
            /* Achieved perplexity of the returned row, e^{-sum p ln p}. */
            double H = 0.0;
            for (int32_t t = 0; t < K; ++t)
                if (p[t] > 0.0) H -= p[t] * log(p[t]);
            beta[m] = b;
            perp[m] = exp(H);
            flags[m] = f;
        }
        free(delta);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Symmetrisation                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t r, c;
    double v;
} triple_t;

static int cmp_triple(const void* pa, const void* pb) {
    const triple_t* a = (const triple_t*)pa;
    const triple_t* b = (const triple_t*)pb;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

/*
 * Symmetrise conditional rows given as CSR (in_ptr[N+1], in_col, in_val:
 * row i holds p_{j|i} for j in its neighbour set) into the joint
 * p_ij = (p_{j|i} + p_{i|j}) / (2N) of Eq. 2 / Eq. 10.  Output CSR with
 * ascending columns: out_ptr[N+1], out_col/out_val with capacity cap.
 * Returns nnz >= 0, or -1 on bad arguments / insufficient capacity.
 */
int64_t atsne_oracle_symmetrize(const int64_t* in_ptr, const int32_t* in_col,
                                const double* in_val, int64_t N, int64_t* out_ptr,
                                int32_t* out_col, double* out_val, int64_t cap) {
    if (!in_ptr || !in_col || !in_val || !out_ptr || N < 1) return -1;
    int64_t nin = in_ptr[N];
    triple_t* t = (triple_t*)malloc(sizeof(triple_t) * (size_t)(2 * nin + 1));
    if (!t) return -1;
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t e = in_ptr[i]; e < in_ptr[i + 1]; ++e) {
            int32_t j = in_col[e];
            if (j < 0 || j >= N) {
                free(t);
                return -1;
            }
            double p = in_val[e];
            t[n].r = (int32_t)i; /* p_{j|i} lands on (i, j) ... */
            t[n].c = j;
            t[n].v = p;
            ++n;
#if ORACLE_MUTANT == 9
            /* planted: mirrored term dropped */
#else
            t[n].r = j; /* ... and, mirrored, on (j, i) */
            t[n].c = (int32_t)i;
            t[n].v = p;
            ++n;
#endif
        }
    }
    qsort(t, (size_t)n, sizeof(triple_t), cmp_triple);
    int64_t nnz = 0;
    for (int64_t i = 0; i <= N; ++i) out_ptr[i] = 0;
    const double norm = 2.0 * (double)N;
    for (int64_t a = 0; a < n;) {
        int64_t b = a;
        double s = 0.0;
        while (b < n && t[b].r == t[a].r && t[b].c == t[a].c) s += t[b++].v;
        if (nnz >= cap) {
            free(t);
            return -1;
        }
        out_col[nnz] = t[a].c;
#if ORACLE_MUTANT == 8
        out_val[nnz] = s / (double)N; /* planted: normaliser N instead of 2N */
#else
        out_val[nnz] = s / norm;
#endif
        out_ptr[t[a].r + 1]++;
        ++nnz;
        a = b;
    }
    for (int64_t i = 0; i < N; ++i) out_ptr[i + 1] += out_ptr[i];
    free(t);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Attractive forces of the gradient (Eq. 5, Eq. 6, Eq. 7)                   */
/* ------------------------------------------------------------------------ */

/*
 * Exaggeration multiplier of point i at iteration t_now: the global factor
 * (early exaggeration) times the selective one of Sec. 4.3, which is tau at
 * the iteration t_ref the point was refined and decays exponentially to 1
 * with time constant `decay` iterations.  t_ref < 0 or t_ref > t_now: no
 * selective exaggeration.
 */
static double exaggeration(const int32_t* t_ref, int64_t i, double tau, double decay, int32_t t_now,
                           double global) {
    double m = global;
    if (t_ref && t_ref[i] >= 0 && t_ref[i] <= t_now)
        m *= 1.0 + (tau - 1.0) * exp(-(double)(t_now - t_ref[i]) / decay);
    return m;
}

/*
 * F_i = m_i * sum_j p_ij q_ij Z (y_i - y_j), with q_ij Z = 1 / (1 + |y_i - y_j|^2)
 * (Eq. 5, Eq. 6): the attractive term of the gradient of Eq. 7 (without the
 * factor 4), over the sparse symmetric P given as CSR (row_ptr[N+1], col,
 * val).  Y is N x dims (row-major), F is N x dims.  Returns 0, or -1 on bad
 * arguments.
 */
int atsne_oracle_attractive(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t N,
                            const double* Y, int32_t dims, const int32_t* t_ref, double tau, double decay,
                            int32_t t_now, double global, double* F) {
    if (!row_ptr || !col || !val || !Y || !F || N < 1 || dims < 1 || dims > 8 || !(decay > 0.0)) return -1;
    for (int64_t i = 0; i < N; ++i) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (j < 0 || j >= N) return -1;
            double d2 = 0.0;
            for (int32_t d = 0; d < dims; ++d) {
                const double t = Y[i * dims + d] - Y[(int64_t)j * dims + d];
                d2 += t * t;
            }
#if ORACLE_MUTANT == 10
            const double w = val[e] / (1.0 + sqrt(d2)); /* planted: distance instead of squared distance */
#else
            const double w = val[e] / (1.0 + d2);
#endif
            for (int32_t d = 0; d < dims; ++d) {
#if ORACLE_MUTANT == 11
                acc[d] += w * (Y[(int64_t)j * dims + d] - Y[i * dims + d]); /* planted: wrong direction */
#else
                acc[d] += w * (Y[i * dims + d] - Y[(int64_t)j * dims + d]);
#endif
            }
        }
        const double m = exaggeration(t_ref, i, tau, decay, t_now, global);
        for (int32_t d = 0; d < dims; ++d) F[i * dims + d] = m * acc[d];
    }
    return 0;
}

int atsne_oracle_mutant(void) { return ORACLE_MUTANT; }

int atsne_oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
