/*
 * atsne.h -- C ABI of the MI355X (gfx950) A-tSNE high-dimensional similarity
 * library, libatsne.so.
 *
 * The library computes the exact sparse joint-probability matrix P that tSNE
 * and its approximated variant A-tSNE start from (Pezzotti et al.,
 * "Approximated and User Steerable tSNE for Progressive Visual Analytics",
 * arXiv:1512.01655):
 *   1. the K nearest neighbours of every point (Sec. 3.1, Eq. 8; squared
 *      Euclidean distance of Eq. 3), K = floor(3 * perplexity);
 *   2. per point, the Gaussian precision beta_i = 1/(2 sigma_i^2) that makes
 *      the row's perplexity equal the target (Eq. 3, Eq. 4), and the
 *      conditional probabilities p_{j|i} over the neighbour set;
 *   3. the symmetric joint p_ij = (p_{j|i} + p_{i|j}) / (2N) (Eq. 2, Eq. 10).
 * plus a serving loop for the paper's steerable, progressive use: point
 * insertion (Sec. 5.3, Eq. 13) and per-point exact refinement of user
 * selections (Sec. 4.3, Sec. 5.1).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless stated
 *     otherwise; the library never frees them.  Matrices are row-major.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on it unless documented to synchronise.
 *   - `ws`/`ws_bytes`: scratch memory owned by the caller, at least the size
 *     reported by the matching *_workspace_size query, 256-byte aligned.
 *     ws == NULL asks the library to allocate (stream-ordered) and release it
 *     inside the call.
 *   - Return value: atsne_status.  On error nothing is launched, outputs are
 *     untouched, and atsne_last_error() returns a message (thread-local).
 *     No C++ exception crosses this boundary.
 *   - Indices are int32 (N < 2^31); CSR row pointers are int64.
 *   - Per-row outcome flags (uint8, device) use the ATSNE_FLAG_* bits.
 */
#ifndef ATSNE_H
#define ATSNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum atsne_status {
    ATSNE_OK = 0,
    ATSNE_E_INVALID_ARG = 1,   /* null pointer, bad size, bad stride, bad precision */
    ATSNE_E_K_RANGE = 2,       /* k < 1, k > N-1, k_cand out of range, perplexity < 1 or >= k */
    ATSNE_E_NOMEM = 3,         /* workspace too small, or an internal allocation failed */
    ATSNE_E_HIP = 4,           /* a HIP runtime call or kernel launch failed */
    ATSNE_E_NOT_CONVERGED = 5, /* strict calibration: some row did not converge */
    ATSNE_E_BUSY = 6,          /* serving: request still pending / results unreleased */
    ATSNE_E_UNSUPPORTED = 7    /* feature or precision not available on this device */
} atsne_status;

/* Arithmetic of the distance contraction (a2).  The neighbour distances
 * returned are always FP32 direct differences of the FP32 source. */
typedef enum atsne_precision {
    ATSNE_PREC_FP32 = 0,     /* exact path: FP32 MFMA, certified candidate margin */
    ATSNE_PREC_BF16 = 1,     /* BF16 (round-to-nearest-even) MFMA, FP32 accumulate */
    ATSNE_PREC_FP8_E4M3 = 2, /* OCP FP8 e4m3 with per-row absmax scales, FP32 accumulate */
    ATSNE_PREC_FP32X3 = 3    /* exact path: each FP32 value split into BF16 hi + BF16 lo
                                (x = hi + lo + r, |r| <= 2^-18 |x|), contraction
                                hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulate;
                                results identical to ATSNE_PREC_FP32 (same FP32 direct-
                                difference distances, same certificate with this
                                contraction's error bound, same exact-scan fallback) */
} atsne_precision;

/* Per-row flags. */
#define ATSNE_FLAG_FP64_RERANKED 0x01u /* k-th/(k+1)-th gap below FP32 resolution: ranked in FP64 */
#define ATSNE_FLAG_NOT_CONVERGED 0x02u /* bisection hit max_iter before reaching tol */
#define ATSNE_FLAG_DEGENERATE 0x04u    /* target perplexity unreachable (equal or repeated distances) */
#define ATSNE_FLAG_EXACT_SCAN 0x08u    /* FP32 path: candidate margin not certified; row redone by exact scan */
#define ATSNE_FLAG_TOL_LIMITED 0x10u   /* bisection ended at adjacent FP32 betas before |e^H - mu| <= tol */

/* Thread-local description of the last error on this thread ("" if none). */
const char* atsne_last_error(void);
/* Library version string. */
const char* atsne_version(void);
/* Device info for measurement: CU count and peak engine clock (kHz) of the current device. */
atsne_status atsne_device_info(int32_t* n_cu, int32_t* clock_khz, int32_t* gcn_arch_major);

/* Kernel timing for measurement (not needed for results).  When enabled,
 * every kernel the library launches is bracketed by HIP events recorded on
 * the stream it runs on; atsne_profile_read synchronises those events and
 * returns, for kernels whose name starts with `name`, the summed elapsed
 * time (ms) and the launch count.  Enabling clears earlier records. */
atsne_status atsne_profile_enable(int32_t on);
atsne_status atsne_profile_read(const char* name, double* total_ms, int64_t* count);

/* ------------------------------------------------------------------ kNN -- */

/* Scratch bytes needed by atsne_knn / atsne_knn_subset for a corpus of N rows
 * of dimension D, M query rows, k neighbours and k_cand candidates
 * (0 = the precision's default), on the current device: the candidate slots
 * take up to a sixteenth of its memory (between 2 and 16 GiB), and query
 * rows beyond what that holds are searched in batches. */
atsne_status atsne_knn_workspace_size(int64_t N, int64_t M, int32_t D, atsne_precision prec, int32_t k,
                                      int32_t k_cand, size_t* bytes);

/* Exact K nearest neighbours of every row of X among the other rows
 * (Sec. 3.1, Eq. 8; squared Euclidean distance of Eq. 3).
 *   X        [N x ld] FP32, row i = point x_i (first D columns used).
 *   prec     arithmetic of the candidate search; see atsne_precision.
 *   k        neighbours per row (the paper's K = floor(3 mu)), 1 <= k <= N-1.
 *   k_cand   candidates re-ranked per row, k <= k_cand <= min(N-1, 1024);
 *            0 selects the default (FP32: k + max(32, k/2); BF16/FP8: 2k).
 *   nbr_idx  [N x k] int32 out: neighbour indices, ascending by (d, j).
 *   nbr_d2   [N x k] FP32 out: squared distances of the FP32 rows, a
 *            compensated FP32 direct difference rounded to FP32 (FP64 when
 *            ATSNE_FLAG_FP64_RERANKED).
 *   nbr_d2_lo [N x k] FP32 out (may be NULL): each distance's residual, so
 *            that nbr_d2 + nbr_d2_lo is the distance to well below FP32
 *            resolution; atsne_calibrate_p takes it to resolve distance
 *            differences that FP32 rounding of nbr_d2 would blur.
 *   flags    [N] uint8 out (may be NULL): ATSNE_FLAG_FP64_RERANKED,
 *            ATSNE_FLAG_EXACT_SCAN.
 * Self is excluded by index; exact duplicates are neighbours at distance 0;
 * equal distances are ordered by the lower index.  Asynchronous, except a
 * seeded search (below), which synchronises the stream.
 * Seeding (ATSNE_PREC_FP8_E4M3, N >= 2^18 contiguous rows, ld == D): the
 *   search first bounds each row's k_cand-th smallest key code from the
 *   keys near it (a k-means partition of about N/1000 clusters, the row's
 *   own cluster and its 7 nearest searched with the same FP8 tile), so its
 *   tiles keep about k_cand keys per row from the start instead of every
 *   key below a threshold that tightens as the corpus streams past.  The
 *   outputs are those of the unseeded search bit for bit.  The pass
 *   allocates its own device memory (about 9 GB at its peak for N = 10^6,
 *   freed before the search) whatever ws is.  Without that memory, for D
 *   above 4096, or when the cells would cover more than a tenth of all row
 *   pairs, the search runs unseeded; ATSNE_FP8_SEED=0 in the environment
 *   turns the pass off.  With kernel timing on, the pass is one "seed_total"
 *   record, plus an empty "seed_declined" record when it stepped aside.
 */
atsne_status atsne_knn(const float* X, int64_t N, int32_t D, int64_t ld, atsne_precision prec, int32_t k,
                       int32_t k_cand, int32_t* nbr_idx, float* nbr_d2, float* nbr_d2_lo, uint8_t* flags, void* ws,
                       size_t ws_bytes, void* stream);

/* As atsne_knn for the M query rows query_ids[0..M) (device int32, each in
 * [0, N)) of the corpus X[0..N); each query excludes itself.  Outputs are
 * [M x k] and [M]; with M = 0 the call checks its sizes and returns, and
 * query_ids and the outputs may be NULL.  This is the per-point exact refinement of Sec. 4.3
 * applied to a selection (Sec. 5.1). */
atsne_status atsne_knn_subset(const float* X, int64_t N, int32_t D, int64_t ld, const int32_t* query_ids,
                              int64_t M, atsne_precision prec, int32_t k, int32_t k_cand, int32_t* nbr_idx,
                              float* nbr_d2, float* nbr_d2_lo, uint8_t* flags, void* ws, size_t ws_bytes,
                              void* stream);

/* ----------------------------------------------------------- calibration -- */

/* Perplexity calibration (Eq. 3, Eq. 4 restricted to the neighbour set of
 * Eq. 8), one wavefront per row, bisection on beta in FP32.
 *   nbr_d2     [N x k] FP32 squared neighbour distances (any order).
 *   nbr_d2_lo  [N x k] FP32 residuals of nbr_d2 (as written by atsne_knn), or
 *              NULL: the row's distances are then nbr_d2 + nbr_d2_lo.  With
 *              them, p_{j|i} matches an FP64 calibration of the exact
 *              distances to about 2e-7 on rows whose distances are close
 *              together relative to their size (the image-like workload);
 *              from FP32 distances alone the shift d_j - min d carries their
 *              rounding (up to one ulp of d) into p.
 *   perplexity target mu, 1 <= mu < k.
 *   tol        stop when |e^H - mu| <= tol (<= 0: default 1e-5), judged on
 *              H = ln Z + beta <delta> evaluated in FP32; bisection also
 *              stops when the bracket collapses to adjacent floats, and then
 *              flags the row ATSNE_FLAG_TOL_LIMITED.  Accuracy: H carries its
 *              FP32 rounding (the spacing of floats near ln mu plus the
 *              summation over k terms), so the achieved perplexity of the
 *              returned P is within about 1e-6 mu of mu whatever tol asks:
 *              within 1e-4 for mu <= 100 (the paper uses 5-50), within
 *              2e-6 mu above (3.8e-4 measured at mu = 333, k = 1000), with
 *              or without the flag.
 *   max_iter   bisection cap (<= 0: default 200).
 *   strict     nonzero: synchronise the stream and return
 *              ATSNE_E_NOT_CONVERGED if any row carries NOT_CONVERGED.
 *   P_cond     [N x k] FP32 out: p_{j|i}, aligned with nbr_d2; rows sum to 1.
 *   beta       [N] FP32 out: 1/(2 sigma_i^2) (+inf for a degenerate row whose
 *              limit is beta -> inf; 0 when all distances are equal).
 *   perp       [N] FP32 out (may be NULL): achieved perplexity e^H of the row.
 *   flags      [N] uint8 in/out (may be NULL): NOT_CONVERGED, DEGENERATE and
 *              TOL_LIMITED are OR-ed into the existing bits.
 * Rows whose minimum-distance multiplicity m satisfies m >= mu cannot reach
 * mu: they get the beta -> inf limit (uniform over the m) and DEGENERATE.
 * An entry of +inf is absent (a removed neighbour, Sec. 5.3): it gets p = 0
 * and the row is calibrated over its present entries; a row with no more
 * than mu present entries is uniform over them and DEGENERATE. */
atsne_status atsne_calibrate_p(const float* nbr_d2, const float* nbr_d2_lo, int64_t N, int32_t k, float perplexity,
                               float tol, int32_t max_iter, int32_t strict, float* P_cond, float* beta, float* perp,
                               uint8_t* flags, void* stream);

/* -------------------------------------------------------- symmetrisation -- */

/* Scratch bytes for atsne_symmetrize / atsne_symmetrize_csr with N rows and
 * at most nnz_in conditional entries (N*k for the fixed-k form). */
atsne_status atsne_symmetrize_workspace_size(int64_t N, int64_t nnz_in, size_t* bytes);

/* Symmetric joint P of Eq. 2 (equivalently the split form of Eq. 10):
 * p_ij = (p_{j|i} + p_{i|j}) / (2N) on the union of the neighbour patterns.
 *   nbr_idx, P_cond  [N x k] neighbour indices and p_{j|i} (from atsne_knn
 *                    and atsne_calibrate_p); indices in [0, N), no self.
 *   row_ptr  [N+1] int64 out; col [2*N*k] int32 out; val [2*N*k] FP32 out
 *            (capacity 2*N*k; the first *nnz_host entries are written).
 *            Columns ascending within a row, no diagonal entries.
 *   nnz_host HOST int64 out: number of stored entries, N*k <= nnz <= 2*N*k.
 * Synchronises the stream once (to read nnz). */
atsne_status atsne_symmetrize(const int32_t* nbr_idx, const float* P_cond, int64_t N, int32_t k,
                              int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* ws,
                              size_t ws_bytes, void* stream);

/* As atsne_symmetrize, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument, and the call allocates nothing.  Its
 * scratch is a 64 MiB device array inside the library, one per GPU, held
 * until the process ends; that limits it to about 1.8 million conditional
 * entries (N * k), and larger inputs return ATSNE_E_NOMEM before any work.
 * Calls that overlap on one GPU share that array and race: serialise them.
 * Same outputs, bit for bit, as atsne_symmetrize; synchronises the stream
 * once (to read nnz). */
atsne_status atsne_symmetrize_noalloc(const int32_t* nbr_idx, const float* P_cond, int64_t N, int32_t k,
                                      int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_host, void* stream);

/* As atsne_symmetrize for conditional rows of varying length given as CSR:
 * in_ptr [N+1] int64 with in_ptr[0] = 0, in_col/in_val [in_ptr[N]] (device),
 * columns distinct within a row, in [0, N), no self.  Output capacity
 * 2*in_ptr[N]; nnz_in_host is in_ptr[N] (host copy, so no extra sync). */
atsne_status atsne_symmetrize_csr(const int64_t* in_ptr, const int32_t* in_col, const float* in_val,
                                  int64_t N, int64_t nnz_in_host, int64_t* row_ptr, int32_t* col, float* val,
                                  int64_t* nnz_host, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------- attractive forces -- */

/* Attractive term of the gradient (Eq. 7) over the sparse symmetric P, the
 * consumer of atsne_symmetrize's output:
 *   F_i = m_i * sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2)
 * with q_ij Z = 1/(1 + |y_i - y_j|^2) from Eq. 5 and Eq. 6; the factor 4 of
 * Eq. 7 is left to the caller.  m_i = global_exaggeration, times
 * 1 + (tau - 1) exp(-(t_now - t_ref[i]) / decay) when 0 <= t_ref[i] <= t_now:
 * the selective exaggeration with exponential decay of Sec. 4.3 (a point
 * refined at iteration t_ref[i] starts at tau).
 *   row_ptr [N+1] int64, col [nnz] int32, val [nnz] FP32: device CSR of P
 *           (as written by atsne_symmetrize); entries whose column is outside
 *           [0, N) are skipped, row ends are clamped to nnz.
 *   Y       [N x dims] FP32 device, row-major embedding; dims is 2 or 3.
 *   t_ref   [N] int32 device iteration of each point's last refinement
 *           (negative: never), or NULL for no selective exaggeration.
 *   F       [N x dims] FP32 device out.
 * Asynchronous on `stream`.  Errors: E_INVALID_ARG (null pointers, negative
 * sizes, decay <= 0 with t_ref), E_UNSUPPORTED (dims). */
atsne_status atsne_attractive_forces(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t N,
                                     int64_t nnz, const float* Y, int32_t dims, const int32_t* t_ref, float tau,
                                     float decay, int32_t t_now, float global_exaggeration, float* F,
                                     void* stream);

/* ------------------------------------ precision-controlled approximate kNN -- */

/* The paper reaches a user precision rho (Eq. 9) with a randomized kd-forest
 * whose parameters are fitted to rho (Sec. 4.2).  This library reaches it
 * with a cluster-pruned brute-force search on the matrix cores:
 *   build  k-means (Lloyd, `iters` updates) from the caller's initial points
 *          init_ids_host[n_clusters] (distinct, in [0, N)); each update sets a
 *          centroid to the mean of its members (an empty cluster keeps its
 *          centroid); the assignment is the exact nearest centroid by
 *          (squared distance, index), taken again after the last update.  The
 *          corpus is sorted by (cluster, index); each cluster's probe order is
 *          itself, then the other clusters by (centroid distance, index).
 *   knn    every point's candidate clusters are its cluster's first n_probe
 *          probe clusters, with further probe clusters added until their rows
 *          number at least k + 1; the search covers the 256-row tiles of the
 *          sorted corpus that overlap those clusters' rows (a superset of
 *          them: the tile kernel works on whole tiles), and the result is the
 *          exact FP32 kNN over the covered rows (same re-rank, tie rule and
 *          FP64 near-tie handling as atsne_knn; the contraction is FP32X3,
 *          whose results equal FP32's).  n_probe >= n_clusters gives the
 *          exact kNN.
 *   fit    the smallest n_probe whose precision (Eq. 9, against the exact
 *          kNN) over all points of the sample clusters reaches rho; precision
 *          never decreases with n_probe, so it is found by bisection.
 * X is a device FP32 [N x D] corpus (copied; the index owns its memory).
 * Limits: 2 <= n_clusters <= min(N, 1024), D <= 4096, k + max(32, k/2) <= 1024.
 * All calls synchronise `stream`. */
typedef struct atsne_ivf atsne_ivf;
atsne_status atsne_ivf_build(const float* X, int64_t N, int32_t D, int32_t n_clusters, const int32_t* init_ids_host,
                             int32_t iters, atsne_ivf** out, void* stream);
/* The partition: assign [N] int32 device, centroids [n_clusters x D] FP32
 * device, cluster_start_host [n_clusters + 1] (rows of the sorted corpus),
 * probe_host [n_clusters x n_clusters]; any pointer may be NULL. */
atsne_status atsne_ivf_partition(const atsne_ivf* ix, int32_t* assign, float* centroids, int64_t* cluster_start_host,
                                 int32_t* probe_host, void* stream);
/* Approximate kNN of all N points, in the layout of atsne_knn (neighbour ids
 * are corpus ids; a row with fewer than k candidates would end in -1/+inf,
 * which the k + 1 rule prevents).  *candidate_fraction_host (may be NULL):
 * mean candidate rows per point / N, the work relative to the exact search. */
atsne_status atsne_ivf_knn(atsne_ivf* ix, int32_t k, int32_t n_probe, int32_t* nbr_idx, float* nbr_d2,
                           uint8_t* flags, double* candidate_fraction_host, void* stream);
atsne_status atsne_ivf_fit(atsne_ivf* ix, int32_t k, float rho, const int32_t* sample_clusters_host, int32_t n_sample,
                           int32_t* n_probe_out, float* rho_sample_out, void* stream);
atsne_status atsne_ivf_destroy(atsne_ivf* ix);

/* -------------------------------------------------- refinement ordering -- */

/* Orderings of Sec. 5.1 that decide which points to refine first (the
 * caller then issues refine requests in that order).  Scratch: at most
 * atsne_order_workspace_size(max(N, M)) bytes; ws may be NULL (then the
 * library allocates stream-ordered scratch). */
atsne_status atsne_order_workspace_size(int64_t N, size_t* bytes);

/* Density-based refinement (Sec. 5.1): the selection `ids` (device int32
 * [M], or NULL for all N points, M == N) sorted by sigma_i descending, i.e.
 * beta_i ascending (sigma_i = 1/sqrt(2 beta_i), beta from
 * atsne_calibrate_p), ties by index: points of sparse regions first.
 *   beta       [N] FP32 device.
 *   order_out  [M] int32 device out.
 * Asynchronous, except that a selection is validated with one
 * synchronisation (E_INVALID_ARG if an id is outside [0, N)). */
atsne_status atsne_order_density(const float* beta, int64_t N, const int32_t* ids, int64_t M, int32_t* order_out,
                                 void* ws, size_t ws_bytes, void* stream);

/* Breadth-first refinement (Sec. 5.1): a visit of the graph of the kNN
 * relationships (edge i -> j for every j in N_i; index -1 is no edge) from
 * the user selection `seeds`.
 *   weighted = 0: hop count from the nearest seed (the breadth-first visit);
 *                 max_depth >= 0 stops the visit at that many hops.
 *   weighted = 1: the visit driven by a priority queue on high-dimensional
 *                 distance: shortest path length from the selection with
 *                 edge weight ||x_i - x_j|| = sqrt(nbr_d2) (FP32 sums; the
 *                 result is the least fixed point, independent of
 *                 scheduling); max_depth must be negative.
 *   nbr_idx [N x k] int32, nbr_d2 [N x k] FP32 device (as from atsne_knn).
 *   seeds   [n_seeds] int32 device, in [0, N) (else E_INVALID_ARG).
 *   key_out [N] FP32 device out (may be NULL): hop count or path length,
 *           +inf for points the visit does not reach.
 *   order_out [N] int32 device out: the reached points sorted by
 *           (key, index); *n_reached_host (HOST) receives their number.
 * Synchronises once per visited level. */
atsne_status atsne_order_neighbourhood(const int32_t* nbr_idx, const float* nbr_d2, int64_t N, int32_t k,
                                       const int32_t* seeds, int64_t n_seeds, int32_t weighted, int32_t max_depth,
                                       float* key_out, int32_t* order_out, int64_t* n_reached_host, void* ws,
                                       size_t ws_bytes, void* stream);

/* --------------------------------------------------------------- serving -- */
/* A server owns a device-resident corpus and its exact similarity state
 * (neighbour lists, conditional rows, beta) and processes requests with
 * continuous batching: requests that arrive while others run are admitted as
 * slots and HBM budget free up, and their row tiles share the same batched
 * kernel launches.  Two request kinds follow the paper's steerable use:
 *   insert  (Sec. 5.3, Eq. 13): B new points join the corpus; their exact
 *           neighbours are computed against the corpus (and each other), and
 *           every resident row i takes a new point a when ||x_a - x_i|| is
 *           below its current farthest neighbour d_i^Max, evicting it.
 *   refine  (Sec. 4.3, Sec. 5.1): the exact neighbourhood and P row of a
 *           user selection of M resident points is recomputed at a requested
 *           perplexity (K_i = floor(3 mu_i) per row).
 *   delete  (Sec. 5.3): points leave the corpus; every resident list drops
 *           them without a replacement, the row's precision rho_i falls by
 *           1/K per removed neighbour, and changed rows are re-calibrated.
 *           A shortened list stays short: Eq. 13 compares with, and evicts,
 *           the farthest neighbour still listed.  Inserting new
 *           points and deleting the oldest gives the sliding window of Sec. 8.
 * Inserts and deletes are commits, applied in arrival order.  Every request
 * carries a view (`epoch`): the number of commits submitted before it.  A
 * request sees exactly the corpus those commits define, so its result does
 * not depend on what else shares the GPU.
 * Latency stamps (atsne_result.t_*_ms) start at the caller's submit call.
 * Failure: if a batched launch or a commit fails, the server stops serving:
 * it waits for its streams to drain, completes every admitted and queued
 * request with that status, and refuses later submissions (and snapshots)
 * with it; results already delivered stay valid until released. */

typedef struct atsne_server atsne_server;

typedef struct atsne_serve_config {
    size_t hbm_budget_bytes; /* cap on request scratch in flight (0 = 4 GiB) */
    int32_t max_slots;       /* max requests in flight at once (0 = 8) */
    int64_t capacity_rows;   /* corpus rows the server can grow to (0 = 2 * N) */
    int32_t max_batch_rows;  /* rows per batched launch (0 = 8192); a request with more rows
                                is split across launches */
    int32_t device;          /* HIP device ordinal (-1 = current) */
} atsne_serve_config;

typedef struct atsne_result {
    uint64_t req_id;
    int32_t kind;            /* 0 insert, 1 refine, 2 delete */
    int32_t status;          /* atsne_status of the request */
    uint64_t epoch;          /* corpus version the request ran against */
    int64_t n_rows;          /* rows in the result (B or M) */
    int32_t k;               /* neighbours per row */
    float perplexity;
    const int32_t* row_ids;  /* device [n_rows]: corpus ids of the result rows */
    const int32_t* nbr_idx;  /* device [n_rows x k] */
    const float* nbr_d2;     /* device [n_rows x k] */
    const float* P_cond;     /* device [n_rows x k] */
    const float* beta;       /* device [n_rows] */
    const uint8_t* flags;    /* device [n_rows] */
    int64_t n_changed;       /* insert/delete: resident rows whose list changed */
    const int32_t* changed;  /* device [n_changed] corpus ids (insert/delete) */
    double t_submit_ms, t_admit_ms, t_complete_ms; /* host clock, ms since server start */
} atsne_result;

typedef struct atsne_serve_stats {
    uint64_t submitted, completed, released;
    uint64_t launches;        /* batched kNN launches issued */
    uint64_t rows_processed;
    int64_t corpus_rows;
    size_t bytes_in_flight;
    size_t peak_bytes_in_flight;
    int32_t max_concurrent;   /* most requests admitted (in flight) at once */
    int32_t max_requests_per_launch; /* most distinct requests sharing one batched launch */
} atsne_serve_stats;

/* Create a server over a copy of corpus [N x D] (device or host FP32, row
 * stride D), with its exact kNN at perplexity mu (k = floor(3 mu)) computed
 * at creation.  Every search of the server runs the FP32X3 contraction; its
 * results equal those of atsne_knn with ATSNE_PREC_FP32.  *out receives the
 * handle. */
atsne_status atsne_serve_create(const atsne_serve_config* cfg, const float* corpus, int64_t N, int32_t D,
                                float perplexity, atsne_server** out);
/* Queue an insert of B points X_new [B x D] (device FP32).  Returns at once
 * with *req_id; the data is copied before return. */
atsne_status atsne_serve_submit_insert(atsne_server* s, const float* X_new, int32_t B, uint64_t* req_id);
/* Queue a delete of M corpus ids (host int32 array, alive at submission). */
atsne_status atsne_serve_submit_delete(atsne_server* s, const int32_t* ids_host, int32_t M, uint64_t* req_id);
/* Queue a refine of M corpus ids (host int32 array) at perplexity mu. */
atsne_status atsne_serve_submit_refine(atsne_server* s, const int32_t* ids_host, int32_t M, float perplexity,
                                       uint64_t* req_id);
/* Non-blocking: ATSNE_E_BUSY while pending, else fills *out. */
atsne_status atsne_serve_poll(atsne_server* s, uint64_t req_id, atsne_result* out);
/* Blocking wait for completion, then fills *out. */
atsne_status atsne_serve_wait(atsne_server* s, uint64_t req_id, atsne_result* out);
/* Free a completed request's result buffers (server-owned until then). */
atsne_status atsne_serve_release(atsne_server* s, uint64_t req_id);
atsne_status atsne_serve_stats_get(atsne_server* s, atsne_serve_stats* out);
/* Snapshot of the server's state once every submitted commit is applied:
 * copies the corpus rows, the resident k-lists (absent entries are index -1,
 * distance +inf, P 0; deleted rows are all absent), their conditional P and
 * beta, the per-row precision rho (present entries / k: 1 for an exact row,
 * 1/k less per removed neighbour, 0 for a deleted row) and the alive flags
 * into caller device buffers of capacity cap_rows (any pointer may be NULL).
 * Synchronises. */
atsne_status atsne_serve_snapshot(atsne_server* s, int64_t cap_rows, float* corpus, int32_t* nbr_idx,
                                  float* nbr_d2, float* P_cond, float* beta, float* rho, uint8_t* alive,
                                  int64_t* n_rows, uint64_t* epoch);
/* Destroy: waits for in-flight work; ATSNE_E_BUSY if results are unreleased
 * and force == 0. */
atsne_status atsne_serve_destroy(atsne_server* s, int32_t force);

#ifdef __cplusplus
}
#endif

#endif /* ATSNE_H */
