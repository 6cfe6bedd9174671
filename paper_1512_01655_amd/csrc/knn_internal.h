// Internal C++ interface of the kNN search, shared by the C ABI entry points
// (knn.hip) and the serving loop (serve.cpp).  Not part of the public ABI.
#pragma once

#include "common.h"

namespace atsne {

constexpr int KNN_KT = 256;  // keys per tile; corpus rows are padded to a multiple

// A device-resident corpus prepared for the contraction: padded copy in the
// contraction's element type, row norms, per-row scales (FP8) and the prefix
// maximum of the norms (pmax[i] = max_{j <= i} n_j, used by the error bound).
struct Corpus {
    int prec = ATSNE_PREC_FP32;
    const float* X = nullptr;  // FP32 source rows (re-rank reads these)
    int64_t ld = 0;
    int32_t D = 0, Dp = 0;
    int n_chunks = 0;
    int64_t row_units = 0;  // 16-byte units per padded row
    int64_t rows_cap = 0;   // padded row capacity (multiple of KNN_KT)
    void* Xp = nullptr;
    float* norms = nullptr;
    float* scales = nullptr;
    float* pmax = nullptr;
    float* pmax_blk = nullptr;  // chunk carries of the prefix max (scratch of corpus_prep)
    // Optional per-row deletion stamps (serving): row j is visible to a
    // request whose view is v iff death[j] >= v (INT32_MAX = never deleted).
    const int32_t* death = nullptr;
};

size_t corpus_bytes(int prec, int64_t rows_cap, int32_t D);
// Carve the corpus buffers out of `mem` (corpus_bytes bytes, 256-aligned).
void corpus_bind(Corpus& c, int prec, const float* X, int64_t ld, int32_t D, int64_t rows_cap, void* mem);
// Prepare rows [r0, r1) (r1 <= rows_cap; rows >= n_live are zero padding).
// pmax is extended from pmax[r0 - 1], so earlier rows must be prepared.
atsne_status corpus_prep(const Corpus& c, int64_t r0, int64_t r1, int64_t n_live, hipStream_t st);

// One launch worth of query rows.  Per-row arrays are device pointers; a
// null pointer selects the uniform value next to it.
struct Batch {
    int64_t M = 0;
    const int32_t* qids = nullptr;  // corpus id of row m (also its self id); null: m0 + m
    int64_t m0 = 0;
    const int32_t* nlims = nullptr;  // keys valid below nlims[m]; null: nlim
    int64_t nlim = 0;
    int64_t key_lo = 0;  // keys valid at or above key_lo
    const int32_t* ks = nullptr;
    int k = 0;
    const int32_t* kcs = nullptr;
    int kc = 0;
    const float* tau0 = nullptr;  // reverse mode: per-row distance that candidates must beat
    int64_t tau0_stride = 0;      // element stride of tau0 (rows' d_max inside a neighbour table)
    const int32_t* views = nullptr;  // per-row view for deletion visibility; null: view
    int32_t view = 0;
    // Seeded threshold (plain search): tau_seed[q] (indexed by corpus id) is
    // at least the k'-th smallest key code d' of row q over all keys, so the
    // tile keeps only keys with d' <= tau_seed[q] from the start; the
    // candidates, and so every output, are those of the unseeded search.
    const float* tau_seed = nullptr;
    // Threshold mode (seeding pass): the select writes, for batch row m with
    // corpus id q, the k'-th smallest d' of its candidates (+inf with fewer)
    // to tau_out[tau_map ? tau_map[q] : q] and writes no neighbour lists.
    float* tau_out = nullptr;
    const int32_t* tau_map = nullptr;
    // Select order (full search in one batch): the select takes batch rows
    // in the order sel_order[0..M) (a permutation of [0, M)), e.g. grouped
    // by cluster so that consecutive rows gather overlapping candidate rows
    // through the caches; outputs stay at their rows.
    const int32_t* sel_order = nullptr;
    // Tile lists (restricted search, FP32, FP32X3, FP8): block b holds batch rows
    // [blk_q[b], blk_q[b+1]) (at most KNN_KT of them) and searches the key
    // tiles tl_idx[blk_t[b] .. blk_t[b+1]) (distinct; ascending where the
    // exact scan may walk them, any order in threshold mode); row_blk[m] is
    // the block of row m.  Null blk_q: every row searches [key_lo, nlim).
    int64_t n_blocks = 0;
    const int32_t* blk_q = nullptr;
    const int32_t* blk_t = nullptr;
    const int32_t* tl_idx = nullptr;
    const int32_t* row_blk = nullptr;
    int32_t* out_idx = nullptr;
    float* out_d2 = nullptr;
    float* out_d2_lo = nullptr;  // residuals of out_d2 (may be null)
    uint8_t* out_flags = nullptr;
    int64_t out_stride = 0;
};

struct SearchPlan {
    int MB = 0, S = 1, tiles_per_split = 1, tile_lo = 0, tile_hi = 0, cap = 0, kc_max = 0, k_max = 0, qb = 256;
    bool small = false;  // 128 x 128 tile geometry (plain search only)
    // balanced schedule (plain search, large geometry): `stream_wgs`
    // workgroups, one per CU, each an equal share of the (query block, key
    // tile) units; 0 = the task grid
    int stream_wgs = 0;
    int kt = KNN_KT;     // keys per tile
    int64_t M = 0;
    size_t ws_bytes = 0;
};

// Plan a search of M rows over keys [key_lo, key_hi) of a corpus prepared
// for `prec`, with at most kc_max candidates and k_max neighbours per row.
// s_max > 0 caps the number of key splits (to fit a fixed workspace).
// allow_small lets a small plain search take the 128 x 128 tile geometry;
// stream lets a large plain search take the balanced schedule (one
// workgroup per CU over equal shares of the work).
SearchPlan plan_search(int prec, int64_t M, int64_t key_lo, int64_t key_hi, int k_max, int kc_max, int s_max = 0,
                       bool allow_small = false, bool stream = false);

// Forward search: exact k nearest neighbours of every batch row (candidate
// contraction, FP32 re-rank, certificate + exact scan on the FP32 path).
atsne_status knn_search(const Corpus& c, const Batch& b, const SearchPlan& p, void* ws, hipStream_t st);

// Reverse merge (Eq. 13): batch rows are resident rows whose neighbour lists
// live in (res_idx, res_d2) with stride res_stride and k = b.k; keys are the
// newly inserted rows [key_lo, key_hi).  Every new row strictly closer than a
// resident row's farthest neighbour enters its list, evicting the farthest;
// ids of changed rows are appended to changed[*n_changed].
atsne_status knn_reverse(const Corpus& c, const Batch& b, const SearchPlan& p, int32_t* res_idx, float* res_d2,
                         float* res_d2_lo, uint8_t* res_flags, int64_t res_stride, int32_t* changed,
                         int32_t* n_changed, void* ws, hipStream_t st);

// Calibrate rows of a neighbour table in place: row r is table row
// (row_ids ? row_ids[r] : r); d2/P rows have stride `stride`, k entries;
// d2_lo (may be null) holds the distances' residuals.
atsne_status calibrate_table(const float* d2, const float* d2_lo, int64_t stride, const int32_t* row_ids,
                             const int32_t* n_rows_dev, int64_t n_rows, int k, float mu, float tol, int max_iter,
                             float* P, float* beta, float* perp, uint8_t* flags, hipStream_t st);

// Ascending 64-bit key sort (hand-written LSD radix over bits [begin_bit,
// end_bit), keys equal elsewhere; stable), optionally carrying a 32-bit value
// per key; tmp holds sort_u64_temp_bytes(n) bytes; in and out must not
// overlap.
size_t sort_u64_temp_bytes(int64_t n);
atsne_status sort_u64(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, int64_t n, hipStream_t st,
                      int begin_bit = 0, int end_bit = 64);
atsne_status sort_pairs_u64(void* tmp, size_t tmp_bytes, const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                            uint32_t* vout, int64_t n, hipStream_t st, int begin_bit = 0, int end_bit = 64);

// Plan a search restricted to per-block tile lists (Batch::blk_q set):
// M rows in n_blocks blocks, S splits per block.
SearchPlan plan_list_search(int64_t M, int64_t n_blocks, int k_max, int kc_max, int S);

// Seeding pass of a large FP8 search (the k-means partition of the
// approximate search; each point's own cluster and its nearest clusters,
// searched in FP8 with the same tile kernel): tau[i] = the kc-th smallest
// key code d' of point i over those keys, an upper bound of its kc-th
// smallest over all keys.  tau is device [N]; the pass allocates its index.
// order (device [N], may be null) receives the points in cluster order.
atsne_status fp8_seed_thresholds(const float* X, int64_t N, int32_t D, int64_t ld, int kc, float* tau,
                                 int32_t* order, hipStream_t st);

// Serving-loop data manipulation (Sec. 5.3); resident lists have k entries
// per row, present entries first, absent ones (index -1, +inf) last.
atsne_status serve_fill_death(int32_t* death, int64_t n, hipStream_t st);
atsne_status serve_mark_deleted(int32_t* death, const int32_t* ids, int64_t M, int32_t c, hipStream_t st);
atsne_status serve_purge_deleted(int32_t* res_idx, float* res_d2, float* res_d2_lo, float* res_P, float* res_beta,
                                 uint8_t* res_flags, int k, int64_t n_rows, const int32_t* death, int32_t c,
                                 int32_t* changed, int32_t* n_changed, hipStream_t st);
atsne_status serve_farthest(const int32_t* res_idx, const float* res_d2, int k, int64_t n_rows, float* dmax,
                            hipStream_t st);
atsne_status serve_state(const int32_t* res_idx, int k, int64_t n_rows, const int32_t* death, float* rho,
                         uint8_t* alive, hipStream_t st);

}  // namespace atsne
