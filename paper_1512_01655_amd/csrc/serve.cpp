// Serving loop for the steerable, progressive use of the similarity path:
// streamed point insertion (Sec. 5.3, Eq. 13), point deletion (Sec. 5.3) and
// exact refinement of user selections (Sec. 4.3, Sec. 5.1) against a
// device-resident corpus.  Inserting new points and deleting the oldest ones
// is the sliding-window stream of Sec. 8.
//
// Continuous batching with iteration-level scheduling: a worker thread admits
// queued requests while request slots and the HBM budget allow, then packs
// row segments from every admitted request into one batched kNN launch (each
// row carries its own corpus id, corpus prefix, k and k_cand).  Two batch
// streams keep consecutive launches overlapped on the device; requests join
// and leave between launches.  Inserts and deletes are commits, applied in
// arrival order on a commit stream without a host synchronisation: an
// insert's rows enter the resident neighbour table, the Eq. 13 reverse merge
// updates every resident row that a new point beats, and the changed rows are
// re-calibrated; a delete removes its points from every resident list (no
// replacement: the row's precision falls by 1/K per removed neighbour) and
// re-calibrates the rows it changed.
//
// Determinism: every request carries a view, the number of commits submitted
// before it.  Its rows search exactly the corpus that view defines (the rows
// reserved before it, minus the rows deleted by earlier commits: a deleted
// row keeps its storage and carries the index of the deleting commit), every
// row's arithmetic is independent of the rows it shares a launch with, and
// the contraction's error bound uses the prefix maximum of the norms, so a request's
// result is bitwise the same alone or in any mix.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "knn_internal.h"

namespace atsne {
namespace {

constexpr float SERVE_MAX_PERPLEXITY = 50.0f;
// The corpus's contraction: FP32X3 (each FP32 value as BF16 hi + lo, three
// BF16 matrix-core products per element pair), at about twice the FP32
// tile's speed at D = 784.  Its candidates are certified against its own
// error bound, rows the bound cannot certify take the exact FP32 scan, and
// the FP32 re-rank and tie test are shared, so every result equals the FP32
// contraction's.
constexpr int SERVE_PREC = ATSNE_PREC_FP32X3;

double now_ms(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit sub-allocator over one device arena; its size is the HBM budget
// for request results.
class Arena2 {
   public:
    void init(char* base, size_t cap) {
        base_ = base;
        cap_ = cap;
        free_.clear();
        free_[0] = cap;
    }
    char* alloc(size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(char* p, size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        size_t off = (size_t)(p - base_);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t cap() const { return cap_; }

   private:
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

enum ReqState { PENDING, ADMITTED, FORWARD_DONE, FINISHING, DONE };

struct Request {
    uint64_t id = 0;
    int kind = 0;  // 0 insert, 1 refine, 2 delete
    uint64_t epoch = 0;  // view: commits submitted before it (inserts/deletes: own commit index)
    int64_t n = 0;
    int k = 0, kc = 0;
    float mu = 0.f;
    int64_t nlim = 0;
    int64_t row0 = 0;
    std::vector<int32_t> ids_host;
    size_t bytes = 0;
    char* mem = nullptr;
    int32_t* row_ids = nullptr;
    int32_t* nbr_idx = nullptr;
    float* nbr_d2 = nullptr;
    float* nbr_d2_lo = nullptr;  // residuals of nbr_d2 (calibration input)
    float* P = nullptr;
    float* beta = nullptr;
    uint8_t* flags = nullptr;
    int32_t* changed = nullptr;
    int32_t* n_changed_dev = nullptr;
    int32_t* n_changed_host = nullptr;  // pinned
    int64_t next_row = 0, rows_done = 0;
    int state = PENDING;
    atsne_status status = ATSNE_OK;
    double t_submit = 0, t_admit = 0, t_complete = 0;
    hipEvent_t fin = nullptr;
    bool released = false;
};

struct Seg {
    Request* r;
    int64_t r0, n, b0;
};

struct BatchSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Seg> segs;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t* d_desc = nullptr;  // qids | nlims | ks | kcs | views, each max_rows
    int32_t* h_desc = nullptr;  // pinned staging
    int32_t* b_idx = nullptr;
    float* b_d2 = nullptr;
    float* b_d2_lo = nullptr;
    uint8_t* b_flags = nullptr;
};

}  // namespace
}  // namespace atsne

struct atsne_server {
    int device = 0;
    int32_t D = 0;
    float mu0 = 30.f;
    int K0 = 90, kc0 = 135;
    int kmax = 150, kcmax = 225;
    int64_t cap_rows = 0;
    int32_t max_batch_rows = 8192;
    int32_t max_slots = 8;
    std::chrono::steady_clock::time_point t0;

    float* X = nullptr;
    atsne::Corpus corpus;
    void* corpus_mem = nullptr;
    int32_t* res_idx = nullptr;
    float* res_d2 = nullptr;
    float* res_d2_lo = nullptr;  // residuals of res_d2 (calibration input)
    float* res_P = nullptr;
    float* res_beta = nullptr;
    uint8_t* res_flags = nullptr;
    float* res_dmax = nullptr;  // farthest present neighbour (Eq. 13 threshold)
    int32_t* death = nullptr;   // per row: index of the deleting commit, INT_MAX if alive
    int32_t* del_ids = nullptr;  // device staging of a delete's ids
    void* res_mem = nullptr;
    std::vector<int32_t> h_death;  // host copy of death

    hipStream_t s_copy = nullptr, s_commit = nullptr, s_finish = nullptr;
    atsne::BatchSlot slot[2];
    void* rev_ws = nullptr;
    size_t rev_ws_bytes = 0;
    char* arena_mem = nullptr;
    atsne::Arena2 arena;

    std::mutex mu, submit_mu;
    std::condition_variable cv, cv_done;
    std::deque<atsne::Request*> pending;
    std::vector<atsne::Request*> active;
    std::map<uint64_t, atsne::Request*> all;
    uint64_t next_id = 1;
    uint64_t commits_submitted = 0, next_commit = 0;
    int64_t n_reserved = 0, n_committed = 0, n_deleted = 0;
    bool stop = false;
    std::thread worker;
    atsne_serve_stats stats{};
    atsne_status fatal = ATSNE_OK;
    // test hook: the n-th batch launch fails with E_NOMEM before touching the
    // device (ATSNE_SERVE_FAIL_LAUNCH=n at creation; 0 = never)
    int64_t fail_launch_at = 0, launch_attempts = 0;
};

namespace atsne {
namespace {

atsne_status alloc_dev(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        return ATSNE_E_NOMEM;
    }
    return ATSNE_OK;
}

size_t request_bytes(const Request& r) {
    Arena a;
    a.take<int32_t>(r.n);
    a.take<int32_t>(r.n * r.k);
    a.take<float>(r.n * r.k);
    a.take<float>(r.n * r.k);
    a.take<float>(r.n * r.k);
    a.take<float>(r.n);
    a.take<uint8_t>(r.n);
    if (r.kind != 1) {
        a.take<int32_t>(std::max<int64_t>(r.kind == 0 ? r.row0 : r.nlim, 1));
        a.take<int32_t>(1);
    }
    return a.used;
}

void carve_request(Request& r) {
    Arena a(r.mem, r.bytes);
    r.row_ids = a.take<int32_t>(r.n);
    r.nbr_idx = a.take<int32_t>(r.n * r.k);
    r.nbr_d2 = a.take<float>(r.n * r.k);
    r.nbr_d2_lo = a.take<float>(r.n * r.k);
    r.P = a.take<float>(r.n * r.k);
    r.beta = a.take<float>(r.n);
    r.flags = a.take<uint8_t>(r.n);
    if (r.kind != 1) {
        r.changed = a.take<int32_t>(std::max<int64_t>(r.kind == 0 ? r.row0 : r.nlim, 1));
        r.n_changed_dev = a.take<int32_t>(1);
    }
}

// Launch one batch of row segments on a batch slot the worker has reserved
// (called without the server lock: it reads only fields fixed at submission
// and the slot's own buffers).
atsne_status launch_batch(atsne_server* s, BatchSlot& b, const std::vector<Seg>& segs, int64_t rows) {
    if (s->fail_launch_at > 0 && ++s->launch_attempts == s->fail_launch_at) {
        set_error("injected failure of batch launch %lld (ATSNE_SERVE_FAIL_LAUNCH)", (long long)s->fail_launch_at);
        return ATSNE_E_NOMEM;
    }
    const int64_t R = s->max_batch_rows;
    int32_t* hq = b.h_desc;
    int32_t* hn = hq + R;
    int32_t* hk = hn + R;
    int32_t* hc = hk + R;
    int32_t* hv = hc + R;
    int64_t key_hi = 0;
    for (const Seg& g : segs) {
        for (int64_t i = 0; i < g.n; ++i) {
            const int64_t row = g.r0 + i;
            hq[g.b0 + i] = g.r->ids_host[row];
            hn[g.b0 + i] = (int32_t)g.r->nlim;
            hk[g.b0 + i] = g.r->k;
            hc[g.b0 + i] = g.r->kc;
            hv[g.b0 + i] = (int32_t)g.r->epoch;
        }
        key_hi = std::max(key_hi, g.r->nlim);
    }
    ATSNE_HIP(hipMemcpyAsync(b.d_desc, b.h_desc, sizeof(int32_t) * 5 * R, hipMemcpyHostToDevice, b.st));
    const int s_fit = 64;
    SearchPlan p = plan_search(SERVE_PREC, rows, 0, key_hi, s->kmax, s->kcmax, s_fit);
    while (p.ws_bytes > b.ws_bytes && p.S > 1) p = plan_search(SERVE_PREC, rows, 0, key_hi, s->kmax, s->kcmax, p.S - 1);
    ATSNE_REQUIRE(p.ws_bytes <= b.ws_bytes, ATSNE_E_NOMEM, "batch workspace too small");
    Batch bt;
    bt.M = rows;
    bt.qids = b.d_desc;
    bt.nlims = b.d_desc + R;
    bt.ks = b.d_desc + 2 * R;
    bt.kcs = b.d_desc + 3 * R;
    bt.views = b.d_desc + 4 * R;
    bt.k = s->kmax;
    bt.kc = s->kcmax;
    bt.nlim = key_hi;
    bt.key_lo = 0;
    bt.out_idx = b.b_idx;
    bt.out_d2 = b.b_d2;
    bt.out_d2_lo = b.b_d2_lo;
    bt.out_flags = b.b_flags;
    bt.out_stride = s->kmax;
    ATSNE_TRY(knn_search(s->corpus, bt, p, b.ws, b.st));
    for (const Seg& g : segs) {
        const int k = g.r->k;
        ATSNE_HIP(hipMemcpy2DAsync(g.r->nbr_idx + g.r0 * k, k * 4, b.b_idx + g.b0 * s->kmax, s->kmax * 4, k * 4,
                                   g.n, hipMemcpyDeviceToDevice, b.st));
        ATSNE_HIP(hipMemcpy2DAsync(g.r->nbr_d2 + g.r0 * k, k * 4, b.b_d2 + g.b0 * s->kmax, s->kmax * 4, k * 4, g.n,
                                   hipMemcpyDeviceToDevice, b.st));
        ATSNE_HIP(hipMemcpy2DAsync(g.r->nbr_d2_lo + g.r0 * k, k * 4, b.b_d2_lo + g.b0 * s->kmax, s->kmax * 4, k * 4,
                                   g.n, hipMemcpyDeviceToDevice, b.st));
        ATSNE_HIP(hipMemcpyAsync(g.r->flags + g.r0, b.b_flags + g.b0, g.n, hipMemcpyDeviceToDevice, b.st));
    }
    ATSNE_HIP(hipEventRecord(b.ev, b.st));
    return ATSNE_OK;
}

// Finish a refine: calibrate its rows at its own perplexity.
atsne_status finish_refine(atsne_server* s, Request& r) {
    ATSNE_TRY(calibrate_table(r.nbr_d2, r.nbr_d2_lo, r.k, nullptr, nullptr, r.n, r.k, r.mu, 1e-5f, 200, r.P, r.beta, nullptr,
                              r.flags, s->s_finish));
    ATSNE_HIP(hipEventRecord(r.fin, s->s_finish));
    return ATSNE_OK;
}

// Commit an insert (in epoch order, on the commit stream).
atsne_status commit_insert(atsne_server* s, Request& r) {
    hipStream_t st = s->s_commit;
    const int K = s->K0;
    const int64_t r0 = r.row0, B = r.n;
    // 1. the new rows' exact lists enter the resident table and are calibrated
    ATSNE_HIP(hipMemcpyAsync(s->res_idx + r0 * K, r.nbr_idx, sizeof(int32_t) * B * K, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(s->res_d2 + r0 * K, r.nbr_d2, sizeof(float) * B * K, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(s->res_d2_lo + r0 * K, r.nbr_d2_lo, sizeof(float) * B * K, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(s->res_flags + r0, r.flags, B, hipMemcpyDeviceToDevice, st));
    ATSNE_TRY(calibrate_table(s->res_d2 + r0 * K, s->res_d2_lo + r0 * K, K, nullptr, nullptr, B, K, s->mu0, 1e-5f, 200, s->res_P + r0 * K,
                              s->res_beta + r0, nullptr, s->res_flags + r0, st));
    // 2. Eq. 13 over the residents that existed before this insert; the
    // threshold of a row is its farthest present neighbour
    ATSNE_HIP(hipMemsetAsync(r.n_changed_dev, 0, sizeof(int32_t), st));
    if (r0 > 0) {
        ATSNE_TRY(serve_farthest(s->res_idx, s->res_d2, K, r0, s->res_dmax, st));
        SearchPlan p = plan_search(SERVE_PREC, r0, r0, r0 + B, K, K);
        while (p.ws_bytes > s->rev_ws_bytes && p.S > 1) p = plan_search(SERVE_PREC, r0, r0, r0 + B, K, K, p.S - 1);
        ATSNE_REQUIRE(p.ws_bytes <= s->rev_ws_bytes, ATSNE_E_NOMEM, "reverse workspace too small");
        Batch bt;
        bt.M = r0;
        bt.m0 = 0;
        bt.nlim = r0 + B;
        bt.key_lo = r0;
        bt.k = K;
        bt.kc = K;
        bt.tau0 = s->res_dmax;
        bt.tau0_stride = 1;
        bt.view = (int32_t)r.epoch;
        ATSNE_TRY(knn_reverse(s->corpus, bt, p, s->res_idx, s->res_d2, s->res_d2_lo, s->res_flags, K, r.changed, r.n_changed_dev,
                              s->rev_ws, st));
        // 3. re-calibrate the changed rows in place (count stays on the device)
        ATSNE_TRY(calibrate_table(s->res_d2, s->res_d2_lo, K, r.changed, r.n_changed_dev, r0, K, s->mu0, 1e-5f, 200, s->res_P,
                                  s->res_beta, nullptr, s->res_flags, st));
    }
    // 4. the result carries the new rows' calibrated state
    ATSNE_HIP(hipMemcpyAsync(r.P, s->res_P + r0 * K, sizeof(float) * B * K, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(r.beta, s->res_beta + r0, sizeof(float) * B, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(r.flags, s->res_flags + r0, B, hipMemcpyDeviceToDevice, st));
    ATSNE_HIP(hipMemcpyAsync(r.n_changed_host, r.n_changed_dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ATSNE_HIP(hipEventRecord(r.fin, st));
    return ATSNE_OK;
}

// Commit a delete (in commit order, on the commit stream): every resident row
// reserved before it drops the deleted points, the deleted rows are emptied,
// and the changed rows are re-calibrated over their remaining neighbours.
atsne_status commit_delete(atsne_server* s, Request& r) {
    hipStream_t st = s->s_commit;
    const int K = s->K0;
    ATSNE_HIP(hipMemsetAsync(r.n_changed_dev, 0, sizeof(int32_t), st));
    ATSNE_TRY(serve_purge_deleted(s->res_idx, s->res_d2, s->res_d2_lo, s->res_P, s->res_beta, s->res_flags, K, r.nlim, s->death,
                                  (int32_t)r.epoch, r.changed, r.n_changed_dev, st));
    ATSNE_TRY(calibrate_table(s->res_d2, s->res_d2_lo, K, r.changed, r.n_changed_dev, r.nlim, K, s->mu0, 1e-5f, 200, s->res_P,
                              s->res_beta, nullptr, s->res_flags, st));
    ATSNE_HIP(hipMemcpyAsync(r.n_changed_host, r.n_changed_dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ATSNE_HIP(hipEventRecord(r.fin, st));
    return ATSNE_OK;
}

void fail_request(atsne_server* s, Request& r, atsne_status st) {
    r.status = st;
    r.state = DONE;
    r.t_complete = now_ms(s->t0);
    s->stats.completed++;
}

// A launch or commit failed: the server stops serving.  Every stream is
// drained first (without the lock), so no copy or kernel still writes into a
// request's result memory when that request is failed and may be released;
// then every admitted and queued request fails with `st`, and later
// submissions are refused.
void fail_server(atsne_server* s, std::unique_lock<std::mutex>& lk, atsne_status st) {
    s->fatal = st;
    lk.unlock();
    for (auto& b : s->slot)
        if (b.st) (void)hipStreamSynchronize(b.st);
    for (hipStream_t q : {s->s_copy, s->s_commit, s->s_finish})
        if (q) (void)hipStreamSynchronize(q);
    lk.lock();
    for (auto& b : s->slot) {
        b.segs.clear();
        b.busy = false;
    }
    for (Request* r : s->active)
        if (r->state != DONE) fail_request(s, *r, st);
    for (Request* r : s->pending) fail_request(s, *r, st);
    s->active.clear();
    s->pending.clear();
    s->cv_done.notify_all();
}

// The worker: admission, batch formation and commit ordering under the server
// lock; every GPU call (copies, launches, commits) with the lock released, so
// submitters and waiters never queue behind device work.  Only the worker
// changes a request's progress fields, so they need no lock while it runs.
void worker_loop(atsne_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    struct Job {
        BatchSlot* b;
        std::vector<Seg> segs;
        int64_t rows;
    };
    for (;;) {
        bool progress = false;
        std::vector<Request*> admitted, finishing;
        std::vector<Job> jobs;
        if (s->fatal == ATSNE_OK) {
            // 1. admission: request slots and the result arena (HBM budget)
            while (!s->pending.empty() && (int)s->active.size() < s->max_slots) {
                Request* r = s->pending.front();
                r->mem = s->arena.alloc(r->bytes);
                if (!r->mem) break;  // wait for releases
                s->pending.pop_front();
                carve_request(*r);
                r->state = r->kind == 2 ? FORWARD_DONE : ADMITTED;  // a delete searches nothing
                r->t_admit = now_ms(s->t0);
                admitted.push_back(r);
                s->active.push_back(r);
                s->stats.bytes_in_flight = s->arena.used();
                s->stats.peak_bytes_in_flight = std::max(s->stats.peak_bytes_in_flight, s->arena.used());
                s->stats.max_concurrent = std::max<int32_t>(s->stats.max_concurrent, (int32_t)s->active.size());
            }
            // 2. batch formation on free slots: row segments from every admitted request
            for (auto& b : s->slot) {
                if (b.busy) continue;
                Job j{&b, {}, 0};
                for (Request* r : s->active) {
                    if (r->state != ADMITTED || r->next_row >= r->n) continue;
                    const int64_t take = std::min<int64_t>(r->n - r->next_row, s->max_batch_rows - j.rows);
                    if (take <= 0) break;
                    j.segs.push_back(Seg{r, r->next_row, take, j.rows});
                    r->next_row += take;
                    j.rows += take;
                }
                if (j.rows == 0) break;
                b.busy = true;
                b.segs = j.segs;
                jobs.push_back(std::move(j));
            }
            // 3. finishing: refines calibrate; inserts and deletes commit in order
            for (Request* r : s->active) {
                if (r->state != FORWARD_DONE) continue;
                if (r->kind != 1) {
                    if (r->epoch != s->next_commit) continue;
                    s->next_commit++;
                }
                r->state = FINISHING;
                finishing.push_back(r);
            }
        }
        progress = !admitted.empty() || !jobs.empty() || !finishing.empty();
        if (progress) {
            lk.unlock();
            atsne_status err = ATSNE_OK;
            for (Request* r : admitted)
                if (err == ATSNE_OK && hipMemcpyAsync(r->row_ids, r->ids_host.data(), sizeof(int32_t) * r->n,
                                                      hipMemcpyHostToDevice, s->s_copy) != hipSuccess) {
                    set_error("row id copy failed");
                    err = ATSNE_E_HIP;
                }
            if (!admitted.empty() && err == ATSNE_OK && hipStreamSynchronize(s->s_copy) != hipSuccess) {
                set_error("row id copy failed");
                err = ATSNE_E_HIP;
            }
            for (Job& j : jobs)
                if (err == ATSNE_OK) err = launch_batch(s, *j.b, j.segs, j.rows);
            for (Request* r : finishing)
                if (err == ATSNE_OK)
                    err = r->kind == 1 ? finish_refine(s, *r) : (r->kind == 0 ? commit_insert(s, *r) : commit_delete(s, *r));
            lk.lock();
            for (const Job& j : jobs) {
                s->stats.launches++;
                s->stats.rows_processed += j.rows;
                int distinct = 0;
                const Request* last = nullptr;
                for (const Seg& g : j.segs)
                    if (g.r != last) {
                        ++distinct;
                        last = g.r;
                    }
                s->stats.max_requests_per_launch = std::max<int32_t>(s->stats.max_requests_per_launch, distinct);
            }
            if (err != ATSNE_OK) {
                fail_server(s, lk, err);
                continue;
            }
        }
        // 4. batch completions
        for (auto& b : s->slot) {
            if (!b.busy || hipEventQuery(b.ev) != hipSuccess) continue;
            for (const Seg& g : b.segs) {
                g.r->rows_done += g.n;
                if (g.r->rows_done == g.r->n && g.r->state == ADMITTED) g.r->state = FORWARD_DONE;
            }
            b.segs.clear();
            b.busy = false;
            progress = true;
        }
        // 5. finished requests
        for (size_t i = 0; i < s->active.size();) {
            Request* r = s->active[i];
            if (r->state == FINISHING && hipEventQuery(r->fin) == hipSuccess) {
                r->state = DONE;
                r->t_complete = now_ms(s->t0);
                if (r->kind == 0) s->n_committed = std::max(s->n_committed, r->row0 + r->n);
                s->stats.completed++;
                progress = true;
            }
            if (r->state == DONE) {
                s->active.erase(s->active.begin() + i);
                s->cv_done.notify_all();
            } else {
                ++i;
            }
        }
        if (s->stop && s->pending.empty() && s->active.empty() && !s->slot[0].busy && !s->slot[1].busy) break;
        if (!progress) s->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

Request* find(atsne_server* s, uint64_t id) {
    auto it = s->all.find(id);
    return it == s->all.end() ? nullptr : it->second;
}

void fill_result(const Request& r, atsne_result* o) {
    o->req_id = r.id;
    o->kind = r.kind;
    o->status = r.status;
    o->epoch = r.epoch;
    o->n_rows = r.n;
    o->k = r.k;
    o->perplexity = r.mu;
    o->row_ids = r.row_ids;
    const bool rows = r.kind != 2;
    o->nbr_idx = rows ? r.nbr_idx : nullptr;
    o->nbr_d2 = rows ? r.nbr_d2 : nullptr;
    o->P_cond = rows ? r.P : nullptr;
    o->beta = rows ? r.beta : nullptr;
    o->flags = rows ? r.flags : nullptr;
    o->n_changed = (r.kind != 1 && r.n_changed_host) ? *r.n_changed_host : 0;
    o->changed = r.changed;
    o->t_submit_ms = r.t_submit;
    o->t_admit_ms = r.t_admit;
    o->t_complete_ms = r.t_complete;
}

void free_request(atsne_server* s, Request* r) {
    if (r->mem) s->arena.release(r->mem, r->bytes);
    if (r->fin) (void)hipEventDestroy(r->fin);
    if (r->n_changed_host) (void)hipHostFree(r->n_changed_host);
    delete r;
}

}  // namespace
}  // namespace atsne

using namespace atsne;

static void destroy_impl(atsne_server* s);

extern "C" atsne_status atsne_serve_create(const atsne_serve_config* cfg, const float* corpus, int64_t N, int32_t D,
                                           float perplexity, atsne_server** out) {
    clear_error();
    ATSNE_REQUIRE(corpus && out && N >= 2 && D >= 1, ATSNE_E_INVALID_ARG, "bad arguments");
    ATSNE_REQUIRE(perplexity >= 1.f && perplexity <= SERVE_MAX_PERPLEXITY, ATSNE_E_K_RANGE,
                  "perplexity %g outside [1, %g]", (double)perplexity, (double)SERVE_MAX_PERPLEXITY);
    const int K0 = (int)std::floor(3.0 * perplexity);
    ATSNE_REQUIRE(K0 <= N - 1 && perplexity < K0, ATSNE_E_K_RANGE, "k=%d out of range for N=%lld", K0, (long long)N);
    atsne_serve_config c{};
    if (cfg) c = *cfg;
    auto* s = new atsne_server();
    s->t0 = std::chrono::steady_clock::now();
    if (c.device >= 0) {
        if (hipSetDevice(c.device) != hipSuccess) {
            delete s;
            set_error("hipSetDevice(%d) failed", c.device);
            return ATSNE_E_HIP;
        }
    }
    (void)hipGetDevice(&s->device);
    s->D = D;
    s->mu0 = perplexity;
    s->K0 = K0;
    s->kc0 = K0 + std::max(32, K0 / 2);
    s->kmax = (int)std::floor(3.0 * SERVE_MAX_PERPLEXITY);
    s->kcmax = s->kmax + std::max(32, s->kmax / 2);
    s->cap_rows = c.capacity_rows > 0 ? std::max<int64_t>(c.capacity_rows, N) : 2 * N;
    s->max_batch_rows = c.max_batch_rows > 0 ? c.max_batch_rows : 8192;
    s->max_slots = c.max_slots > 0 ? c.max_slots : 8;
    if (const char* f = std::getenv("ATSNE_SERVE_FAIL_LAUNCH")) s->fail_launch_at = std::atoll(f);
    const size_t budget = c.hbm_budget_bytes > 0 ? c.hbm_budget_bytes : ((size_t)4 << 30);
    auto fail = [&](atsne_status st) {
        destroy_impl(s);
        return st;
    };
    const int64_t cap = ceil_div(s->cap_rows, KNN_KT) * KNN_KT;
    atsne_status st;
    if ((st = alloc_dev((void**)&s->X, sizeof(float) * cap * D)) != ATSNE_OK) return fail(st);
    if ((st = alloc_dev(&s->corpus_mem, corpus_bytes(SERVE_PREC, cap, D))) != ATSNE_OK) return fail(st);
    corpus_bind(s->corpus, SERVE_PREC, s->X, D, D, cap, s->corpus_mem);
    {
        Arena a;
        a.take<int32_t>(cap * K0);
        a.take<float>(cap * K0);
        a.take<float>(cap * K0);
        a.take<float>(cap * K0);
        a.take<float>(cap);
        a.take<uint8_t>(cap);
        a.take<float>(cap);
        a.take<int32_t>(cap);
        a.take<int32_t>(cap);
        if ((st = alloc_dev(&s->res_mem, a.used)) != ATSNE_OK) return fail(st);
        Arena b(s->res_mem, a.used);
        s->res_idx = b.take<int32_t>(cap * K0);
        s->res_d2 = b.take<float>(cap * K0);
        s->res_d2_lo = b.take<float>(cap * K0);
        s->res_P = b.take<float>(cap * K0);
        s->res_beta = b.take<float>(cap);
        s->res_flags = b.take<uint8_t>(cap);
        s->res_dmax = b.take<float>(cap);
        s->death = b.take<int32_t>(cap);
        s->del_ids = b.take<int32_t>(cap);
        s->corpus.death = s->death;
        s->h_death.assign(cap, INT_MAX);
    }
    if (hipStreamCreateWithFlags(&s->s_copy, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_commit, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_finish, hipStreamNonBlocking) != hipSuccess) {
        set_error("stream creation failed");
        return fail(ATSNE_E_HIP);
    }
    const int64_t R = s->max_batch_rows;
    {
        // batch workspace: enough for the largest batch with a few splits
        SearchPlan p = plan_search(SERVE_PREC, R, 0, cap, s->kmax, s->kcmax, 4);
        for (auto& b : s->slot) {
            b.ws_bytes = p.ws_bytes;
            if ((st = alloc_dev(&b.ws, b.ws_bytes)) != ATSNE_OK) return fail(st);
            if ((st = alloc_dev((void**)&b.d_desc, sizeof(int32_t) * 5 * R)) != ATSNE_OK) return fail(st);
            if ((st = alloc_dev((void**)&b.b_idx, sizeof(int32_t) * R * s->kmax)) != ATSNE_OK) return fail(st);
            if ((st = alloc_dev((void**)&b.b_d2, sizeof(float) * R * s->kmax)) != ATSNE_OK) return fail(st);
            if ((st = alloc_dev((void**)&b.b_d2_lo, sizeof(float) * R * s->kmax)) != ATSNE_OK) return fail(st);
            if ((st = alloc_dev((void**)&b.b_flags, R)) != ATSNE_OK) return fail(st);
            if (hipHostMalloc((void**)&b.h_desc, sizeof(int32_t) * 5 * R, hipHostMallocDefault) != hipSuccess ||
                hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
                set_error("batch slot setup failed");
                return fail(ATSNE_E_HIP);
            }
        }
        SearchPlan rp = plan_search(SERVE_PREC, cap, 0, 4096 + KNN_KT, K0, K0, 1);
        s->rev_ws_bytes = rp.ws_bytes;
        if ((st = alloc_dev(&s->rev_ws, s->rev_ws_bytes)) != ATSNE_OK) return fail(st);
    }
    if ((st = alloc_dev((void**)&s->arena_mem, budget)) != ATSNE_OK) return fail(st);
    s->arena.init(s->arena_mem, budget);

    // Corpus copy (host or device source), preparation, and its exact state.
    hipStream_t cs = s->s_commit;
    if (hipMemcpyAsync(s->X, corpus, sizeof(float) * N * D, hipMemcpyDefault, cs) != hipSuccess ||
        hipMemsetAsync(s->X + N * D, 0, sizeof(float) * (cap - N) * D, cs) != hipSuccess) {
        set_error("corpus copy failed");
        return fail(ATSNE_E_HIP);
    }
    if ((st = serve_fill_death(s->death, cap, cs)) != ATSNE_OK) return fail(st);
    if ((st = corpus_prep(s->corpus, 0, cap, N, cs)) != ATSNE_OK) return fail(st);
    {
        SearchPlan p = plan_search(SERVE_PREC, std::min<int64_t>(N, 65536), 0, N, K0, s->kc0);
        void* ws = nullptr;
        if ((st = alloc_dev(&ws, p.ws_bytes)) != ATSNE_OK) return fail(st);
        for (int64_t m0 = 0; m0 < N && st == ATSNE_OK; m0 += p.M) {
            Batch bt;
            bt.M = std::min<int64_t>(p.M, N - m0);
            bt.m0 = m0;
            bt.nlim = N;
            bt.k = K0;
            bt.kc = s->kc0;
            bt.out_idx = s->res_idx + m0 * K0;
            bt.out_d2 = s->res_d2 + m0 * K0;
            bt.out_d2_lo = s->res_d2_lo + m0 * K0;
            bt.out_flags = s->res_flags + m0;
            bt.out_stride = K0;
            st = knn_search(s->corpus, bt, p, ws, cs);
        }
        if (st == ATSNE_OK)
            st = calibrate_table(s->res_d2, s->res_d2_lo, K0, nullptr, nullptr, N, K0, perplexity, 1e-5f, 200, s->res_P,
                                 s->res_beta, nullptr, s->res_flags, cs);
        hipError_t e = hipStreamSynchronize(cs);
        (void)hipFree(ws);
        if (st != ATSNE_OK) return fail(st);
        if (e != hipSuccess) {
            set_error("initial similarity failed: %s", hipGetErrorString(e));
            return fail(ATSNE_E_HIP);
        }
    }
    s->n_reserved = s->n_committed = N;
    s->stats.corpus_rows = N;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_submit_insert(atsne_server* s, const float* X_new, int32_t B, uint64_t* req_id) {
    clear_error();
    ATSNE_REQUIRE(s && X_new && req_id && B >= 1, ATSNE_E_INVALID_ARG, "bad arguments");
    // latency is measured from the caller's call, staging included
    const double t_call = now_ms(s->t0);
    std::lock_guard<std::mutex> sl(s->submit_mu);
    int64_t row0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        ATSNE_REQUIRE(!s->stop, ATSNE_E_INVALID_ARG, "server is shutting down");
        ATSNE_REQUIRE(s->fatal == ATSNE_OK, s->fatal, "the server stopped after a failed launch or commit");
        ATSNE_REQUIRE(s->n_reserved + B <= s->cap_rows, ATSNE_E_NOMEM, "corpus capacity %lld rows exceeded",
                      (long long)s->cap_rows);
        row0 = s->n_reserved;
    }
    auto* r = new Request();
    r->kind = 0;
    r->n = B;
    r->k = s->K0;
    r->kc = s->kc0;
    r->mu = s->mu0;
    r->row0 = row0;
    r->nlim = row0 + B;
    r->ids_host.resize(B);
    for (int32_t i = 0; i < B; ++i) r->ids_host[i] = (int32_t)(row0 + i);
    r->bytes = request_bytes(*r);
    if (r->bytes > s->arena.cap()) {
        delete r;
        set_error("request needs %zu bytes, above the HBM budget", request_bytes(Request()));
        return ATSNE_E_NOMEM;
    }
    // data enters the corpus now (arrival order); the rows are prepared
    // before any later request can search them
    if (hipMemcpyAsync(s->X + row0 * s->D, X_new, sizeof(float) * B * s->D, hipMemcpyDefault, s->s_copy) !=
            hipSuccess ||
        corpus_prep(s->corpus, row0, row0 + B, row0 + B, s->s_copy) != ATSNE_OK ||
        hipStreamSynchronize(s->s_copy) != hipSuccess || hipEventCreateWithFlags(&r->fin, hipEventDisableTiming) !=
                                                              hipSuccess ||
        hipHostMalloc((void**)&r->n_changed_host, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        delete r;
        set_error("insert staging failed");
        return ATSNE_E_HIP;
    }
    *r->n_changed_host = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->epoch = s->commits_submitted++;
        r->t_submit = t_call;
        s->n_reserved += B;
        s->stats.corpus_rows = s->n_reserved;
        s->stats.submitted++;
        s->all[r->id] = r;
        s->pending.push_back(r);
        *req_id = r->id;
    }
    s->cv.notify_all();
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_submit_refine(atsne_server* s, const int32_t* ids_host, int32_t M,
                                                  float perplexity, uint64_t* req_id) {
    clear_error();
    ATSNE_REQUIRE(s && ids_host && req_id && M >= 1, ATSNE_E_INVALID_ARG, "bad arguments");
    ATSNE_REQUIRE(perplexity >= 1.f && perplexity <= SERVE_MAX_PERPLEXITY, ATSNE_E_K_RANGE,
                  "perplexity %g outside [1, %g]", (double)perplexity, (double)SERVE_MAX_PERPLEXITY);
    const int k = (int)std::floor(3.0 * perplexity);
    const double t_call = now_ms(s->t0);
    std::lock_guard<std::mutex> sl(s->submit_mu);
    auto* r = new Request();
    r->kind = 1;
    r->n = M;
    r->k = k;
    r->kc = k + std::max(32, k / 2);
    r->mu = perplexity;
    int64_t n_alive;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->nlim = s->n_reserved;
        r->epoch = s->commits_submitted;
        n_alive = s->n_reserved - s->n_deleted;
    }
    if (!(perplexity < k) || k > n_alive - 1) {
        delete r;
        set_error("k=%d out of range for a corpus of %lld live points", k, (long long)n_alive);
        return ATSNE_E_K_RANGE;
    }
    r->kc = (int)std::min<int64_t>(r->kc, n_alive - 1);
    r->ids_host.assign(ids_host, ids_host + M);
    // deletes are submitted under submit_mu too, so h_death is stable here
    for (int32_t v : r->ids_host)
        if (v < 0 || v >= r->nlim || s->h_death[v] != INT_MAX) {
            delete r;
            set_error("refine id %d is not a live point of the corpus [0, %lld)", v, (long long)r->nlim);
            return ATSNE_E_INVALID_ARG;
        }
    r->bytes = request_bytes(*r);
    if (r->bytes > s->arena.cap()) {
        delete r;
        set_error("request needs more than the HBM budget");
        return ATSNE_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&r->fin, hipEventDisableTiming) != hipSuccess) {
        delete r;
        set_error("event creation failed");
        return ATSNE_E_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || s->fatal != ATSNE_OK) {
            const atsne_status st = s->stop ? ATSNE_E_INVALID_ARG : s->fatal;
            free_request(s, r);
            set_error(s->stop ? "server is shutting down" : "the server stopped after a failed launch or commit");
            return st;
        }
        r->id = s->next_id++;
        r->t_submit = t_call;
        s->stats.submitted++;
        s->all[r->id] = r;
        s->pending.push_back(r);
        *req_id = r->id;
    }
    s->cv.notify_all();
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_submit_delete(atsne_server* s, const int32_t* ids_host, int32_t M,
                                                  uint64_t* req_id) {
    clear_error();
    ATSNE_REQUIRE(s && ids_host && req_id && M >= 1, ATSNE_E_INVALID_ARG, "bad arguments");
    const double t_call = now_ms(s->t0);
    std::lock_guard<std::mutex> sl(s->submit_mu);
    auto* r = new Request();
    r->kind = 2;
    r->n = M;
    r->k = 0;
    r->mu = s->mu0;
    int64_t n_alive;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || s->fatal != ATSNE_OK) {
            const atsne_status st = s->stop ? ATSNE_E_INVALID_ARG : s->fatal;
            delete r;
            set_error(s->stop ? "server is shutting down" : "the server stopped after a failed launch or commit");
            return st;
        }
        r->nlim = s->n_reserved;
        n_alive = s->n_reserved - s->n_deleted;
    }
    if (n_alive - M < (int64_t)s->K0 + 1) {
        delete r;
        set_error("deleting %d of %lld live points leaves fewer than k+1 = %d", M, (long long)n_alive, s->K0 + 1);
        return ATSNE_E_K_RANGE;
    }
    r->ids_host.assign(ids_host, ids_host + M);
    {
        std::vector<int32_t> sorted(r->ids_host);
        std::sort(sorted.begin(), sorted.end());
        for (size_t i = 0; i < sorted.size(); ++i) {
            const int32_t v = sorted[i];
            if (v < 0 || v >= r->nlim || s->h_death[v] != INT_MAX || (i > 0 && sorted[i - 1] == v)) {
                delete r;
                set_error("delete id %d is not a distinct live point of the corpus [0, %lld)", v, (long long)r->nlim);
                return ATSNE_E_INVALID_ARG;
            }
        }
    }
    r->bytes = request_bytes(*r);
    if (r->bytes > s->arena.cap()) {
        delete r;
        set_error("request needs more than the HBM budget");
        return ATSNE_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&r->fin, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&r->n_changed_host, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        free_request(s, r);
        set_error("delete staging failed");
        return ATSNE_E_HIP;
    }
    *r->n_changed_host = 0;
    // The deletion stamp is written now: requests submitted later never see
    // these rows, earlier ones still do (their view is at most this index).
    uint64_t c;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        c = s->commits_submitted;
    }
    if (c >= (uint64_t)INT_MAX) {  // deletion stamps are int32 commit indices
        free_request(s, r);
        set_error("commit index space exhausted");
        return ATSNE_E_K_RANGE;
    }
    if (hipMemcpyAsync(s->del_ids, r->ids_host.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s->s_copy) !=
            hipSuccess ||
        serve_mark_deleted(s->death, s->del_ids, M, (int32_t)c, s->s_copy) != ATSNE_OK ||
        hipStreamSynchronize(s->s_copy) != hipSuccess) {
        free_request(s, r);
        set_error("delete staging failed");
        return ATSNE_E_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int32_t v : r->ids_host) s->h_death[v] = (int32_t)c;
        r->id = s->next_id++;
        r->epoch = s->commits_submitted++;
        r->t_submit = t_call;
        s->n_deleted += M;
        s->stats.submitted++;
        s->all[r->id] = r;
        s->pending.push_back(r);
        *req_id = r->id;
    }
    s->cv.notify_all();
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_poll(atsne_server* s, uint64_t req_id, atsne_result* out) {
    clear_error();
    ATSNE_REQUIRE(s && out, ATSNE_E_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = find(s, req_id);
    ATSNE_REQUIRE(r && !r->released, ATSNE_E_INVALID_ARG, "unknown request %llu", (unsigned long long)req_id);
    if (r->state != DONE) return ATSNE_E_BUSY;
    fill_result(*r, out);
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_wait(atsne_server* s, uint64_t req_id, atsne_result* out) {
    clear_error();
    ATSNE_REQUIRE(s && out, ATSNE_E_INVALID_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    Request* r = find(s, req_id);
    ATSNE_REQUIRE(r && !r->released, ATSNE_E_INVALID_ARG, "unknown request %llu", (unsigned long long)req_id);
    s->cv.notify_all();
    s->cv_done.wait(lk, [&] { return r->state == DONE; });
    fill_result(*r, out);
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_release(atsne_server* s, uint64_t req_id) {
    clear_error();
    ATSNE_REQUIRE(s, ATSNE_E_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = find(s, req_id);
    ATSNE_REQUIRE(r && !r->released, ATSNE_E_INVALID_ARG, "unknown request %llu", (unsigned long long)req_id);
    if (r->state != DONE) return ATSNE_E_BUSY;
    s->all.erase(req_id);
    free_request(s, r);
    s->stats.released++;
    s->stats.bytes_in_flight = s->arena.used();
    s->cv.notify_all();
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_stats_get(atsne_server* s, atsne_serve_stats* out) {
    clear_error();
    ATSNE_REQUIRE(s && out, ATSNE_E_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_snapshot(atsne_server* s, int64_t cap_rows, float* corpus, int32_t* nbr_idx,
                                             float* nbr_d2, float* P_cond, float* beta, float* rho,
                                             uint8_t* alive, int64_t* n_rows, uint64_t* epoch) {
    clear_error();
    ATSNE_REQUIRE(s && n_rows && epoch, ATSNE_E_INVALID_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    // wait for every submitted commit to be applied
    s->cv.notify_all();
    s->cv_done.wait(lk, [&] {
        if (s->fatal != ATSNE_OK) return true;
        if (s->next_commit != s->commits_submitted) return false;
        for (Request* r : s->active)
            if (r->kind != 1) return false;
        for (Request* r : s->pending)
            if (r->kind != 1) return false;
        return true;
    });
    ATSNE_REQUIRE(s->fatal == ATSNE_OK, s->fatal, "the server stopped after a failed launch or commit");
    const int64_t n = s->n_committed;
    *n_rows = n;
    *epoch = s->commits_submitted;
    ATSNE_REQUIRE(cap_rows >= n, ATSNE_E_NOMEM, "snapshot needs %lld rows", (long long)n);
    ATSNE_HIP(hipStreamSynchronize(s->s_commit));
    if (corpus) ATSNE_HIP(hipMemcpy(corpus, s->X, sizeof(float) * n * s->D, hipMemcpyDeviceToDevice));
    if (nbr_idx) ATSNE_HIP(hipMemcpy(nbr_idx, s->res_idx, sizeof(int32_t) * n * s->K0, hipMemcpyDeviceToDevice));
    if (nbr_d2) ATSNE_HIP(hipMemcpy(nbr_d2, s->res_d2, sizeof(float) * n * s->K0, hipMemcpyDeviceToDevice));
    if (P_cond) ATSNE_HIP(hipMemcpy(P_cond, s->res_P, sizeof(float) * n * s->K0, hipMemcpyDeviceToDevice));
    if (beta) ATSNE_HIP(hipMemcpy(beta, s->res_beta, sizeof(float) * n, hipMemcpyDeviceToDevice));
    ATSNE_TRY(serve_state(s->res_idx, s->K0, n, s->death, rho, alive, s->s_commit));
    ATSNE_HIP(hipStreamSynchronize(s->s_commit));
    return ATSNE_OK;
}

extern "C" atsne_status atsne_serve_destroy(atsne_server* s, int32_t force) {
    clear_error();
    if (!s) return ATSNE_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (!force) {
            for (auto& kv : s->all)
                if (kv.second->state == DONE && !kv.second->released)
                    ATSNE_REQUIRE(false, ATSNE_E_BUSY, "request %llu has unreleased results",
                                  (unsigned long long)kv.first);
        }
    }
    destroy_impl(s);
    return ATSNE_OK;
}

static void destroy_impl(atsne_server* s) {
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // requests not yet admitted are cancelled; admitted ones finish
        for (Request* r : s->pending) fail_request(s, *r, ATSNE_E_BUSY);
        s->pending.clear();
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->all) free_request(s, kv.second);
    s->all.clear();
    for (auto& b : s->slot) {
        if (b.st) (void)hipStreamSynchronize(b.st);
        (void)hipFree(b.ws);
        (void)hipFree(b.d_desc);
        (void)hipFree(b.b_idx);
        (void)hipFree(b.b_d2);
        (void)hipFree(b.b_d2_lo);
        (void)hipFree(b.b_flags);
        if (b.h_desc) (void)hipHostFree(b.h_desc);
        if (b.ev) (void)hipEventDestroy(b.ev);
        if (b.st) (void)hipStreamDestroy(b.st);
    }
    for (hipStream_t st : {s->s_copy, s->s_commit, s->s_finish})
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    (void)hipFree(s->rev_ws);
    (void)hipFree(s->arena_mem);
    (void)hipFree(s->res_mem);
    (void)hipFree(s->corpus_mem);
    (void)hipFree(s->X);
    delete s;
}
