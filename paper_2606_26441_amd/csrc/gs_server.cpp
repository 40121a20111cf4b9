// Continuous-batching request loop over one resident index (the paper's
// future work (3), Sec. 8: streaming query batching for serving).
//
// Requests are queued as they are submitted. Admission is by memory: the
// server owns one workspace arena of `rows` query rows (each row: the score
// array of one query plus its selection scratch, the memory a query's score
// buffer needs), sized to the memory budget. A scheduler thread owns `n_slots`
// slots (a HIP stream, a reusable batch of max_batch queries, step counters,
// output rows on the device and pinned host rows). Whenever a slot is free and
// requests are waiting, the scheduler takes a contiguous run of free arena
// rows, moves as many waiting requests (FIFO, at most max_batch) into the slot,
// and enqueues their search, the copy of results and diagnostics, and an event
// on the slot's stream; slots run concurrently on the device. When a slot's
// event completes, its requests get their results and latency (submission to
// completion) and its rows return to the arena. A request that arrives while
// others are on the GPU is admitted as soon as a slot and rows are free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gpusparse.h"
#include "gs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t ticket = 0;
    std::vector<int32_t> terms;
    std::vector<float> weights;
    int32_t k = 0;
    Clock::time_point t_submit;
};

struct Result {
    std::vector<int32_t> ids;
    std::vector<uint8_t> scores;  // k * score size bytes
    double latency_ms = 0.0;
    int32_t status = GS_OK;
    std::string msg;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    gs_batch batch = nullptr;
    uint32_t* counters = nullptr;  // device: this slot's step counters
    int32_t* d_ids = nullptr;
    void* d_scores = nullptr;
    int32_t* h_ids = nullptr;    // pinned
    void* h_scores = nullptr;    // pinned
    int32_t* h_diag = nullptr;   // pinned: per-query selection diagnostics of the step
    std::vector<Request> reqs;   // in flight
    int64_t row0 = 0;            // arena rows [row0, row0 + reqs.size()) held by the step
    bool busy = false;
};

// Free runs of arena rows: start -> length, adjacent runs merged.
struct RowRuns {
    std::map<int64_t, int64_t> free;
    int64_t in_use = 0;
    void init(int64_t n) {
        free.clear();
        if (n > 0) free[0] = n;
    }
    // The first run of at least `want` rows, else the longest run: returns its start and
    // sets *got to the rows taken (0 when every row is in use).
    int64_t take(int64_t want, int64_t* got) {
        auto best = free.end();
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= want) { best = it; break; }
            if (best == free.end() || it->second > best->second) best = it;
        }
        *got = 0;
        if (best == free.end()) return 0;
        const int64_t start = best->first, len = best->second;
        *got = std::min(want, len);
        free.erase(best);
        if (len > *got) free[start + *got] = len - *got;
        in_use += *got;
        return start;
    }
    void give(int64_t start, int64_t n) {
        if (n <= 0) return;
        in_use -= n;
        auto next = free.lower_bound(start);
        int64_t s = start, len = n;
        if (next != free.end() && next->first == s + len) {
            len += next->second;
            next = free.erase(next);
        }
        if (next != free.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == s) {
                s = prev->first;
                len += prev->second;
                free.erase(prev);
            }
        }
        free[s] = len;
    }
};

int32_t sfail(int32_t code, const std::string& m) { return gs::set_error(code, m); }

}  // namespace

struct gs_server_s {
    gs_index index = nullptr;
    gs_server_opts opts{};
    size_t score_size = 4;
    int device = 0;
    int64_t n_docs = 0;
    int32_t precision = 0;
    std::vector<Slot> slots;
    void* arena = nullptr;  // device: the workspace rows of every in-flight query
    int64_t arena_rows = 0;
    size_t arena_bytes = 0;
    RowRuns rows;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request> pending;
    std::unordered_map<int64_t, Result> done;
    std::vector<bool> collected;  // per ticket: its result was handed out
    int64_t next_ticket = 0;
    int waiters = 0;
    bool stop = false;
    std::thread sched;
    // stats
    int64_t n_done = 0, n_failed = 0, n_steps = 0, queries_in_steps = 0, max_inflight = 0;

    void run();
    void launch(Slot& s);
    void finish(Slot& s, int32_t status, const std::string& msg);
    ~gs_server_s();
};

void gs_server_s::launch(Slot& s) {
    // host CSR of the requests taken into this slot
    const int32_t n = (int32_t)s.reqs.size();
    std::vector<int64_t> rp((size_t)n + 1, 0);
    std::vector<int32_t> terms, k((size_t)n);
    std::vector<float> w;
    for (int32_t i = 0; i < n; i++) {
        const Request& r = s.reqs[(size_t)i];
        terms.insert(terms.end(), r.terms.begin(), r.terms.end());
        w.insert(w.end(), r.weights.begin(), r.weights.end());
        rp[(size_t)i + 1] = (int64_t)terms.size();
        k[(size_t)i] = r.k;
    }
    // the copies are staged in pinned memory and ordered before the search on the slot's stream
    int32_t rc = gs::batch_update(s.batch, rp.data(), n, terms.data(), w.data(), (int64_t)terms.size(), k.data(),
                                  s.stream, false);
    if (rc == GS_OK)
        rc = gs::search_rows(index, s.batch, arena, arena_rows, s.row0, s.counters, &opts.search, s.d_ids,
                             s.d_scores, s.stream);
    hipError_t e = hipSuccess;
    const size_t out_rows = (size_t)n * (size_t)opts.k_max;
    if (rc == GS_OK) e = hipMemcpyAsync(s.h_ids, s.d_ids, out_rows * 4, hipMemcpyDeviceToHost, s.stream);
    if (rc == GS_OK && e == hipSuccess)
        e = hipMemcpyAsync(s.h_scores, s.d_scores, out_rows * score_size, hipMemcpyDeviceToHost, s.stream);
    if (rc == GS_OK && e == hipSuccess)
        e = hipMemcpyAsync(s.h_diag, gs::batch_diag(s.batch), (size_t)n * gs::kDiagWords * 4, hipMemcpyDeviceToHost,
                           s.stream);
    if (rc == GS_OK && e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (rc != GS_OK || e != hipSuccess) {
        // the step's requests fail; the slot and its rows stay usable
        const std::string msg = rc != GS_OK ? std::string(gs_last_error()) : std::string(hipGetErrorString(e));
        finish(s, rc != GS_OK ? rc : GS_EHIP, msg);
        return;
    }
    s.busy = true;
}

// Hand the slot's requests their results (status GS_OK) or the failure, return its rows.
void gs_server_s::finish(Slot& s, int32_t status, const std::string& msg) {
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> l(mu);
    for (size_t i = 0; i < s.reqs.size(); i++) {
        const Request& r = s.reqs[i];
        Result res;
        res.status = status;
        res.msg = msg;
        if (status == GS_OK && s.h_diag[i * gs::kDiagWords + 3]) {
            res.status = GS_ECAPACITY;
            res.msg = "more than 32768 documents inside the bf16 error band of the k-th score";
        }
        if (res.status == GS_OK) {
            res.ids.assign(s.h_ids + i * (size_t)opts.k_max, s.h_ids + i * (size_t)opts.k_max + (size_t)r.k);
            const uint8_t* sc = (const uint8_t*)s.h_scores + i * (size_t)opts.k_max * score_size;
            res.scores.assign(sc, sc + (size_t)r.k * score_size);
            res.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
            n_done++;
        } else {
            n_failed++;
        }
        done[r.ticket] = std::move(res);
    }
    if (status == GS_OK) {
        n_steps++;
        queries_in_steps += (int64_t)s.reqs.size();
    }
    rows.give(s.row0, (int64_t)s.reqs.size());
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
}

void gs_server_s::run() {
    (void)hipSetDevice(device);
    for (;;) {
        // completions
        bool any_busy = false;
        for (Slot& s : slots) {
            if (!s.busy) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipSuccess) finish(s, GS_OK, "");
            else if (q == hipErrorNotReady) any_busy = true;
            else finish(s, GS_EHIP, hipGetErrorString(q));
        }
        // admissions: a free slot takes a run of free rows and as many waiting requests
        std::vector<Slot*> to_launch;
        {
            std::unique_lock<std::mutex> l(mu);
            if (stop) break;
            for (Slot& s : slots) {
                if (s.busy || pending.empty()) continue;
                int64_t got = 0;
                const int64_t want = std::min<int64_t>((int64_t)pending.size(), opts.max_batch);
                const int64_t r0 = rows.take(want, &got);
                if (got == 0) break;  // every row is in use: wait for a completion
                s.row0 = r0;
                for (int64_t i = 0; i < got; i++) {
                    s.reqs.push_back(std::move(pending.front()));
                    pending.pop_front();
                }
                to_launch.push_back(&s);
            }
            if (to_launch.empty()) {
                if (any_busy) cv_sched.wait_for(l, std::chrono::microseconds(20));
                else cv_sched.wait(l, [&] { return stop || !pending.empty(); });
                continue;
            }
            max_inflight = std::max(max_inflight, rows.in_use);
        }
        for (Slot* s : to_launch) launch(*s);
    }
}

gs_server_s::~gs_server_s() {
    {
        std::unique_lock<std::mutex> l(mu);
        stop = true;
        cv_sched.notify_all();
        cv_done.notify_all();
        // callers blocked in gs_server_wait return (the server is stopping) before it is freed
        cv_done.wait(l, [&] { return waiters == 0; });
    }
    if (sched.joinable()) sched.join();
    (void)hipSetDevice(device);
    for (Slot& s : slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.batch) gs_batch_free(s.batch);
        if (s.counters) (void)hipFree(s.counters);
        if (s.d_ids) (void)hipFree(s.d_ids);
        if (s.d_scores) (void)hipFree(s.d_scores);
        if (s.h_ids) (void)hipHostFree(s.h_ids);
        if (s.h_scores) (void)hipHostFree(s.h_scores);
        if (s.h_diag) (void)hipHostFree(s.h_diag);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    if (arena) (void)hipFree(arena);
}

namespace {

// Wait for (timeout_ms < 0: no limit; 0: poll) and collect one ticket's result.
int32_t collect(gs_server s, int64_t ticket, int32_t timeout_ms, int32_t* out_ids, void* out_scores,
                double* latency_ms) {
    std::unique_lock<std::mutex> l(s->mu);
    if (ticket < 0 || ticket >= s->next_ticket) return sfail(GS_EINVAL, "unknown ticket");
    if (s->collected[(size_t)ticket]) return sfail(GS_EINVAL, "ticket already collected");
    s->waiters++;
    auto ready = [&] { return s->stop || s->done.count(ticket) != 0 || s->collected[(size_t)ticket]; };
    bool ok = true;
    if (timeout_ms < 0) s->cv_done.wait(l, ready);
    else ok = s->cv_done.wait_for(l, std::chrono::milliseconds(timeout_ms), ready);
    int32_t rc = GS_OK;
    Result res;
    if (!ok) {
        rc = sfail(GS_ETIMEOUT, "request not finished");
    } else if (s->done.count(ticket)) {
        res = std::move(s->done[ticket]);
        s->done.erase(ticket);
        s->collected[(size_t)ticket] = true;
    } else if (s->collected[(size_t)ticket]) {
        rc = sfail(GS_EINVAL, "ticket collected by another caller");
    } else {
        rc = sfail(GS_EINVAL, "server stopped before the request finished");
    }
    s->waiters--;
    if (s->stop) s->cv_done.notify_all();
    l.unlock();
    if (rc != GS_OK) return rc;
    if (res.status != GS_OK) return sfail(res.status, "search failed: " + res.msg);
    if (out_ids) std::memcpy(out_ids, res.ids.data(), res.ids.size() * 4);
    if (out_scores) std::memcpy(out_scores, res.scores.data(), res.scores.size());
    if (latency_ms) *latency_ms = res.latency_ms;
    return GS_OK;
}

}  // namespace

extern "C" {

int32_t gs_server_create(gs_index index, const gs_server_opts* opts, gs_server* out) {
    gs::set_error(GS_OK, "");
    if (!index || !opts || !out) return sfail(GS_EINVAL, "null argument");
    *out = nullptr;
    gs_server_opts o = *opts;
    if (o.reserved != 0) return sfail(GS_EINVAL, "reserved field must be 0");
    if (o.max_batch < 1 || o.n_slots < 1 || o.k_max < 1 || o.k_max > GS_MAX_K || o.memory_budget < 0)
        return sfail(GS_EINVAL, "max_batch, n_slots, k_max must be >= 1, k_max <= GS_MAX_K, budget >= 0");
    gs_index_info_t info;
    if (gs_index_info(index, &info) != GS_OK) return sfail(GS_EINVAL, "bad index");
    size_t one = 0;
    int32_t rc = gs_workspace_size(index, 1, &o.search, &one);  // also validates the options
    if (rc != GS_OK) return sfail(rc, gs_last_error());
    // admission by memory: the arena holds as many query rows as the budget allows (without a
    // budget, every slot's full batch)
    int64_t n_rows = (int64_t)o.n_slots * o.max_batch;
    if (o.memory_budget > 0) {
        if (gs::arena_bytes(info.n_docs, 1, info.precision) > (size_t)o.memory_budget)
            return sfail(GS_ECAPACITY, "memory budget below one query's score buffer");
        int64_t lo = 1, hi = n_rows;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (gs::arena_bytes(info.n_docs, mid, info.precision) <= (size_t)o.memory_budget) lo = mid;
            else hi = mid - 1;
        }
        n_rows = lo;
    }
    gs_server s = new (std::nothrow) gs_server_s();
    if (!s) return sfail(GS_ENOMEM, "host allocation failed");
    s->index = index;
    s->opts = o;
    s->n_docs = info.n_docs;
    s->precision = info.precision;
    s->score_size = info.precision == GS_BF16 ? 8 : 4;
    (void)hipGetDevice(&s->device);
    auto bail = [&](int32_t code, const std::string& m) {
        delete s;
        return sfail(code, m);
    };
    s->arena_rows = n_rows;
    s->arena_bytes = gs::arena_bytes(info.n_docs, n_rows, info.precision);
    if (gs::dev_malloc(&s->arena, s->arena_bytes) != hipSuccess) {
        s->arena = nullptr;
        return bail(GS_ENOMEM, "device allocation of the workspace arena failed");
    }
    s->rows.init(n_rows);
    s->slots.resize((size_t)o.n_slots);
    const size_t out_rows = (size_t)o.max_batch * (size_t)o.k_max;
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return bail(GS_EHIP, "stream/event creation failed");
        if (gs::dev_malloc((void**)&sl.counters, 16 * 4) != hipSuccess ||
            gs::dev_malloc((void**)&sl.d_ids, out_rows * 4) != hipSuccess ||
            gs::dev_malloc(&sl.d_scores, out_rows * s->score_size) != hipSuccess)
            return bail(GS_ENOMEM, "device allocation for a slot failed");
        if (gs::pinned_malloc((void**)&sl.h_ids, out_rows * 4) != hipSuccess ||
            gs::pinned_malloc(&sl.h_scores, out_rows * s->score_size) != hipSuccess ||
            gs::pinned_malloc((void**)&sl.h_diag, (size_t)o.max_batch * gs::kDiagWords * 4) != hipSuccess)
            return bail(GS_ENOMEM, "pinned host allocation for a slot failed");
        rc = gs_batch_reserve(index, o.max_batch, (int64_t)o.max_batch * GS_MAX_QUERY_NNZ, o.k_max, &sl.batch);
        if (rc != GS_OK) return bail(rc, gs_last_error());
    }
    s->sched = std::thread([s] { s->run(); });
    *out = s;
    return GS_OK;
}

int64_t gs_server_submit(gs_server s, const int32_t* term_ids, const float* weights, int32_t nnz, int32_t k) {
    gs::set_error(GS_OK, "");
    if (!s) return sfail(GS_EINVAL, "server is null");
    if (nnz < 0 || nnz > GS_MAX_QUERY_NNZ || (nnz > 0 && (!term_ids || !weights)))
        return sfail(GS_EINVAL, "bad query");
    if (k < 0 || k > s->opts.k_max) return sfail(GS_EINVAL, "k outside [0, k_max]");
    gs_index_info_t info;
    (void)gs_index_info(s->index, &info);
    for (int32_t j = 0; j < nnz; j++) {
        if (term_ids[j] < 0 || term_ids[j] >= info.vocab_size) return sfail(GS_EINVAL, "term id out of range");
        if (!(weights[j] >= 0.0f) || weights[j] > 3.4e38f) return sfail(GS_EINVAL, "weight negative or not finite");
        for (int32_t i = 0; i < j; i++)
            if (term_ids[i] == term_ids[j]) return sfail(GS_EINVAL, "duplicate term");
    }
    Request r;
    r.terms.assign(term_ids, term_ids + nnz);
    r.weights.assign(weights, weights + nnz);
    r.k = k;
    r.t_submit = Clock::now();
    int64_t t;
    {
        std::lock_guard<std::mutex> l(s->mu);
        if (s->stop) return sfail(GS_EINVAL, "server is stopping");
        t = s->next_ticket++;
        s->collected.push_back(false);
        r.ticket = t;
        s->pending.push_back(std::move(r));
    }
    s->cv_sched.notify_one();
    return t;
}

int32_t gs_server_wait(gs_server s, int64_t ticket, int32_t timeout_ms, int32_t* out_ids, void* out_scores,
                       double* latency_ms) {
    gs::set_error(GS_OK, "");
    if (!s) return sfail(GS_EINVAL, "server is null");
    return collect(s, ticket, timeout_ms, out_ids, out_scores, latency_ms);
}

int32_t gs_server_poll(gs_server s, int64_t ticket, int32_t* out_ids, void* out_scores, double* latency_ms) {
    gs::set_error(GS_OK, "");
    if (!s) return sfail(GS_EINVAL, "server is null");
    return collect(s, ticket, 0, out_ids, out_scores, latency_ms);
}

int32_t gs_server_stats(gs_server s, gs_server_stats_t* out) {
    gs::set_error(GS_OK, "");
    if (!s || !out) return sfail(GS_EINVAL, "null argument");
    std::lock_guard<std::mutex> l(s->mu);
    out->n_slots = (int32_t)s->slots.size();
    out->max_batch = s->opts.max_batch;
    out->completed = s->n_done;
    out->failed = s->n_failed;
    out->device_steps = s->n_steps;
    out->mean_batch = s->n_steps ? (double)s->queries_in_steps / (double)s->n_steps : 0.0;
    out->max_in_flight = s->max_inflight;
    out->pending = (int64_t)s->pending.size();
    out->arena_rows = s->arena_rows;
    out->arena_bytes = (int64_t)s->arena_bytes;
    out->row_bytes = s->arena_rows ? (int64_t)(s->arena_bytes / (size_t)s->arena_rows) : 0;
    return GS_OK;
}

void gs_server_destroy(gs_server s) { delete s; }

}  // extern "C"
