// Continuous-batching request loop over one resident index (the paper's
// future work (3), Sec. 8: streaming query batching for serving).
//
// Requests are queued as they are submitted. A scheduler thread owns
// `n_slots` device slots; each slot has its own HIP stream, a reusable query
// batch of `max_batch` queries, a workspace (one score array per query plus
// selection scratch: the memory a query's score buffer needs), device output
// rows and pinned host rows. Whenever a slot is free and requests are waiting,
// the scheduler moves up to `max_batch` of them (FIFO) into the slot, enqueues
// the search and the copy of the results on the slot's stream and records an
// event; slots run concurrently on the device. Completed slots are detected by
// their events, results are handed to the waiting callers with their latency
// (submission to completion), and the slot takes the next requests. The number
// of slots is bounded by the device-memory budget, so admission is by the
// memory the queries' score buffers need.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    gs_batch batch = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t* d_ids = nullptr;
    void* d_scores = nullptr;
    int32_t* h_ids = nullptr;   // pinned
    void* h_scores = nullptr;   // pinned
    std::vector<Request> reqs;  // in flight
    bool busy = false;
};

int32_t sfail(int32_t code, const std::string& m) { return gs::set_error(code, m); }

}  // namespace

struct gs_server_s {
    gs_index index = nullptr;
    gs_server_opts opts{};
    size_t score_size = 4;
    int device = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request> pending;
    std::unordered_map<int64_t, Result> done;
    int64_t next_ticket = 0;
    bool stop = false;
    std::thread sched;
    // stats
    int64_t n_done = 0, n_steps = 0, queries_in_steps = 0, max_inflight = 0;
    std::string fatal;

    void run();
    void launch(Slot& s);
    void finish(Slot& s);
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
        rc = gs_search_batch(index, s.batch, s.ws, s.ws_bytes, s.d_ids, s.d_scores, &opts.search, s.stream);
    hipError_t e = hipSuccess;
    const size_t rows = (size_t)n * (size_t)opts.k_max;
    if (rc == GS_OK) e = hipMemcpyAsync(s.h_ids, s.d_ids, rows * 4, hipMemcpyDeviceToHost, s.stream);
    if (rc == GS_OK && e == hipSuccess)
        e = hipMemcpyAsync(s.h_scores, s.d_scores, rows * score_size, hipMemcpyDeviceToHost, s.stream);
    if (rc == GS_OK && e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (rc != GS_OK || e != hipSuccess) {
        // requests fail individually; the slot stays usable
        const std::string msg = rc != GS_OK ? std::string(gs_last_error()) : std::string(hipGetErrorString(e));
        std::lock_guard<std::mutex> l(mu);
        for (Request& r : s.reqs) {
            Result res;
            res.status = rc != GS_OK ? rc : GS_EHIP;
            done[r.ticket] = std::move(res);
        }
        s.reqs.clear();
        fatal = msg;
        cv_done.notify_all();
        return;
    }
    s.busy = true;
}

void gs_server_s::finish(Slot& s) {
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> l(mu);
    for (size_t i = 0; i < s.reqs.size(); i++) {
        const Request& r = s.reqs[i];
        Result res;
        res.ids.assign(s.h_ids + i * (size_t)opts.k_max, s.h_ids + i * (size_t)opts.k_max + (size_t)r.k);
        const uint8_t* sc = (const uint8_t*)s.h_scores + i * (size_t)opts.k_max * score_size;
        res.scores.assign(sc, sc + (size_t)r.k * score_size);
        res.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
        done[r.ticket] = std::move(res);
        n_done++;
    }
    n_steps++;
    queries_in_steps += (int64_t)s.reqs.size();
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
            if (q == hipSuccess) finish(s);
            else if (q == hipErrorNotReady) any_busy = true;
            else {
                std::lock_guard<std::mutex> l(mu);
                fatal = hipGetErrorString(q);
                for (Request& r : s.reqs) {
                    Result res;
                    res.status = GS_EHIP;
                    done[r.ticket] = std::move(res);
                }
                s.reqs.clear();
                s.busy = false;
                cv_done.notify_all();
            }
        }
        // admissions: every free slot takes up to max_batch waiting requests
        std::vector<Slot*> to_launch;
        {
            std::unique_lock<std::mutex> l(mu);
            if (stop) break;
            for (Slot& s : slots) {
                if (s.busy || pending.empty()) continue;
                const size_t take = std::min(pending.size(), (size_t)opts.max_batch);
                for (size_t i = 0; i < take; i++) {
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
        }
        for (Slot* s : to_launch) launch(*s);
        int64_t inflight = 0;
        for (Slot& s : slots) inflight += s.busy ? (int64_t)s.reqs.size() : 0;
        std::lock_guard<std::mutex> l(mu);
        max_inflight = std::max(max_inflight, inflight);
    }
}

gs_server_s::~gs_server_s() {
    {
        std::lock_guard<std::mutex> l(mu);
        stop = true;
    }
    cv_sched.notify_all();
    if (sched.joinable()) sched.join();
    (void)hipSetDevice(device);
    for (Slot& s : slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.batch) gs_batch_free(s.batch);
        if (s.ws) (void)hipFree(s.ws);
        if (s.d_ids) (void)hipFree(s.d_ids);
        if (s.d_scores) (void)hipFree(s.d_scores);
        if (s.h_ids) (void)hipHostFree(s.h_ids);
        if (s.h_scores) (void)hipHostFree(s.h_scores);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
}

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
    size_t ws_bytes = 0;
    int32_t rc = gs_workspace_size(index, o.max_batch, &o.search, &ws_bytes);
    if (rc != GS_OK) return sfail(rc, gs_last_error());
    // admission by memory: slots whose score buffers fit the budget
    if (o.memory_budget > 0) {
        const int64_t fit = o.memory_budget / (int64_t)ws_bytes;
        if (fit < 1) return sfail(GS_ECAPACITY, "memory budget below one slot's score buffers");
        o.n_slots = (int32_t)std::min<int64_t>(o.n_slots, fit);
    }
    gs_server s = new (std::nothrow) gs_server_s();
    if (!s) return sfail(GS_ENOMEM, "host allocation failed");
    s->index = index;
    s->opts = o;
    s->score_size = info.precision == GS_BF16 ? 8 : 4;
    (void)hipGetDevice(&s->device);
    s->slots.resize((size_t)o.n_slots);
    auto bail = [&](int32_t code, const std::string& m) {
        delete s;
        return sfail(code, m);
    };
    const size_t rows = (size_t)o.max_batch * (size_t)o.k_max;
    for (Slot& sl : s->slots) {
        sl.ws_bytes = ws_bytes;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return bail(GS_EHIP, "stream/event creation failed");
        if (hipMalloc(&sl.ws, ws_bytes) != hipSuccess || hipMalloc((void**)&sl.d_ids, rows * 4) != hipSuccess ||
            hipMalloc(&sl.d_scores, rows * s->score_size) != hipSuccess)
            return bail(GS_ENOMEM, "device allocation for a slot failed");
        if (hipHostMalloc((void**)&sl.h_ids, rows * 4, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.h_scores, rows * s->score_size, hipHostMallocDefault) != hipSuccess)
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
        t = s->next_ticket++;
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
    std::unique_lock<std::mutex> l(s->mu);
    if (ticket < 0 || ticket >= s->next_ticket) return sfail(GS_EINVAL, "unknown ticket");
    auto ready = [&] { return s->done.count(ticket) != 0; };
    if (timeout_ms < 0) s->cv_done.wait(l, ready);
    else if (!s->cv_done.wait_for(l, std::chrono::milliseconds(timeout_ms), ready))
        return sfail(GS_ETIMEOUT, "request not finished");
    Result res = std::move(s->done[ticket]);
    s->done.erase(ticket);
    l.unlock();
    if (res.status != GS_OK) return sfail(res.status, "search failed: " + s->fatal);
    if (out_ids) std::memcpy(out_ids, res.ids.data(), res.ids.size() * 4);
    if (out_scores) std::memcpy(out_scores, res.scores.data(), res.scores.size());
    if (latency_ms) *latency_ms = res.latency_ms;
    return GS_OK;
}

int32_t gs_server_stats(gs_server s, gs_server_stats_t* out) {
    gs::set_error(GS_OK, "");
    if (!s || !out) return sfail(GS_EINVAL, "null argument");
    std::lock_guard<std::mutex> l(s->mu);
    out->n_slots = (int32_t)s->slots.size();
    out->max_batch = s->opts.max_batch;
    out->completed = s->n_done;
    out->device_steps = s->n_steps;
    out->mean_batch = s->n_steps ? (double)s->queries_in_steps / (double)s->n_steps : 0.0;
    out->max_in_flight = s->max_inflight;
    out->pending = (int64_t)s->pending.size();
    out->slot_bytes = (int64_t)(s->slots.empty() ? 0 : s->slots[0].ws_bytes);
    return GS_OK;
}

void gs_server_destroy(gs_server s) { delete s; }

}  // extern "C"
