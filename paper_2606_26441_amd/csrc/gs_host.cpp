// Host side of libgpusparse.so: argument validation, the term-major posting
// layout (paper Sec. 3.2), device residency of the index and of query
// batches, workspace carving and the per-tile launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <limits>
#include <thread>
#include <vector>

#include "../../include/gpusparse.h"
#include "gs_internal.h"

using namespace gs;

namespace gs {
thread_local const char* g_failed_launch = "";
int32_t set_error(int32_t code, const std::string& msg);

namespace {
// fault injection for tests: allocations left before one fails (-1: none fails)
std::atomic<int64_t> g_alloc_countdown{-1};

bool inject_alloc_failure() {
    int64_t v = g_alloc_countdown.load();
    while (v >= 0) {
        if (g_alloc_countdown.compare_exchange_weak(v, v - 1)) return v == 0;
    }
    return false;
}
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
    if (inject_alloc_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(void** p, size_t bytes) {
    if (inject_alloc_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}
}  // namespace gs

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define GS_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(e_ == hipErrorOutOfMemory ? GS_ENOMEM : GS_EHIP,                              \
                        std::string(#call) + ": " + hipGetErrorString(e_));                           \
    } while (0)

int n_workers() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min(h, 16u);
}

template <typename F>
void parallel_for(int64_t n, F f) {
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(n_workers(), n / 4096 + 1));
    if (T == 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; t++) {
        const int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([=, &f] { f(t, a, b); });
    }
    for (auto& x : th) x.join();
}

inline uint16_t bf16_rne(float w) {
    uint32_t u;
    std::memcpy(&u, &w, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

inline float bf16_widen(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// uint8 impact: round(w * 255 / 3) with ties to even, saturated to [0, 255].
inline uint8_t q8(float w) {
    const double x = std::nearbyint((double)w * 85.0);
    return x > 255.0 ? 255 : (x > 0.0 ? (uint8_t)x : 0);
}

}  // namespace

int32_t gs::set_error(int32_t code, const std::string& msg) { return fail(code, msg); }

namespace {

// ------------------------------------------------- fixed-point plan ------
//
// Per-query scale of the fixed-point sums (fp32 and bf16 weights; Sec. 4.1's
// scatter-add of w_q(t) * w_d(t) done in integers). Products are rounded to
// units of 2^-F and summed exactly.
//  * fp32 (64-bit sums): every product of the query below 2^51 units, from the
//    largest stored weight of each query term, so a sum of at most 256 products
//    stays below 2^59.
//  * bf16 (32-bit sums): every doc's sum below 2^32 units. A sum is at most
//    sumprod * 2^F (sumprod: the query weights times their terms' largest stored
//    weights) plus half a unit of rounding per product; F is the largest with
//    sumprod * 2^F + m + 2 < 2^32.
// abs_err bounds |fixed-point score - exact score|: half a unit per product plus
// the conversions, (m + 1) units. wide_lim: the selection sends the query to the
// fp64 pass when its k-th approximate score may lie below abs_err / rho, rho the
// relative budget of that error (fp32: 2^-18, so that two scores compared across
// the k-th boundary stay within the 1e-5 rule; bf16: 2^-12, small beside the
// error band's bf16 width). A positive score is at least the smallest positive
// product (query weight times its term's smallest positive stored weight); when
// that is at or above the limit, no score can miss the budget and wide_lim is 0.
struct FixedPlan {
    int F = 0;
    double scale = 1.0, abs_err = 0.0, wide_lim = 0.0;
};

FixedPlan fixed_point_plan(int precision, int64_t m, const float* w, const float* tmax, const float* tmin) {
    FixedPlan p;
    double maxprod = 0.0, sumprod = 0.0, minprod = std::numeric_limits<double>::infinity();
    for (int64_t j = 0; j < m; j++) {
        const double pm = (double)w[j] * (double)tmax[j];
        maxprod = std::max(maxprod, pm);
        sumprod += pm;
        if (w[j] > 0.0f && std::isfinite(tmin[j])) minprod = std::min(minprod, (double)w[j] * (double)tmin[j]);
    }
    int ex = 0;
    if (precision == kBF16) {
        if (sumprod > 0.0) {
            (void)std::frexp((4294967296.0 - (double)m - 3.0) / (sumprod * (1.0 + 1e-9)), &ex);
            p.F = ex - 1;  // 2^F <= (2^32 - m - 3) / sumprod
        }
    } else {
        if (maxprod > 0.0) (void)std::frexp(maxprod * (1.0 + 1e-9), &ex);  // maxprod < 2^ex
        p.F = 51 - ex;
    }
    p.F = std::min(1000, std::max(-1000, p.F));
    p.scale = std::ldexp(1.0, -p.F);
    p.abs_err = (double)(m + 1) * p.scale * (1.0 + 1e-6);
    if (precision != kU8) {
        const double lim = p.abs_err / std::ldexp(1.0, precision == kFP32 ? -18 : -12);
        p.wide_lim = lim <= minprod ? 0.0 : lim;
    }
    return p;
}

// ----------------------------------------------------------- CSR checks --

struct Rows {
    const int64_t* row_ptr;
    const int32_t* term;
    const float* w;
    int64_t n;
    std::vector<int32_t> term_sorted;  // filled when some input row is unsorted
    std::vector<float> w_sorted;
};

// Validate a CSR of (term, weight) rows; when a row is unsorted, keep a sorted copy.
int32_t check_rows(Rows& r, int64_t nnz, int32_t vocab, int64_t max_row, const char* what) {
    if (r.n < 0 || nnz < 0) return fail(GS_EINVAL, std::string(what) + ": negative size");
    if (r.n > 0 || nnz > 0) {
        if (!r.row_ptr) return fail(GS_EINVAL, std::string(what) + ": null row_ptr");
        if (nnz > 0 && (!r.term || !r.w)) return fail(GS_EINVAL, std::string(what) + ": null arrays");
    }
    if (r.row_ptr && r.row_ptr[0] != 0) return fail(GS_EINVAL, std::string(what) + ": row_ptr[0] != 0");
    if (r.row_ptr && r.row_ptr[r.n] != nnz) return fail(GS_EINVAL, std::string(what) + ": row_ptr[n] != nnz");
    for (int64_t i = 0; i < r.n; i++)
        if (r.row_ptr[i + 1] < r.row_ptr[i] || r.row_ptr[i + 1] - r.row_ptr[i] > max_row)
            return fail(GS_EINVAL, std::string(what) + ": row " + std::to_string(i) +
                                       " has a negative length or more than " + std::to_string(max_row) + " terms");
    std::atomic<int> bad{0}, unsorted{0};
    parallel_for(r.n, [&](int, int64_t a, int64_t b) {
        for (int64_t i = a; i < b && !bad.load(std::memory_order_relaxed); i++) {
            for (int64_t j = r.row_ptr[i]; j < r.row_ptr[i + 1]; j++) {
                const float w = r.w[j];
                if (r.term[j] < 0 || r.term[j] >= vocab) { bad = 1; break; }
                if (!std::isfinite(w) || w < 0.0f) { bad = 2; break; }
                if (j > r.row_ptr[i] && r.term[j] <= r.term[j - 1]) {
                    if (r.term[j] == r.term[j - 1]) { bad = 3; break; }
                    unsorted = 1;
                }
            }
        }
    });
    if (bad == 1) return fail(GS_EINVAL, std::string(what) + ": term id out of range");
    if (bad == 2) return fail(GS_EINVAL, std::string(what) + ": weight negative or not finite");
    if (bad == 3) return fail(GS_EINVAL, std::string(what) + ": duplicate term in a row");
    if (unsorted) {
        r.term_sorted.resize((size_t)nnz);
        r.w_sorted.resize((size_t)nnz);
        parallel_for(r.n, [&](int, int64_t a, int64_t b) {
            std::vector<std::pair<int32_t, float>> tmp;
            for (int64_t i = a; i < b; i++) {
                const int64_t s = r.row_ptr[i], e = r.row_ptr[i + 1];
                tmp.clear();
                for (int64_t j = s; j < e; j++) tmp.emplace_back(r.term[j], r.w[j]);
                std::sort(tmp.begin(), tmp.end(),
                          [](const std::pair<int32_t, float>& x, const std::pair<int32_t, float>& y) {
                              return x.first < y.first;
                          });
                for (int64_t j = s; j < e; j++) {
                    r.term_sorted[(size_t)j] = tmp[(size_t)(j - s)].first;
                    r.w_sorted[(size_t)j] = tmp[(size_t)(j - s)].second;
                    if (j > s && tmp[(size_t)(j - s)].first == tmp[(size_t)(j - s - 1)].first) bad = 3;
                }
            }
        });
        if (bad == 3) return fail(GS_EINVAL, std::string(what) + ": duplicate term in a row");
        r.term = r.term_sorted.data();
        r.w = r.w_sorted.data();
    }
    return GS_OK;
}

// ------------------------------------------------------- posting layout --

struct Layout {
    int64_t n_docs = 0, nnz = 0, padded = 0, n_grains = 0;
    int32_t vocab = 0, precision = 0;
    std::vector<int64_t> term_off;   // [V+1]
    std::vector<int32_t> term_len;   // [V]
    std::vector<int32_t> post_doc;   // [padded]
    std::vector<float> w_f32;        // [padded] (GS_FP32)
    std::vector<uint16_t> w_bf16;    // [padded] (GS_BF16)
    std::vector<uint8_t> w_u8;       // [padded] (GS_U8)
    std::vector<float> blk_max;      // [padded / 64]
    std::vector<int32_t> blk_first;  // [padded / 64]
    std::vector<int32_t> tile_off;   // [V][n_grains+1]
};

float stored_weight(const Layout& L, int64_t i) {
    switch (L.precision) {
        case kFP32: return L.w_f32[(size_t)i];
        case kBF16: return bf16_widen(L.w_bf16[(size_t)i]);
        default: return (float)L.w_u8[(size_t)i];
    }
}

int32_t sizes_only(const Rows& r, int32_t vocab, Layout& L) {
    std::vector<int64_t> df((size_t)vocab, 0);
    for (int64_t j = 0; j < r.row_ptr[r.n]; j++) df[(size_t)r.term[j]]++;
    L.padded = 0;
    for (int32_t t = 0; t < vocab; t++) L.padded += (df[(size_t)t] + kBlock - 1) / kBlock * kBlock;
    return GS_OK;
}

int32_t build_layout(const Rows& r, int32_t vocab, int32_t precision, bool tiles, Layout& L) {
    const int64_t N = r.n, nnz = r.n > 0 ? r.row_ptr[r.n] : 0;
    L.n_docs = N;
    L.nnz = nnz;
    L.vocab = vocab;
    L.precision = precision;
    try {
        // term counts per worker over contiguous doc ranges (docs stay in order per term)
        const int T = std::max<int64_t>(1, std::min<int64_t>(n_workers(), N / 4096 + 1));
        std::vector<std::vector<int64_t>> cnt((size_t)T, std::vector<int64_t>((size_t)vocab, 0));
        std::vector<int64_t> lo((size_t)T + 1);
        for (int t = 0; t <= T; t++) lo[(size_t)t] = N * t / T;
        {
            std::vector<std::thread> th;
            for (int t = 0; t < T; t++)
                th.emplace_back([&, t] {
                    auto& c = cnt[(size_t)t];
                    for (int64_t j = r.row_ptr[lo[(size_t)t]]; j < r.row_ptr[lo[(size_t)t + 1]]; j++)
                        c[(size_t)r.term[j]]++;
                });
            for (auto& x : th) x.join();
        }
        L.term_off.assign((size_t)vocab + 1, 0);
        L.term_len.assign((size_t)vocab, 0);
        for (int32_t v = 0; v < vocab; v++) {
            int64_t df = 0;
            for (int t = 0; t < T; t++) df += cnt[(size_t)t][(size_t)v];
            L.term_len[(size_t)v] = (int32_t)df;
            L.term_off[(size_t)v + 1] = L.term_off[(size_t)v] + (df + kBlock - 1) / kBlock * kBlock;
        }
        L.padded = L.term_off[(size_t)vocab];
        // per-worker write cursors
        for (int32_t v = 0; v < vocab; v++) {
            int64_t run = L.term_off[(size_t)v];
            for (int t = 0; t < T; t++) {
                const int64_t c = cnt[(size_t)t][(size_t)v];
                cnt[(size_t)t][(size_t)v] = run;
                run += c;
            }
        }
        L.post_doc.assign((size_t)L.padded, -1);
        if (precision == kFP32) L.w_f32.assign((size_t)L.padded, 0.0f);
        if (precision == kBF16) L.w_bf16.assign((size_t)L.padded, 0);
        if (precision == kU8) L.w_u8.assign((size_t)L.padded, 0);
        {
            std::vector<std::thread> th;
            for (int t = 0; t < T; t++)
                th.emplace_back([&, t] {
                    auto& cur = cnt[(size_t)t];
                    for (int64_t d = lo[(size_t)t]; d < lo[(size_t)t + 1]; d++) {
                        for (int64_t j = r.row_ptr[d]; j < r.row_ptr[d + 1]; j++) {
                            const int64_t p = cur[(size_t)r.term[j]]++;
                            L.post_doc[(size_t)p] = (int32_t)d;
                            if (precision == kFP32) L.w_f32[(size_t)p] = r.w[j];
                            else if (precision == kBF16) L.w_bf16[(size_t)p] = bf16_rne(r.w[j]);
                            else L.w_u8[(size_t)p] = q8(r.w[j]);
                        }
                    }
                });
            for (auto& x : th) x.join();
        }
        // block-max metadata per 64-posting block
        const int64_t nb = L.padded / kBlock;
        L.blk_max.assign((size_t)nb, 0.0f);
        L.blk_first.assign((size_t)nb, -1);
        parallel_for(nb, [&](int, int64_t a, int64_t b) {
            for (int64_t k = a; k < b; k++) {
                float m = 0.0f;
                for (int64_t i = k * kBlock; i < (k + 1) * kBlock; i++) m = std::max(m, stored_weight(L, i));
                L.blk_max[(size_t)k] = m;
                L.blk_first[(size_t)k] = L.post_doc[(size_t)(k * kBlock)];
            }
        });
        // segment table: first posting at or after each 8192-doc grain start
        L.n_grains = (N + (1 << kGrainShift) - 1) >> kGrainShift;
        if (tiles) {
            const int64_t G = L.n_grains + 1;
            L.tile_off.assign((size_t)vocab * (size_t)G, 0);
            parallel_for(vocab, [&](int, int64_t a, int64_t b) {
                for (int64_t v = a; v < b; v++) {
                    const int32_t* docs = L.post_doc.data() + L.term_off[(size_t)v];
                    const int32_t len = L.term_len[(size_t)v];
                    int32_t* row = L.tile_off.data() + v * G;
                    int32_t i = 0;
                    for (int64_t g = 0; g < G; g++) {
                        const int64_t start = g << kGrainShift;
                        while (i < len && docs[i] < start) i++;
                        row[g] = i;
                    }
                }
            });
        }
    } catch (const std::bad_alloc&) {
        return fail(GS_ENOMEM, "host allocation failed while building the posting layout");
    }
    return GS_OK;
}

// Byte form of the doc ids: a term whose every 64-posting block spans at most 256 docs
// ("dense") also stores each id as its distance to the block's first doc.
void byte_form(const Layout& L, std::vector<uint8_t>& dense, std::vector<uint8_t>& b8) {
    dense.assign((size_t)L.vocab, 0);
    b8.assign((size_t)L.padded, 0);
    parallel_for(L.vocab, [&](int, int64_t a, int64_t b) {
        for (int64_t v = a; v < b; v++) {
            const int64_t o = L.term_off[(size_t)v];
            const int64_t len = L.term_len[(size_t)v];
            if (len == 0) continue;
            bool ok = true;
            for (int64_t k = 0; k < len && ok; k += kBlock) {
                const int64_t last = std::min(k + kBlock, len) - 1;
                ok = L.post_doc[(size_t)(o + last)] - L.post_doc[(size_t)(o + k)] <= 255;
            }
            if (!ok) continue;
            dense[(size_t)v] = 1;
            for (int64_t i = 0; i < len; i++)
                b8[(size_t)(o + i)] = (uint8_t)(L.post_doc[(size_t)(o + i)] - L.blk_first[(size_t)((o + i) / kBlock)]);
        }
    });
}

}  // namespace

// ===================================================================== API ==

struct gs_index_s {
    int device = 0;
    int64_t n_docs = 0, nnz = 0, padded = 0, n_grains = 0;
    int64_t n_dense = 0;              // terms whose lists have the byte doc-id form
    std::vector<uint8_t> term_dense;  // [V] host copy of the byte-form flags
    int32_t vocab = 0, precision = 0;
    uint32_t flags = 0;
    size_t bytes = 0;
    std::vector<float> term_max;  // largest stored weight of each term (value of the stored form)
    std::vector<float> term_min;  // smallest positive stored weight of each term (+inf if none)
    std::vector<int32_t> term_len;  // postings per term (host copy, for work estimates)
    std::vector<void*> allocs;
    DevIndex dev{};
    ~gs_index_s() {
        for (void* p : allocs) (void)hipFree(p);
    }
};

// Byte offsets of a batch's arrays inside its one device allocation (and the
// pinned host stage of the same layout): the per-query arrays first (copied
// whole on every update), then the per-term arrays (copied up to the terms in use).
struct BatchLayout {
    size_t rp = 0, k = 0, fs = 0, delta = 0, scale = 0, err = 0, wide = 0, work = 0, diag = 0, head = 0;
    size_t gcount = 0, gmember = 0, grow = 0;
    size_t term = 0, w = 0, w8 = 0, fx = 0, ubcum = 0, gterm = 0, gwfx = 0, gw8 = 0, total = 0;
    BatchLayout(size_t nq, size_t nz) {
        size_t at = 0;
        auto take = [&](size_t bytes) {
            const size_t o = at;
            at = (at + std::max<size_t>(bytes, 8) + 255) / 256 * 256;
            return o;
        };
        rp = take((nq + 1) * 8);
        k = take(nq * 4);
        fs = take(nq * 4);
        delta = take(nq * 4);
        scale = take(nq * 8);
        err = take(nq * 8);
        wide = take(nq * 8);
        work = take(nq * 8);
        diag = take(nq * kDiagWords * 4);
        gcount = take(4);
        gmember = take((nq + kGroupMax) * 4);
        grow = take((nq + 2) * 4);
        head = at;
        term = take(nz * 4);
        w = take(nz * 4);
        w8 = take(nz * 4);
        fx = take(nz * 8);
        ubcum = take(nz * 8);
        gterm = take(nz * 4);
        gwfx = take(nz * kGroupMax * 4);
        gw8 = take(nz * kGroupMax * 4);
        total = at;
    }
};

struct gs_batch_s {
    gs_index index = nullptr;          // borrowed: must outlive searches, not needed to free the batch
    int device = 0;                    // device holding the batch's memory
    int32_t n_queries = 0, k_max = 0;  // capacity in queries (launch shapes use it)
    int64_t q_nnz = 0;                 // capacity in query terms
    int32_t n_active = 0;              // queries set by the last update
    BatchLayout lay{0, 0};
    uint8_t* dmem = nullptr;    // device: every array of the batch
    uint8_t* stage = nullptr;   // pinned host copy of the same layout (update staging)
    hipEvent_t copied = nullptr;  // recorded after the last update's copies
    bool copy_pending = false;
    DevBatch dev{};
    int32_t* diag = nullptr;  // [n_queries * kDiagWords] (inside dmem)
    ~gs_batch_s() {
        if (copy_pending) (void)hipEventSynchronize(copied);
        if (copied) (void)hipEventDestroy(copied);
        if (dmem) (void)hipFree(dmem);
        if (stage) (void)hipHostFree(stage);
    }
};

namespace {

template <typename T>
int32_t dev_upload(std::vector<void*>& allocs, size_t& bytes, const T* host, size_t n, T** out, hipStream_t s,
                   size_t slack = 0) {
    *out = nullptr;
    const size_t copy = n;
    if (n == 0) n = 1;  // keep a valid pointer for empty arrays
    n += slack;         // zeroed entries past the end
    void* p = nullptr;
    GS_HIP(dev_malloc(&p, n * sizeof(T)));
    allocs.push_back(p);
    bytes += n * sizeof(T);
    if (host && copy) GS_HIP(hipMemcpyAsync(p, host, copy * sizeof(T), hipMemcpyHostToDevice, s));
    if (n > copy) GS_HIP(hipMemsetAsync((T*)p + copy, 0, (n - copy) * sizeof(T), s));
    *out = (T*)p;
    return GS_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// ---- kernel timing (measurement only) ----
struct TimedSpan {
    hipEvent_t a, b;
    int kind;     // 0 scoring, 1 selection
    bool counts;  // counts as one launch of its kind
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedSpan> g_spans;

bool timing_on() {
    std::lock_guard<std::mutex> l(g_timing_mu);
    return g_timing_on;
}

struct SpanRecorder {
    TimedSpan span{};
    bool active = false;
    // counts: whether the span counts as one launch of its kind (a scoring pass split into
    // two launches records the first one without counting it)
    SpanRecorder(int kind, hipStream_t s, bool counts = true) {
        if (kind < 0 || !timing_on()) return;
        span.kind = kind;
        span.counts = counts;
        if (hipEventCreate(&span.a) != hipSuccess) return;
        if (hipEventCreate(&span.b) != hipSuccess) {
            (void)hipEventDestroy(span.a);
            return;
        }
        active = hipEventRecord(span.a, s) == hipSuccess;
    }
    void end(hipStream_t s) {
        if (!active) return;
        if (hipEventRecord(span.b, s) == hipSuccess) {
            std::lock_guard<std::mutex> l(g_timing_mu);
            g_spans.push_back(span);
        } else {
            (void)hipEventDestroy(span.a);
            (void)hipEventDestroy(span.b);
        }
        active = false;
    }
};

}  // namespace

namespace gs {

// Workspace of `rows` query rows. Every per-query array is indexed by row, so a search of n
// queries may run on rows [r0, r0 + n) of a larger workspace (the server's arena): the
// work-prefix array of the global-atomic kernel takes kMaxQueryNnz + 1 entries per row for
// that reason. One block of step counters follows (a search on rows of an arena brings its own).
size_t arena_bytes(int64_t n_docs, int64_t rows, int32_t precision) {
    const size_t ld = (size_t)((n_docs + 63) / 64 * 64), R = (size_t)rows;
    size_t b = 0;
    b += align256(R * ld * 4);
    b += 2 * align256(R * kHistBins * 4);
    b += align256(R * sizeof(SelState));
    b += align256(R * kCandCap * 8);
    if (precision == kBF16) {
        b += align256(R * kCandCap * 8);
        b += align256(R * kCandCap * 4);
    }
    b += align256(R * (kMaxQueryNnz + 1) * 8);
    b += align256(R * kMaxQueryNnz * 4);
    b += align256(R * 4);
    b += align256(16 * 4);
    b += align256(R * 4);
    return b;
}

void carve_rows(void* base, int64_t n_docs, int64_t rows, int32_t precision, int64_t r0, Workspace* ws) {
    const size_t ld = (size_t)((n_docs + 63) / 64 * 64), R = (size_t)rows, o = (size_t)r0;
    char* p = (char*)base;
    auto take = [&](size_t n) {
        char* r = p;
        p += align256(n);
        return r;
    };
    ws->ld = (int64_t)ld;
    ws->scores = (uint32_t*)take(R * ld * 4) + o * ld;
    ws->hist1 = (uint32_t*)take(R * kHistBins * 4) + o * kHistBins;
    ws->hist_ref = (uint32_t*)take(R * kHistBins * 4) + o * kHistBins;
    ws->state = (SelState*)take(R * sizeof(SelState)) + o;
    ws->cand = (unsigned long long*)take(R * kCandCap * 8) + o * kCandCap;
    ws->band_s = nullptr;
    ws->band_id = nullptr;
    if (precision == kBF16) {
        ws->band_s = (double*)take(R * kCandCap * 8) + o * kCandCap;
        ws->band_id = (int32_t*)take(R * kCandCap * 4) + o * kCandCap;
    }
    ws->work_prefix = (int64_t*)take(R * (kMaxQueryNnz + 1) * 8) + o * (kMaxQueryNnz + 1);
    ws->work_pair_q = (int32_t*)take(R * kMaxQueryNnz * 4) + o * kMaxQueryNnz;
    ws->order = (int32_t*)take(R * 4) + o;
    ws->counters = (uint32_t*)take(16 * 4);
    ws->rescore_list = (int32_t*)take(R * 4) + o;
}

size_t workspace_bytes(int64_t n_docs, int32_t qt, int32_t precision) { return arena_bytes(n_docs, qt, precision); }

void carve_workspace(void* base, int64_t n_docs, int32_t qt, int32_t precision, Workspace* ws) {
    carve_rows(base, n_docs, qt, precision, 0, ws);
}

}  // namespace gs

extern "C" {

const char* gs_version(void) { return "gpusparse-mi355x 0.1 (gfx950)"; }

const char* gs_status_string(int32_t s) {
    switch (s) {
        case GS_OK: return "ok";
        case GS_EINVAL: return "invalid argument";
        case GS_ENOMEM: return "out of memory";
        case GS_EHIP: return "HIP runtime error";
        case GS_ECAPACITY: return "capacity exceeded";
        case GS_EUNSUPPORTED: return "unsupported";
        case GS_ETIMEOUT: return "timeout";
    }
    return "unknown status";
}

const char* gs_last_error(void) { return g_err.c_str(); }

int32_t gs_debug_fail_alloc(int64_t n) {
    g_alloc_countdown.store(n < 0 ? -1 : n);
    return GS_OK;
}

int32_t gs_layout_host(const int64_t* row_ptr, int64_t n_docs, const int32_t* term_ids, const float* weights,
                       int64_t nnz, int32_t vocab_size, int32_t precision, int64_t* out_padded_nnz, int64_t* term_off,
                       int32_t* term_len, int32_t* post_doc, float* post_w, float* blk_max, int32_t* blk_first_doc,
                       uint8_t* term_dense, uint8_t* post_b8) {
    g_err.clear();
    if (vocab_size < 1) return fail(GS_EINVAL, "vocab_size < 1");
    if (precision < kFP32 || precision > kU8) return fail(GS_EINVAL, "unknown precision");
    if (n_docs >= (int64_t)1 << 31) return fail(GS_EINVAL, "n_docs must be < 2^31");
    Rows r{row_ptr, term_ids, weights, n_docs, {}, {}};
    int32_t rc = check_rows(r, nnz, vocab_size, vocab_size, "documents");
    if (rc != GS_OK) return rc;
    Layout L;
    const bool want_arrays =
        term_off || term_len || post_doc || post_w || blk_max || blk_first_doc || term_dense || post_b8;
    if (!want_arrays) {
        if (!out_padded_nnz) return fail(GS_EINVAL, "nothing requested");
        sizes_only(r, vocab_size, L);
        *out_padded_nnz = L.padded;
        return GS_OK;
    }
    rc = build_layout(r, vocab_size, precision, false, L);
    if (rc != GS_OK) return rc;
    if (out_padded_nnz) *out_padded_nnz = L.padded;
    if (term_off) std::memcpy(term_off, L.term_off.data(), L.term_off.size() * 8);
    if (term_len) std::memcpy(term_len, L.term_len.data(), L.term_len.size() * 4);
    if (post_doc) std::memcpy(post_doc, L.post_doc.data(), L.post_doc.size() * 4);
    if (post_w)
        for (int64_t i = 0; i < L.padded; i++) post_w[i] = stored_weight(L, i);
    if (blk_max) std::memcpy(blk_max, L.blk_max.data(), L.blk_max.size() * 4);
    if (blk_first_doc) std::memcpy(blk_first_doc, L.blk_first.data(), L.blk_first.size() * 4);
    if (term_dense || post_b8) {
        std::vector<uint8_t> dense, b8;
        try {
            byte_form(L, dense, b8);
        } catch (const std::bad_alloc&) {
            return fail(GS_ENOMEM, "host memory for the byte doc offsets");
        }
        if (term_dense) std::memcpy(term_dense, dense.data(), dense.size());
        if (post_b8) std::memcpy(post_b8, b8.data(), b8.size());
    }
    return GS_OK;
}

int32_t gs_query_plan_host(int32_t precision, const float* q_weights, const float* term_max, const float* term_min,
                           int32_t nnz, int32_t* out_F, double* out_abs_err, double* out_wide_lim) {
    g_err.clear();
    if (precision != kFP32 && precision != kBF16) return fail(GS_EINVAL, "precision must be GS_FP32 or GS_BF16");
    if (nnz < 0 || nnz > kMaxQueryNnz) return fail(GS_EINVAL, "nnz outside [0, GS_MAX_QUERY_NNZ]");
    if (nnz > 0 && (!q_weights || !term_max || !term_min)) return fail(GS_EINVAL, "null array");
    for (int32_t j = 0; j < nnz; j++)
        if (!(q_weights[j] >= 0.0f) || !std::isfinite(q_weights[j]) || !(term_max[j] >= 0.0f) ||
            !std::isfinite(term_max[j]) || !(term_min[j] > 0.0f))
            return fail(GS_EINVAL, "weights must be finite and >= 0, term_min > 0 (+inf for an all-zero list)");
    const FixedPlan p = fixed_point_plan(precision, nnz, q_weights, term_max, term_min);
    if (out_F) *out_F = p.F;
    if (out_abs_err) *out_abs_err = p.abs_err;
    if (out_wide_lim) *out_wide_lim = p.wide_lim;
    return GS_OK;
}

int32_t gs_build_index(const int64_t* row_ptr, int64_t n_docs, const int32_t* term_ids, const float* weights,
                       int64_t nnz, int32_t vocab_size, int32_t precision, uint32_t flags, void* hip_stream,
                       gs_index* out) {
    g_err.clear();
    if (!out) return fail(GS_EINVAL, "out is null");
    *out = nullptr;
    if (vocab_size < 1) return fail(GS_EINVAL, "vocab_size < 1");
    if (precision < kFP32 || precision > kU8) return fail(GS_EINVAL, "unknown precision");
    if (flags & ~(uint32_t)(GS_KEEP_FORWARD | GS_KEEP_DOC_IDS)) return fail(GS_EINVAL, "unknown flag");
    if (n_docs >= (int64_t)1 << 31) return fail(GS_EINVAL, "n_docs must be < 2^31");
    Rows r{row_ptr, term_ids, weights, n_docs, {}, {}};
    int32_t rc = check_rows(r, nnz, vocab_size, vocab_size, "documents");
    if (rc != GS_OK) return rc;
    Layout L;
    rc = build_layout(r, vocab_size, precision, true, L);
    if (rc != GS_OK) return rc;

    hipStream_t s = (hipStream_t)hip_stream;
    gs_index ix = new (std::nothrow) gs_index_s();
    if (!ix) return fail(GS_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&ix->device);
    ix->n_docs = n_docs;
    ix->nnz = nnz;
    ix->padded = L.padded;
    ix->n_grains = L.n_grains;
    ix->vocab = vocab_size;
    ix->precision = precision;
    if (precision == kBF16) flags |= GS_KEEP_FORWARD;
    ix->flags = flags;
    ix->term_len = L.term_len;
    ix->term_max.assign((size_t)vocab_size, 0.0f);
    for (int32_t v = 0; v < vocab_size; v++)
        for (int64_t k = L.term_off[(size_t)v] / kBlock; k < L.term_off[(size_t)v + 1] / kBlock; k++)
            ix->term_max[(size_t)v] = std::max(ix->term_max[(size_t)v], L.blk_max[(size_t)k]);
    ix->term_min.assign((size_t)vocab_size, std::numeric_limits<float>::infinity());
    parallel_for(vocab_size, [&](int, int64_t a, int64_t b) {
        for (int64_t v = a; v < b; v++) {
            float m = std::numeric_limits<float>::infinity();
            for (int64_t i = L.term_off[(size_t)v]; i < L.term_off[(size_t)v] + L.term_len[(size_t)v]; i++) {
                const float w = stored_weight(L, i);
                if (w > 0.0f) m = std::min(m, w);
            }
            ix->term_min[(size_t)v] = m;
        }
    });
    DevIndex& d = ix->dev;
    d.n_docs = n_docs;
    d.vocab = vocab_size;
    d.precision = precision;
    d.n_grains = L.n_grains;
    auto done = [&](int32_t code) {
        if (code != GS_OK) delete ix;
        return code;
    };
    int64_t* term_off = nullptr;
    int32_t *term_len = nullptr, *post_doc = nullptr, *tile_off = nullptr;
    if ((rc = dev_upload(ix->allocs, ix->bytes, L.term_off.data(), L.term_off.size(), &term_off, s))) return done(rc);
    if ((rc = dev_upload(ix->allocs, ix->bytes, L.term_len.data(), L.term_len.size(), &term_len, s))) return done(rc);
    // 32-bit doc ids only for the global-atomic kernel: the doc-tiled kernels read 16- or 8-bit ones
    if (flags & GS_KEEP_DOC_IDS)
        if ((rc = dev_upload(ix->allocs, ix->bytes, L.post_doc.data(), L.post_doc.size(), &post_doc, s)))
            return done(rc);
    if ((rc = dev_upload(ix->allocs, ix->bytes, L.tile_off.data(), L.tile_off.size(), &tile_off, s))) return done(rc);
    d.term_off = term_off;
    d.term_len = term_len;
    d.post_doc = post_doc;
    d.tile_off = tile_off;
    {
        uint16_t* lo = nullptr;
        std::vector<uint16_t> low;
        try {
            low.resize(L.post_doc.size());
        } catch (const std::bad_alloc&) {
            return done(set_error(GS_ENOMEM, "host memory for the 16-bit doc offsets"));
        }
        const int64_t n = (int64_t)low.size();
        const int T = std::max<int64_t>(1, std::min<int64_t>(n_workers(), n / (1 << 20) + 1));
        std::vector<std::thread> th;
        for (int t = 0; t < T; t++)
            th.emplace_back([&, t] {
                for (int64_t i = n * t / T; i < n * (t + 1) / T; i++)
                    low[(size_t)i] = (uint16_t)((uint32_t)L.post_doc[(size_t)i] & 0xFFFFu);
            });
        for (auto& x : th) x.join();
        if ((rc = dev_upload(ix->allocs, ix->bytes, low.data(), low.size(), &lo, s, kPostSlack))) return done(rc);
        d.post_lo = lo;
        // the upload is asynchronous: `low` must outlive it
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return done(fail(GS_EHIP, std::string("upload: ") + hipGetErrorString(e)));
    }
    if (precision == kFP32) {
        float* p = nullptr;
        if ((rc = dev_upload(ix->allocs, ix->bytes, L.w_f32.data(), L.w_f32.size(), &p, s, kPostSlack))) return done(rc);
        d.post_w = p;
    } else if (precision == kBF16) {
        uint16_t* p = nullptr;
        if ((rc = dev_upload(ix->allocs, ix->bytes, L.w_bf16.data(), L.w_bf16.size(), &p, s, kPostSlack))) return done(rc);
        d.post_w = p;
    } else {
        uint8_t* p = nullptr;
        if ((rc = dev_upload(ix->allocs, ix->bytes, L.w_u8.data(), L.w_u8.size(), &p, s, kPostSlack))) return done(rc);
        d.post_w = p;
    }
    float* blk_max = nullptr;
    int32_t* blk_first = nullptr;
    if ((rc = dev_upload(ix->allocs, ix->bytes, L.blk_max.data(), L.blk_max.size(), &blk_max, s))) return done(rc);
    if ((rc = dev_upload(ix->allocs, ix->bytes, L.blk_first.data(), L.blk_first.size(), &blk_first, s)))
        return done(rc);
    d.blk_first = blk_first;
    d.blk_max = blk_max;
    {
        // Byte form of the doc ids: a term whose every 64-posting block spans at most 256 docs
        // stores each id as its distance to the block's first doc.
        std::vector<uint8_t> dense, b8;
        try {
            byte_form(L, dense, b8);
        } catch (const std::bad_alloc&) {
            return done(set_error(GS_ENOMEM, "host memory for the byte doc offsets"));
        }
        uint8_t *pd = nullptr, *pb = nullptr;
        if ((rc = dev_upload(ix->allocs, ix->bytes, dense.data(), dense.size(), &pd, s))) return done(rc);
        // only the fp32 and bf16 kernels read the byte form; a uint8 index keeps a placeholder
        const bool keep_b8 = precision != kU8;
        if ((rc = dev_upload(ix->allocs, ix->bytes, keep_b8 ? b8.data() : nullptr, keep_b8 ? b8.size() : 0, &pb, s,
                             keep_b8 ? kPostSlack : 0)))
            return done(rc);
        d.term_dense = pd;
        d.post_b8 = pb;
        ix->n_dense = 0;
        for (int32_t v = 0; v < vocab_size; v++) ix->n_dense += dense[(size_t)v];
        ix->term_dense = dense;
        // the uploads above are asynchronous: keep the host buffers until the stream is done
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return done(fail(GS_EHIP, std::string("upload: ") + hipGetErrorString(e)));
    }
    if (flags & GS_KEEP_FORWARD) {
        int64_t* frp = nullptr;
        int32_t* ft = nullptr;
        float* fw = nullptr;
        if ((rc = dev_upload(ix->allocs, ix->bytes, r.row_ptr, (size_t)n_docs + 1, &frp, s))) return done(rc);
        if ((rc = dev_upload(ix->allocs, ix->bytes, r.term, (size_t)nnz, &ft, s))) return done(rc);
        if ((rc = dev_upload(ix->allocs, ix->bytes, r.w, (size_t)nnz, &fw, s))) return done(rc);
        d.fwd_row_ptr = frp;
        d.fwd_term = ft;
        d.fwd_w = fw;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(fail(GS_EHIP, std::string("upload: ") + hipGetErrorString(e)));
    *out = ix;
    return GS_OK;
}

int32_t gs_index_info(gs_index ix, gs_index_info_t* out) {
    g_err.clear();
    if (!ix || !out) return fail(GS_EINVAL, "null argument");
    out->n_docs = ix->n_docs;
    out->nnz = ix->nnz;
    out->padded_nnz = ix->padded;
    out->device_bytes = (int64_t)ix->bytes;
    out->vocab_size = ix->vocab;
    out->precision = ix->precision;
    out->flags = ix->flags;
    out->tile_grain = 1 << kGrainShift;
    out->n_tiles = ix->n_grains;
    out->n_dense_terms = ix->n_dense;
    return GS_OK;
}

int32_t gs_index_dense_terms(gs_index ix, uint8_t* out, int32_t vocab_size) {
    g_err.clear();
    if (!ix || !out) return fail(GS_EINVAL, "null argument");
    if (vocab_size != ix->vocab) return fail(GS_EINVAL, "vocab_size differs from the index's");
    std::memcpy(out, ix->term_dense.data(), (size_t)ix->vocab);
    return GS_OK;
}

void gs_free_index(gs_index ix) {
    if (!ix) return;
    DeviceGuard g(ix->device);
    delete ix;
}

int32_t gs_batch_reserve(gs_index ix, int32_t max_queries, int64_t max_nnz, int32_t k_max, gs_batch* out) {
    g_err.clear();
    if (!out) return fail(GS_EINVAL, "out is null");
    *out = nullptr;
    if (!ix) return fail(GS_EINVAL, "index is null");
    if (max_queries < 0 || max_nnz < 0) return fail(GS_EINVAL, "negative capacity");
    if (k_max < 0 || k_max > GS_MAX_K) return fail(GS_EINVAL, "k_max must be in [0, GS_MAX_K]");
    DeviceGuard g(ix->device);
    gs_batch b = new (std::nothrow) gs_batch_s();
    if (!b) return fail(GS_ENOMEM, "host allocation failed");
    b->index = ix;
    b->device = ix->device;
    b->n_queries = max_queries;
    b->k_max = k_max;
    b->q_nnz = max_nnz;
    auto done = [&](int32_t code) {
        if (code != GS_OK) delete b;
        return code;
    };
    const size_t nq = (size_t)max_queries, nz = (size_t)max_nnz;
    b->lay = BatchLayout(nq, nz);
    const BatchLayout& L = b->lay;
    {
        hipError_t e = dev_malloc((void**)&b->dmem, L.total);
        if (e == hipSuccess) e = pinned_malloc((void**)&b->stage, L.total);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
        if (e != hipSuccess)
            return done(fail(e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EHIP,
                             std::string("batch allocation: ") + hipGetErrorString(e)));
    }
    uint8_t* m = b->dmem;
    DevBatch& d = b->dev;
    d.n_queries = max_queries;
    d.k_max = k_max;
    d.q_row_ptr = (const int64_t*)(m + L.rp);
    d.q_term = (const int32_t*)(m + L.term);
    d.q_w = (const float*)(m + L.w);
    d.q_w8 = (const int32_t*)(m + L.w8);
    d.q_fx = (const double*)(m + L.fx);
    d.q_ub_cum = (const unsigned long long*)(m + L.ubcum);
    d.k = (const int32_t*)(m + L.k);
    d.first_shift = (const int32_t*)(m + L.fs);
    d.delta = (const float*)(m + L.delta);
    d.q_scale = (const double*)(m + L.scale);
    d.q_abs_err = (const double*)(m + L.err);
    d.q_wide_lim = (const double*)(m + L.wide);
    d.g_count = (const int32_t*)(m + L.gcount);
    d.g_member = (const int32_t*)(m + L.gmember);
    d.g_row = (const int32_t*)(m + L.grow);
    d.g_term = (const int32_t*)(m + L.gterm);
    d.g_wq = (const float*)(m + L.gwfx);
    d.g_w8 = (const int32_t*)(m + L.gw8);
    d.q_work = (const int64_t*)(m + L.work);
    b->diag = (int32_t*)(m + L.diag);
    // an empty batch until the first update: every slot is a query with no terms and k = 0
    std::vector<int64_t> zero_rp(nq + 1, 0);
    int32_t rc2 = gs_batch_update(b, zero_rp.data(), 0, nullptr, nullptr, 0, nullptr, nullptr);
    if (rc2 != GS_OK) return done(rc2);
    *out = b;
    return GS_OK;
}

}  // extern "C"

namespace gs {

int32_t batch_update(gs_batch b, const int64_t* q_row_ptr, int32_t n_queries, const int32_t* q_term_ids,
                     const float* q_weights, int64_t q_nnz, const int32_t* k, void* hip_stream, bool wait) {
    g_err.clear();
    if (!b) return fail(GS_EINVAL, "batch is null");
    gs_index ix = b->index;
    if (n_queries < 0 || n_queries > b->n_queries)
        return fail(GS_EINVAL, "n_queries outside [0, batch capacity]");
    if (q_nnz < 0 || q_nnz > b->q_nnz) return fail(GS_EINVAL, "q_nnz exceeds the batch capacity");
    if (n_queries > 0 && !k) return fail(GS_EINVAL, "k is null");
    for (int32_t q = 0; q < n_queries; q++)
        if (k[q] < 0 || k[q] > b->k_max) return fail(GS_EINVAL, "k[" + std::to_string(q) + "] outside [0, k_max]");
    Rows r{q_row_ptr, q_term_ids, q_weights, n_queries, {}, {}};
    int32_t rc = check_rows(r, q_nnz, ix->vocab, kMaxQueryNnz, "queries");
    if (rc != GS_OK) return rc;
    const int32_t cap = b->n_queries;
    DeviceGuard g(ix->device);
    // the stage may still be read by the previous update's copies
    if (b->copy_pending) {
        GS_HIP(hipEventSynchronize(b->copied));
        b->copy_pending = false;
    }
    const BatchLayout& L = b->lay;
    uint8_t* h = b->stage;
    int64_t* rp = (int64_t*)(h + L.rp);
    int32_t* kk = (int32_t*)(h + L.k);
    int32_t* fshift = (int32_t*)(h + L.fs);
    float* delta = (float*)(h + L.delta);
    double* qscale = (double*)(h + L.scale);
    double* qerr = (double*)(h + L.err);
    double* qwide = (double*)(h + L.wide);
    int64_t* qwork = (int64_t*)(h + L.work);
    int32_t* w8 = (int32_t*)(h + L.w8);
    double* qfx = (double*)(h + L.fx);
    unsigned long long* qub = (unsigned long long*)(h + L.ubcum);
    // slots past n_queries become empty queries with k = 0 (no work, padding-only rows)
    for (int32_t q = 0; q <= cap; q++) rp[q] = q <= n_queries ? (q_row_ptr ? q_row_ptr[q] : 0) : q_nnz;
    for (int32_t q = 0; q < cap; q++) kk[q] = q < n_queries ? k[q] : 0;
    std::memset(h + L.diag, 0, (size_t)cap * kDiagWords * 4);
    if (q_nnz > 0) {
        std::memcpy(h + L.term, r.term, (size_t)q_nnz * 4);
        std::memcpy(h + L.w, r.w, (size_t)q_nnz * 4);
    }
    std::vector<float> tmax, tmin;
    for (int32_t q = 0; q < cap; q++) {
        uint64_t maxs = 0;
        const int64_t m = rp[q + 1] - rp[q];
        qwork[q] = 0;
        tmax.resize((size_t)m);
        tmin.resize((size_t)m);
        for (int64_t j = rp[q]; j < rp[q + 1]; j++) {
            qwork[q] += ix->term_len[(size_t)r.term[j]];
            w8[j] = q8(r.w[j]);
            maxs += (uint64_t)w8[j] * 255u;
            tmax[(size_t)(j - rp[q])] = ix->term_max[(size_t)r.term[j]];
            tmin[(size_t)(j - rp[q])] = ix->term_min[(size_t)r.term[j]];
        }
        if (ix->precision == kU8) {
            int hb = 0;
            while (hb < 64 && (maxs >> hb) != 0) hb++;
            fshift[q] = 32 + std::max(hb, kHistBits) - kHistBits;
        } else {
            fshift[q] = kFirstShiftFloat;
        }
        const FixedPlan fp = fixed_point_plan(ix->precision, m, r.w + rp[q], tmax.data(), tmin.data());
        qscale[q] = fp.scale;
        qerr[q] = fp.abs_err;
        qwide[q] = fp.wide_lim;
        for (int64_t j = rp[q]; j < rp[q + 1]; j++) qfx[j] = std::ldexp((double)r.w[j], fp.F);
        // Block-max pruning: each term's upper bound on its product with any doc (fixed-point
        // units: the largest stored weight times w_q 2^F, rounded up, plus one for the product's
        // rounding; uint8: the exact integer product), then per term the sum of the bounds of
        // the terms up to it in ascending order of bound (ties by position).
        {
            std::vector<std::pair<unsigned long long, int64_t>> ub;
            ub.reserve((size_t)m);
            for (int64_t j = rp[q]; j < rp[q + 1]; j++) {
                const double tm = (double)ix->term_max[(size_t)r.term[j]];
                const unsigned long long u = ix->precision == kU8
                                                 ? (unsigned long long)w8[j] * (unsigned long long)tm
                                                 : (unsigned long long)std::ceil(qfx[j] * tm) + 1ull;
                ub.emplace_back(u, j);
            }
            std::sort(ub.begin(), ub.end());
            unsigned long long run = 0;
            for (const auto& e : ub) {
                run += e.first;
                qub[e.second] = run;
            }
        }
        // bf16 form: relative error of a stored weight (2^-8) and of the fp32 score (2^-24, with margin)
        delta[q] = (float)(((1.0 + std::ldexp(1.0, -8)) * (1.0 + std::ldexp(1.0, -23)) - 1.0) * (1.0 + 1e-6));
    }
    // Groups of the group kernel: the queries with k > 0 by descending work (ties by index),
    // G consecutive ones per group, and per group the ascending union of the members' terms
    // with each member's weight w_q (0 where it lacks the term; the kernel scales it by 2^F of
    // the member). Terms are ascending per query.
    const int G = 2;  // the group kernel's group size, every precision
    int32_t* gcnt = (int32_t*)(h + L.gcount);
    int32_t* gmem = (int32_t*)(h + L.gmember);
    int32_t* grow = (int32_t*)(h + L.grow);
    int32_t* gterm = (int32_t*)(h + L.gterm);
    float* gwq = (float*)(h + L.gwfx);
    int32_t* gw8 = (int32_t*)(h + L.gw8);
    int64_t n_union = 0;
    {
        std::vector<int32_t> ord;
        for (int32_t q = 0; q < n_queries; q++)
            if (kk[q] > 0) ord.push_back(q);
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return qwork[a] > qwork[b]; });
        const int32_t ng = (int32_t)((ord.size() + G - 1) / G);
        *gcnt = ng;
        grow[0] = 0;
        for (int32_t g = 0; g < ng; g++) {
            int64_t at[kGroupMax], end[kGroupMax];
            for (int m = 0; m < G; m++) {
                const size_t i = (size_t)g * G + m;
                const int32_t q = i < ord.size() ? ord[i] : -1;
                gmem[g * G + m] = q;
                at[m] = q >= 0 ? rp[q] : 0;
                end[m] = q >= 0 ? rp[q + 1] : 0;
            }
            for (;;) {  // merge of the members' ascending term lists
                int32_t t = INT32_MAX;
                for (int m = 0; m < G; m++)
                    if (at[m] < end[m]) t = std::min(t, r.term[at[m]]);
                if (t == INT32_MAX) break;
                gterm[n_union] = t;
                for (int m = 0; m < G; m++) {
                    const bool has = at[m] < end[m] && r.term[at[m]] == t;
                    gwq[n_union * G + m] = has ? r.w[at[m]] : 0.0f;
                    gw8[n_union * G + m] = has ? w8[at[m]] : 0;
                    if (has) at[m]++;
                }
                n_union++;
            }
            grow[g + 1] = (int32_t)n_union;
        }
    }
    // copies on the caller's stream, ordered after the searches already enqueued on it
    hipStream_t s = (hipStream_t)hip_stream;
    auto up = [&](size_t off, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(b->dmem + off, h + off, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    hipError_t e = up(0, L.head);
    if (e == hipSuccess) e = up(L.term, (size_t)q_nnz * 4);
    if (e == hipSuccess) e = up(L.w, (size_t)q_nnz * 4);
    if (e == hipSuccess) e = up(L.w8, (size_t)q_nnz * 4);
    if (e == hipSuccess) e = up(L.fx, (size_t)q_nnz * 8);
    if (e == hipSuccess) e = up(L.ubcum, (size_t)q_nnz * 8);
    if (e == hipSuccess) e = up(L.gterm, (size_t)n_union * 4);
    if (e == hipSuccess) e = up(L.gwfx, (size_t)n_union * G * 4);
    if (e == hipSuccess) e = up(L.gw8, (size_t)n_union * G * 4);
    if (e == hipSuccess) e = hipEventRecord(b->copied, s);
    if (e == hipSuccess) {
        b->copy_pending = true;
        if (wait) {
            e = hipEventSynchronize(b->copied);
            if (e == hipSuccess) b->copy_pending = false;
        }
    }
    if (e != hipSuccess) return fail(GS_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
    b->n_active = n_queries;
    return GS_OK;
}

}  // namespace gs

extern "C" {

int32_t gs_batch_update(gs_batch b, const int64_t* q_row_ptr, int32_t n_queries, const int32_t* q_term_ids,
                        const float* q_weights, int64_t q_nnz, const int32_t* k, void* hip_stream) {
    return gs::batch_update(b, q_row_ptr, n_queries, q_term_ids, q_weights, q_nnz, k, hip_stream, true);
}

int32_t gs_batch_create(gs_index ix, const int64_t* q_row_ptr, int32_t n_queries, const int32_t* q_term_ids,
                        const float* q_weights, int64_t q_nnz, const int32_t* k, int32_t k_max, void* hip_stream,
                        gs_batch* out) {
    g_err.clear();
    if (!out) return fail(GS_EINVAL, "out is null");
    *out = nullptr;
    if (n_queries < 0 || q_nnz < 0) return fail(GS_EINVAL, "negative size");
    gs_batch b = nullptr;
    int32_t rc = gs_batch_reserve(ix, n_queries, q_nnz, k_max, &b);
    if (rc != GS_OK) return rc;
    rc = gs_batch_update(b, q_row_ptr, n_queries, q_term_ids, q_weights, q_nnz, k, hip_stream);
    if (rc != GS_OK) {
        gs_batch_free(b);
        return rc;
    }
    *out = b;
    return GS_OK;
}

void gs_batch_free(gs_batch b) {
    if (!b) return;
    DeviceGuard g(b->device);
    delete b;
}

static int32_t resolve_opts(gs_index ix, const gs_search_opts* o, ScoreOpts* so) {
    so->kernel = GS_KERNEL_TILED;
    // 64 KiB of LDS accumulators: 8192 fixed-point (fp32, bf16) or 16384 int32 (uint8) documents
    so->tile_shift = ix->precision == kFP32 ? 13 : 14;
    so->chunk = 1024;  // measured fastest for both doc-tiled forms at every tile size
    so->seed_stride = 1;  // fused filtering wanted (the stride itself is chosen per search)
    if (!o) return GS_OK;
    for (int i = 0; i < 2; i++)
        if (o->reserved[i] != 0) return fail(GS_EINVAL, "reserved option fields must be 0");
    if (o->prune != 0 && o->prune != 1) return fail(GS_EINVAL, "prune must be 0 or 1");
    if (o->no_fused_filter != 0 && o->no_fused_filter != 1) return fail(GS_EINVAL, "no_fused_filter must be 0 or 1");
    if (o->no_fused_filter) so->seed_stride = 0;
    if (o->kernel < GS_KERNEL_AUTO || o->kernel > GS_KERNEL_GROUP) return fail(GS_EINVAL, "unknown kernel");
    if (o->kernel != GS_KERNEL_AUTO) so->kernel = o->kernel;
    if (so->kernel == GS_KERNEL_DOCPAR && !(ix->flags & GS_KEEP_FORWARD))
        return fail(GS_EUNSUPPORTED, "document-parallel kernel needs an index built with GS_KEEP_FORWARD");
    if (so->kernel == GS_KERNEL_ATOMIC && !(ix->flags & GS_KEEP_DOC_IDS))
        return fail(GS_EUNSUPPORTED, "global-atomic kernel needs an index built with GS_KEEP_DOC_IDS");
    if (o->query_tile < 0) return fail(GS_EINVAL, "query_tile < 0");
    switch (o->tile_docs) {
        case 0: break;
        case 8192: so->tile_shift = 13; break;
        case 16384: so->tile_shift = 14; break;
        case 32768: so->tile_shift = 15; break;
        default: return fail(GS_EINVAL, "tile_docs must be 0, 8192, 16384 or 32768");
    }
    if (so->tile_shift == 15 && ix->precision == kFP32)
        return fail(GS_EUNSUPPORTED, "tile_docs 32768 is not available for GS_FP32 (LDS capacity)");
    switch (o->chunk) {
        case 0: break;
        case 64: case 128: case 256: case 512: case 1024: so->chunk = o->chunk; break;
        default: return fail(GS_EINVAL, "chunk must be 0, 64, 128, 256, 512 or 1024");
    }
    if (o->prune) {
        const int def_shift = ix->precision == kFP32 ? 13 : 14;
        if (so->kernel != GS_KERNEL_TILED || ix->precision == kBF16 || so->tile_shift != def_shift ||
            so->chunk != 1024)
            return fail(GS_EUNSUPPORTED,
                        "pruning needs GS_KERNEL_TILED, fp32 or uint8 weights, the default tile and chunk 1024");
        so->prune = 1;
    }
    if (so->kernel == GS_KERNEL_GROUP) {
        if (o->tile_docs != 0 && o->tile_docs != (1 << kGroupTileShift))
            return fail(GS_EUNSUPPORTED, "the group kernel works on 8192-doc tiles");
        // measured: chunks of 1024 for uint8; the fixed-point forms spill registers at 1024
        if (o->chunk == 0) so->chunk = ix->precision == kU8 ? 1024 : 512;
        if (so->chunk < 256) return fail(GS_EUNSUPPORTED, "the group kernel takes chunks of 256, 512 or 1024");
        so->tile_shift = kGroupTileShift;
    }
    return GS_OK;
}

int32_t gs_search_workspace_size(gs_index ix, int32_t n_queries, int64_t q_nnz, int32_t k_max,
                                 const gs_search_opts* opts, size_t* bytes) {
    g_err.clear();
    if (!ix || !bytes) return fail(GS_EINVAL, "null argument");
    if (n_queries < 0 || q_nnz < 0 || q_nnz > (int64_t)n_queries * kMaxQueryNnz)
        return fail(GS_EINVAL, "n_queries < 0, or q_nnz outside [0, n_queries * GS_MAX_QUERY_NNZ]");
    if (k_max < 0 || k_max > GS_MAX_K) return fail(GS_EINVAL, "k_max outside [0, GS_MAX_K]");
    ScoreOpts so;
    int32_t rc = resolve_opts(ix, opts, &so);
    if (rc != GS_OK) return rc;
    int32_t live = std::max(n_queries, 1);
    if (opts && opts->query_tile > 0) live = std::min(live, opts->query_tile);
    *bytes = workspace_bytes(ix->n_docs, live, ix->precision);
    return GS_OK;
}

int32_t gs_workspace_size(gs_index ix, int32_t query_tile, const gs_search_opts* opts, size_t* bytes) {
    g_err.clear();
    if (!ix || !bytes) return fail(GS_EINVAL, "null argument");
    if (query_tile < 1) return fail(GS_EINVAL, "query_tile < 1");
    ScoreOpts so;
    int32_t rc = resolve_opts(ix, opts, &so);
    if (rc != GS_OK) return rc;
    *bytes = workspace_bytes(ix->n_docs, query_tile, ix->precision);
    return GS_OK;
}

}  // extern "C"

namespace {

// Validate a search request and pick the query-tile size the workspace allows.
int32_t plan_search(gs_index ix, gs_batch b, size_t workspace_bytes_, const gs_search_opts* opts, ScoreOpts* so,
                    int32_t* qt) {
    if (!ix || !b) return fail(GS_EINVAL, "null index or batch");
    if (b->index != ix) return fail(GS_EINVAL, "batch was created for another index");
    int32_t rc = resolve_opts(ix, opts, so);
    if (rc != GS_OK) return rc;
    if ((!opts || opts->kernel == GS_KERNEL_AUTO) && b->n_active >= 32) so->kernel = GS_KERNEL_SHARED;
    if (workspace_bytes(ix->n_docs, 1, ix->precision) > workspace_bytes_)
        return fail(GS_ECAPACITY, "workspace smaller than gs_workspace_size(index, 1)");
    const int32_t nq = std::max(b->n_queries, 1);
    int32_t lo = 1, hi = nq;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes(ix->n_docs, mid, ix->precision) <= workspace_bytes_) lo = mid; else hi = mid - 1;
    }
    *qt = lo;
    if (opts && opts->query_tile > 0) *qt = std::min(*qt, opts->query_tile);
    return GS_OK;
}

// Enqueue the whole search on stream s (no host synchronisation; capturable).
// Queries [0, nq) are searched; output rows [nq, capacity) are written as padding
// (id -1, score 0). A direct search passes the queries of the last update, a
// graph the whole capacity (it is replayed after updates of any size).
int32_t enqueue_search(gs_index ix, gs_batch b, int32_t nq, const Workspace& ws, int32_t qt, const ScoreOpts& so_in,
                       int32_t* out_ids, void* out_scores, hipStream_t s, bool timing) {
    ScoreOpts so = so_in;
    // Fused candidate filtering (doc-tiled kernels): every stride-th tile seeds a lower bound
    // of the k-th composite; the other tiles append their candidates while they are scored.
    // The seed tiles should hold several times k documents: stride 8 up to k = 1024, 4 up to
    // 2048, else off; it needs at least two seed tiles. It adds five launches to a search,
    // which a few queries' row scans do not repay: searches of fewer than 32 queries scan.
    // the group kernel's groups span the whole batch: with query tiles it gives way to the
    // shared-traversal kernel
    if (so.kernel == GS_KERNEL_GROUP && qt < nq) so.kernel = GS_KERNEL_SHARED;
    {
        const bool tiled = so.kernel == GS_KERNEL_TILED || so.kernel == GS_KERNEL_SHARED || so.kernel == GS_KERNEL_GROUP;
        const int64_t n_tiles = (ix->n_docs + (1ll << so.tile_shift) - 1) >> so.tile_shift;
        int stride = b->k_max <= 1024 ? 8 : (b->k_max <= 2048 ? 4 : 0);
        if (!tiled || so.seed_stride == 0 || n_tiles < 2 * (int64_t)stride || nq < 32) stride = 0;
        so.seed_stride = stride;
    }
    (void)hipGetLastError();  // launches below report their own status; drop any earlier, unrelated one
    g_failed_launch = "";
    for (int32_t q0 = 0; q0 < nq; q0 += qt) {
        const int32_t n = std::min(qt, nq - q0);
        hipError_t e = launch_clear(ws, n, s);
        if (e == hipSuccess && ix->n_docs > 0) {
            const bool group = so.kernel == GS_KERNEL_GROUP;
            if (so.seed_stride == 0 || so.kernel == GS_KERNEL_ATOMIC || so.kernel == GS_KERNEL_DOCPAR) {
                SpanRecorder rec(timing ? 0 : -1, s);
                if (so.kernel == GS_KERNEL_ATOMIC) e = launch_score_atomic(ix->dev, b->dev, q0, n, so, ws, s);
                else if (so.kernel == GS_KERNEL_DOCPAR) e = launch_score_docpar(ix->dev, b->dev, q0, n, so, ws, s);
                else if (group) e = launch_score_group(ix->dev, b->dev, so, ws, s, 0);
                else e = launch_score_tiled(ix->dev, b->dev, q0, n, so, ws, s);
                rec.end(s);
            } else {
                // fused filtering: seed tiles, their bound (selection work), then the other tiles
                {
                    SpanRecorder rec(timing ? 0 : -1, s, false);
                    e = group ? launch_score_group(ix->dev, b->dev, so, ws, s, 1)
                              : launch_score_tiled(ix->dev, b->dev, q0, n, so, ws, s, 1);
                    rec.end(s);
                }
                if (e == hipSuccess) {
                    SpanRecorder rec(timing ? 1 : -1, s, false);
                    e = launch_seed_bound(ix->dev, b->dev, q0, n, ws, s, so.tile_shift, so.seed_stride);
                    rec.end(s);
                }
                if (e == hipSuccess) {
                    SpanRecorder rec(timing ? 0 : -1, s);
                    e = group ? launch_score_group(ix->dev, b->dev, so, ws, s, 2)
                              : launch_score_tiled(ix->dev, b->dev, q0, n, so, ws, s, 2);
                    rec.end(s);
                }
            }
        }
        if (e == hipSuccess) {
            SpanRecorder rec(timing ? 1 : -1, s);
            // Between the two first-digit selection passes: the rows of the listed queries.
            // Fused queries that fell back get their non-seed tiles scored (phase 3);
            // fixed-point queries found wide range get every tile scored in fp64 (phase 4).
            const bool doc_tiled =
                so.kernel == GS_KERNEL_TILED || so.kernel == GS_KERNEL_SHARED || so.kernel == GS_KERNEL_GROUP;
            const bool fixed = doc_tiled && ix->precision != kU8;
            const bool phase3 = so.seed_stride > 0;
            const int acc = ix->precision == kU8 ? kAccInteger : (doc_tiled ? kAccFixed : kAccFloat);
            e = launch_select(ix->dev, b->dev, q0, n, ws, out_ids, out_scores, b->diag, s, acc, so.tile_shift,
                              so.seed_stride, phase3 ? &so : nullptr, fixed);
            rec.end(s);
        }
        if (e != hipSuccess)
            return fail(GS_EHIP, std::string("launch of ") + g_failed_launch + ": " + hipGetErrorString(e));
    }
    if (nq < b->n_queries) {
        const int64_t rows = (int64_t)(b->n_queries - nq) * b->k_max;
        const int64_t words = ix->precision == kBF16 ? 2 : 1;
        hipError_t e = launch_fill(out_ids + (int64_t)nq * b->k_max, rows, 0xFFFFFFFFu, s);
        if (e == hipSuccess)
            e = launch_fill((uint32_t*)out_scores + (int64_t)nq * b->k_max * words, rows * words, 0u, s);
        if (e != hipSuccess)
            return fail(GS_EHIP, std::string("launch of ") + g_failed_launch + ": " + hipGetErrorString(e));
    }
    return GS_OK;
}

}  // namespace

namespace gs {

int32_t search_rows(gs_index ix, gs_batch b, void* arena, int64_t rows, int64_t r0, uint32_t* counters,
                    const gs_search_opts* opts, int32_t* out_ids, void* out_scores, hipStream_t s) {
    if (!ix || !b || !arena || !counters) return fail(GS_EINVAL, "null argument");
    if (b->index != ix) return fail(GS_EINVAL, "batch was created for another index");
    const int32_t n = b->n_active;
    if (r0 < 0 || r0 + n > rows) return fail(GS_EINVAL, "rows outside the arena");
    ScoreOpts so;
    int32_t rc = resolve_opts(ix, opts, &so);
    if (rc != GS_OK) return rc;
    if ((!opts || opts->kernel == GS_KERNEL_AUTO) && n >= 32) so.kernel = GS_KERNEL_SHARED;
    if (b->n_queries == 0 || b->k_max == 0 || n == 0) return GS_OK;
    DeviceGuard g(ix->device);
    Workspace ws;
    carve_rows(arena, ix->n_docs, rows, ix->precision, r0, &ws);
    ws.counters = counters;
    return enqueue_search(ix, b, n, ws, n, so, out_ids, out_scores, s, false);
}

const int32_t* batch_diag(const gs_batch_s* b) { return b->diag; }

}  // namespace gs

namespace {

// After a synchronised search: GS_ECAPACITY when the rescored band of some query did not
// fit its buffer (bf16; that row holds padding), else GS_OK.
int32_t check_overflow(gs_batch b) {
    if (b->n_active == 0) return GS_OK;
    std::vector<int32_t> d((size_t)b->n_active * kDiagWords);
    const hipError_t e = hipMemcpy(d.data(), b->diag, d.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(GS_EHIP, std::string("diagnostics: ") + hipGetErrorString(e));
    for (int32_t q = 0; q < b->n_active; q++)
        if (d[(size_t)q * kDiagWords + 3])
            return fail(GS_ECAPACITY, "query " + std::to_string(q) + ": more than " + std::to_string(kCandCap) +
                                          " documents inside the bf16 error band of its k-th score");
    return GS_OK;
}

}  // namespace

struct gs_graph_s {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~gs_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" {

int32_t gs_search_batch(gs_index ix, gs_batch b, void* workspace, size_t workspace_bytes_, int32_t* out_ids,
                        void* out_scores, const gs_search_opts* opts, void* hip_stream) {
    g_err.clear();
    ScoreOpts so;
    int32_t qt = 1;
    int32_t rc = plan_search(ix, b, workspace_bytes_, opts, &so, &qt);
    if (rc != GS_OK) return rc;
    if (b->n_queries == 0 || b->k_max == 0) return GS_OK;
    if (!out_ids || !out_scores) return fail(GS_EINVAL, "null output");
    if (!workspace) return fail(GS_EINVAL, "null workspace");
    DeviceGuard g(ix->device);
    Workspace ws;
    carve_workspace(workspace, ix->n_docs, qt, ix->precision, &ws);
    return enqueue_search(ix, b, b->n_active, ws, qt, so, out_ids, out_scores, (hipStream_t)hip_stream, true);
}

int32_t gs_search_batch_noalloc(gs_index ix, gs_batch b, int32_t* out_ids, void* out_scores,
                                const gs_search_opts* opts, void* hip_stream) {
    g_err.clear();
    if (!ix || !b) return fail(GS_EINVAL, "null index or batch");
    const size_t one = workspace_bytes(ix->n_docs, 1, ix->precision);
    if (one > kScratchBytes)
        return fail(GS_ECAPACITY, "a one-query workspace of this index (" + std::to_string(one) +
                                      " bytes) exceeds the fixed scratch array (" + std::to_string(kScratchBytes) +
                                      " bytes)");
    DeviceGuard g(ix->device);
    void* scratch = nullptr;
    const hipError_t e = scratch_address(ix->device, &scratch);
    if (e != hipSuccess) return fail(GS_EHIP, std::string("scratch array address: ") + hipGetErrorString(e));
    ScoreOpts so;
    int32_t qt = 1;
    int32_t rc = plan_search(ix, b, kScratchBytes, opts, &so, &qt);
    if (rc != GS_OK) return rc;
    if (b->n_queries == 0 || b->k_max == 0) return GS_OK;
    if (!out_ids || !out_scores) return fail(GS_EINVAL, "null output");
    // no timing events: nothing is created or allocated on this path
    Workspace ws;
    carve_workspace(scratch, ix->n_docs, qt, ix->precision, &ws);
    return enqueue_search(ix, b, b->n_active, ws, qt, so, out_ids, out_scores, (hipStream_t)hip_stream, false);
}

int32_t gs_graph_create(gs_index ix, gs_batch b, void* workspace, size_t workspace_bytes_, int32_t* out_ids,
                        void* out_scores, const gs_search_opts* opts, void* hip_stream, gs_graph* out) {
    g_err.clear();
    if (!out) return fail(GS_EINVAL, "out is null");
    *out = nullptr;
    ScoreOpts so;
    int32_t qt = 1;
    int32_t rc = plan_search(ix, b, workspace_bytes_, opts, &so, &qt);
    if (rc != GS_OK) return rc;
    if (b->n_queries == 0 || b->k_max == 0) return fail(GS_EINVAL, "empty batch");
    if (!out_ids || !out_scores || !workspace) return fail(GS_EINVAL, "null workspace or output");
    DeviceGuard g(ix->device);
    hipStream_t s = (hipStream_t)hip_stream;
    Workspace ws;
    carve_workspace(workspace, ix->n_docs, qt, ix->precision, &ws);
    // one eager run first: one-time kernel attributes and occupancy queries happen outside the capture
    rc = enqueue_search(ix, b, b->n_queries, ws, qt, so, out_ids, out_scores, s, false);
    if (rc != GS_OK) return rc;
    GS_HIP(hipStreamSynchronize(s));
    gs_graph gr = new (std::nothrow) gs_graph_s();
    if (!gr) return fail(GS_ENOMEM, "host allocation failed");
    gr->device = ix->device;
    // capture on a private stream (the legacy default stream cannot be captured)
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        if (cs) (void)hipStreamDestroy(cs);
        delete gr;
        return fail(GS_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    rc = enqueue_search(ix, b, b->n_queries, ws, qt, so, out_ids, out_scores, cs, false);
    e = hipStreamEndCapture(cs, &gr->graph);
    (void)hipStreamDestroy(cs);
    if (rc != GS_OK) {
        delete gr;
        return rc;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        delete gr;
        return fail(GS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = gr;
    return GS_OK;
}

int32_t gs_autotune(gs_index ix, gs_batch b, void* workspace, size_t workspace_bytes_, int32_t* out_ids,
                    void* out_scores, int32_t reps, void* hip_stream, gs_search_opts* best, gs_search_opts* cands,
                    float* times_ms, int32_t max_candidates, int32_t* n_candidates) {
    g_err.clear();
    if (!ix || !b || !best) return fail(GS_EINVAL, "null argument");
    if (reps < 1) return fail(GS_EINVAL, "reps < 1");
    std::vector<gs_search_opts> cand;
    const int kernels[2] = {GS_KERNEL_TILED, GS_KERNEL_SHARED};
    std::vector<int> tiles = {8192, 16384};
    if (ix->precision != kFP32) tiles.push_back(32768);
    for (int k : kernels)
        for (int t : tiles)
            for (int c : {128, 256, 512, 1024}) {
                gs_search_opts o{};
                o.kernel = k;
                o.tile_docs = t;
                o.chunk = c;
                cand.push_back(o);
            }
    for (int c : {256, 512, 1024}) {  // the group kernel: 8192-doc tiles
        gs_search_opts o{};
        o.kernel = GS_KERNEL_GROUP;
        o.tile_docs = 1 << kGroupTileShift;
        o.chunk = c;
        cand.push_back(o);
    }
    DeviceGuard g(ix->device);
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GS_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GS_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
    }
    float best_ms = 0.0f;
    int best_i = -1;
    int32_t rc = GS_OK;
    for (size_t i = 0; i < cand.size() && rc == GS_OK; i++) {
        ScoreOpts so;
        int32_t qt = 1;
        rc = plan_search(ix, b, workspace_bytes_, &cand[i], &so, &qt);
        if (rc != GS_OK) break;
        Workspace ws;
        carve_workspace(workspace, ix->n_docs, qt, ix->precision, &ws);
        rc = enqueue_search(ix, b, b->n_active, ws, qt, so, out_ids, out_scores, s, false);  // untimed
        if (rc != GS_OK) break;
        he = hipEventRecord(e0, s);
        for (int r = 0; r < reps && rc == GS_OK && he == hipSuccess; r++)
            rc = enqueue_search(ix, b, b->n_active, ws, qt, so, out_ids, out_scores, s, false);
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) rc = fail(GS_EHIP, std::string("autotune timing: ") + hipGetErrorString(he));
        if (rc != GS_OK) break;
        ms /= (float)reps;
        if ((int32_t)i < max_candidates) {
            if (cands) cands[i] = cand[i];
            if (times_ms) times_ms[i] = ms;
        }
        if (best_i < 0 || ms < best_ms) {
            best_ms = ms;
            best_i = (int)i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GS_OK) return rc;
    // the outputs are the best option set's result: run it once more, last
    {
        ScoreOpts so;
        int32_t qt = 1;
        rc = plan_search(ix, b, workspace_bytes_, &cand[(size_t)best_i], &so, &qt);
        if (rc != GS_OK) return rc;
        Workspace ws;
        carve_workspace(workspace, ix->n_docs, qt, ix->precision, &ws);
        rc = enqueue_search(ix, b, b->n_active, ws, qt, so, out_ids, out_scores, s, false);
        if (rc != GS_OK) return rc;
        GS_HIP(hipStreamSynchronize(s));
    }
    if (n_candidates) *n_candidates = (int32_t)cand.size();
    *best = cand[(size_t)best_i];
    return GS_OK;
}

int32_t gs_graph_launch(gs_graph gr, void* hip_stream) {
    g_err.clear();
    if (!gr) return fail(GS_EINVAL, "graph is null");
    DeviceGuard g(gr->device);
    GS_HIP(hipGraphLaunch(gr->exec, (hipStream_t)hip_stream));
    return GS_OK;
}

void gs_graph_free(gs_graph gr) {
    if (!gr) return;
    DeviceGuard g(gr->device);
    delete gr;
}

int32_t gs_search(gs_index ix, const int64_t* q_row_ptr, int32_t n_queries, const int32_t* q_term_ids,
                  const float* q_weights, int64_t q_nnz, const int32_t* k, int32_t k_max, void* workspace,
                  size_t workspace_bytes_, int32_t* out_ids, void* out_scores, const gs_search_opts* opts,
                  void* hip_stream) {
    gs_batch b = nullptr;
    int32_t rc = gs_batch_create(ix, q_row_ptr, n_queries, q_term_ids, q_weights, q_nnz, k, k_max, hip_stream, &b);
    if (rc != GS_OK) return rc;
    rc = gs_search_batch(ix, b, workspace, workspace_bytes_, out_ids, out_scores, opts, hip_stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (rc == GS_OK && e != hipSuccess) rc = fail(GS_EHIP, std::string("search: ") + hipGetErrorString(e));
    if (rc == GS_OK) rc = check_overflow(b);
    gs_batch_free(b);
    return rc;
}

int32_t gs_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> l(g_timing_mu);
    g_timing_on = on != 0;
    return GS_OK;
}

int32_t gs_timing_read(double* score_ms, int64_t* score_launches, double* select_ms, int64_t* select_launches) {
    g_err.clear();
    std::vector<TimedSpan> spans;
    {
        std::lock_guard<std::mutex> l(g_timing_mu);
        spans.swap(g_spans);
    }
    double ms[2] = {0.0, 0.0};
    int64_t cnt[2] = {0, 0};
    hipError_t err = hipSuccess;
    for (auto& sp : spans) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(sp.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, sp.a, sp.b);
        if (e == hipSuccess) {
            ms[sp.kind] += t;
            cnt[sp.kind] += sp.counts ? 1 : 0;
        } else {
            err = e;
        }
        (void)hipEventDestroy(sp.a);
        (void)hipEventDestroy(sp.b);
    }
    if (score_ms) *score_ms = ms[0];
    if (score_launches) *score_launches = cnt[0];
    if (select_ms) *select_ms = ms[1];
    if (select_launches) *select_launches = cnt[1];
    if (err != hipSuccess) return fail(GS_EHIP, std::string("timing: ") + hipGetErrorString(err));
    return GS_OK;
}

int32_t gs_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
    g_err.clear();
    if (!dst || !src) return fail(GS_EINVAL, "null pointer");
    if (bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return fail(GS_EINVAL, "copy needs 16-byte sizes and alignment");
    (void)hipGetLastError();
    GS_HIP(launch_copy16(dst, src, (int64_t)(bytes / 16), (hipStream_t)hip_stream));
    return GS_OK;
}

int32_t gs_lds_atomic_probe(int32_t op, int32_t pattern, int32_t workgroups, int32_t iters, void* sink,
                            void* hip_stream, int64_t* lane_ops) {
    g_err.clear();
    if (op < 0 || op > 3) return fail(GS_EINVAL, "op must be 0 (uint32), 1 (uint64), 2 (float) or 3 (double)");
    if (pattern != 0 && pattern != 1) return fail(GS_EINVAL, "pattern must be 0 or 1");
    if (workgroups < 1 || iters < 16 || iters % 16) return fail(GS_EINVAL, "workgroups >= 1, iters a positive multiple of 16");
    if (!sink) return fail(GS_EINVAL, "null sink");
    (void)hipGetLastError();
    GS_HIP(launch_lds_atomic(op, pattern, workgroups, iters, sink, (hipStream_t)hip_stream));
    if (lane_ops) *lane_ops = (int64_t)workgroups * 512 * iters;
    return GS_OK;
}

int32_t gs_batch_diagnostics(gs_batch b, int32_t* out) {
    g_err.clear();
    if (!b || !out) return fail(GS_EINVAL, "null argument");
    if (b->n_queries == 0) return GS_OK;
    DeviceGuard g(b->device);
    GS_HIP(hipMemcpy(out, b->diag, (size_t)b->n_queries * kDiagWords * 4, hipMemcpyDeviceToHost));
    return GS_OK;
}

}  // extern "C"
