// Host paths of libgpusparse under AddressSanitizer and UndefinedBehaviorSanitizer (built
// and run by tests/test_host_sanitized.py on the CPU, without a GPU). It drives the input
// validation, the host posting layout, the fixed-point plan and the error paths of every
// entry point that reaches the device (which fail here: there is no GPU), so that an out
// of bounds access, a use after free, a leak or undefined behaviour in that code aborts.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "../../include/gpusparse.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, gs_last_error());
        failures++;
    }
}

struct Csr {
    std::vector<int64_t> rp;
    std::vector<int32_t> term;
    std::vector<float> w;
};

Csr random_csr(std::mt19937_64& rng, int n, int vocab, int max_row, bool sorted) {
    Csr c;
    c.rp.push_back(0);
    std::uniform_int_distribution<int> len(0, max_row);
    std::uniform_real_distribution<float> wd(0.0f, 3.0f);
    for (int i = 0; i < n; i++) {
        std::vector<int32_t> row;
        const int m = std::min(len(rng), vocab);
        std::vector<int32_t> all(vocab);
        for (int t = 0; t < vocab; t++) all[t] = t;
        std::shuffle(all.begin(), all.end(), rng);
        row.assign(all.begin(), all.begin() + m);
        if (sorted) std::sort(row.begin(), row.end());
        for (int32_t t : row) {
            c.term.push_back(t);
            c.w.push_back(wd(rng) * (rng() % 7 == 0 ? 0.0f : 1.0f));
        }
        c.rp.push_back((int64_t)c.term.size());
    }
    return c;
}

void layout(const Csr& c, int vocab, int precision, int32_t expect_rc) {
    const int64_t n = (int64_t)c.rp.size() - 1;
    int64_t padded = 0;
    int32_t rc = gs_layout_host(c.rp.data(), n, c.term.data(), c.w.data(), (int64_t)c.term.size(), vocab, precision,
                                &padded, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    expect(rc == expect_rc, "layout sizes status");
    if (rc != GS_OK) return;
    std::vector<int64_t> off(vocab + 1);
    std::vector<int32_t> len(vocab), doc(padded), bfirst(padded / 64);
    std::vector<float> w(padded), bmax(padded / 64);
    std::vector<uint8_t> dense(vocab), b8(padded);
    rc = gs_layout_host(c.rp.data(), n, c.term.data(), c.w.data(), (int64_t)c.term.size(), vocab, precision, &padded,
                        off.data(), len.data(), doc.data(), w.data(), bmax.data(), bfirst.data(), dense.data(),
                        b8.data());
    expect(rc == GS_OK, "layout arrays");
    int64_t real = 0;
    for (int t = 0; t < vocab; t++) real += len[t];
    expect(real == (int64_t)c.term.size(), "every posting placed");
}

}  // namespace

int main() {
    std::mt19937_64 rng(7);
    for (int s = 0; s < 40; s++) {
        const int vocab = 1 + (int)(rng() % 300);
        const int n = (int)(rng() % 3000);
        Csr c = random_csr(rng, n, vocab, 40, s % 2 == 0);
        layout(c, vocab, (int)(s % 3), GS_OK);
    }
    // malformed inputs are rejected
    {
        Csr c = random_csr(rng, 50, 20, 6, true);
        Csr bad = c;
        if (!bad.term.empty()) {
            bad.term[0] = 20;  // out of range
            layout(bad, 20, GS_FP32, GS_EINVAL);
            bad = c;
            bad.w[0] = std::numeric_limits<float>::quiet_NaN();
            layout(bad, 20, GS_FP32, GS_EINVAL);
            bad = c;
            bad.w[0] = -1.0f;
            layout(bad, 20, GS_U8, GS_EINVAL);
        }
        bad = c;
        bad.rp[1] = bad.rp[2] + 1;  // not monotone
        layout(bad, 20, GS_BF16, GS_EINVAL);
        Csr dup;
        dup.rp = {0, 2};
        dup.term = {3, 3};
        dup.w = {1.0f, 2.0f};
        layout(dup, 20, GS_FP32, GS_EINVAL);
        Csr empty;
        empty.rp = {0};
        layout(empty, 1, GS_FP32, GS_OK);
    }
    // the fixed-point plan
    for (int s = 0; s < 200; s++) {
        const int m = (int)(rng() % 257);
        std::vector<float> q(m), tmax(m), tmin(m);
        std::uniform_real_distribution<double> e(-12.0, 0.5);
        for (int j = 0; j < m; j++) {
            q[j] = (float)std::pow(10.0, e(rng));
            tmin[j] = (float)std::pow(10.0, e(rng));
            tmax[j] = tmin[j] * 4.0f;
        }
        int32_t F = 0;
        double err = 0, lim = 0;
        expect(gs_query_plan_host(GS_FP32, q.data(), tmax.data(), tmin.data(), m, &F, &err, &lim) == GS_OK, "plan fp32");
        expect(gs_query_plan_host(GS_BF16, q.data(), tmax.data(), tmin.data(), m, &F, &err, &lim) == GS_OK, "plan bf16");
    }
    expect(gs_query_plan_host(GS_FP32, nullptr, nullptr, nullptr, 257, nullptr, nullptr, nullptr) == GS_EINVAL,
           "plan nnz bound");
    // entry points that need the device: argument errors, then the device error paths
    gs_index ix = nullptr;
    expect(gs_build_index(nullptr, 0, nullptr, nullptr, 0, 0, GS_FP32, 0, nullptr, &ix) == GS_EINVAL, "vocab < 1");
    {
        Csr c = random_csr(rng, 500, 50, 12, false);
        const int32_t rc = gs_build_index(c.rp.data(), 500, c.term.data(), c.w.data(), (int64_t)c.term.size(), 50,
                                          GS_U8, GS_KEEP_DOC_IDS, nullptr, &ix);
        expect(rc != GS_OK && ix == nullptr, "no device: the build fails without an index");
        gs_debug_fail_alloc(0);
        const int32_t rc2 = gs_build_index(c.rp.data(), 500, c.term.data(), c.w.data(), (int64_t)c.term.size(), 50,
                                           GS_FP32, 0, nullptr, &ix);
        expect(rc2 != GS_OK && ix == nullptr, "injected allocation failure");
        gs_debug_fail_alloc(-1);
    }
    gs_batch b = nullptr;
    expect(gs_batch_reserve(nullptr, 4, 16, 10, &b) == GS_EINVAL && b == nullptr, "batch without index");
    size_t bytes = 0;
    expect(gs_search_workspace_size(nullptr, 1, 1, 1, nullptr, &bytes) == GS_EINVAL, "workspace without index");
    gs_server srv = nullptr;
    gs_server_opts so{};
    expect(gs_server_create(nullptr, &so, &srv) == GS_EINVAL && srv == nullptr, "server without index");
    expect(gs_server_poll(nullptr, 0, nullptr, nullptr, nullptr) == GS_EINVAL, "poll without server");
    for (int32_t st = 1; st >= -7; st--) expect(gs_status_string(st) != nullptr, "status string");
    gs_free_index(nullptr);
    gs_batch_free(nullptr);
    gs_server_destroy(nullptr);
    std::printf("host paths: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
