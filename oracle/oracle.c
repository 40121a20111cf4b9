/*
 * CPU oracle for exact learned-sparse retrieval (plain C, fp64 and int64).
 *
 * TEST INFRASTRUCTURE. This file is the slow, obviously correct reference that
 * the GPU library is checked against. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load it; the product path never does. It
 * shares no code, header or table with the GPU library.
 *
 * What it computes (paper Sec. 2.1 "Learned Sparse Retrieval": the retrieval
 * score is the inner product of the query's and the document's sparse
 * vectors; Sec. 4.1, first equation: score(q,d) = sum over the query's terms
 * t_i of w_i * s_d(t_i), with s_d(t) = 0 when t is absent from d):
 *
 *   S(q,d) = sum_{t in q and d} w_q(t) * w_d(t)
 *
 * evaluated in fp64 for every document d of the collection, by walking d's own
 * term list in ascending term id and adding qw[t] * w_d(t), where qw is the
 * query scattered into a dense vector (0 for terms absent from the query, so
 * those products add +0.0 and leave the sum unchanged). Each product of two
 * fp32 values is exact in fp64.
 *
 * The ranking (Sec. 4.3: exact scoring, every document is scored, nothing is
 * pruned) is the full sort of all N documents by (score descending, doc id
 * ascending); the answer for (q, k) is its first min(k, N) entries. Slots from
 * min(k, N) to k_max are id -1, score 0.
 *
 * The integer form (uint8 impacts; the paper names quantised posting scores as
 * future work in Sec. 8) quantises every weight as q8(w) = round(w * 255 / 3)
 * with ties to even, saturated to [0, 255], and accumulates exact int64 sums
 * of q8(w_q(t)) * q8(w_d(t)) over shared terms, ranked the same way.
 *
 * Error codes: 0 ok, -1 invalid argument (term id out of range, duplicate
 * term in a query, k < 0, k > k_max, non-finite weight), -2 allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ q8 -- */

uint8_t oracle_q8(float w) {
    double x = rint((double)w * 85.0); /* 255/3 = 85; the product is exact in fp64 */
    if (!(x > 0.0)) return 0;          /* also maps NaN to 0 (callers reject NaN) */
    if (x > 255.0) return 255;
    return (uint8_t)x;
}

void oracle_q8_array(const float* w, int64_t n, uint8_t* out) {
    for (int64_t i = 0; i < n; i++) out[i] = oracle_q8(w[i]);
}

/* ------------------------------------------------------- row traversal -- */

/* Returns 1 when the row's term ids are strictly ascending. */
static int row_sorted(const int32_t* t, int64_t n) {
    for (int64_t j = 1; j < n; j++)
        if (t[j] <= t[j - 1]) return 0;
    return 1;
}

typedef struct { int32_t t; float w; } entry_t;

static int cmp_entry(const void* a, const void* b) {
    int32_t x = ((const entry_t*)a)->t, y = ((const entry_t*)b)->t;
    return (x > y) - (x < y);
}

/* Copy a row into buf sorted by ascending term id (buf holds >= n entries). */
static void sorted_copy(const int32_t* t, const float* w, int64_t n, entry_t* buf) {
    for (int64_t j = 0; j < n; j++) { buf[j].t = t[j]; buf[j].w = w[j]; }
    qsort(buf, (size_t)n, sizeof(entry_t), cmp_entry);
}

static int64_t max_row_len(const int64_t* row_ptr, int64_t n_rows) {
    int64_t m = 0;
    for (int64_t i = 0; i < n_rows; i++)
        if (row_ptr[i + 1] - row_ptr[i] > m) m = row_ptr[i + 1] - row_ptr[i];
    return m;
}

/* Scatter a query into a dense fp64 vector. Rejects bad ids, duplicates and non-finite weights. */
static int scatter_query_f64(const int32_t* qt, const float* qw, int64_t qn, int32_t vocab, double* dense,
                             unsigned char* mark) {
    memset(dense, 0, sizeof(double) * (size_t)vocab);
    memset(mark, 0, (size_t)vocab);
    for (int64_t j = 0; j < qn; j++) {
        if (qt[j] < 0 || qt[j] >= vocab || mark[qt[j]] || !isfinite(qw[j])) return -1;
        mark[qt[j]] = 1;
        dense[qt[j]] = (double)qw[j];
    }
    return 0;
}

static int scatter_query_i64(const int32_t* qt, const float* qw, int64_t qn, int32_t vocab, int64_t* dense,
                             unsigned char* mark) {
    memset(dense, 0, sizeof(int64_t) * (size_t)vocab);
    memset(mark, 0, (size_t)vocab);
    for (int64_t j = 0; j < qn; j++) {
        if (qt[j] < 0 || qt[j] >= vocab || mark[qt[j]] || !isfinite(qw[j])) return -1;
        mark[qt[j]] = 1;
        dense[qt[j]] = (int64_t)oracle_q8(qw[j]);
    }
    return 0;
}

/* S(q,d) in fp64 for one document, terms visited in ascending id. */
static double doc_score_f64(const int32_t* t, const float* w, int64_t n, int32_t vocab, const double* qdense,
                            entry_t* buf, int* bad) {
    double s = 0.0;
    if (row_sorted(t, n)) {
        for (int64_t j = 0; j < n; j++) {
            if (t[j] < 0 || t[j] >= vocab) { *bad = 1; return 0.0; }
            s += qdense[t[j]] * (double)w[j];
        }
    } else {
        sorted_copy(t, w, n, buf);
        for (int64_t j = 0; j < n; j++) {
            if (buf[j].t < 0 || buf[j].t >= vocab) { *bad = 1; return 0.0; }
            s += qdense[buf[j].t] * (double)buf[j].w;
        }
    }
    return s;
}

static int64_t doc_score_i64(const int32_t* t, const float* w, int64_t n, int32_t vocab, const int64_t* qdense,
                             int* bad) {
    int64_t s = 0;
    for (int64_t j = 0; j < n; j++) {
        if (t[j] < 0 || t[j] >= vocab) { *bad = 1; return 0; }
        s += qdense[t[j]] * (int64_t)oracle_q8(w[j]);
    }
    return s;
}

/* ----------------------------------------------------------- all docs -- */

/* Dense scores of one query against every document (fp64). out[n_docs]. */
int oracle_scores_f64(const int64_t* row_ptr, const int32_t* terms, const float* weights, int64_t n_docs,
                      int32_t vocab, const int32_t* q_terms, const float* q_weights, int64_t q_nnz,
                      double* out) {
    double* dense = (double*)malloc(sizeof(double) * (size_t)vocab);
    unsigned char* mark = (unsigned char*)malloc((size_t)vocab);
    int64_t ml = max_row_len(row_ptr, n_docs);
    entry_t* buf = (entry_t*)malloc(sizeof(entry_t) * (size_t)(ml > 0 ? ml : 1));
    if (!dense || !mark || !buf) { free(dense); free(mark); free(buf); return -2; }
    int rc = scatter_query_f64(q_terms, q_weights, q_nnz, vocab, dense, mark);
    int bad = 0;
    for (int64_t d = 0; rc == 0 && d < n_docs; d++) {
        int64_t a = row_ptr[d], b = row_ptr[d + 1];
        out[d] = doc_score_f64(terms + a, weights + a, b - a, vocab, dense, buf, &bad);
    }
    free(dense); free(mark); free(buf);
    return rc != 0 ? rc : (bad ? -1 : 0);
}

/* Dense integer scores of one query against every document. out[n_docs]. */
int oracle_scores_i64(const int64_t* row_ptr, const int32_t* terms, const float* weights, int64_t n_docs,
                      int32_t vocab, const int32_t* q_terms, const float* q_weights, int64_t q_nnz,
                      int64_t* out) {
    int64_t* dense = (int64_t*)malloc(sizeof(int64_t) * (size_t)vocab);
    unsigned char* mark = (unsigned char*)malloc((size_t)vocab);
    if (!dense || !mark) { free(dense); free(mark); return -2; }
    int rc = scatter_query_i64(q_terms, q_weights, q_nnz, vocab, dense, mark);
    int bad = 0;
    for (int64_t d = 0; rc == 0 && d < n_docs; d++) {
        int64_t a = row_ptr[d], b = row_ptr[d + 1];
        out[d] = doc_score_i64(terms + a, weights + a, b - a, vocab, dense, &bad);
    }
    free(dense); free(mark);
    return rc != 0 ? rc : (bad ? -1 : 0);
}

/* Scores of one query against a list of documents (fp64 and int64 forms). */
int oracle_pair_scores(const int64_t* row_ptr, const int32_t* terms, const float* weights, int64_t n_docs,
                       int32_t vocab, const int32_t* q_terms, const float* q_weights, int64_t q_nnz,
                       const int32_t* docs, int64_t n, double* out_f64, int64_t* out_i64) {
    double* dense = (double*)malloc(sizeof(double) * (size_t)vocab);
    int64_t* idense = (int64_t*)malloc(sizeof(int64_t) * (size_t)vocab);
    unsigned char* mark = (unsigned char*)malloc((size_t)vocab);
    entry_t* buf = (entry_t*)malloc(sizeof(entry_t) * 4096);
    if (!dense || !idense || !mark || !buf) { free(dense); free(idense); free(mark); free(buf); return -2; }
    int rc = scatter_query_f64(q_terms, q_weights, q_nnz, vocab, dense, mark);
    if (rc == 0) rc = scatter_query_i64(q_terms, q_weights, q_nnz, vocab, idense, mark);
    int bad = 0;
    for (int64_t i = 0; rc == 0 && i < n; i++) {
        int64_t d = docs[i];
        if (d < 0 || d >= n_docs) { rc = -1; break; }
        int64_t a = row_ptr[d], b = row_ptr[d + 1];
        if (b - a > 4096) { rc = -1; break; }
        if (out_f64) out_f64[i] = doc_score_f64(terms + a, weights + a, b - a, vocab, dense, buf, &bad);
        if (out_i64) out_i64[i] = doc_score_i64(terms + a, weights + a, b - a, vocab, idense, &bad);
    }
    free(dense); free(idense); free(mark); free(buf);
    return rc != 0 ? rc : (bad ? -1 : 0);
}

/* ------------------------------------------------------------- top-k -- */

typedef struct { double s; int32_t id; } fpair_t;
typedef struct { int64_t s; int32_t id; } ipair_t;

/* score descending, then doc id ascending */
static int cmp_fpair(const void* a, const void* b) {
    const fpair_t* x = (const fpair_t*)a;
    const fpair_t* y = (const fpair_t*)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int cmp_ipair(const void* a, const void* b) {
    const ipair_t* x = (const ipair_t*)a;
    const ipair_t* y = (const ipair_t*)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/*
 * Exact top-k for a batch of queries (fp64 scores).
 * Queries: CSR q_row_ptr[n_q+1], q_terms, q_weights. k[n_q] with 0 <= k <= k_max.
 * Outputs (row-major [n_q, k_max]): out_ids (-1 padded), out_scores (0 padded).
 * n_threads <= 0 lets OpenMP decide.
 */
int oracle_topk_f64(const int64_t* row_ptr, const int32_t* terms, const float* weights, int64_t n_docs,
                    int32_t vocab, const int64_t* q_row_ptr, int32_t n_q, const int32_t* q_terms,
                    const float* q_weights, const int32_t* k, int32_t k_max, int32_t* out_ids,
                    double* out_scores, int32_t n_threads) {
    if (n_docs < 0 || n_q < 0 || k_max < 0) return -1;
    for (int32_t q = 0; q < n_q; q++)
        if (k[q] < 0 || k[q] > k_max) return -1;
    int64_t ml = max_row_len(row_ptr, n_docs);
    int err = 0;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : omp_get_max_threads())
    {
        double* dense = (double*)malloc(sizeof(double) * (size_t)vocab);
        unsigned char* mark = (unsigned char*)malloc((size_t)vocab);
        entry_t* buf = (entry_t*)malloc(sizeof(entry_t) * (size_t)(ml > 0 ? ml : 1));
        fpair_t* all = (fpair_t*)malloc(sizeof(fpair_t) * (size_t)(n_docs > 0 ? n_docs : 1));
        int local_err = (!dense || !mark || !buf || !all) ? -2 : 0;
#pragma omp for schedule(dynamic, 1)
        for (int32_t q = 0; q < n_q; q++) {
            if (local_err) continue;
            int64_t qa = q_row_ptr[q], qb = q_row_ptr[q + 1];
            if (scatter_query_f64(q_terms + qa, q_weights + qa, qb - qa, vocab, dense, mark) != 0) {
                local_err = -1;
                continue;
            }
            int bad = 0;
            for (int64_t d = 0; d < n_docs; d++) {
                int64_t a = row_ptr[d], b = row_ptr[d + 1];
                all[d].s = doc_score_f64(terms + a, weights + a, b - a, vocab, dense, buf, &bad);
                all[d].id = (int32_t)d;
            }
            if (bad) { local_err = -1; continue; }
            qsort(all, (size_t)n_docs, sizeof(fpair_t), cmp_fpair);
            int64_t take = k[q] < n_docs ? k[q] : n_docs;
            for (int64_t i = 0; i < k_max; i++) {
                out_ids[(int64_t)q * k_max + i] = i < take ? all[i].id : -1;
                out_scores[(int64_t)q * k_max + i] = i < take ? all[i].s : 0.0;
            }
        }
        if (local_err) {
#pragma omp critical
            err = local_err;
        }
        free(dense); free(mark); free(buf); free(all);
    }
    return err;
}

/* Exact top-k for a batch of queries on uint8 impacts with int64 accumulation. */
int oracle_topk_i64(const int64_t* row_ptr, const int32_t* terms, const float* weights, int64_t n_docs,
                    int32_t vocab, const int64_t* q_row_ptr, int32_t n_q, const int32_t* q_terms,
                    const float* q_weights, const int32_t* k, int32_t k_max, int32_t* out_ids,
                    int64_t* out_scores, int32_t n_threads) {
    if (n_docs < 0 || n_q < 0 || k_max < 0) return -1;
    for (int32_t q = 0; q < n_q; q++)
        if (k[q] < 0 || k[q] > k_max) return -1;
    int err = 0;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : omp_get_max_threads())
    {
        int64_t* dense = (int64_t*)malloc(sizeof(int64_t) * (size_t)vocab);
        unsigned char* mark = (unsigned char*)malloc((size_t)vocab);
        ipair_t* all = (ipair_t*)malloc(sizeof(ipair_t) * (size_t)(n_docs > 0 ? n_docs : 1));
        int local_err = (!dense || !mark || !all) ? -2 : 0;
#pragma omp for schedule(dynamic, 1)
        for (int32_t q = 0; q < n_q; q++) {
            if (local_err) continue;
            int64_t qa = q_row_ptr[q], qb = q_row_ptr[q + 1];
            if (scatter_query_i64(q_terms + qa, q_weights + qa, qb - qa, vocab, dense, mark) != 0) {
                local_err = -1;
                continue;
            }
            int bad = 0;
            for (int64_t d = 0; d < n_docs; d++) {
                int64_t a = row_ptr[d], b = row_ptr[d + 1];
                all[d].s = doc_score_i64(terms + a, weights + a, b - a, vocab, dense, &bad);
                all[d].id = (int32_t)d;
            }
            if (bad) { local_err = -1; continue; }
            qsort(all, (size_t)n_docs, sizeof(ipair_t), cmp_ipair);
            int64_t take = k[q] < n_docs ? k[q] : n_docs;
            for (int64_t i = 0; i < k_max; i++) {
                out_ids[(int64_t)q * k_max + i] = i < take ? all[i].id : -1;
                out_scores[(int64_t)q * k_max + i] = i < take ? all[i].s : 0;
            }
        }
        if (local_err) {
#pragma omp critical
            err = local_err;
        }
        free(dense); free(mark); free(all);
    }
    return err;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
