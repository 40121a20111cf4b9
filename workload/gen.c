/*
 * Seeded synthetic learned-sparse collections and query batches.
 *
 * Input synthesis only: this file holds none of the retrieval method's
 * arithmetic (no scoring, no quantisation, no ranking). Both the CPU oracle
 * and the GPU library consume the arrays it writes.
 *
 * Shapes follow the paper's workload (Sec. 6.1 "Data": SPLADE vectors over a
 * 30,522-term vocabulary, ~127 terms per passage, ~50 per query, weights of the
 * form log(1+ReLU(.)) in [0, 3.5]) with a Zipf term law:
 *   - doc nnz ~ Poisson(mean) clipped to [lo, hi];
 *   - query nnz ~ Poisson(mean) clipped, or lognormal(median, sigma) rounded
 *     and clipped (long-tailed batches);
 *   - distinct term ids: weighted sampling without replacement, weight of rank
 *     r proportional to r^-s (r = 1..V), ranks mapped to term ids through a
 *     seeded permutation of the vocabulary; ids stored ascending per row;
 *   - weight = float(log1p(exp(sigma_w * z))), z ~ N(0,1), capped at w_cap.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) run as one counter stream per row, keyed by
 * (seed, stream kind, row index), so the output does not depend on the number
 * of threads. Zipf draws use Walker's alias method (Vose's construction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline rng_t rng_for(uint64_t seed, uint64_t kind, uint64_t index) {
    rng_t r;
    r.s = mix64(seed * GOLDEN_GAMMA + 0x632be59bd9b4e019ULL) ^ mix64((kind << 56) ^ (index + 1) * 0xd1b54a32d192ed03ULL);
    return r;
}

static inline uint64_t rng_u64(rng_t* r) {
    r->s += GOLDEN_GAMMA;
    return mix64(r->s);
}

/* uniform in (0, 1) */
static inline double rng_unif(rng_t* r) {
    return ((double)(rng_u64(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static inline double rng_normal(rng_t* r) {
    double u1 = rng_unif(r), u2 = rng_unif(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

static int64_t rng_poisson(rng_t* r, double lam) {
    /* inversion by sequential search; fine for the means used here (<= 500) */
    double u = rng_unif(r);
    double p = exp(-lam), F = p;
    int64_t k = 0;
    while (u > F && k < 100000) {
        k++;
        p *= lam / (double)k;
        F += p;
        if (p == 0.0 && F < u) break;
    }
    return k;
}

/* ---------------- Zipf sampler (alias table) + vocab permutation ---------- */

typedef struct {
    int32_t V;
    double* prob;    /* alias acceptance probability per column */
    int32_t* alias;  /* alias column */
    int32_t* perm;   /* rank index (0-based) -> term id */
} zipf_t;

static void zipf_free(zipf_t* z) {
    free(z->prob); free(z->alias); free(z->perm);
    memset(z, 0, sizeof(*z));
}

static int zipf_init(zipf_t* z, int32_t V, double s, uint64_t perm_seed) {
    z->V = V;
    z->prob = (double*)malloc(sizeof(double) * (size_t)V);
    z->alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
    z->perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
    double* q = (double*)malloc(sizeof(double) * (size_t)V);
    int32_t* small = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
    int32_t* large = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
    if (!z->prob || !z->alias || !z->perm || !q || !small || !large) {
        free(q); free(small); free(large); zipf_free(z); return -1;
    }
    double tot = 0.0;
    for (int32_t r = 0; r < V; r++) { q[r] = pow((double)(r + 1), -s); tot += q[r]; }
    int32_t ns = 0, nl = 0;
    for (int32_t r = 0; r < V; r++) {
        q[r] = q[r] * (double)V / tot;
        if (q[r] < 1.0) small[ns++] = r; else large[nl++] = r;
    }
    while (ns > 0 && nl > 0) {
        int32_t a = small[--ns], g = large[--nl];
        z->prob[a] = q[a];
        z->alias[a] = g;
        q[g] = (q[g] + q[a]) - 1.0;
        if (q[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { int32_t g = large[--nl]; z->prob[g] = 1.0; z->alias[g] = g; }
    while (ns > 0) { int32_t a = small[--ns]; z->prob[a] = 1.0; z->alias[a] = a; }
    /* Fisher-Yates permutation of the vocabulary, its own stream (kind 0) */
    rng_t r = rng_for(perm_seed, 0, 0);
    for (int32_t i = 0; i < V; i++) z->perm[i] = i;
    for (int32_t i = V - 1; i > 0; i--) {
        int32_t j = (int32_t)(rng_u64(&r) % (uint64_t)(i + 1));
        int32_t t = z->perm[i]; z->perm[i] = z->perm[j]; z->perm[j] = t;
    }
    free(q); free(small); free(large);
    return 0;
}

static inline int32_t zipf_draw(const zipf_t* z, rng_t* r) {
    uint64_t x = rng_u64(r);
    int32_t col = (int32_t)(((x >> 32) * (uint64_t)z->V) >> 32);
    double u = (double)(x & 0xffffffffULL) * (1.0 / 4294967296.0);
    return u < z->prob[col] ? col : z->alias[col];
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Row-length laws. law 0: Poisson(mean) clipped; law 1: lognormal(median, sigma) rounded, clipped. */
static int64_t draw_nnz(rng_t* r, int32_t law, double a, double b, int64_t lo, int64_t hi) {
    int64_t n;
    if (law == 0) n = rng_poisson(r, a);
    else n = (int64_t)llround(exp(log(a) + b * rng_normal(r)));
    if (n < lo) n = lo;
    if (n > hi) n = hi;
    return n;
}

/*
 * Pass 1: row lengths. kind selects the stream family (1 = docs, 2 = queries,
 * others free for callers). Writes nnz[n_rows].
 */
int wl_row_nnz(uint64_t seed, int32_t kind, int64_t n_rows, int32_t law, double a, double b,
               int64_t lo, int64_t hi, int32_t vocab, int64_t* nnz_out) {
    if (n_rows < 0 || lo < 0 || hi < lo || hi > vocab) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; i++) {
        rng_t r = rng_for(seed, (uint64_t)kind, (uint64_t)i);
        nnz_out[i] = draw_nnz(&r, law, a, b, lo, hi);
    }
    return 0;
}

/*
 * Pass 2: fill term ids (ascending per row) and weights given row_ptr from the
 * lengths of pass 1 (same seed/kind/law arguments). perm_seed keys the
 * vocabulary permutation; docs and queries of one workload share it so that
 * both follow the same term law.
 */
int wl_fill_rows(uint64_t seed, int32_t kind, int64_t n_rows, int32_t law, double a, double b,
                 int64_t lo, int64_t hi, int32_t vocab, double zipf_s, uint64_t perm_seed,
                 double w_sigma, float w_cap,
                 const int64_t* row_ptr, int32_t* terms, float* weights) {
    zipf_t z;
    if (zipf_init(&z, vocab, zipf_s, perm_seed) != 0) return -2;
    int err = 0;
#pragma omp parallel
    {
        uint64_t* seen = (uint64_t*)calloc(((size_t)vocab + 63) / 64, sizeof(uint64_t));
        if (!seen) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n_rows; i++) {
            if (!seen) continue;
            rng_t r = rng_for(seed, (uint64_t)kind, (uint64_t)i);
            int64_t n = draw_nnz(&r, law, a, b, lo, hi);
            if (n != row_ptr[i + 1] - row_ptr[i]) {
#pragma omp atomic write
                err = -3;
                continue;
            }
            int32_t* t = terms + row_ptr[i];
            float* w = weights + row_ptr[i];
            int64_t got = 0;
            while (got < n) {
                int32_t rk = zipf_draw(&z, &r);
                if (seen[rk >> 6] & (1ULL << (rk & 63))) continue;
                seen[rk >> 6] |= 1ULL << (rk & 63);
                t[got++] = rk;
            }
            for (int64_t j = 0; j < n; j++) {
                int32_t rk = t[j];
                seen[rk >> 6] &= ~(1ULL << (rk & 63));
                t[j] = z.perm[rk];
            }
            qsort(t, (size_t)n, sizeof(int32_t), cmp_i32);
            for (int64_t j = 0; j < n; j++) {
                float v = (float)log1p(exp(w_sigma * rng_normal(&r)));
                w[j] = v > w_cap ? w_cap : v;
            }
        }
        free(seen);
    }
    zipf_free(&z);
    return err;
}
