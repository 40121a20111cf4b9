// Internal declarations shared by the host side (gs_host.cpp) and the HIP
// kernels (gs_score.hip, gs_topk.hip, gs_yardstick.hip) of libgpusparse.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

struct gs_batch_s;
struct gs_index_s;
struct gs_search_opts;

namespace gs {

constexpr int kWave = 64;             // CDNA wavefront
constexpr int kBlock = 64;            // postings per padded block (one wavefront)
constexpr int kGrainShift = 13;       // segment-table doc-tile granularity: 8192 docs
constexpr int kMaxQueryNnz = 256;     // GS_MAX_QUERY_NNZ
constexpr int kMaxChunk = 1024;       // largest chunk of the doc-tiled kernels (postings)
// post_lo and post_w carry kMaxChunk zeroed entries past the last posting, so a
// chunk's full-width loads stay inside the arrays (lanes past its end are masked).
constexpr size_t kPostSlack = kMaxChunk;
constexpr int kMaxK = 4096;           // GS_MAX_K
constexpr int kHistBits = 11;         // selection digit width (first digit fused into scoring)
constexpr int kHistBins = 1 << kHistBits;
constexpr int kCandCap = 32768;       // candidates kept per query by the filter pass
constexpr int kFusedCap = 24576;      // of which appended while scoring (fused filtering)
constexpr int kRefinePasses = 6;      // enough to resolve any 64-bit composite key
constexpr int kFirstShiftFloat = 52;  // first digit of a float key: bits 30..20
constexpr int kDiagWords = 8;         // per-query words of gs_batch_diagnostics
// Group kernel (GS_KERNEL_GROUP): 8192-doc tiles, at most 4 queries per group, so at most
// 4 x 256 distinct terms per group.
constexpr int kGroupTileShift = 13;
constexpr int kGroupMax = 4;
constexpr int kGroupMaxTerms = kGroupMax * kMaxQueryNnz;
constexpr int kGroupChunkTab = 1024;  // chunk table entries of a group work item (two workgroups per CU keep fitting the LDS)
// Fixed scratch array of the allocation-free search (gs_search_batch_noalloc): one per
// device, 128 MiB (a one-query workspace for collections up to about 33M documents).
constexpr size_t kScratchBytes = (size_t)128 << 20;

enum Precision { kFP32 = 0, kBF16 = 1, kU8 = 2 };

// Record the message returned by gs_last_error() on this thread; returns code.
int32_t set_error(int32_t code, const std::string& msg);

// Device and pinned host allocations of the library go through these, so that a test can
// make the n-th one fail (gs_debug_fail_alloc) and check the GS_ENOMEM paths.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t pinned_malloc(void** p, size_t bytes);

// Name of the kernel whose launch failed last on this thread (for error messages).
extern thread_local const char* g_failed_launch;

#define GS_CHECK_LAUNCH(name)                      \
    do {                                           \
        const hipError_t e_ = hipGetLastError();   \
        if (e_ != hipSuccess) {                    \
            ::gs::g_failed_launch = (name);        \
            return e_;                             \
        }                                          \
    } while (0)

// Index arrays on the device (plain pointers; passed by value to kernels).
struct DevIndex {
    int64_t n_docs;
    int32_t vocab;
    int32_t precision;
    const int64_t* term_off;   // [V+1] start of each padded list
    const int32_t* term_len;   // [V]   real postings per term
    const int32_t* post_doc;   // [padded_nnz], -1 in padding (GS_KEEP_DOC_IDS only, else null)
    // [padded_nnz] doc id modulo 65536. A doc tile of at most 32768 docs, aligned to its
    // size, lies inside one 65536-aligned range, so the doc-tiled kernels read 2 bytes per
    // posting for the id and recover the offset in the tile from the tile's base.
    const uint16_t* post_lo;
    // Byte form of the doc ids of dense terms (every 64-posting block of the list spans at
    // most 256 docs): post_b8[i] = doc(i) - blk_first[i / 64]. The doc-tiled kernels read
    // these lists in whole blocks, 1 byte per posting for the id instead of 2.
    const uint8_t* post_b8;    // [padded_nnz] (0 outside dense lists)
    const int32_t* blk_first;  // [padded_nnz / 64] doc of each block's first posting (-1 if empty)
    const float* blk_max;      // [padded_nnz / 64] largest stored weight of each block (as float)
    const uint8_t* term_dense; // [V] 1 if the term's list has the byte form
    const void* post_w;        // [padded_nnz] float | bf16 bits (uint16) | uint8
    const int32_t* tile_off;   // [V][n_grains+1] posting offset (relative to the list start)
    int64_t n_grains;          // ceil(n_docs / 8192)
    const int64_t* fwd_row_ptr;  // [N+1] forward rows (sorted by term), or null
    const int32_t* fwd_term;
    const float* fwd_w;
};

// A query batch on the device.
struct DevBatch {
    int32_t n_queries;
    int32_t k_max;
    const int64_t* q_row_ptr;  // [n+1]
    const int32_t* q_term;     // [q_nnz], ascending within each query
    const float* q_w;          // [q_nnz]
    const int32_t* q_w8;       // [q_nnz] uint8 impacts as int (GS_U8), else null
    const int32_t* k;          // [n]
    const int32_t* first_shift;  // [n] position of the first selection digit in the composite key
    const float* delta;        // [n] bf16 relative error bound per query (GS_BF16), else null
    // fixed-point accumulation (GS_FP32, GS_BF16): each product w_q * w_d is rounded to an
    // integer number of units 2^-F(q) and summed exactly as an unsigned integer (64-bit for
    // fp32, every product below 2^51 units; 32-bit for bf16, every doc's sum below 2^32 units).
    const double* q_fx;        // [q_nnz] w_q * 2^F(q) (exact)
    const double* q_scale;     // [n] 2^-F(q)
    const double* q_abs_err;   // [n] bound on |fixed-point sum - exact sum|
    // [n] wide-range check of the fixed-point sums: a query whose k-th approximate score may
    // lie below this value (its error bound over the relative budget of its precision) is
    // scored again with fp64 accumulation; 0 when the bound holds for every positive score.
    const double* q_wide_lim;
    const int64_t* q_work;     // [n] postings of the query's terms (work estimate)
    // Block-max pruning (opt-in): per query term, the sum of the upper bounds of the query's
    // terms (w_q times the term's largest stored weight, in fixed-point units or as an exact
    // uint8 product) taken in ascending order of bound, up to and including this term.
    const unsigned long long* q_ub_cum;  // [q_nnz]
    // Groups of the group kernel (built on the host at each update): the queries with k > 0
    // by descending work, G consecutive per group (G = 2 for fp32, 4 for bf16 and uint8);
    // per group the ascending union of its members' terms with each member's weight
    // (w_q, scaled by the member's 2^F in the kernel, or the uint8 impact; 0 where the member
    // lacks the term).
    const int32_t* g_count;    // [1] number of groups
    const int32_t* g_member;   // [groups * G] query of each member (-1: none)
    const int32_t* g_row;      // [groups + 1] start of each group's union terms
    const int32_t* g_term;     // [union terms]
    const float* g_wq;         // [union terms * G] (fp32, bf16)
    const int32_t* g_w8;       // [union terms * G] (uint8)
};

// Per-query selection state in the workspace.
struct SelState {
    unsigned long long prefix;  // bucket: composites c with (c >> shift) == (prefix >> shift)
    unsigned long long lo;      // filter threshold (inclusive) once resolved
    int32_t shift;
    int32_t k_rem;              // still needed from the bucket
    int32_t resolved;           // 0 refine, 1 filter with lo, 2 nothing to select (k == 0)
    int32_t n_cand;             // candidates appended by the filter
    int32_t passes;             // refinement passes over the score array
    int32_t band;               // bf16: candidates inside the error band
    int32_t overflow;           // candidate or band buffer overflow
    int32_t need_band_pass;     // bf16: band reaches below the filter threshold
    double tau;                 // bf16: band threshold on approximate scores
    // fused candidate filtering: a lower bound of the k-th composite from the seed tiles;
    // the other tiles append every composite >= bound while they are scored
    unsigned long long bound;
    int32_t fused;              // 1 while the appended candidates stand in for the row scan
    int32_t fused_over;         // the appends passed kFusedCap
    // 1: fell back from fused filtering after its non-seed rows were left unwritten (score
    // them again, fixed point); 2: wide range (score every tile again, fp64 accumulation)
    int32_t rescore;
    int32_t pruned;             // 64-posting blocks skipped by block-max pruning
};

// Workspace carve-up for a tile of qt queries.
struct Workspace {
    uint32_t* scores;             // [qt][N] fp32 bits or int32
    uint32_t* hist1;              // [qt][kHistBins]
    uint32_t* hist_ref;           // [qt][kHistBins]
    SelState* state;              // [qt]
    unsigned long long* cand;     // [qt][kCandCap]
    double* band_s;               // [qt][kCandCap] (bf16)
    int32_t* band_id;             // [qt][kCandCap] (bf16)
    int64_t* work_prefix;         // [qt * kMaxQueryNnz + 1] (atomic kernel)
    int32_t* work_pair_q;         // [qt * kMaxQueryNnz]
    int32_t* order;               // [qt] persistent kernel: query order within the tile
    uint32_t* counters;           // [16]: [0..7] persistent kernel per-XCD work counters,
                                  // [8] queries in rescore_list
    int32_t* rescore_list;        // [qt] queries whose rows are scored again (SelState::rescore)
    int64_t ld;                   // row stride of the score arrays (n_docs rounded up to 64)
};

size_t workspace_bytes(int64_t n_docs, int32_t qt, int32_t precision);
void carve_workspace(void* base, int64_t n_docs, int32_t qt, int32_t precision, Workspace* ws);
// A workspace of `rows` query rows in which a search may use any run [r0, r0 + n) (server arena).
size_t arena_bytes(int64_t n_docs, int64_t rows, int32_t precision);
void carve_rows(void* base, int64_t n_docs, int64_t rows, int32_t precision, int64_t r0, Workspace* ws);

struct ScoreOpts {
    int kernel;
    int tile_shift;   // doc tile of the TILED/SHARED kernels = 1 << tile_shift docs
    int chunk;        // postings per work item
    int seed_stride = 0;  // fused candidate filtering: every seed_stride-th doc tile seeds the bound (0: off)
    int prune = 0;        // block-max pruning of the non-seed tiles (TILED, fp32 and uint8)
};

// Doc tiles of a scoring launch: phase 0 all tiles, phase 1 the seed tiles
// (multiples of stride), phase 2 the others, phase 3 the others again for the
// queries that fell back from fused filtering (their rows), phase 4 all tiles
// again for the wide-range queries (fp64 accumulation), phase 5 the others again
// for the bf16 queries whose error band reaches below their fused candidates
// (their rows, for the band pass). v is the launch's tile index.
__host__ __device__ inline int64_t phase_tiles(int phase, int stride, int64_t n_tiles) {
    if (phase == 0 || phase == 4) return n_tiles;
    const int64_t seeds = (n_tiles + stride - 1) / stride;
    return phase == 1 ? seeds : n_tiles - seeds;
}
__host__ __device__ inline int64_t phase_tile(int phase, int stride, int64_t v) {
    if (phase == 0 || phase == 4) return v;
    if (phase == 1) return v * stride;
    return (v / (stride - 1)) * stride + v % (stride - 1) + 1;
}

// Upload a query batch (gs_batch_update). With wait == false it returns once the
// copies are enqueued on hip_stream (staged in pinned memory), for callers that
// search on that same stream.
int32_t batch_update(struct ::gs_batch_s* b, const int64_t* q_row_ptr, int32_t n_queries,
                     const int32_t* q_term_ids, const float* q_weights, int64_t q_nnz, const int32_t* k,
                     void* hip_stream, bool wait);

// Search the queries of the batch's last update on rows [r0, r0 + n) of an arena of `rows`
// rows, with the caller's step counters (16 words, device); asynchronous on s. (Server steps.)
int32_t search_rows(struct ::gs_index_s* ix, struct ::gs_batch_s* b, void* arena, int64_t rows, int64_t r0,
                    uint32_t* counters, const struct gs_search_opts* opts, int32_t* out_ids, void* out_scores,
                    hipStream_t s);
// Device array of the batch's per-query diagnostics (kDiagWords words per query).
const int32_t* batch_diag(const struct ::gs_batch_s* b);

// ---- launchers (gs_score.hip) ----
hipError_t launch_clear(const Workspace& ws, int32_t qt, hipStream_t s);
hipError_t launch_score_tiled(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                              const ScoreOpts& o, const Workspace& ws, hipStream_t s, int phase = 0);
// group kernel (GS_KERNEL_GROUP): phases 0, 1 and 2 of a search whose queries form one tile
hipError_t launch_score_group(const DevIndex& ix, const DevBatch& qb, const ScoreOpts& o, const Workspace& ws,
                              hipStream_t s, int phase);
// fp64-accumulating pass over every doc tile for the queries listed as wide range
// (fp32, bf16); a no-op when none is listed
hipError_t launch_score_wide(const DevIndex& ix, const DevBatch& qb, int32_t q0, const Workspace& ws, hipStream_t s);
hipError_t launch_score_atomic(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                               const ScoreOpts& o, const Workspace& ws, hipStream_t s);
hipError_t launch_score_docpar(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                               const ScoreOpts& o, const Workspace& ws, hipStream_t s);
hipError_t launch_hist1(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                        const Workspace& ws, hipStream_t s);
// ---- gs_noalloc.hip ----
// Device address of `device`'s copy of the fixed scratch array (kScratchBytes), looked up
// once per device with that device current (the caller makes it current).
hipError_t scratch_address(int device, void** out);

// ---- launchers (gs_yardstick.hip) ----
hipError_t launch_copy16(void* dst, const void* src, int64_t n16, hipStream_t s);
// LDS atomic-add throughput: op 0 uint32, 1 uint64, 2 float, 3 double; pattern 0 scattered, 1 consecutive
hipError_t launch_lds_atomic(int op, int pattern, int workgroups, int iters, void* sink, hipStream_t s);
hipError_t launch_fill(void* p, int64_t n_words, uint32_t v, hipStream_t s);  // p[0..n) = v (a kernel, capturable)

// ---- launchers (gs_topk.hip) ----
// Accumulation behind the scores: fixed point (doc-tiled kernels, fp32 and bf16 weights:
// absolute error bound, wide-range check), float (global-atomic and document-parallel
// kernels: relative error bound) or integer (uint8 impacts: exact).
enum AccKind { kAccFixed = 0, kAccFloat = 1, kAccInteger = 2 };
// Between the two k_select_first passes, the rows of the listed queries are scored again:
// with phase3 (non-null) the fused fp32 / uint8 queries that fell back (phase 3 of
// launch_score_tiled with these options), with wide the wide-range queries (fp64 pass).
hipError_t launch_select(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                         const Workspace& ws, int32_t* out_ids, void* out_scores, int32_t* diag,
                         hipStream_t s, int acc, int tile_shift = 0, int seed_stride = 0,
                         const ScoreOpts* phase3 = nullptr, bool wide = false);
// fused filtering: the bound of every query of the tile from its seed-tile histogram
hipError_t launch_seed_bound(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt,
                             const Workspace& ws, hipStream_t s, int tile_shift, int stride);

}  // namespace gs
