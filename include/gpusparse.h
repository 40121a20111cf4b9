/*
 * gpusparse.h - exact learned-sparse retrieval on one MI355X (gfx950).
 *
 * C ABI of libgpusparse.so. What it computes is the paper's scoring method
 * (GPUSparse, "GPU-Accelerated Learned Sparse Retrieval with Parallel Inverted
 * Indices"):
 *
 *   score(q, d) = sum over the query's terms t of w_q(t) * w_d(t)      (Sec. 2.1; Sec. 4.1, first eq.)
 *
 * evaluated for every document through a term-major inverted index (Sec. 3.2)
 * by scatter-adding w_q(t) * w_d(t) into one score array per query
 * (Sec. 4.1, second eq.; Sec. 4.2), followed by an exact per-query top-k.
 * Nothing is pruned (Sec. 4.3).
 *
 * Conventions for every entry point:
 *  - Return value: GS_OK (0) or a negative gs_status. On error no output
 *    buffer is written and gs_last_error() holds a message for the calling
 *    thread.
 *  - "host" pointers are read during the call only and stay owned by the
 *    caller. "device" pointers are HIP device memory owned by the caller
 *    (for example torch tensors); the library never frees them.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the legacy default
 *    stream). Device work is enqueued on it; calls documented as
 *    "asynchronous" return before the device finishes.
 *  - Ranking order: score descending, then doc id ascending. Row q of a
 *    result holds min(k[q], n_docs) entries; the remaining slots up to k_max
 *    are id -1 with score 0. Documents sharing no term with the query have
 *    score 0 and are ranked like any other document.
 */
#ifndef GPUSPARSE_H
#define GPUSPARSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_index_s* gs_index;
typedef struct gs_batch_s* gs_batch;

enum gs_status {
    GS_OK = 0,
    GS_EINVAL = -1,       /* malformed input (see each call) */
    GS_ENOMEM = -2,       /* host or device allocation failed */
    GS_EHIP = -3,         /* a HIP runtime call failed */
    GS_ECAPACITY = -4,    /* workspace or output too small */
    GS_EUNSUPPORTED = -5, /* option not available for this index */
    GS_ETIMEOUT = -6      /* gs_server_wait: the request has not finished in time */
};

/* Posting-weight storage (the paper stores fp32, Sec. 3.1; compressed
 * posting scores are its future work (2), Sec. 8). */
enum gs_precision {
    GS_FP32 = 0, /* fp32 weights; scores are float, each within 1e-5 relative of the
                    exact score. The doc-tiled kernels sum products in 64-bit fixed
                    point (one scale per query: absolute error about 2^-51 of the
                    query's largest product, times its term count); a query whose
                    k-th score is too small for that error to stay within 2^-18 of
                    it is summed again with fp64 accumulation of exact fp64 products */
    GS_BF16 = 1, /* bf16 weights (round to nearest even); approximate scores from
                    32-bit fixed-point sums (per-query scale bounding every doc's
                    sum below 2^32 units; the same wide-range check with 2^-12), then
                    fp64 rescoring of every candidate within the bf16 error band of
                    the k-th score from the fp32 forward rows; scores are double and
                    equal the fp64 sum over shared terms in ascending term order */
    GS_U8 = 2    /* uint8 impacts q8(w) = round(w*255/3) (ties to even, saturated
                    at 255) for document and query weights, exact int32
                    accumulation; scores are int32 */
};

enum gs_build_flags {
    GS_KEEP_FORWARD = 1, /* keep the fp32 doc-major rows on the device (needed by the
                            document-parallel kernel; always kept for GS_BF16) */
    GS_KEEP_DOC_IDS = 2  /* keep 32-bit doc ids of every posting on the device (needed by
                            the global-atomic kernel only: the doc-tiled kernels read
                            16-bit or 8-bit ids, so by default they are not uploaded) */
};

/* Scoring kernels (Sec. 5.2 term-parallel scatter-add; Sec. 5.3 document-parallel). */
enum gs_kernel {
    GS_KERNEL_AUTO = 0,   /* library choice */
    GS_KERNEL_TILED = 1,  /* term-parallel, per (query, doc tile): posting segments
                             scatter-added into an LDS tile, one coalesced write per doc */
    GS_KERNEL_ATOMIC = 2, /* term-parallel, per (query, term, posting chunk): global
                             atomics into the score array (the paper's Sec. 5.2 form) */
    GS_KERNEL_DOCPAR = 3, /* document-parallel: per (query, doc) gather over the
                             forward rows, no atomics (Sec. 5.3); needs GS_KEEP_FORWARD */
    GS_KERNEL_SHARED = 4, /* batched shared traversal: the TILED work items on a
                             persistent grid, taken tile by tile (every query of a
                             doc tile on one XCD, longest queries first), so a
                             tile's posting segments are read from HBM once and
                             from that XCD's L2 for the other queries holding them */
    GS_KERNEL_GROUP = 5   /* batched shared traversal with explicit sharing: per (doc tile
                             of 8192, group of 2 queries), the segments of
                             the union of the group's terms; each posting chunk is loaded
                             once and added into the LDS tile of every query of the group
                             holding its term. Tile 8192 and chunks of 256-1024 only
                             (GS_EUNSUPPORTED otherwise); a search whose workspace holds
                             fewer than all its queries runs GS_KERNEL_SHARED instead */
};

#define GS_MAX_K 4096        /* largest k per query */
#define GS_MAX_QUERY_NNZ 256  /* largest number of terms in one query */

typedef struct gs_search_opts {
    int32_t kernel;      /* gs_kernel */
    int32_t query_tile;  /* most queries whose score arrays are live at once
                            (0 = as many as the workspace holds) */
    int32_t tile_docs;   /* doc tile of the TILED/SHARED kernels: 0 (default),
                            8192, 16384 or 32768 (32768: not for GS_FP32,
                            GS_EUNSUPPORTED) */
    int32_t chunk;       /* postings per work item (TILED/ATOMIC): 0 (default),
                            64, 128, 256, 512 or 1024 */
    int32_t no_fused_filter; /* TILED/SHARED, searches of 32+ queries: 0 (default)
                                appends candidates while scoring (a bound from every
                                8th doc tile, then only those tiles' scores are
                                scanned and, for fp32 and uint8, written); 1 writes
                                and scans every score row */
    int32_t prune;       /* 1: exact block-max pruning in the non-seed tiles (Sec. 5.3 leaves
                            GPU pruning aside; built here as an option). Needs GS_KERNEL_TILED,
                            GS_FP32 or GS_U8, the default tile, chunk 1024 (else
                            GS_EUNSUPPORTED) and fused filtering (a search of 32+ queries,
                            k <= 2048; otherwise nothing is pruned). Per query, the terms
                            whose upper bounds (w_q times the term's largest weight) sum below
                            the seed bound's score are non-essential; after the others are
                            scored, each 64-posting block of a non-essential term is skipped
                            unread when no doc it can hold can reach the bound. The results
                            are the same as without it, bit for bit */
    int32_t reserved[2]; /* must be 0 */
} gs_search_opts;

typedef struct gs_index_info_t {
    int64_t n_docs;
    int64_t nnz;          /* real postings */
    int64_t padded_nnz;   /* postings after padding each list to a multiple of 64 */
    int64_t device_bytes; /* device memory held by the index */
    int32_t vocab_size;
    int32_t precision;    /* gs_precision */
    uint32_t flags;       /* gs_build_flags in effect */
    int32_t tile_grain;   /* doc-tile granularity of the segment table (docs) */
    int64_t n_tiles;      /* tiles of tile_grain docs covering the collection */
    int64_t n_dense_terms; /* terms whose every 64-posting block spans at most 256 docs:
                              the doc-tiled kernels read their doc ids as one byte per
                              posting (distance to the block's first doc) */
} gs_index_info_t;

/* ------------------------------------------------------------------ misc -- */

const char* gs_version(void);
const char* gs_status_string(int32_t status);
/* Message of the last failing call on this thread ("" if none). */
const char* gs_last_error(void);

/* Test hook (fault injection, not for production use): after n more device or pinned
 * host allocations made by the library, the next one fails as out of memory, once;
 * n < 0 disarms it. Process-wide. Lets tests check the GS_ENOMEM paths (no leaks,
 * no partial objects). Always returns GS_OK. */
int32_t gs_debug_fail_alloc(int64_t n);

/* ------------------------------------------------------------ index build -- */

/*
 * Build the GPU-resident inverted index (paper Sec. 3.2) from a doc-major CSR.
 *
 * row_ptr [n_docs+1] (host, int64): row_ptr[0] = 0, non-decreasing, row_ptr[n_docs] = nnz.
 * term_ids [nnz] (host, int32): term of each entry, in [0, vocab_size); no term
 *     twice in one row; rows need not be sorted.
 * weights [nnz] (host, float): finite and >= 0 (learned sparse weights are
 *     non-negative, Sec. 2.1).
 * precision: gs_precision. flags: gs_build_flags.
 *
 * Layout built (all device-resident, owned by the index):
 *  - posting lists term-major, each sorted by doc id (Sec. 3.2), padded with
 *    (doc -1, weight 0) entries to a multiple of 64 (one wavefront); their
 *    32-bit doc ids only with GS_KEEP_DOC_IDS;
 *  - term_off[V+1] (int64) list starts, term_len[V] real lengths;
 *  - per 64-posting block: the largest weight and the first doc id;
 *  - per term and per tile of tile_grain docs: the offset of the first
 *    posting at or after the tile start (segment table for doc-tiled kernels);
 *  - doc ids again as 16-bit values (doc id modulo 65536), and, for the lists
 *    whose every 64-posting block spans at most 256 docs ("dense" terms), as
 *    one byte per posting: the distance to the block's first doc. The
 *    doc-tiled kernels read 2 or 1 bytes per posting for the id instead of 4.
 * Synchronous: returns once the index is on the device.
 * Errors: GS_EINVAL (any check above, vocab_size < 1, n_docs < 0,
 *   n_docs >= 2^31, unknown precision or flag), GS_ENOMEM, GS_EHIP.
 */
int32_t gs_build_index(const int64_t* row_ptr, int64_t n_docs, const int32_t* term_ids,
                       const float* weights, int64_t nnz, int32_t vocab_size, int32_t precision,
                       uint32_t flags, void* hip_stream, gs_index* out);

/* Sizes of a built index (Sec. 3.2 arrays; device memory as in Sec. 3.3's
 * memory model plus the segment table and block metadata). out (host,
 * caller-owned) receives them. Errors: GS_EINVAL (null argument). */
int32_t gs_index_info(gs_index index, gs_index_info_t* out);

/*
 * Byte-form flags of the index's terms (see n_dense_terms): out [vocab_size]
 * (host, caller-owned) receives 1 for a term whose every 64-posting block spans at
 * most 256 docs, else 0. For measurement: the doc-tiled kernels with fp32 or bf16
 * weights read such a term's doc ids as 1 byte per posting plus one 4-byte block
 * base per 64 postings. Errors: GS_EINVAL (null argument, vocab_size differs from
 * the index's).
 */
int32_t gs_index_dense_terms(gs_index index, uint8_t* out, int32_t vocab_size);
/* Releases the index's device memory (the resident index of Sec. 3.2). NULL is a
 * no-op. Batches created for it may still be freed afterwards, not searched. */
void gs_free_index(gs_index index);

/*
 * Host-only form of the posting layout gs_build_index puts on the device
 * (same code path), for inspection and tests. Call first with
 * out_padded_nnz != NULL and every array NULL to get the sizes, then again
 * with caller-allocated arrays:
 *   term_off [vocab_size+1] int64, term_len [vocab_size] int32,
 *   post_doc [padded_nnz] int32, post_w [padded_nnz] float (the stored weight
 *   converted back to float: fp32 as is, bf16 widened, uint8 as its integer),
 *   blk_max [padded_nnz/64] float, blk_first_doc [padded_nnz/64] int32,
 *   term_dense [vocab_size] uint8 (1 for a term whose every 64-posting block
 *   spans at most 256 docs), post_b8 [padded_nnz] uint8 (for those terms' real
 *   postings: doc id minus the block's first doc id; 0 elsewhere).
 * Any array may be NULL. Errors as gs_build_index.
 */
int32_t gs_layout_host(const int64_t* row_ptr, int64_t n_docs, const int32_t* term_ids,
                       const float* weights, int64_t nnz, int32_t vocab_size, int32_t precision,
                       int64_t* out_padded_nnz, int64_t* term_off, int32_t* term_len,
                       int32_t* post_doc, float* post_w, float* blk_max, int32_t* blk_first_doc,
                       uint8_t* term_dense, uint8_t* post_b8);

/*
 * Host-only form of the per-query fixed-point plan that gs_batch_create computes
 * (same code), for inspection and tests. The scatter-add of Sec. 4.1 (second
 * eq.) is done in integers: each product w_q(t) * w_d(t) is rounded to units of
 * 2^-F and the units are summed exactly.
 * precision: GS_FP32 (64-bit sums: every product of the query below 2^51 units)
 *   or GS_BF16 (32-bit sums: every document's sum below 2^32 units).
 * q_weights [nnz], term_max [nnz], term_min [nnz] (host): per query term, its
 *   weight, the largest stored weight of its posting list and the smallest
 *   positive one (+inf if the list has none).
 * out_F: the scale exponent. out_abs_err: bound on |fixed-point score - exact
 *   score| for every document. out_wide_lim: the search sums the query again in
 *   fp64 when its k-th approximate score may lie below this value (out_abs_err
 *   over 2^-18 for fp32, 2^-12 for bf16); 0 when every positive score (at least
 *   the smallest positive product) clears it. Any output may be NULL.
 * Errors: GS_EINVAL (precision, nnz outside [0, GS_MAX_QUERY_NNZ], negative or
 *   non-finite weights, term_min not positive).
 */
int32_t gs_query_plan_host(int32_t precision, const float* q_weights, const float* term_max, const float* term_min,
                           int32_t nnz, int32_t* out_F, double* out_abs_err, double* out_wide_lim);

/* --------------------------------------------------------- query batches -- */

/*
 * Validate a CSR batch of queries and copy it to the device (owned by the batch).
 * q_row_ptr [n_queries+1] (host, int64), q_term_ids / q_weights [q_nnz] (host),
 * k [n_queries] (host, int32) with 0 <= k[q] <= k_max <= GS_MAX_K.
 * Query rows follow the same rules as document rows (terms in range, no
 * duplicates, finite non-negative weights, at most GS_MAX_QUERY_NNZ terms).
 * Synchronous. Errors: GS_EINVAL, GS_ENOMEM, GS_EHIP.
 */
int32_t gs_batch_create(gs_index index, const int64_t* q_row_ptr, int32_t n_queries,
                        const int32_t* q_term_ids, const float* q_weights, int64_t q_nnz,
                        const int32_t* k, int32_t k_max, void* hip_stream, gs_batch* out);
/* Frees a batch (also after its index was freed). A batch may only be searched
 * while the index it was created for is alive. */
void gs_batch_free(gs_batch batch);

/*
 * A batch with fixed capacity, for reuse across searches (hipGraph replays,
 * serving slots): room for max_queries queries holding max_nnz terms in total,
 * k <= k_max. Until filled, every slot is an empty query with k = 0.
 * Errors: GS_EINVAL, GS_ENOMEM, GS_EHIP.
 */
int32_t gs_batch_reserve(gs_index index, int32_t max_queries, int64_t max_nnz, int32_t k_max,
                         gs_batch* out);

/*
 * Replace the queries of a batch in place (same rules as gs_batch_create),
 * n_queries <= capacity, q_nnz <= capacity. Slots n_queries..capacity-1 become
 * empty queries with k = 0: no scoring work, their result rows are padding.
 * Waits for work already enqueued on hip_stream (which may read the batch),
 * then copies synchronously. Launch shapes depend only on the capacity, so a
 * graph made by gs_graph_create keeps working after an update.
 * Errors: GS_EINVAL (nothing is changed), GS_EHIP.
 */
int32_t gs_batch_update(gs_batch batch, const int64_t* q_row_ptr, int32_t n_queries,
                        const int32_t* q_term_ids, const float* q_weights, int64_t q_nnz,
                        const int32_t* k, void* hip_stream);

/*
 * Device workspace (bytes) for a search of a batch of n_queries queries with
 * q_nnz terms in total and k <= k_max: one score array of n_docs 32-bit words
 * per live query (Sec. 4.2's per-query accumulators) plus selection scratch,
 * for all n_queries at once, or for opts->query_tile of them when that is set
 * (opts may be NULL). A smaller workspace still works down to
 * gs_workspace_size(index, 1, opts): queries then run in tiles (score arrays
 * tiled to fit memory). Errors: GS_EINVAL (negative sizes, k_max outside
 * [0, GS_MAX_K], q_nnz above n_queries x GS_MAX_QUERY_NNZ, bad opts),
 * GS_EUNSUPPORTED (as gs_search_batch).
 */
int32_t gs_search_workspace_size(gs_index index, int32_t n_queries, int64_t q_nnz, int32_t k_max,
                                 const gs_search_opts* opts, size_t* bytes);

/*
 * Device workspace (bytes) needed to search query_tile queries at once with
 * these options (opts may be NULL). It holds one score array of n_docs 32-bit
 * words per live query plus selection scratch.
 */
int32_t gs_workspace_size(gs_index index, int32_t query_tile, const gs_search_opts* opts,
                          size_t* bytes);

/*
 * Search a prepared batch: exact top-k per query. Scores are the inner product
 * of Sec. 2.1 over the query's terms, accumulated per query as in Sec. 4.1
 * (second eq.) and Sec. 4.2; the top-k is exact (Sec. 4.3).
 * workspace: device, workspace_bytes >= gs_workspace_size(index, 1, opts);
 *   queries are processed in tiles of as many as the workspace holds
 *   (score arrays tiled to fit memory).
 * out_ids [n_queries * k_max] (device, int32).
 * out_scores [n_queries * k_max] (device): float for GS_FP32, double for
 *   GS_BF16, int32 for GS_U8.
 * Asynchronous on hip_stream. The index and batch are only read, so searches
 * with separate workspaces and outputs may run concurrently on different streams.
 * Errors: GS_EINVAL (NULL arguments, bad opts), GS_ECAPACITY (workspace too
 *   small), GS_EUNSUPPORTED (kernel not available for this index), GS_EHIP.
 */
int32_t gs_search_batch(gs_index index, gs_batch batch, void* workspace, size_t workspace_bytes,
                        int32_t* out_ids, void* out_scores, const gs_search_opts* opts,
                        void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): gs_search_batch with
 * the library's fixed scratch array as the workspace. It calls no hipMalloc,
 * hipFree or other allocating routine. The array is 128 MiB per GPU, held from
 * the first call on that GPU until the process ends; queries are processed in
 * tiles of as many as fit in it (at 8.8M documents: 3 at a time). Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and give undefined results. Calls on one stream
 * are ordered and safe. Arguments, outputs and asynchrony as gs_search_batch.
 * Errors: GS_ECAPACITY (a one-query workspace of this index exceeds 128 MiB:
 * collections above about 33M documents), GS_EINVAL, GS_EUNSUPPORTED, GS_EHIP.
 */
int32_t gs_search_batch_noalloc(gs_index index, gs_batch batch, int32_t* out_ids, void* out_scores,
                                const gs_search_opts* opts, void* hip_stream);

/*
 * Convenience form (the search of Sec. 4.2 from a host CSR of queries):
 * gs_batch_create + gs_search_batch + gs_batch_free.
 * Synchronous (the stream is synchronised before returning). Returns
 * GS_ECAPACITY when the fp64-rescored error band of some query (GS_BF16) held
 * more than 32768 documents: that query's row is then padding (see
 * gs_batch_diagnostics); the other rows are valid.
 */
int32_t gs_search(gs_index index, const int64_t* q_row_ptr, int32_t n_queries,
                  const int32_t* q_term_ids, const float* q_weights, int64_t q_nnz,
                  const int32_t* k, int32_t k_max, void* workspace, size_t workspace_bytes,
                  int32_t* out_ids, void* out_scores, const gs_search_opts* opts,
                  void* hip_stream);

/*
 * hipGraph form of gs_search_batch: the full launch sequence for this batch
 * (at its capacity), workspace and outputs is run once on hip_stream and then
 * captured into a graph; gs_graph_launch replays it on any stream. The graph
 * holds the pointers given here (the batch included): they must stay valid,
 * and the batch may be refilled with gs_batch_update between launches. No
 * memset or host work is captured (buffers are cleared by kernels). The
 * fixed-point kernels come in two forms, with and without the raise of a
 * positive product that rounds to 0 units; the graph captures the form the
 * batch needs at capture time, and a launch after a refill that needs the
 * other form enqueues the same search directly instead (same results).
 * Errors: as gs_search_batch, plus GS_EHIP for capture or instantiation
 * failures.
 */
typedef struct gs_graph_s* gs_graph;
int32_t gs_graph_create(gs_index index, gs_batch batch, void* workspace, size_t workspace_bytes,
                        int32_t* out_ids, void* out_scores, const gs_search_opts* opts,
                        void* hip_stream, gs_graph* out);
int32_t gs_graph_launch(gs_graph graph, void* hip_stream);
void gs_graph_free(gs_graph graph);

/*
 * Autotuner: runs this batch with every candidate option set - scoring kernel
 * (GS_KERNEL_TILED, GS_KERNEL_SHARED) x tile_docs (8192, 16384; plus 32768 for
 * GS_BF16 and GS_U8) x chunk (128, 256, 512, 1024) - one untimed run then `reps` timed runs
 * each (HIP events on hip_stream), and writes the fastest option set to *best.
 * Optional host outputs: cands[max_candidates] (the option sets tried, in
 * order), times_ms[max_candidates] (mean search time of each), n_candidates.
 * Synchronous; overwrites out_ids / out_scores. Errors: as gs_search_batch.
 */
int32_t gs_autotune(gs_index index, gs_batch batch, void* workspace, size_t workspace_bytes,
                    int32_t* out_ids, void* out_scores, int32_t reps, void* hip_stream,
                    gs_search_opts* best, gs_search_opts* cands, float* times_ms,
                    int32_t max_candidates, int32_t* n_candidates);

/*
 * Per-query selection diagnostics of the last gs_search_batch on this batch
 * (host copy; call after the stream has been synchronised).
 * out [n_queries * 8] int32 (host, caller-owned), per query:
 *   [0] candidates kept by the filter (with fused filtering: those appended
 *       while scoring plus the seed tiles');
 *   [1] refinement passes over the score array;
 *   [2] bf16 band size (0 for other precisions);
 *   [3] overflow flag: 1 if more than 32768 documents lay inside the bf16 error
 *       band of the k-th score (only when a huge number of documents tie
 *       within that band). The buffer size is fixed, so the row is padding
 *       (ids -1) and no workspace size avoids it; gs_search and the server
 *       report GS_ECAPACITY for it;
 *   [4] rows scored again: 0 no, 1 fallback of fused candidate filtering,
 *       2 wide range (fixed-point error too large for the k-th score: every
 *       tile summed again in fp64), 3 (GS_BF16) the error band reached below
 *       the fused candidates: the other tiles' rows scored for the band pass;
 *   [5] 1 if fused candidate filtering produced the candidates;
 *   [6] 64-posting blocks skipped by pruning (opts.prune);
 *   [7] 0.
 */
int32_t gs_batch_diagnostics(gs_batch batch, int32_t* out);

/*
 * Kernel timing for measurement. While enabled (on != 0), gs_search_batch
 * records a HIP event pair on its stream around every scoring launch and
 * around every selection (top-k) sequence. With fused candidate filtering a
 * scoring pass is two launches (seed tiles, then the rest), timed apart and
 * counted as one; the seed bound between them is selection time.
 * gs_timing_read synchronises those events, returns the summed milliseconds
 * and launch counts since the previous read (any output pointer may be NULL)
 * and releases the events.
 * Process-wide; thread-safe. Errors: GS_EHIP.
 */
int32_t gs_timing_enable(int32_t on);
int32_t gs_timing_read(double* score_ms, int64_t* score_launches, double* select_ms,
                       int64_t* select_launches);

/*
 * Plain device-to-device copy of `bytes` (a multiple of 16; both pointers
 * 16-byte aligned) with 16-byte vector loads and stores: the yardstick that
 * hardware traffic counters are calibrated against (it moves exactly `bytes`
 * in each direction). Asynchronous. Errors: GS_EINVAL, GS_EHIP.
 */
int32_t gs_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/*
 * LDS atomic-add throughput yardstick. The doc-tiled kernels scatter-add one
 * product per posting into an LDS copy of a doc tile (the on-chip accumulation
 * the paper leaves to future work (1), Sec. 8); the accumulator type is chosen
 * by these rates. `workgroups` workgroups of 512 lanes each issue `iters`
 * no-return atomic adds (iters a positive multiple of 16) into a 64 KiB LDS
 * array. op: 0 uint32, 1 uint64, 2 float, 3 double. pattern: 0 scattered
 * addresses (a per-lane pseudo-random sequence, as postings of many terms land
 * in a tile), 1 consecutive words across each wavefront. sink (device, at least
 * workgroups x 8 bytes) receives one value per workgroup. *lane_ops (may be
 * NULL) receives workgroups x 512 x iters. Asynchronous on hip_stream; time it
 * with events on that stream. Errors: GS_EINVAL, GS_EHIP.
 */
int32_t gs_lds_atomic_probe(int32_t op, int32_t pattern, int32_t workgroups, int32_t iters, void* sink,
                            void* hip_stream, int64_t* lane_ops);

/* ------------------------------------------------------------- serving -- */

/*
 * Continuous-batching request loop over one resident index (the paper lists
 * streaming query batching for serving as future work (3), Sec. 8).
 * Requests queue as they arrive. Admission is by memory: the server holds one
 * workspace arena of query rows (a row: the n_docs x 4 B score array of one
 * query plus its selection scratch, the memory a query's score buffer needs),
 * as many rows as memory_budget allows (without a budget, n_slots x max_batch).
 * A scheduler thread owns n_slots slots, each with its own HIP stream, a
 * reusable batch of max_batch queries and pinned result rows. Whenever a slot
 * is free and requests wait, it takes a contiguous run of free rows and as many
 * waiting requests (oldest first, at most max_batch) and runs their search while
 * other slots keep running; the rows return to the arena when the step ends. So
 * requests that arrive while others are on the GPU are admitted as slots and
 * memory free up, and at most arena_rows queries are on the device at once.
 * Results are identical to a search of the same query alone (the integer and
 * fixed-point sums do not depend on the batch).
 */
typedef struct gs_server_s* gs_server;

typedef struct gs_server_opts {
    int32_t max_batch;     /* most queries in one device step */
    int32_t n_slots;       /* concurrent device steps (streams) */
    int32_t k_max;         /* largest k a request may ask for (<= GS_MAX_K) */
    int32_t reserved;      /* must be 0 */
    int64_t memory_budget; /* device bytes for the in-flight queries' rows (0: n_slots x max_batch rows) */
    gs_search_opts search; /* kernel options used for every step */
} gs_server_opts;

typedef struct gs_server_stats_t {
    int32_t n_slots;
    int32_t max_batch;
    int64_t completed;     /* requests finished with results */
    int64_t failed;        /* requests finished with an error status */
    int64_t device_steps;  /* searches run */
    double mean_batch;     /* requests per search */
    int64_t max_in_flight; /* most requests on the device at once (at most arena_rows) */
    int64_t pending;       /* requests waiting for a slot or rows now */
    int64_t arena_rows;    /* queries whose rows fit the budget at once */
    int64_t arena_bytes;   /* device bytes of the arena */
    int64_t row_bytes;     /* arena bytes per query row */
} gs_server_stats_t;

/* Allocates the arena and every slot up front (device and pinned memory) and
 * starts the scheduler. Errors: GS_EINVAL, GS_ECAPACITY (budget below one
 * query's row), GS_ENOMEM, GS_EHIP. */
int32_t gs_server_create(gs_index index, const gs_server_opts* opts, gs_server* out);

/* Queue one query (host arrays, copied). Returns a ticket >= 0, or a negative
 * gs_status (GS_EINVAL: bad term, weight, duplicate, nnz > GS_MAX_QUERY_NNZ,
 * k outside [0, k_max], server stopping). Thread-safe. */
int64_t gs_server_submit(gs_server server, const int32_t* term_ids, const float* weights, int32_t nnz,
                         int32_t k);

/* Wait for a ticket (timeout_ms < 0: no limit), then copy its k ids and scores
 * (host, caller-owned: k int32 ids; k floats, doubles for GS_BF16, int32 for
 * GS_U8) and give its latency from submission to completion in ms (any output
 * may be NULL). Each ticket is collected once. Thread-safe. Errors: GS_EINVAL
 * (unknown ticket, already collected, or the server was destroyed first),
 * GS_ETIMEOUT (not finished in time; the ticket stays collectable), or the
 * status of its failed search (GS_ECAPACITY: a bf16 band overflow). */
int32_t gs_server_wait(gs_server server, int64_t ticket, int32_t timeout_ms, int32_t* out_ids,
                       void* out_scores, double* latency_ms);

/* Non-blocking form of gs_server_wait: GS_OK and the result if the request has
 * finished, GS_ETIMEOUT if it has not (the ticket stays collectable). */
int32_t gs_server_poll(gs_server server, int64_t ticket, int32_t* out_ids, void* out_scores,
                       double* latency_ms);

int32_t gs_server_stats(gs_server server, gs_server_stats_t* out);

/* Stops the scheduler after the steps on the device finish; requests still
 * waiting for a slot are dropped, and callers blocked in gs_server_wait return
 * GS_EINVAL before the server is freed. */
void gs_server_destroy(gs_server server);

#ifdef __cplusplus
}
#endif

#endif /* GPUSPARSE_H */
