// Scoring kernels: fill one score array per query with
//   S[q][d] = sum over the query's terms t of w_q(t) * w_d(t)
// (paper Sec. 4.1: the score decomposes into one scatter-add per query term).
//
// Forms:
//  * k_score_tiled  - term-parallel, work = (query, doc tile). Each query term's
//    posting list is doc-sorted, so the postings that fall into a doc tile are
//    one contiguous segment (found in the per-term segment table). The
//    workgroup streams every segment of its query through coalesced loads and
//    scatter-adds w_q * w_d into an LDS copy of the tile with LDS atomics, then
//    writes the tile once (coalesced) and builds the histogram of the first
//    selection digit. No global atomics, no zeroing pass. This is the hybrid
//    of scatter-add and on-chip accumulation listed as future work (1) in Sec. 8.
//  * k_score_persistent - the same work items on a resident grid, taken tile by
//    tile (all queries of a tile on one XCD while its postings sit in that L2):
//    the shared traversal of a batch.
//  * k_score_atomic - term-parallel, work = (query, term, chunk of postings);
//    global atomic adds into a zeroed score array, as in the paper's Sec. 5.2
//    kernel (one program per query term looping over posting chunks), with
//    long lists split into chunks so that head terms do not serialise.
//  * k_score_docpar - document-parallel (Sec. 5.3): per (query, doc) a gather
//    over the doc's forward row with the query's weights in a dense LDS table;
//    each output cell is written once, no atomics.
//
// Weight forms of the doc-tiled kernels: fp32 (products rounded to units of a
// per-query scale and summed exactly in 64-bit fixed point), bf16 (stored as the
// upper 16 bits of the fp32 pattern; 32-bit fixed point, then fp64 rescoring of
// the candidates) and uint8 impacts (int32 products and sums, exact). Doc ids are
// read as 16-bit offsets, or, for dense terms in k_score_tiled with fp32 and bf16
// weights, as one byte per posting from the 64-block's first doc. With fused
// candidate filtering a search runs them in phases: the seed tiles, then the
// other tiles appending candidates at or above a bound while they flush, then a
// pass that writes the rows of the queries that fell back (k_score_listed; see
// gs_topk.hip).
#include <algorithm>
#include <type_traits>

#include "gs_internal.h"

namespace gs {

namespace {

template <int P> struct WF;
template <> struct WF<kFP32> {
    using Acc = float;
    static __device__ __forceinline__ float load(const void* p, int64_t i) { return ((const float*)p)[i]; }
    static __device__ __forceinline__ float from_fp32(float w) { return w; }
    static __device__ __forceinline__ float qweight(const DevBatch& qb, int64_t j) { return qb.q_w[j]; }
    static __device__ __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
};
template <> struct WF<kBF16> {
    using Acc = float;
    static __device__ __forceinline__ float load(const void* p, int64_t i) {
        return __uint_as_float((uint32_t)((const uint16_t*)p)[i] << 16);
    }
    static __device__ __forceinline__ float from_fp32(float w) {
        // round to nearest even on the upper 16 bits (weights are finite and >= 0)
        uint32_t u = __float_as_uint(w);
        u += 0x7fffu + ((u >> 16) & 1u);
        return __uint_as_float(u & 0xffff0000u);
    }
    static __device__ __forceinline__ float qweight(const DevBatch& qb, int64_t j) { return qb.q_w[j]; }
    static __device__ __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
};
template <> struct WF<kU8> {
    using Acc = int;
    static __device__ __forceinline__ int load(const void* p, int64_t i) { return ((const uint8_t*)p)[i]; }
    static __device__ __forceinline__ int from_fp32(float w) {
        double x = __builtin_rint((double)w * 85.0);
        return x > 255.0 ? 255 : (x > 0.0 ? (int)x : 0);
    }
    static __device__ __forceinline__ int qweight(const DevBatch& qb, int64_t j) { return qb.q_w8[j]; }
    static __device__ __forceinline__ uint32_t bits(int v) { return (uint32_t)v; }
};

// A wave-uniform double moved into scalar registers: the predicated per-posting
// blocks that use it then carry no wait on the LDS read that produced it.
__device__ __forceinline__ double uniform_f64(double v) {
    const long long b = __double_as_longlong(v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(b >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ unsigned long long comp_key(uint32_t key, uint32_t id) {
    return ((unsigned long long)key << 32) | (unsigned long long)(~id);
}

__device__ __forceinline__ void glb_add(uint32_t* a, float v) { unsafeAtomicAdd(reinterpret_cast<float*>(a), v); }
__device__ __forceinline__ void glb_add(uint32_t* a, int v) { atomicAdd(reinterpret_cast<int*>(a), v); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Fixed-point product of a query weight pre-scaled by 2^F (qd = w_q * 2^F, exact
// in fp64) and a stored document weight given by its fp32 bit pattern (bf16
// weights are widened first). One fp64 FMA forms qd * w_d + 2^52 with a single
// rounding; the per-query F keeps every product below 2^51, so the result lies in
// [2^52, 2^53) where the fp64 spacing is 1 and its low bits are the product
// rounded to the nearest integer (within half a unit of it). A product below half
// a unit becomes 0; the selection's wide-range check covers the queries where
// that could matter (their rows are summed again in fp64).
__device__ __forceinline__ unsigned long long fx_product(double qd, uint32_t wbits) {
    constexpr double kTwo52 = 4503599627370496.0;
    const double wd = (double)__uint_as_float(wbits);
    return (unsigned long long)__double_as_longlong(__builtin_fma(qd, wd, kTwo52)) - 0x4330000000000000ull;
}

__device__ __forceinline__ uint32_t stored_bits(const void* p, int64_t i, std::integral_constant<int, kFP32>) {
    return ((const uint32_t*)p)[i];
}
__device__ __forceinline__ uint32_t stored_bits(const void* p, int64_t i, std::integral_constant<int, kBF16>) {
    return (uint32_t)((const uint16_t*)p)[i] << 16;
}

// Write a finished LDS tile to the score array (fp32 bits or int32) and add its
// first-digit histogram (composite key (score bits, ~doc id), digit at fs).
// Accumulator forms: kAccInt (int32 sums, written as they are), kAccFx32 and
// kAccFx64 (unsigned fixed point in units of `scale`, written as fp32 bits), kAccF64
// (fp64 sums of exact fp64 products, the wide-range pass, written as fp32 bits).
enum AccForm { kAccInt = 0, kAccFx32 = 1, kAccFx64 = 2, kAccF64 = 3 };

// Fused candidate filtering: append the composites c >= bound of the lanes that
// take one to the query's candidate buffer (one atomic per wavefront; hits are
// rare once the bound is set). Past kFusedCap the query is flagged instead.
__device__ __forceinline__ void append_candidates(bool take, unsigned long long c, SelState* st,
                                                  unsigned long long* C) {
    const unsigned long long m = __ballot(take);
    if (m == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = __ffsll((long long)__ballot(1)) - 1;
    int slot = 0;
    if (lane == leader) {
        slot = atomicAdd(&st->n_cand, __popcll(m));
        if (slot + __popcll(m) > kFusedCap) st->fused_over = 1;
    }
    slot = __shfl(slot, leader, kWave) + __popcll(m & ((1ull << lane) - 1ull));
    if (take && slot < kFusedCap) C[slot] = c;
}

// write: store the scores in the row; count: add the tile to the first-digit histogram.
// Q: 0 for a plain tile (doc d in accumulator d); else a tile in quarters (doc d in
// accumulator (d % 4) * Q + d / 4, Q = tile size / 4), as the four-postings-per-lane loads of
// score_tile leave it.
// stg (optional): 2 + BS / 64 LDS words (a base, unused, and a count per wavefront) and an LDS
// stage of stage_cap entries. With it, a flush that appends stages its candidates, each
// wavefront in its own slice with its count in a scalar register (no LDS round trip per hit),
// and takes one range of the query's buffer for all of them at the end (one global atomic per
// tile instead of one per wavefront and hit, whose round trips otherwise hold up the tile's
// last wavefront); candidates past a wavefront's slice go to the buffer directly.
// TD: the tile's size in docs (0: not known here). With it, the scan's read-ahead rounds stay
// inside the tile by construction and are issued without a per-read guard.
template <int BS, int AF, int Q = 0, int TD = 0>
__device__ __forceinline__ void flush_tile(const void* acc_v, uint32_t* hist, int tile_n, int64_t base, uint32_t* Sq,
                                           int fs, double scale, uint32_t* hist_out, bool append,
                                           unsigned long long bound, SelState* st, unsigned long long* C,
                                           bool write, bool count, int* stg = nullptr,
                                           unsigned long long* stage = nullptr, int stage_cap = 0) {
    const int tid = threadIdx.x;
    const bool staged = stg != nullptr && append;
    constexpr int NWF = BS / kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int per_w = stage_cap / NWF;
    unsigned long long* my_stage = stage + wv * per_w;
    // The wavefront's staged candidates. Lanes that leave a scan loop early keep an old value,
    // so the count is always taken from the first active lane: every loop here keeps a prefix
    // of the lanes active, so that is lane 0, which takes part in every append.
    int w_cnt = 0;
    auto put = [&](bool take, unsigned long long c) {
        if (!staged) {
            append_candidates(take, c, st, C);
            return;
        }
        const unsigned long long m = __ballot(take);
        if (m == 0) return;
        const int wc = __builtin_amdgcn_readfirstlane(w_cnt);
        const int slot = wc + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (take && slot < per_w) my_stage[slot] = c;
        const int pc = __popcll(m);
        if (wc + pc > per_w) append_candidates(take && slot >= per_w, c, st, C);  // past the slice
        w_cnt = min(wc + pc, per_w);
    };
    auto drain = [&]() {
        if (!staged) return;
        const int wc = __builtin_amdgcn_readfirstlane(w_cnt);
        if ((tid & (kWave - 1)) == 0) stg[2 + wv] = wc;
        __syncthreads();
        int n = 0, off = 0;
#pragma unroll
        for (int w = 0; w < NWF; w++) {
            const int cw = stg[2 + w];
            off += w < wv ? cw : 0;
            n += cw;
        }
        if (n == 0) return;
        if (tid == 0) {
            const int b = atomicAdd(&st->n_cand, n);
            if (b + n > kFusedCap) st->fused_over = 1;
            stg[0] = b;
        }
        __syncthreads();
        const int b = stg[0] + off;
        for (int i = tid & (kWave - 1); i < wc; i += kWave)
            if (b + i < kFusedCap) C[b + i] = my_stage[i];
    };
    const int n4 = tile_n >> 2;
    auto at4 = [](int i, int j) { return Q ? j * Q + i : 4 * i + j; };   // doc 4 i + j
    auto at = [](int d) { return Q ? (d & 3) * Q + (d >> 2) : d; };
    if constexpr (AF == kAccFx64) {
        if (!write && !count) {
            // Only candidates matter (no row, no histogram). A doc whose float score
            // float(acc * scale) reaches the bound's score s_b has acc * scale >= s_b (1 - 2^-24),
            // and converting the sum to double loses at most 2^-53 more, so a sum below t_lo
            // (taken with margin) cannot reach the bound: test the raw sums first and convert
            // only where a wavefront holds a sum at or above t_lo.
            if (!append) return;
            const double sb = (double)__uint_as_float((uint32_t)(bound >> 32));
            const unsigned long long t_lo = (unsigned long long)fmax(0.0, floor(sb * (1.0 - 0x1p-22) / scale));
            const unsigned long long* acc = (const unsigned long long*)acc_v;
            // two rounds of reads issued before the first test (one LDS round trip per two); in a
            // tile of TD docs every round reads inside the tile (TD / 4 is a multiple of 2 BS), so
            // the reads need no guard (rounds past a short last tile's end are not tested)
            constexpr bool FULL = TD > 0 && (TD / 4) % (2 * BS) == 0;
            constexpr int R = 2;
            for (int i0 = tid; i0 < n4; i0 += R * BS) {
                unsigned long long a[R][4];
#pragma unroll
                for (int h = 0; h < R; h++) {
                    const int i = i0 + h * BS;
#pragma unroll
                    for (int j = 0; j < 4; j++) a[h][j] = (FULL || i < n4) ? acc[at4(i, j)] : 0ull;
                }
#pragma unroll
                for (int h = 0; h < R; h++) {
                    const int i = i0 + h * BS;
                    const unsigned long long m01 = a[h][0] > a[h][1] ? a[h][0] : a[h][1];
                    const unsigned long long m23 = a[h][2] > a[h][3] ? a[h][2] : a[h][3];
                    if (!__ballot(i < n4 && (m01 > m23 ? m01 : m23) >= t_lo)) continue;
                    const uint32_t d0 = (uint32_t)(base + 4 * i);
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t v = __float_as_uint((float)((double)a[h][j] * scale));
                        const unsigned long long c = comp_key(v, d0 + j);
                        put(i < n4 && c >= bound, c);
                    }
                }
            }
            for (int i = (n4 << 2) + tid; i < tile_n; i += BS) {
                const uint32_t v = __float_as_uint((float)((double)acc[at(i)] * scale));
                const unsigned long long c = comp_key(v, (uint32_t)(base + i));
                put(c >= bound, c);
            }
            drain();
            return;
        }
    }
    // docs 4 i .. 4 i + 3 with their scores v: row store, histogram, candidates
    auto emit = [&](int i, const uint32_t* v) {
        if (write) reinterpret_cast<uint4*>(Sq)[i] = make_uint4(v[0], v[1], v[2], v[3]);
        const uint32_t d0 = (uint32_t)(base + 4 * i);
        if (count) {
#pragma unroll
            for (int j = 0; j < 4; j++) atomicAdd(&hist[(comp_key(v[j], d0 + j) >> fs) & (kHistBins - 1)], 1u);
        }
        // a composite reaches the bound only if its score bits reach the bound's: one test
        // of the lane's largest score first, the exact per-document test only then
        if (append && __ballot(max(max(v[0], v[1]), max(v[2], v[3])) >= (uint32_t)(bound >> 32))) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const unsigned long long c = comp_key(v[j], d0 + j);
                put(c >= bound, c);
            }
        }
    };
    int i_first = 0;
    if constexpr (Q != 0 && (AF == kAccInt || AF == kAccFx32)) {
        // a tile in quarters: 16 docs 16 g .. 16 g + 15 per lane, one 16-byte read from each
        // quarter (word 4 g + m of quarter j is doc 16 g + 4 m + j); two rounds of reads issued
        // before the first test where a tile's Q / 4 groups are a multiple of 2 BS, else one.
        // Every round then reads inside the tile (no guard per read); a round past a short
        // last tile's end is read but not tested.
        const uint32_t* acc = (const uint32_t*)acc_v;
        const int n16 = tile_n >> 4;
        constexpr int IT = (Q / 4) % (2 * BS) == 0 ? 2 : 1;
        for (int g0 = tid; g0 < n16; g0 += IT * BS) {
            uint4 r[IT][4];
#pragma unroll
            for (int it = 0; it < IT; it++) {
                const int g = g0 + it * BS;
#pragma unroll
                for (int j = 0; j < 4; j++) r[it][j] = *reinterpret_cast<const uint4*>(acc + j * Q + 4 * g);
            }
#pragma unroll
            for (int it = 0; it < IT; it++) {
                const int g = g0 + it * BS;
                if (g >= n16) break;
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    uint32_t v[4];
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        v[j] = m == 0 ? r[it][j].x : m == 1 ? r[it][j].y : m == 2 ? r[it][j].z : r[it][j].w;
                    if constexpr (AF == kAccFx32) {
#pragma unroll
                        for (int j = 0; j < 4; j++) v[j] = __float_as_uint((float)((double)v[j] * scale));
                    }
                    emit(4 * g + m, v);
                }
            }
        }
        i_first = n16 * 4;
    }
    for (int i = i_first + tid; i < n4; i += BS) {
        uint32_t v[4];
        if constexpr (AF == kAccFx64) {
            const unsigned long long* acc = (const unsigned long long*)acc_v;
#pragma unroll
            for (int j = 0; j < 4; j++) v[j] = __float_as_uint((float)((double)acc[at4(i, j)] * scale));
        } else if constexpr (AF == kAccF64) {
            const double* acc = (const double*)acc_v;
#pragma unroll
            for (int j = 0; j < 4; j++) v[j] = __float_as_uint((float)acc[at4(i, j)]);
        } else if constexpr (Q != 0) {
            const uint32_t* acc = (const uint32_t*)acc_v;
#pragma unroll
            for (int j = 0; j < 4; j++) v[j] = acc[at4(i, j)];
            if constexpr (AF == kAccFx32) {
#pragma unroll
                for (int j = 0; j < 4; j++) v[j] = __float_as_uint((float)((double)v[j] * scale));
            }
        } else {
            const uint4 u = reinterpret_cast<const uint4*>(acc_v)[i];
            v[0] = u.x; v[1] = u.y; v[2] = u.z; v[3] = u.w;
            if constexpr (AF == kAccFx32) {
#pragma unroll
                for (int j = 0; j < 4; j++) v[j] = __float_as_uint((float)((double)v[j] * scale));
            }
        }
        emit(i, v);
    }
    for (int i = (n4 << 2) + tid; i < tile_n; i += BS) {
        uint32_t v;
        const int ai = at(i);
        if constexpr (AF == kAccFx64) v = __float_as_uint((float)((double)((const unsigned long long*)acc_v)[ai] * scale));
        else if constexpr (AF == kAccF64) v = __float_as_uint((float)((const double*)acc_v)[ai]);
        else if constexpr (AF == kAccFx32) v = __float_as_uint((float)((double)((const uint32_t*)acc_v)[ai] * scale));
        else v = ((const uint32_t*)acc_v)[ai];
        if (write) Sq[i] = v;
        const unsigned long long c = comp_key(v, (uint32_t)(base + i));
        if (count) atomicAdd(&hist[(c >> fs) & (kHistBins - 1)], 1u);
        if (append) put(c >= bound, c);
    }
    drain();
    if (!count) return;
    __syncthreads();
    for (int b = tid; b < kHistBins; b += BS)
        if (hist[b]) atomicAdd(&hist_out[b], hist[b]);
}

// ------------------------------------------------------------- tiled --
//
// One workgroup per (query, doc tile of 2^TS docs). LDS holds the tile's
// accumulators: unsigned fixed point for fp32 (64-bit) and bf16 (32-bit) weights
// (LDS integer atomics run far faster than LDS float atomics on this GPU, and
// integer sums do not depend on the order of the updates), int32 for uint8
// impacts. Work inside
// the workgroup: the query's posting segments for this tile are cut into chunks
// of CH postings; wavefronts take chunks round-robin, each lane loads CH/64
// postings (coalesced across the wavefront) before issuing its LDS adds.

// fp32 weights: 64-bit fixed point. Its error is absolute, (m+1) half-units of
// 2^-F with 2^-F about 2^-51 of the query's largest product: far inside the 1e-5
// relative rule for scores near the query's scale, not for scores many orders of
// magnitude below it. The selection checks each query's k-th score against that
// bound and sends the queries where it could fail to the fp64 pass (W).
// bf16 weights: 32-bit fixed point, whose scores only choose the candidates that
// are rescored in fp64 (the same check keeps the error band narrow). uint8
// impacts: int32, exact. W: fp64 accumulation of exact fp64 products.
template <int P, bool W = false>
constexpr int acc_form() {
    return W ? kAccF64 : (P == kFP32 ? kAccFx64 : (P == kBF16 ? kAccFx32 : kAccInt));
}

// Queries per work item of the group kernel. Two: 64 KiB of 32-bit accumulators over
// 8192 docs (bf16, uint8), so that two workgroups share a CU and one accumulates while the
// other flushes; 128 KiB of 64-bit ones (fp32). (Four queries with 32-bit sums, 128 KiB and
// one workgroup per CU, measured slower.)
template <int P>
constexpr int group_size() {
    return 2;
}

// Word 3 of a raw buffer descriptor on the gfx9 family (gfx950 included): no stride,
// no swizzle, 32-bit data format; the hardware range-checks each lane's byte offset
// against the record count and returns 0 past it.
constexpr int kRawBufferWord3 = 0x00020000;

// Segments of a (query, tile) work item, dense terms first: a dense term's segment is
// widened to whole 64-posting blocks (seg_edge = postings before | after the real
// segment << 8), the others are exact.
struct TileShared {
    int64_t seg_beg[kMaxQueryNnz];
    int32_t seg_len[kMaxQueryNnz];
    int32_t seg_cpre[kMaxQueryNnz + 1];
    double seg_qd[kMaxQueryNnz];   // w_q * 2^F (fixed point)
    uint32_t seg_q8[kMaxQueryNnz]; // uint8 query impact
    uint16_t seg_edge[kMaxQueryNnz];
    unsigned long long dmask[kMaxQueryNnz / kWave];  // dense terms per wavefront of the setup
    unsigned long long wmax[kMaxQueryNnz / kWave];   // pruning: largest bound sum per wavefront
    // what the flush needs of the query (its selection state and histogram scaling)
    unsigned long long fl_bound;
    double fl_scale;
    int fl_fused, fl_over, fl_shift;
    int stg[2 + 512 / kWave];  // the flush's candidate stage: base, unused, a count per wavefront
};
static_assert(kMaxQueryNnz <= 512 && kMaxQueryNnz % kWave == 0, "segment setup: one thread per query term");

// Chunk c of a tile's work (c is the same on every lane of the wavefront):
// segment index, first posting and length, kept in scalar registers. The
// segment comes from the chunk table when the tile has one, else from a binary
// search over the chunk prefix.
template <bool TAB>
__device__ __forceinline__ void chunk_at(const TileShared& sh, const uint8_t* tab, int nq, int c, int ch, int* seg,
                                         int64_t* p0, int* n, int* off_out) {
    int lo;
    if constexpr (TAB) {
        lo = tab[c];
    } else {
        lo = 0;
        int hi = nq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.seg_cpre[mid] <= c) lo = mid; else hi = mid - 1;
        }
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int off = __builtin_amdgcn_readfirstlane((c - sh.seg_cpre[lo]) * ch);
    *off_out = off;
    *seg = lo;
    *n = __builtin_amdgcn_readfirstlane(min(ch, sh.seg_len[lo] - off));
    const int64_t p = sh.seg_beg[lo] + off;
    *p0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(p >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)p));
}

// Score one (query, doc tile) work item into LDS and flush it. Every thread of
// the workgroup calls this; it ends after the flush (callers that loop must
// synchronise before reusing the LDS). DB: read the byte doc ids of dense terms.
// That saves HBM bytes but adds scalar work and a second chunk loop per item, so
// it pays only where the kernel waits on HBM (the per-query kernel with fp32 or
// bf16 weights), not where it is bound by instruction issue (shared traversal,
// uint8 weights). W: the wide-range pass (fp64 products w_q * w_d, fp64 sums).
// PR: block-max pruning (MaxScore over 64-posting blocks) in the non-seed tiles of a query
// with a seed bound, for fp32 and uint8 weights (no byte doc ids, DB false). The query's
// terms with the smallest bounds w_q * maxw, as long as their bounds sum to less than the
// bound's raw score t_lo, are non-essential: no doc that holds none of the others can be a
// candidate. The essential terms are scored first; then each 64-doc group of the tile gets
// its largest partial sum, and a block of a non-essential term is skipped (not even read)
// when every doc it can hold has partial sum + the non-essential bounds' sum below t_lo. A
// doc of a skipped block can then not reach the bound, so it is no candidate, and every
// candidate's sum is complete: the result is exact.
// QD: the 2-byte-id segments are read four postings per lane: one 8-byte load of ids and
// one load of four weights (4, 8 or 16 bytes) cover a lane's postings 4l .. 4l + 3 of each
// 256 postings of the chunk, a quarter of the vector memory instructions of one posting per
// lane and load (those instructions, not HBM or the LDS, bound the shared traversal). Segment
// starts are rounded down to a multiple of 4 (the postings before the real start are
// masked). So that the 64 lanes of an add still touch consecutive LDS words where doc ids run
// consecutively, the tile is kept in quarters: doc x of the tile is accumulator
// (x % 4) * TILE / 4 + x / 4 (flush_tile reads it back in doc order).
template <int P, int TS, int CH, bool DB, bool W = false, bool PR = false, bool QD = false>
__device__ __forceinline__ void score_tile(const DevIndex& ix, const DevBatch& qb, int32_t q0, int64_t tile, int ql,
                                           uint32_t* __restrict__ S, int64_t ld, uint32_t* __restrict__ hist1,
                                           uint32_t* lds, TileShared& sh, int phase, SelState* state,
                                           unsigned long long* cand) {
    constexpr int BS = 512, NW = BS / kWave, TILE = 1 << TS, U = CH / kWave, GPT = TS - kGrainShift;
    constexpr bool FX = P != kU8;                  // fixed-point (or, W, fp64) products (fp32, bf16)
    constexpr int AF = acc_form<P, W>();
    constexpr int AW = (AF == kAccFx64 || AF == kAccF64) ? 2 : 1;  // accumulator words per doc
    unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(lds);  // [TILE] (fp32)
    uint32_t* acc32 = lds;                                                   // [TILE] (bf16, uint8)
    uint32_t* hist = lds + TILE * AW;                                        // [kHistBins]

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: chunk bookkeeping stays scalar
    const int q = q0 + ql;
    if (qb.k[q] == 0) return;  // nothing is selected for it (also every padding slot of a batch)
    if (phase == 3 && state[ql].rescore != 1) return;  // only the queries that fell back
    if (phase == 4 && state[ql].rescore != 2) return;  // only the wide-range queries
    if (phase == 5 && state[ql].rescore != 3) return;  // only the bf16 band passes of fused queries
    // What the flush needs of the query: one thread loads it now, so that the latency passes
    // under the setup, and leaves it in LDS (registers are what the accumulation runs short
    // of). The state is set before this launch; the cap flag may be set during it by other
    // workgroups, and a stale 0 only costs appends that the cap check drops.
    int fl_fused = 0, fl_over = 0, fl_shift = 0;
    unsigned long long fl_bound = 0;
    double fl_scale = 1.0;
    if (threadIdx.x == BS - 1) {
        const SelState* stq0 = state + ql;
        fl_fused = stq0->fused;
        fl_over = stq0->fused_over;
        fl_bound = stq0->bound;
        fl_shift = qb.first_shift[q];
        fl_scale = (FX && !W) ? qb.q_scale[q] : 1.0;
    }
    const int64_t N = ix.n_docs;
    const int64_t base = tile << TS;
    const int tile_n = (int)min((int64_t)TILE, N - base);
    static_assert(TS <= 16, "a doc tile must lie inside one 65536-doc range");
    const int lbase = (int)(base & 0xFFFF);  // the tile's offset inside its 65536-doc range

    for (int i = tid; i < TILE * AW / 4; i += BS) reinterpret_cast<uint4*>(lds)[i] = make_uint4(0u, 0u, 0u, 0u);

    const int64_t qa = qb.q_row_ptr[q];
    const int nq = (int)(qb.q_row_ptr[q + 1] - qa);
    const int64_t g0 = tile << GPT;
    const int64_t g1 = min(g0 + (int64_t)(1 << GPT), ix.n_grains);
    static_assert(!(PR && DB), "pruning reads 2-byte doc ids");
    static_assert(!QD || (!PR && !W && CH % 256 == 0), "quad loads: chunks of 256-posting rows");
    static_assert(!PR || (P != kBF16 && !W), "pruning: fp32 and uint8 fixed-point or integer sums");
    // Pruning applies to the non-seed tiles of a query whose seed bound is set; t_lo is the
    // bound's score as a raw sum (no sum below it can give a candidate, see flush_tile).
    bool prune_item = false;
    unsigned long long t_lo = 0;
    if constexpr (PR) {
        const SelState* stq = state + ql;
        if (phase == 2 && stq->fused == 1) {
            const uint32_t sb = (uint32_t)(stq->bound >> 32);
            if constexpr (P == kU8) t_lo = sb;
            else t_lo = (unsigned long long)fmax(0.0, floor((double)__uint_as_float(sb) * (1.0 - 0x1p-22) / qb.q_scale[q]));
            prune_item = t_lo > 0;
        }
    }
    // One thread per query term. Dense terms take the first segment slots (in query
    // order), so their chunks come first and run in the byte-offset loop. With pruning the
    // essential terms come first (exact segments) and the non-essential ones after them
    // (whole 64-posting blocks, each skipped or read).
    const int t = tid;
    const bool live = t < nq;
    int term = 0, a = 0, b = 0;
    bool dense = false;  // first loop: byte doc ids (DB), or the essential terms (PR)
    unsigned long long ub_cum = 0;
    if (live) {
        term = qb.q_term[qa + t];
        const int32_t* row = ix.tile_off + (int64_t)term * (ix.n_grains + 1);
        a = row[g0];
        b = row[g1];
        dense = DB && ix.term_dense[term] != 0 && b > a;
        if constexpr (PR) {
            ub_cum = qb.q_ub_cum[qa + t];
            dense = !prune_item || !(ub_cum < t_lo);
        }
    }
    if (t < kMaxQueryNnz) {
        const unsigned long long m = __ballot(live && dense);
        if (lane == 0) sh.dmask[wave] = m;
        if constexpr (PR) {
            // the bound sum of the non-essential terms: the largest cumulative bound among them
            unsigned long long v = (live && !dense) ? ub_cum : 0ull;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const unsigned long long o = __shfl_xor(v, d, kWave);
                v = o > v ? o : v;
            }
            if (lane == 0) sh.wmax[wave] = v;
        }
    }
    __syncthreads();
    if (live) {
        int before = 0, nd = 0;
#pragma unroll
        for (int w = 0; w < kMaxQueryNnz / kWave; w++) {
            const int pc = __popcll(sh.dmask[w]);
            nd += pc;
            if (w < wave) before += pc;
        }
        before += __popcll(sh.dmask[wave] & ((1ull << lane) - 1ull));
        const int slot = dense ? before : nd + (t - before);
        bool zero_weight;
        if constexpr (FX) {
            const double qd = W ? (double)qb.q_w[qa + t] : qb.q_fx[qa + t];
            sh.seg_qd[slot] = qd;
            zero_weight = !(qd > 0.0);
        } else {
            const uint32_t q8 = (uint32_t)qb.q_w8[qa + t];
            sh.seg_q8[slot] = q8;
            zero_weight = q8 == 0u;
        }
        int beg = a, len = b - a, edge = 0;
        if constexpr (QD) {  // quads: the segment starts at a multiple of 4, edge postings masked
            beg = a & ~3;
            len = b - beg;
            edge = a - beg;
        }
        if (PR ? (!dense && b > a) : dense) {  // whole blocks: lists start 64-aligned and are padded to 64
            beg = a & ~(kBlock - 1);
            const int end = (b + kBlock - 1) & ~(kBlock - 1);
            len = end - beg;
            edge = (a - beg) | ((end - b) << 8);
        }
        sh.seg_beg[slot] = ix.term_off[term] + beg;
        sh.seg_len[slot] = zero_weight ? 0 : len;  // a zero query weight adds nothing
        sh.seg_edge[slot] = (uint16_t)edge;
    }
    if (tid == BS - 1) {
        sh.fl_fused = fl_fused;
        sh.fl_over = fl_over;
        sh.fl_bound = fl_bound;
        sh.fl_shift = fl_shift;
        sh.fl_scale = fl_scale;
    }
    __syncthreads();
    {
        // Every wavefront computes the chunk prefix of all segments (lane l: segments
        // 4 l .. 4 l + 3) and writes its eighth of the chunk table; wavefront 0 also stores
        // the prefix.
        int c[4];
        int s = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int t = lane * 4 + u;
            c[u] = t < nq ? (sh.seg_len[t] + CH - 1) / CH : 0;
            s += c[u];
        }
        // Exclusive prefix of s over the lanes, one bit plane at a time: a ballot of bit b
        // and the count of the lower lanes that hold it (no cross-lane traffic through the
        // LDS, whose queue the other workgroup's atomics keep long).
        int run = 0, total = 0;
        for (int b = 0; __ballot((s >> b) != 0) != 0ull; b++) {
            const unsigned long long m = __ballot((s >> b) & 1);
            run += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
            total += __popcll(m) << b;
        }
        // Chunk table: during accumulation the histogram's LDS holds the segment index
        // of every chunk (one byte each), so a wavefront finds its chunk's segment with
        // one LDS read; tiles with more chunks than it holds fall back to a search.
        uint8_t* t8 = reinterpret_cast<uint8_t*>(hist);
        const bool table = total <= kHistBins * 4;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (wave == 0) sh.seg_cpre[lane * 4 + u] = run;
            if (table)
                for (int j = wave; j < c[u]; j += NW) t8[run + j] = (uint8_t)(lane * 4 + u);
            run += c[u];
        }
        if (tid == 0) sh.seg_cpre[kMaxQueryNnz] = total;
    }
    __syncthreads();

    // Chunks go round-robin to the wavefronts. Each wavefront keeps two chunks in
    // flight: the loads of its next chunk are issued before the LDS adds of the
    // current one (two register sets, alternating).
    const int total = sh.seg_cpre[nq];
    const uint8_t* tab = total <= kHistBins * 4 ? reinterpret_cast<const uint8_t*>(hist) : nullptr;
    struct Chunk {
        uint32_t doc[U];  // doc id modulo 65536, or (dense) distance to the block's first doc
        uint32_t w[U];    // stored weight as fp32 bits, or the uint8 impact
        int32_t blk;      // (dense) lane u < U: first doc of the chunk's block u
        int seg, n, lo;   // postings [lo, n) of the chunk are the segment's (lo > 0: first slot only)
        uint32_t skip;    // (pruned blocks) bit u: block u of the chunk is skipped
        int32_t bq[CH >= 256 ? CH / 256 : 1];  // (quad loads, dense) the block base of the lane's quad q
    };
    // Chunk forms: 0 exact segment, 2-byte ids; 1 dense term, whole blocks, 1-byte ids;
    // 2 non-essential term under pruning, whole blocks, 2-byte ids, skipped blocks not read.
    using FExact = std::integral_constant<int, 0>;
    using FDense = std::integral_constant<int, 1>;
    using FPrune = std::integral_constant<int, 2>;
    // pruning: per 64-doc group of the tile, the largest sum of the essential terms (in the
    // histogram area's last 2 KiB, which the chunk table leaves free for pruned items)
    unsigned long long* gmax = reinterpret_cast<unsigned long long*>(hist) + (kHistBins / 2 - 256);
    unsigned long long u_n = 0;  // the bound sum of the non-essential terms
    const int tbase = __builtin_amdgcn_readfirstlane((int)base);
    using WT = std::conditional_t<P == kU8, uint8_t, std::conditional_t<P == kBF16, uint16_t, uint32_t>>;
    // Loads are straight-line (no branch around them, so the compiler can wait for
    // the older chunk only): lanes past the end of a chunk read 0, and an empty slot
    // reads nothing (record count 0). The chunk's base is wave-uniform (a buffer
    // descriptor in scalar registers), so no address arithmetic is done per posting.
    // The chunk lookup is branch-free with the chunk table (an invalid slot looks up
    // chunk 0 and gets length 0). A dense chunk covers whole blocks: it reads 1-byte
    // distances, plus one block base per 64 postings.
    auto load = [&](auto use_tab, auto form, int c, Chunk& k, bool valid) {
        constexpr bool DENSE = decltype(form)::value == 1;
        constexpr bool PRUNED = decltype(form)::value == 2;
        int64_t p0 = 0;
        int n = 0, off = 0;
        chunk_at<decltype(use_tab)::value>(sh, tab, nq, valid ? c : 0, CH, &k.seg, &p0, &n, &off);
        k.skip = 0u;
        if constexpr (QD && DENSE) {
            // whole 64-posting blocks (p0 and n multiples of 64): four 1-byte ids per lane and load,
            // the block base of each of the lane's quads (block 4 q + lane / 16 of the chunk), and
            // the weights as for the 2-byte form below
            const int edge = __builtin_amdgcn_readfirstlane((int)sh.seg_edge[k.seg]);
            const int real_end = sh.seg_len[k.seg] - (edge >> 8) - off;
            k.lo = off == 0 ? (edge & 0xFF) : 0;
            k.n = valid ? min(n, real_end) : 0;
            const int nrec = valid ? n : 0;
            const __amdgpu_buffer_rsrc_t rid = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint8_t*>(ix.post_b8 + p0), (short)0, nrec, kRawBufferWord3);
            const __amdgpu_buffer_rsrc_t rbk = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<int32_t*>(ix.blk_first + (p0 >> 6)), (short)0, (nrec >> 6) * 4, kRawBufferWord3);
            const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<WT*>(reinterpret_cast<const WT*>(ix.post_w) + p0), (short)0, nrec * (int)sizeof(WT),
                kRawBufferWord3);
            const int z = (int)((uint64_t)p0 >> 48);  // 0, keeps one lane offset per chunk
            const int vid = lane * 4 + z;
            const int vbk = (lane >> 4) * 4 + z;
            const int vw = lane * 4 * (int)sizeof(WT) + z;
#pragma unroll
            for (int q = 0; q < CH / 256; q++) {
                k.doc[q] = __builtin_amdgcn_raw_buffer_load_b32(rid, vid + q * 256, 0, 0);
                k.bq[q] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rbk, vbk + q * 16, 0, 0);
                if constexpr (sizeof(WT) == 1) {
                    k.w[q] = __builtin_amdgcn_raw_buffer_load_b32(rw, vw + q * 256, 0, 0);
                } else if constexpr (sizeof(WT) == 2) {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b64(rw, vw + q * 512, 0, 0);
                    k.w[2 * q] = w[0];
                    k.w[2 * q + 1] = w[1];
                } else {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rw, vw + q * 1024, 0, 0);
                    k.w[4 * q] = w[0];
                    k.w[4 * q + 1] = w[1];
                    k.w[4 * q + 2] = w[2];
                    k.w[4 * q + 3] = w[3];
                }
            }
            return;
        }
        if constexpr (QD && !DENSE && !PRUNED) {
            // p0 is a multiple of 4: ids as 8-byte loads, weights as 4-, 8- or 16-byte loads, both
            // covering whole quads (up to 3 postings past the segment, inside the padded list)
            k.lo = off == 0 ? __builtin_amdgcn_readfirstlane((int)sh.seg_edge[k.seg]) : 0;
            k.n = valid ? n : 0;
            const int nrec = valid ? (n + 3) & ~3 : 0;
            const __amdgpu_buffer_rsrc_t rid = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint16_t*>(ix.post_lo + p0), (short)0, nrec * 2, kRawBufferWord3);
            const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<WT*>(reinterpret_cast<const WT*>(ix.post_w) + p0), (short)0, nrec * (int)sizeof(WT),
                kRawBufferWord3);
            const int z = (int)((uint64_t)p0 >> 48);  // 0, keeps one lane offset per chunk (as below)
            const int vid = lane * 8 + z;
            const int vw = lane * 4 * (int)sizeof(WT) + z;
#pragma unroll
            for (int q = 0; q < CH / 256; q++) {
                const auto d = __builtin_amdgcn_raw_buffer_load_b64(rid, vid + q * 512, 0, 0);
                k.doc[2 * q] = d[0];
                k.doc[2 * q + 1] = d[1];
                if constexpr (sizeof(WT) == 1) {
                    k.w[q] = __builtin_amdgcn_raw_buffer_load_b32(rw, vw + q * 256, 0, 0);
                } else if constexpr (sizeof(WT) == 2) {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b64(rw, vw + q * 512, 0, 0);
                    k.w[2 * q] = w[0];
                    k.w[2 * q + 1] = w[1];
                } else {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rw, vw + q * 1024, 0, 0);
                    k.w[4 * q] = w[0];
                    k.w[4 * q + 1] = w[1];
                    k.w[4 * q + 2] = w[2];
                    k.w[4 * q + 3] = w[3];
                }
            }
            return;
        }
        if constexpr (DENSE || PRUNED) {
            const int edge = __builtin_amdgcn_readfirstlane((int)sh.seg_edge[k.seg]);
            const int real_end = sh.seg_len[k.seg] - (edge >> 8) - off;
            k.lo = off == 0 ? (edge & 0xFF) : 0;
            k.n = valid ? min(n, real_end) : 0;
        } else {
            k.lo = 0;
            k.n = valid ? n : 0;
        }
        const int nblk = (n + kBlock - 1) >> 6;
        if constexpr (DENSE) {
            // one register for the chunk's block bases (lane u holds block u); a slot takes
            // its base with a lane read, which keeps scalar registers free
            k.blk = ix.blk_first[(p0 >> 6) + min(lane, max(nblk - 1, 0))];
        }
        if constexpr (PRUNED) {
            // lane u < nblk decides block u: the docs it can hold are [its first doc, the next
            // block's first doc) inside the segment, the tile's end for the segment's last
            // block, clipped to the tile; it is skipped when every 64-doc group they touch has
            // essential sum + u_n below t_lo
            bool sk = false;
            if (valid && lane < nblk) {
                const int64_t blk = (p0 >> 6) + lane;
                const int64_t seg_end_blk = (sh.seg_beg[k.seg] + sh.seg_len[k.seg]) >> 6;
                const int first = ix.blk_first[blk];
                const int last = blk + 1 < seg_end_blk ? ix.blk_first[blk + 1] - 1 : tbase + tile_n - 1;
                const int lo = max(first - tbase, 0), hi = min(last - tbase, tile_n - 1);
                unsigned long long m = 0;
                for (int gi = lo >> 6; gi <= (hi >> 6); gi++) m = gmax[gi] > m ? gmax[gi] : m;
                sk = m + u_n < t_lo;
            }
            k.skip = (uint32_t)__ballot(sk);
            if (k.skip != 0u && lane == 0) atomicAdd(&state[ql].pruned, __popc(k.skip));
        }
        // Buffer loads over the chunk: the descriptor's record count is the chunk's bytes,
        // so lanes past its end read 0 without a clamp, and slot u's offset is the
        // instruction's immediate (one lane-offset register per chunk).
        const int nrec = valid ? n : 0;
        const void* lb = DENSE ? static_cast<const void*>(ix.post_b8 + p0) : static_cast<const void*>(ix.post_lo + p0);
        // a skipped block's lanes get an offset past the record count: the hardware reads nothing
        auto far = [&](int u) { return PRUNED && ((k.skip >> u) & 1u) ? (1 << 30) : 0; };
        const void* wb = static_cast<const void*>(reinterpret_cast<const WT*>(ix.post_w) + p0);
        const __amdgpu_buffer_rsrc_t rid =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(lb), (short)0, nrec * (DENSE ? 1 : 2), kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t rw =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(wb), (short)0, nrec * (int)sizeof(WT), kRawBufferWord3);
        // z is 0 (posting offsets stay far below 2^48) but not a loop invariant, so the
        // compiler keeps one lane offset per chunk and each slot's offset in the
        // instruction, instead of holding a register per slot across the loop.
        const int z = (int)((uint64_t)p0 >> 48);
        const int vid = (lane << (DENSE ? 0 : 1)) + z;
        const int vw = lane * (int)sizeof(WT) + z;
#pragma unroll
        for (int u = 0; u < U; u++) {
            if constexpr (DENSE) k.doc[u] = __builtin_amdgcn_raw_buffer_load_b8(rid, vid + u * kWave, 0, 0);
            else k.doc[u] = __builtin_amdgcn_raw_buffer_load_b16(rid, vid + far(u) + u * kWave * 2, 0, 0);
            uint32_t wv;
            if constexpr (sizeof(WT) == 4) wv = __builtin_amdgcn_raw_buffer_load_b32(rw, vw + far(u) + u * kWave * 4, 0, 0);
            else if constexpr (sizeof(WT) == 2) wv = __builtin_amdgcn_raw_buffer_load_b16(rw, vw + far(u) + u * kWave * 2, 0, 0);
            else wv = __builtin_amdgcn_raw_buffer_load_b8(rw, vw + far(u) + u * kWave, 0, 0);
            k.w[u] = P == kBF16 ? wv << 16 : wv;
        }
    };
    // Accumulator of slot u: exact segments index by doc id modulo 65536 (the tile's offset
    // folded into the base); dense ones by the distance plus the block's first doc relative
    // to the tile (a scalar per slot).
    unsigned long long* acc64f = acc64 - lbase;
    uint32_t* acc32f = acc32 - lbase;
    // A full chunk (every lane holds a posting in every slot) adds without the
    // per-posting predicate; a segment's first (dense) and last chunks are predicated.
    auto apply = [&](auto form, const Chunk& k) {
        constexpr bool DENSE = decltype(form)::value == 1;
        constexpr bool PRUNED = decltype(form)::value == 2;
        // slot u's accumulator: the uniform part (block base) goes into the pointer, so each
        // lane adds only its scaled offset
        auto at = [&](auto* acc, int u) {
            if constexpr (DENSE) return (acc + (__builtin_amdgcn_readlane(k.blk, u) - tbase)) + k.doc[u];
            else return acc + k.doc[u];
        };
        auto add = [&](auto pred) {
            constexpr bool PRED = decltype(pred)::value;
            if constexpr (QD && !PRUNED) {
                // posting q * 256 + 4 lane + j of the chunk; its quarter-tile accumulator. 2-byte
                // ids: relative to acc - lbase / 4 (lbase is a multiple of 4, so d16 % 4 is the tile
                // doc's). 1-byte ids (dense): the quad's block base minus the tile base, plus the id.
                auto okq = [&](int q, int j) {
                    const int idx = q * 256 + lane * 4 + j;
                    return !PRED || (idx >= k.lo && idx < k.n);
                };
                auto slot = [&](int q, int j) -> uint32_t {
                    if constexpr (DENSE) {
                        const uint32_t x = (uint32_t)(k.bq[q] - tbase) + ((k.doc[q] >> (8 * j)) & 0xffu);
                        return ((x & 3u) << (TS - 2)) + (x >> 2);
                    } else {
                        const uint32_t dw = k.doc[2 * q + (j >> 1)];
                        const uint32_t d16 = (j & 1) ? (dw >> 16) : (dw & 0xffffu);
                        return ((d16 & 3u) << (TS - 2)) + (d16 >> 2);
                    }
                };
                auto wbits = [&](int q, int j) -> uint32_t {  // stored weight (fp32 bits or uint8)
                    if constexpr (sizeof(WT) == 1) {
                        return (k.w[q] >> (8 * j)) & 0xffu;
                    } else if constexpr (sizeof(WT) == 2) {
                        const uint32_t h = k.w[2 * q + (j >> 1)];
                        return ((j & 1) ? (h >> 16) : (h & 0xffffu)) << 16;
                    } else {
                        return k.w[4 * q + j];
                    }
                };
                if constexpr (AF == kAccFx64) {
                    unsigned long long* acc = DENSE ? acc64 : acc64 - (lbase >> 2);
                    const double qd = uniform_f64(sh.seg_qd[k.seg]);
#pragma unroll
                    for (int q = 0; q < CH / 256; q++)
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            if (okq(q, j)) atomicAdd(acc + slot(q, j), fx_product(qd, wbits(q, j)));
                } else if constexpr (AF == kAccFx32) {
                    uint32_t* acc = DENSE ? acc32 : acc32 - (lbase >> 2);
                    const double qd = uniform_f64(sh.seg_qd[k.seg]);
#pragma unroll
                    for (int q = 0; q < CH / 256; q++)
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            if (okq(q, j)) atomicAdd(acc + slot(q, j), (uint32_t)fx_product(qd, wbits(q, j)));
                } else if constexpr (AF == kAccInt) {
                    uint32_t* acc = DENSE ? acc32 : acc32 - (lbase >> 2);
                    const uint32_t q8v = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.seg_q8[k.seg]);
#pragma unroll
                    for (int q = 0; q < CH / 256; q++)
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            if (okq(q, j)) atomicAdd(acc + slot(q, j), __umul24(q8v, wbits(q, j)));
                }
                return;
            }
            auto ok = [&](int u) {
                return (!PRUNED || !((k.skip >> u) & 1u)) &&
                       (!PRED || ((u > 0 || lane >= k.lo) && lane + u * kWave < k.n));
            };
            if constexpr (AF == kAccFx64) {
                unsigned long long* acc = DENSE ? acc64 : acc64f;
                const double qd = uniform_f64(sh.seg_qd[k.seg]);
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (ok(u)) atomicAdd(at(acc, u), fx_product(qd, k.w[u]));
            } else if constexpr (AF == kAccF64) {
                // products of two fp32 values (or fp32 and bf16) are exact in fp64
                double* acc = reinterpret_cast<double*>(DENSE ? acc64 : acc64f);
                const double qd = uniform_f64(sh.seg_qd[k.seg]);
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (ok(u)) atomicAdd(at(acc, u), qd * (double)__uint_as_float(k.w[u]));
            } else if constexpr (AF == kAccFx32) {
                // the query's scale keeps every doc's sum below 2^32 units
                uint32_t* acc = DENSE ? acc32 : acc32f;
                const double qd = uniform_f64(sh.seg_qd[k.seg]);
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (ok(u)) atomicAdd(at(acc, u), (uint32_t)fx_product(qd, k.w[u]));
            } else {
                uint32_t* acc = DENSE ? acc32 : acc32f;
                const uint32_t q8v = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.seg_q8[k.seg]);
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (ok(u)) atomicAdd(at(acc, u), __umul24(q8v, k.w[u]));  // both below 256: full rate
            }
        };
        if (k.n == CH && k.lo == 0) add(std::false_type());
        else add(std::true_type());
    };
    // Chunks c = wave, wave + NW, ... below `end`; returns the wavefront's first chunk at
    // or past `end`.
    auto run = [&](auto use_tab, auto form, int c, int end) -> int {
        Chunk A, B;
        load(use_tab, form, c, A, c < end);
        while (c < end) {
            const int cb = c + NW;
            load(use_tab, form, cb, B, cb < end);
            apply(form, A);
            if (cb >= end) return cb;
            const int ca = cb + NW;
            load(use_tab, form, ca, A, ca < end);
            apply(form, B);
            c = ca;
        }
        return c;
    };
    if constexpr (PR) {
        // The chunk table must leave the last 2 KiB of the histogram area to the group maxima;
        // otherwise nothing is skipped (t_lo 0), the non-essential blocks are all read.
        if (prune_item && total > kHistBins * 4 - 2048) {
            prune_item = false;
            t_lo = 0;
        }
        u_n = sh.wmax[0];
#pragma unroll
        for (int w = 1; w < kMaxQueryNnz / kWave; w++) u_n = sh.wmax[w] > u_n ? sh.wmax[w] : u_n;
    }
    if (total > 0) {
        int n_dense = 0;
#pragma unroll
        for (int w = 0; w < kMaxQueryNnz / kWave; w++) n_dense += __popcll(sh.dmask[w]);
        const int total_d = __builtin_amdgcn_readfirstlane(sh.seg_cpre[n_dense]);
        auto two_loops = [&](auto use_tab) {
            int c = wave;
            if constexpr (DB) {
                c = total_d > 0 ? run(use_tab, FDense(), wave, total_d) : wave;
                run(use_tab, FExact(), c, total);
            } else if constexpr (PR) {
                // essential terms, then the largest essential sum of every 64-doc group, then
                // the non-essential terms block by block
                c = total_d > 0 ? run(use_tab, FExact(), wave, total_d) : wave;
                if (total_d < total) {  // non-essential terms exist: whole-block segments
                    __syncthreads();
                    for (int gi = tid >> 2; gi < TILE / 64; gi += BS / 4) {
                        unsigned long long m = 0;
                        for (int j = 0; j < 16; j++) {
                            const int d = gi * 64 + (tid & 3) * 16 + j;
                            if (d < tile_n) {
                                const unsigned long long v =
                                    AF == kAccFx64 ? acc64[d] : (unsigned long long)acc32[d];
                                m = v > m ? v : m;
                            }
                        }
                        unsigned long long o = __shfl_xor(m, 1, kWave);
                        m = o > m ? o : m;
                        o = __shfl_xor(m, 2, kWave);
                        m = o > m ? o : m;
                        if ((tid & 3) == 0 && prune_item) gmax[gi] = m;
                    }
                    __syncthreads();
                    run(use_tab, FPrune(), c, total);
                }
            } else {
                run(use_tab, FExact(), c, total);
            }
        };
        if (tab) two_loops(std::true_type());
        else two_loops(std::false_type());
    }
    __syncthreads();
    for (int i = tid; i < kHistBins; i += BS) hist[i] = 0u;
    __syncthreads();
    // Fused filtering (the non-seed tiles of a query whose seed bound is set): append while
    // flushing, no appends once past the cap, and no score row. A query that falls back gets
    // its rows from phase 3; a bf16 query whose error band reaches below its candidates gets
    // them from phase 5, before the band pass.
    SelState* st = state + ql;
    // the flush's candidate stage: the histogram's LDS when the flush does not count, else the
    // segment starts (the segment table is not read once the adds are done)
    unsigned long long* stage_hist = reinterpret_cast<unsigned long long*>(hist);
    unsigned long long* stage_seg = reinterpret_cast<unsigned long long*>(sh.seg_beg);
    const bool fused_q = phase == 2 && sh.fl_fused == 1;
    const bool app = fused_q && !sh.fl_over;
    const bool write = !fused_q;
    // The first-digit histogram of a fused query keeps the seed tiles' counts only: its
    // selection needs no more, and if it falls back, phase 3 scores these tiles again and
    // counts them then.
    const bool count = !fused_q;
    flush_tile<BS, AF, (QD ? TILE / 4 : 0), TILE>(lds, hist, tile_n, base, S + (int64_t)ql * ld + base, sh.fl_shift,
                       sh.fl_scale, hist1 + (int64_t)ql * kHistBins, app, app ? sh.fl_bound : 0ull, st,
                       cand + (int64_t)ql * kCandCap, write, count, sh.stg, count ? stage_seg : stage_hist,
                       count ? kMaxQueryNnz : kHistBins / 2);
}

// Per-query form: grid (tiles, queries), the tiles of one query are consecutive
// workgroups, so each query streams its own postings from HBM.
// Both scoring kernels are held to 128 VGPRs (four wavefronts per SIMD): two
// 512-thread workgroups per CU, which is what their LDS footprint allows.
// PR: block-max pruning (phase 2).
template <int P, int TS, int CH, bool PR = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_score_tiled(
    DevIndex ix, DevBatch qb, int32_t q0, uint32_t* __restrict__ S, int64_t ld, uint32_t* __restrict__ hist1,
    int phase, int stride, SelState* __restrict__ state, unsigned long long* __restrict__ cand) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ TileShared sh;
    const int64_t tile = phase_tile(phase, stride, (int64_t)blockIdx.x);
    constexpr bool DB = P != kU8 && !PR;
    // four postings per lane and load: uint8 +5 %, bf16 +4 %; fp32 (16-byte weight loads, the
    // HBM-bound form) measured 0.7 % slower and keeps one posting per lane
    constexpr bool QD = !PR && CH % 256 == 0 && P != kFP32;
    score_tile<P, TS, CH, DB, false, PR, QD>(ix, qb, q0, tile, (int)blockIdx.y, S, ld, hist1, lds, sh, phase, state,
                                             cand);
}

// The rows of the listed queries scored again, one workgroup per tile walking the list
// (usually empty): those that fell back from fused filtering (phase 3) or were found wide
// range (phase 4, W: fp64 accumulation). score_tile skips the other kind. A kernel of its
// own, so that the per-query kernel's registers hold one copy of the scoring loop.
template <int P, int TS, int CH, bool W = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_score_listed(
    DevIndex ix, DevBatch qb, int32_t q0, uint32_t* __restrict__ S, int64_t ld, uint32_t* __restrict__ hist1,
    int phase, int stride, SelState* __restrict__ state, unsigned long long* __restrict__ cand,
    const uint32_t* __restrict__ counters, const int32_t* __restrict__ rescore_list) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ TileShared sh;
    const int64_t tile = phase_tile(phase, stride, (int64_t)blockIdx.x);
    constexpr bool DB = P != kU8 && !W;
    const int nres = (int)counters[8];
    for (int r = 0; r < nres; r++) {
        score_tile<P, TS, CH, DB, W>(ix, qb, q0, tile, rescore_list[r], S, ld, hist1, lds, sh, phase, state, cand);
        __syncthreads();
    }
}

// Persistent form of the shared traversal: a grid of (resident workgroups,
// rounded to a multiple of 8) in which workgroup b stays on XCD b % 8 and pulls
// work items from that XCD's counter. XCD x owns the tiles x, x+8, ...; the items
// of a tile are its queries in the order given by `order` (heaviest first), so
// every query of a tile runs on one XCD while the tile's postings are in its L2.
// Every workgroup leaves the loop once its XCD's counter passes the item count.
template <int P, int TS, int CH>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_score_persistent(
    DevIndex ix, DevBatch qb, int32_t q0, int32_t qt, const int32_t* __restrict__ order,
    uint32_t* __restrict__ counters, uint32_t* __restrict__ S, int64_t ld, uint32_t* __restrict__ hist1, int phase,
    int stride, SelState* __restrict__ state, unsigned long long* __restrict__ cand,
    const int32_t* __restrict__ rescore_list) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ TileShared sh;
    __shared__ int64_t item_sh;
    const int x = (int)(blockIdx.x & 7);
    const int64_t n_tiles = phase_tiles(phase, stride, (ix.n_docs + (1 << TS) - 1) >> TS);
    const int64_t tiles_x = n_tiles > x ? (n_tiles - x + 7) / 8 : 0;
    // phases 3 and 5 cover only the listed queries (fused filtering's fallbacks, bf16 band
    // passes; usually none)
    const bool listed = phase == 3 || phase == 5;
    const int nq = listed ? (int)counters[8] : qt;
    const int64_t items = tiles_x * nq;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&counters[x], 1u);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= items) break;
        const int64_t tile = phase_tile(phase, stride, x + 8 * (item / nq));
        const int ql = listed ? rescore_list[item % nq] : order[item % nq];
        // uint8 weights: four postings per lane and load (measured +10 %; the fixed-point forms,
        // with more arithmetic per posting, ran 4-6 % slower that way)
        score_tile<P, TS, CH, false, false, false, (P == kU8 && CH % 256 == 0)>(ix, qb, q0, tile, ql, S, ld, hist1,
                                                                                lds, sh, phase, state, cand);
        __syncthreads();
    }
}

// Work order of a query tile for the persistent kernel: local query indices by
// descending estimated work (postings of the query's terms), ties by index.
__global__ __launch_bounds__(256) void k_work_order(DevBatch qb, int32_t q0, int32_t qt, int32_t* __restrict__ order) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= qt) return;
    const int64_t wi = qb.q_work[q0 + i];
    int r = 0;
    for (int j = 0; j < qt; j++) {
        const int64_t wj = qb.q_work[q0 + j];
        r += (wj > wi) || (wj == wi && j < i);
    }
    order[r] = i;
}

// ------------------------------------------------------------- group --
//
// Shared traversal with explicit sharing: a work item is (doc tile, group of G
// queries). The LDS holds G accumulator tiles of 8192 docs (128 KiB: G = 4 with
// 32-bit sums for bf16 and uint8, G = 2 with 64-bit fixed point for fp32). The
// segments are those of the union of the group's terms (built on the host, with
// each member's weight per union term, 0 where the member lacks the term), so a
// posting chunk is loaded once and scatter-added into the tile of every member
// that holds its term. The items of a tile run on one XCD (tile-major, as in the
// persistent kernel), groups in the host's order (heaviest first).
template <int MT, int G>
struct GroupShared {
    union {
        struct {
            int64_t beg[MT];
            int32_t len[MT];
            int32_t cpre[MT + 1];
        } seg;
        uint32_t hist[kHistBins];  // the flush histogram, once the segments are no longer read
    };
    uint32_t w[MT][G];  // per union term, each member's w_q (fp32 bits) or uint8 impact
    uint16_t tab[kGroupChunkTab];  // chunk -> union term, when the item has at most that many chunks
    int32_t wave_sum[16];
    int64_t item;
};

template <int P, int CH>
__global__ __launch_bounds__(group_size<P>() * kMaxQueryNnz) __attribute__((amdgpu_waves_per_eu(4))) void k_score_group(
    DevIndex ix, DevBatch qb, uint32_t* __restrict__ counters, uint32_t* __restrict__ S, int64_t ld,
    uint32_t* __restrict__ hist1, int phase, int stride, SelState* __restrict__ state,
    unsigned long long* __restrict__ cand) {
    constexpr int G = group_size<P>();
    constexpr int MT = G * kMaxQueryNnz;  // most union terms of a group; one thread each
    constexpr int TS = kGroupTileShift, TILE = 1 << TS, BS = MT, NW = BS / kWave, U = CH / kWave;
    static_assert(NW <= 16, "wave sums");
    constexpr bool FX = P != kU8;
    constexpr int AF = acc_form<P>();
    constexpr int AW = AF == kAccFx64 ? 2 : 1;  // accumulator words per doc
    extern __shared__ __align__(16) uint32_t lds[];  // [G][TILE * AW]
    __shared__ GroupShared<MT, G> sh;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int x = (int)(blockIdx.x & 7);
    const int64_t n_tiles = phase_tiles(phase, stride, (ix.n_docs + TILE - 1) >> TS);
    const int64_t tiles_x = n_tiles > x ? (n_tiles - x + 7) / 8 : 0;
    const int ng = qb.g_count[0];
    const int64_t items = tiles_x * ng;
    using WT = std::conditional_t<P == kU8, uint8_t, std::conditional_t<P == kBF16, uint16_t, uint32_t>>;
    for (;;) {
        if (tid == 0) sh.item = (int64_t)atomicAdd(&counters[x], 1u);
        __syncthreads();
        const int64_t item = sh.item;
        if (item >= items) break;
        const int64_t tile = phase_tile(phase, stride, x + 8 * (item / ng));
        const int g = (int)(item % ng);
        const int64_t base = tile << TS;
        const int tile_n = (int)min((int64_t)TILE, ix.n_docs - base);
        const int lbase = (int)(base & 0xFFFF);
        const int gr = qb.g_row[g], nu = qb.g_row[g + 1] - gr;
        for (int i = tid; i < G * TILE * AW; i += BS) lds[i] = 0u;
        // segments of the union terms in this tile; a term no member weighs adds nothing
        const int64_t g0 = tile << (TS - kGrainShift);
        const int64_t g1 = min(g0 + (int64_t)(1 << (TS - kGrainShift)), ix.n_grains);
        int c = 0;
        if (tid < nu) {
            const int term = qb.g_term[gr + tid];
            const int32_t* row = ix.tile_off + (int64_t)term * (ix.n_grains + 1);
            const int a = row[g0], b = row[g1];
            bool any = false;
#pragma unroll
            for (int m = 0; m < G; m++) {
                uint32_t wv;
                if constexpr (FX) wv = __float_as_uint(qb.g_wq[(int64_t)(gr + tid) * G + m]);
                else wv = (uint32_t)qb.g_w8[(int64_t)(gr + tid) * G + m];
                sh.w[tid][m] = wv;
                any |= wv != 0u;  // weights are >= 0: a zero bit pattern is a zero weight
            }
            sh.seg.beg[tid] = ix.term_off[term] + a;
            sh.seg.len[tid] = any ? b - a : 0;
            c = any ? (b - a + CH - 1) / CH : 0;
        }
        // exclusive prefix of the chunk counts over the union terms (one per thread)
        int incl = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int v = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += v;
        }
        if (lane == kWave - 1) sh.wave_sum[wave] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const int ws_ = sh.wave_sum[w];
            before += w < wave ? ws_ : 0;
            total += ws_;
        }
        if (tid < nu) sh.seg.cpre[tid] = before + incl - c;
        if (tid == 0) sh.seg.cpre[MT] = total;
        // chunk table: each union term writes its chunks' entries
        const bool use_tab = total <= kGroupChunkTab;
        if (use_tab && tid < nu)
            for (int j = 0; j < c; j++) sh.tab[before + incl - c + j] = (uint16_t)tid;
        __syncthreads();
        struct Chunk {
            uint32_t doc[U];
            uint32_t w[U];
            int seg, n;
        };
        auto load = [&](int cc, Chunk& k, bool valid) {
            // segment of chunk cc: the chunk table, else a binary search over the prefix
            const int want = valid ? cc : 0;
            int lo = 0;
            if (use_tab) {
                lo = total > 0 ? (int)sh.tab[want] : 0;
            } else {
                int hi = max(nu - 1, 0);
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.seg.cpre[mid] <= want) lo = mid; else hi = mid - 1;
                }
            }
            lo = __builtin_amdgcn_readfirstlane(lo);
            const int off = __builtin_amdgcn_readfirstlane((want - sh.seg.cpre[lo]) * CH);
            const int n = valid ? __builtin_amdgcn_readfirstlane(min(CH, sh.seg.len[lo] - off)) : 0;
            const int64_t pp = sh.seg.beg[lo] + off;
            const int64_t p0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(pp >> 32)) << 32) |
                                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pp));
            k.seg = lo;
            k.n = n;
            const __amdgpu_buffer_rsrc_t rid = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint16_t*>(ix.post_lo + p0), (short)0, n * 2, kRawBufferWord3);
            const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<WT*>(reinterpret_cast<const WT*>(ix.post_w) + p0), (short)0, n * (int)sizeof(WT),
                kRawBufferWord3);
            const int z = (int)((uint64_t)p0 >> 48);  // 0, but not a loop invariant (see score_tile)
            const int vid = (lane << 1) + z;
            const int vw = lane * (int)sizeof(WT) + z;
#pragma unroll
            for (int u = 0; u < U; u++) {
                k.doc[u] = __builtin_amdgcn_raw_buffer_load_b16(rid, vid + u * kWave * 2, 0, 0);
                uint32_t wv;
                if constexpr (sizeof(WT) == 4) wv = __builtin_amdgcn_raw_buffer_load_b32(rw, vw + u * kWave * 4, 0, 0);
                else if constexpr (sizeof(WT) == 2) wv = __builtin_amdgcn_raw_buffer_load_b16(rw, vw + u * kWave * 2, 0, 0);
                else wv = __builtin_amdgcn_raw_buffer_load_b8(rw, vw + u * kWave, 0, 0);
                k.w[u] = P == kBF16 ? wv << 16 : wv;
            }
        };
        // the members' scales 2^F (fixed point): w_q * 2^F is then exact, as q_fx
        double inv_scale[G];
#pragma unroll
        for (int m = 0; m < G; m++) {
            const int ql = qb.g_member[g * G + m];
            inv_scale[m] = (FX && ql >= 0) ? 1.0 / qb.q_scale[ql] : 0.0;
        }
        // a chunk's postings into the tile of every member holding its term
        auto apply = [&](const Chunk& k) {
            auto add = [&](auto pred) {
                constexpr bool PRED = decltype(pred)::value;
                auto ok = [&](int u) { return !PRED || lane + u * kWave < k.n; };
#pragma unroll
                for (int m = 0; m < G; m++) {
                    const uint32_t wm = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.w[k.seg][m]);
                    if (wm == 0u) continue;
                    if constexpr (AF == kAccFx64) {
                        const double qd = (double)__uint_as_float(wm) * inv_scale[m];
                        unsigned long long* acc = reinterpret_cast<unsigned long long*>(lds) + m * TILE - lbase;
#pragma unroll
                        for (int u = 0; u < U; u++)
                            if (ok(u)) atomicAdd(acc + k.doc[u], fx_product(qd, k.w[u]));
                    } else if constexpr (AF == kAccFx32) {
                        const double qd = (double)__uint_as_float(wm) * inv_scale[m];
                        uint32_t* acc = lds + m * TILE - lbase;
#pragma unroll
                        for (int u = 0; u < U; u++)
                            if (ok(u)) atomicAdd(acc + k.doc[u], (uint32_t)fx_product(qd, k.w[u]));
                    } else {
                        const uint32_t q8v = wm;
                        uint32_t* acc = lds + m * TILE - lbase;
#pragma unroll
                        for (int u = 0; u < U; u++)
                            if (ok(u)) atomicAdd(acc + k.doc[u], __umul24(q8v, k.w[u]));
                    }
                }
            };
            if (k.n == CH) add(std::false_type());
            else add(std::true_type());
        };
        {
            int cc = wave;
            Chunk A, B;
            load(cc, A, cc < total);
            while (cc < total) {
                const int cb = cc + NW;
                load(cb, B, cb < total);
                apply(A);
                if (cb >= total) break;
                const int ca = cb + NW;
                load(ca, A, ca < total);
                apply(B);
                cc = ca;
            }
        }
        __syncthreads();
        // flush every member's tile (the histogram reuses the segment area)
        uint32_t* hist = sh.hist;
        for (int m = 0; m < G; m++) {
            const int ql = qb.g_member[g * G + m];
            if (ql < 0 || qb.k[ql] == 0) continue;  // uniform: read from global memory
            for (int i = tid; i < kHistBins; i += BS) hist[i] = 0u;
            __syncthreads();
            SelState* st = state + ql;
            const bool fused_q = phase == 2 && st->fused == 1;
            const bool app = fused_q && !st->fused_over;
            // as in score_tile: a fused query writes no row and counts no tile here; its
            // fallback (phase 3) or bf16 band pass (phase 5) scores these tiles again
            const bool write = !fused_q;
            const bool count = !fused_q;
            flush_tile<BS, AF>(lds + m * TILE * AW, hist, tile_n, base, S + (int64_t)ql * ld + base,
                               qb.first_shift[ql], FX ? qb.q_scale[ql] : 1.0, hist1 + (int64_t)ql * kHistBins, app,
                               app ? st->bound : 0ull, st, cand + (int64_t)ql * kCandCap, write, count);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------ atomic --

// Exclusive prefix of posting chunks over the (query, term) pairs of a query tile.
__global__ __launch_bounds__(1024) void k_pair_prefix(DevIndex ix, DevBatch qb, int32_t q0, int32_t qt, int chunk,
                                                      int64_t* __restrict__ prefix, int32_t* __restrict__ pair_q) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t a0 = qb.q_row_ptr[q0];
    const int64_t np = qb.q_row_ptr[q0 + qt] - a0;
    const int64_t per = (np + 1023) / 1024;
    const int64_t lo = min(np, tid * per), hi = min(np, lo + per);
    int64_t s = 0;
    for (int64_t p = lo; p < hi; p++) {
        const int term = qb.q_term[a0 + p];
        const int64_t padded = ix.term_off[term + 1] - ix.term_off[term];
        s += (padded + chunk - 1) / chunk;
    }
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    int ql = 0;
    for (int64_t p = lo; p < hi; p++) {
        while (qb.q_row_ptr[q0 + ql + 1] - a0 <= p) ql++;
        prefix[p] = run;
        pair_q[p] = ql;
        const int term = qb.q_term[a0 + p];
        const int64_t padded = ix.term_off[term + 1] - ix.term_off[term];
        run += (padded + chunk - 1) / chunk;
    }
    if (tid == 1023) prefix[np] = part[1023];
}

template <int P, int CH>
__global__ __launch_bounds__(256) void k_score_atomic(DevIndex ix, DevBatch qb, int32_t q0, int32_t qt,
                                                      const int64_t* __restrict__ prefix,
                                                      const int32_t* __restrict__ pair_q, uint32_t* __restrict__ S,
                                                      int64_t ld) {
    constexpr int NW = 256 / kWave, U = CH / kWave;
    using Acc = typename WF<P>::Acc;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t a0 = qb.q_row_ptr[q0];
    const int64_t np = qb.q_row_ptr[q0 + qt] - a0;
    const int64_t total = prefix[np];
    for (int64_t c = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6); c < total; c += (int64_t)gridDim.x * NW) {
        int64_t lo = 0, hi = np - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= c) lo = mid; else hi = mid - 1;
        }
        const int term = qb.q_term[a0 + lo];
        const Acc wq = WF<P>::qweight(qb, a0 + lo);
        const int64_t off = (c - prefix[lo]) * (int64_t)CH;
        const int64_t p0 = ix.term_off[term] + off;
        const int n = (int)min((int64_t)CH, ix.term_off[term + 1] - p0);  // a list ends on a 64-posting block
        uint32_t* Sq = S + (int64_t)pair_q[lo] * ld;
        int doc[U];
        Acc w[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int i = lane + u * kWave;
            doc[u] = -1;
            if (i < n) {
                doc[u] = ix.post_doc[p0 + i];
                w[u] = WF<P>::load(ix.post_w, p0 + i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            if (doc[u] >= 0) glb_add(&Sq[doc[u]], wq * w[u]);
    }
}

// ------------------------------------------------------------ docpar --

// 1024 threads per (query, block of docs): the query's weights sit in a dense
// LDS table; a wavefront scores 4 documents at a time, 16 lanes per document,
// each lane walking its document's forward row with stride 16 and four loads
// of (term, weight) in flight, then a 16-lane reduction. Rows are contiguous,
// so the 4 x 16 lanes read 4 short coalesced runs per step.
template <int P>
__global__ __launch_bounds__(1024) void k_score_docpar(DevIndex ix, DevBatch qb, int32_t q0, uint32_t* __restrict__ S,
                                                       int64_t ld, int docs_per_block) {
    using Acc = typename WF<P>::Acc;
    extern __shared__ __align__(16) uint32_t table[];  // [vocab] query weights (dense)
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int ql = blockIdx.y, q = q0 + ql;
    for (int i = tid; i < ix.vocab; i += 1024) table[i] = 0u;
    __syncthreads();
    const int64_t qa = qb.q_row_ptr[q], qn = qb.q_row_ptr[q + 1] - qa;
    for (int t = tid; t < qn; t += 1024) {
        Acc v = WF<P>::qweight(qb, qa + t);
        table[qb.q_term[qa + t]] = WF<P>::bits(v);
    }
    __syncthreads();
    if (qb.k[q] == 0) return;
    const Acc* tab = reinterpret_cast<const Acc*>(table);
    const int64_t d0 = (int64_t)blockIdx.x * docs_per_block;
    const int64_t d1 = min(ix.n_docs, d0 + docs_per_block);
    uint32_t* Sq = S + (int64_t)ql * ld;
    const int grp = lane >> 4, sub = lane & 15;
    for (int64_t dg = d0 + (int64_t)wave * 4; dg < d1; dg += 16 * 4) {
        const int64_t d = dg + grp;
        int64_t a = 0, b = 0;
        if (d < d1) {
            a = ix.fwd_row_ptr[d];
            b = ix.fwd_row_ptr[d + 1];
        }
        Acc s = 0;
        for (int64_t e = a + sub; e < b; e += 64) {
            int t[4];
            float w[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int64_t eu = e + 16 * u;
                t[u] = eu < b ? ix.fwd_term[eu] : 0;
                w[u] = eu < b ? ix.fwd_w[eu] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (e + 16 * u < b) s += tab[t[u]] * WF<P>::from_fp32(w[u]);
        }
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (sub == 0 && d < d1) Sq[d] = WF<P>::bits(s);
    }
}

// ------------------------------------------------------ hist / clear --

__global__ __launch_bounds__(512) void k_hist1(DevBatch qb, int32_t q0, int64_t N, const uint32_t* __restrict__ S,
                                               int64_t ld, int per_block, uint32_t* __restrict__ hist1) {
    __shared__ uint32_t hist[kHistBins];
    const int tid = threadIdx.x, ql = blockIdx.y;
    for (int i = tid; i < kHistBins; i += 512) hist[i] = 0u;
    __syncthreads();
    const int fs = qb.first_shift[q0 + ql];
    const int64_t d0 = (int64_t)blockIdx.x * per_block, d1 = min(N, d0 + per_block);
    const uint32_t* Sq = S + (int64_t)ql * ld;
    for (int64_t d = d0 + tid; d < d1; d += 512)
        atomicAdd(&hist[(comp_key(Sq[d], (uint32_t)d) >> fs) & (kHistBins - 1)], 1u);
    __syncthreads();
    for (int b = tid; b < kHistBins; b += 512)
        if (hist[b]) atomicAdd(&hist1[(int64_t)ql * kHistBins + b], hist[b]);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t fill_u32(void* p, int64_t n_words, hipStream_t s) { return launch_fill(p, n_words, 0u, s); }

template <typename F>
hipError_t by_precision(int p, F f) {
    switch (p) {
        case kFP32: return f(std::integral_constant<int, kFP32>());
        case kBF16: return f(std::integral_constant<int, kBF16>());
        case kU8: return f(std::integral_constant<int, kU8>());
    }
    return hipErrorInvalidValue;
}

template <int P, int TS, int CH>
hipError_t launch_tiled_one(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, bool persistent,
                            const Workspace& ws, int64_t ld, hipStream_t s, int phase, int stride, bool prune) {
    const int64_t n_tiles = phase_tiles(phase, stride, (ix.n_docs + (1 << TS) - 1) >> TS);
    if (n_tiles <= 0) return hipSuccess;
    const size_t lds = (size_t)((1 << TS) * (acc_form<P>() == kAccFx64 ? 2 : 1) + kHistBins) * 4;
    if (lds > 150 * 1024) return hipErrorInvalidValue;
    if (lds > 65536) {
        static const hipError_t attr = [&] {
            hipError_t e = hipFuncSetAttribute((const void*)k_score_tiled<P, TS, CH>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void*)k_score_listed<P, TS, CH>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void*)k_score_persistent<P, TS, CH>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            return e;
        }();
        if (attr != hipSuccess) {
            g_failed_launch = "hipFuncSetAttribute(k_score_tiled)";
            return attr;
        }
    }
    if (!persistent) {
        // block-max pruning (non-seed tiles): the default tile and chunk of fp32 and uint8 only
        constexpr bool kPrunable = ((P == kFP32 && TS == 13) || (P == kU8 && TS == 14)) && CH == 1024;
        if constexpr (kPrunable) {
            if (prune && phase == 2) {
                static const hipError_t pattr = hipFuncSetAttribute(
                    (const void*)k_score_tiled<P, TS, CH, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (pattr != hipSuccess) {
                    g_failed_launch = "hipFuncSetAttribute(k_score_tiled, pruning)";
                    return pattr;
                }
                hipLaunchKernelGGL((k_score_tiled<P, TS, CH, true>), dim3((unsigned)n_tiles, (unsigned)qt),
                                   dim3(512), lds, s, ix, qb, q0, ws.scores, ld, ws.hist1, phase, stride, ws.state,
                                   ws.cand);
                GS_CHECK_LAUNCH("k_score_tiled (pruning)");
                return hipSuccess;
            }
        }
        if (phase == 3 || phase == 5) {
            hipLaunchKernelGGL((k_score_listed<P, TS, CH>), dim3((unsigned)n_tiles, 1u), dim3(512), lds, s, ix, qb, q0,
                               ws.scores, ld, ws.hist1, phase, stride, ws.state, ws.cand, (const uint32_t*)ws.counters,
                               (const int32_t*)ws.rescore_list);
            GS_CHECK_LAUNCH("k_score_listed");
            return hipSuccess;
        }
        hipLaunchKernelGGL((k_score_tiled<P, TS, CH>), dim3((unsigned)n_tiles, (unsigned)qt), dim3(512), lds, s, ix,
                           qb, q0, ws.scores, ld, ws.hist1, phase, stride, ws.state, ws.cand);
        GS_CHECK_LAUNCH("k_score_tiled");
        return hipSuccess;
    }
    // resident workgroups: as many as fit on every CU at once, a multiple of the 8 XCDs
    static const int grid = [&] {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t p{};
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_score_persistent<P, TS, CH>, 512,
                                                         lds) != hipSuccess)
            return 0;
        return std::max(8, (p.multiProcessorCount * std::max(per_cu, 1)) / 8 * 8);
    }();
    if (grid <= 0) return hipErrorInvalidConfiguration;
    if (phase <= 1) {  // the later launches of a fused search keep the first one's order
        hipLaunchKernelGGL(k_work_order, dim3((unsigned)((qt + 255) / 256)), dim3(256), 0, s, qb, q0, qt, ws.order);
        GS_CHECK_LAUNCH("k_work_order");
    } else {
        const hipError_t e = launch_fill(ws.counters, 8, 0u, s);  // the first launch used the counters
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_score_persistent<P, TS, CH>), dim3((unsigned)grid), dim3(512), lds, s, ix, qb, q0, qt,
                       (const int32_t*)ws.order, ws.counters, ws.scores, ld, ws.hist1, phase, stride, ws.state,
                       ws.cand, (const int32_t*)ws.rescore_list);
    GS_CHECK_LAUNCH("k_score_persistent");
    return hipSuccess;
}

template <int P, int TS>
hipError_t tiled_chunk(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, int chunk, bool persistent,
                       const Workspace& ws, int64_t ld, hipStream_t s, int phase, int stride, bool prune) {
    switch (chunk) {
        case 64: return launch_tiled_one<P, TS, 64>(ix, qb, q0, qt, persistent, ws, ld, s, phase, stride, prune);
        case 128: return launch_tiled_one<P, TS, 128>(ix, qb, q0, qt, persistent, ws, ld, s, phase, stride, prune);
        case 256: return launch_tiled_one<P, TS, 256>(ix, qb, q0, qt, persistent, ws, ld, s, phase, stride, prune);
        case 512: return launch_tiled_one<P, TS, 512>(ix, qb, q0, qt, persistent, ws, ld, s, phase, stride, prune);
        case 1024: return launch_tiled_one<P, TS, 1024>(ix, qb, q0, qt, persistent, ws, ld, s, phase, stride, prune);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int64_t score_ld(int64_t n_docs) { return (n_docs + 63) / 64 * 64; }

hipError_t launch_fill(void* p, int64_t n_words, uint32_t v, hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n_words + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n_words, v);
    GS_CHECK_LAUNCH("k_fill_u32");
    return hipSuccess;
}

hipError_t launch_clear(const Workspace& ws, int32_t qt, hipStream_t s) {
    hipError_t e = fill_u32(ws.counters, 16, s);
    if (e == hipSuccess) e = fill_u32(ws.hist1, (int64_t)qt * kHistBins, s);
    if (e == hipSuccess) e = fill_u32(ws.hist_ref, (int64_t)qt * kHistBins, s);
    if (e == hipSuccess) e = fill_u32(ws.state, (int64_t)qt * sizeof(SelState) / 4, s);
    return e;
}

hipError_t launch_score_tiled(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const ScoreOpts& o,
                              const Workspace& ws, hipStream_t s, int phase) {
    const int stride = phase == 0 ? 1 : o.seed_stride;
    const int64_t ld = score_ld(ix.n_docs);
    return by_precision(ix.precision, [&](auto pc) -> hipError_t {
        constexpr int P = decltype(pc)::value;
        const bool persistent = o.kernel == 4;  // GS_KERNEL_SHARED: persistent, tile-major, XCD-aware
        switch (o.tile_shift) {
            case 13: return tiled_chunk<P, 13>(ix, qb, q0, qt, o.chunk, persistent, ws, ld, s, phase, stride, o.prune != 0);
            case 14: return tiled_chunk<P, 14>(ix, qb, q0, qt, o.chunk, persistent, ws, ld, s, phase, stride, o.prune != 0);
            case 15:
                if constexpr (acc_form<P>() != kAccFx64)
                    return tiled_chunk<P, 15>(ix, qb, q0, qt, o.chunk, persistent, ws, ld, s, phase, stride, o.prune != 0);
                return hipErrorInvalidValue;  // 32768 64-bit accumulators exceed one CU's LDS
        }
        return hipErrorInvalidValue;
    });
}

template <int P, int CH>
hipError_t launch_group_one(const DevIndex& ix, const DevBatch& qb, const Workspace& ws, int64_t ld, hipStream_t s,
                            int phase, int stride) {
    constexpr int TS = kGroupTileShift;
    const int64_t n_tiles = phase_tiles(phase, stride, (ix.n_docs + (1 << TS) - 1) >> TS);
    if (n_tiles <= 0) return hipSuccess;
    const size_t lds = (size_t)group_size<P>() * (1 << TS) * (acc_form<P>() == kAccFx64 ? 8 : 4);
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_score_group<P, CH>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) {
        g_failed_launch = "hipFuncSetAttribute(k_score_group)";
        return attr;
    }
    // resident workgroups (one per CU), a multiple of the 8 XCDs
    static const int grid = [&] {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t p{};
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_score_group<P, CH>,
                                                         group_size<P>() * kMaxQueryNnz, lds) !=
            hipSuccess)
            return 0;
        return std::max(8, (p.multiProcessorCount * std::max(per_cu, 1)) / 8 * 8);
    }();
    if (grid <= 0) return hipErrorInvalidConfiguration;
    if (phase > 1) {  // the seed-tile launch used the counters
        const hipError_t e = launch_fill(ws.counters, 8, 0u, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_score_group<P, CH>), dim3((unsigned)grid), dim3(group_size<P>() * kMaxQueryNnz), lds, s,
                       ix, qb, ws.counters,
                       ws.scores, ld, ws.hist1, phase, stride, ws.state, ws.cand);
    GS_CHECK_LAUNCH("k_score_group");
    return hipSuccess;
}

hipError_t launch_score_group(const DevIndex& ix, const DevBatch& qb, const ScoreOpts& o, const Workspace& ws,
                              hipStream_t s, int phase) {
    const int stride = phase == 0 ? 1 : o.seed_stride;
    const int64_t ld = score_ld(ix.n_docs);
    return by_precision(ix.precision, [&](auto pc) -> hipError_t {
        constexpr int P = decltype(pc)::value;
        switch (o.chunk) {
            case 256: return launch_group_one<P, 256>(ix, qb, ws, ld, s, phase, stride);
            case 512: return launch_group_one<P, 512>(ix, qb, ws, ld, s, phase, stride);
            case 1024: return launch_group_one<P, 1024>(ix, qb, ws, ld, s, phase, stride);
        }
        return hipErrorInvalidValue;
    });
}

hipError_t launch_score_wide(const DevIndex& ix, const DevBatch& qb, int32_t q0, const Workspace& ws, hipStream_t s) {
    // 8192 docs of fp64 accumulators (64 KiB of LDS), one workgroup per tile walking the list
    constexpr int TS = 13, CH = 256;
    const int64_t n_tiles = (ix.n_docs + (1 << TS) - 1) >> TS;
    if (n_tiles <= 0) return hipSuccess;
    const size_t lds = (size_t)((1 << TS) * 2 + kHistBins) * 4;
    const int64_t ld = score_ld(ix.n_docs);
    auto go = [&](auto pc) -> hipError_t {
        constexpr int P = decltype(pc)::value;
        static const hipError_t attr = hipFuncSetAttribute((const void*)k_score_listed<P, TS, CH, true>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) {
            g_failed_launch = "hipFuncSetAttribute(k_score_listed, wide)";
            return attr;
        }
        hipLaunchKernelGGL((k_score_listed<P, TS, CH, true>), dim3((unsigned)n_tiles, 1u), dim3(512), lds, s, ix, qb,
                           q0, ws.scores, ld, ws.hist1, 4, 1, ws.state, ws.cand, (const uint32_t*)ws.counters,
                           (const int32_t*)ws.rescore_list);
        GS_CHECK_LAUNCH("k_score_listed (wide)");
        return hipSuccess;
    };
    if (ix.precision == kFP32) return go(std::integral_constant<int, kFP32>());
    if (ix.precision == kBF16) return go(std::integral_constant<int, kBF16>());
    return hipSuccess;  // uint8 sums are exact
}

hipError_t launch_score_atomic(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const ScoreOpts& o,
                               const Workspace& ws, hipStream_t s) {
    const int64_t ld = score_ld(ix.n_docs);
    hipError_t e = fill_u32(ws.scores, (int64_t)qt * ld, s);
    if (e != hipSuccess) return e;
    int64_t* prefix = ws.work_prefix;
    int32_t* pair_q = ws.work_pair_q;
    hipLaunchKernelGGL(k_pair_prefix, dim3(1), dim3(1024), 0, s, ix, qb, q0, qt, o.chunk, prefix, pair_q);
    GS_CHECK_LAUNCH("k_pair_prefix");
    const dim3 grid(2048);
    e = by_precision(ix.precision, [&](auto pc) -> hipError_t {
        constexpr int P = decltype(pc)::value;
        switch (o.chunk) {
            case 64: hipLaunchKernelGGL((k_score_atomic<P, 64>), grid, dim3(256), 0, s, ix, qb, q0, qt, prefix, pair_q, ws.scores, ld); break;
            case 128: hipLaunchKernelGGL((k_score_atomic<P, 128>), grid, dim3(256), 0, s, ix, qb, q0, qt, prefix, pair_q, ws.scores, ld); break;
            case 256: hipLaunchKernelGGL((k_score_atomic<P, 256>), grid, dim3(256), 0, s, ix, qb, q0, qt, prefix, pair_q, ws.scores, ld); break;
            case 512: hipLaunchKernelGGL((k_score_atomic<P, 512>), grid, dim3(256), 0, s, ix, qb, q0, qt, prefix, pair_q, ws.scores, ld); break;
            case 1024: hipLaunchKernelGGL((k_score_atomic<P, 1024>), grid, dim3(256), 0, s, ix, qb, q0, qt, prefix, pair_q, ws.scores, ld); break;
            default: return hipErrorInvalidValue;
        }
        GS_CHECK_LAUNCH("k_score_atomic");
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    return launch_hist1(ix, qb, q0, qt, ws, s);
}

hipError_t launch_score_docpar(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const ScoreOpts& o,
                               const Workspace& ws, hipStream_t s) {
    (void)o;
    const int64_t ld = score_ld(ix.n_docs);
    const int per = 4096;
    const dim3 grid((unsigned)((ix.n_docs + per - 1) / per), (unsigned)qt);
    const size_t lds = (size_t)ix.vocab * 4;
    if (lds > 160 * 1024) return hipErrorInvalidValue;  // dense query table must fit one CU's LDS
    hipError_t e = by_precision(ix.precision, [&](auto pc) -> hipError_t {
        constexpr int P = decltype(pc)::value;
        if (lds > 65536) {
            const hipError_t a = hipFuncSetAttribute((const void*)k_score_docpar<P>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (a != hipSuccess) return a;
        }
        hipLaunchKernelGGL((k_score_docpar<P>), grid, dim3(1024), lds, s, ix, qb, q0, ws.scores, ld, per);
        GS_CHECK_LAUNCH("k_score_docpar");
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    return launch_hist1(ix, qb, q0, qt, ws, s);
}

hipError_t launch_hist1(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const Workspace& ws,
                        hipStream_t s) {
    const int64_t ld = score_ld(ix.n_docs);
    const int per = 65536;
    const dim3 grid((unsigned)((ix.n_docs + per - 1) / per), (unsigned)qt);
    hipLaunchKernelGGL(k_hist1, grid, dim3(512), 0, s, qb, q0, ix.n_docs, (const uint32_t*)ws.scores, ld, per,
                       ws.hist1);
    GS_CHECK_LAUNCH("k_hist1");
    return hipSuccess;
}

}  // namespace gs
