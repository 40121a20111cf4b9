// Exact per-query top-k over the score arrays (paper Sec. 4.2: a top-k over
// each query's accumulator row; Sec. 4.3: the result is exact).
//
// Every document is ranked by the 64-bit composite key
//     c = (score bits << 32) | (uint32)~doc_id
// Non-negative fp32 and int32 scores are monotone in their bit patterns, and
// ~id reverses the id order, so "c descending" is exactly "score descending,
// then doc id ascending", and all composites are distinct: the k largest
// composites are the unique answer, ties included.
//
// Pipeline for a tile of queries (all launches fixed, no host round trip):
//  1. the first 11-bit digit histogram (built by the scoring kernel);
//  2. k_select_first: find the digit bucket holding the k-th composite; if the
//     composites at or above that bucket fit the candidate buffer the query is
//     resolved, otherwise
//  3. k_refine_hist / k_refine_select (up to six rounds): radix-select refinement
//     over the full score array, 11 more bits per round, only for unresolved
//     queries (a degenerate distribution such as a query matching fewer than k
//     documents, where the answer is decided by doc ids);
//  4. k_filter: append every composite >= the threshold to the candidate buffer
//     (wavefront ballot + popcount for the append slot);
//  5. k_final: radix select on the candidates (8-bit digits, LDS histograms) for
//     the exact k-th composite, gather the k winners and place each one by its
//     rank among them (one pass of comparisons, no sort network needed).
// bf16 form: k_final also derives the error band of the k-th approximate score
// and rescores every candidate in the band in fp64 from the fp32 forward rows
// (ascending term order); k_band_filter / k_band_final handle the rare case in
// which the band reaches below the candidate threshold (a fused query first gets
// the rows of its other tiles, scoring phase 5).
//
// Fused candidate filtering (doc-tiled kernels, searches of 32+ queries): the
// seed tiles (every 8th doc tile) are scored first; k_seed_bound / k_seed_hist /
// k_seed_refine derive from them a lower bound of each query's k-th composite
// (a 22-bit bucket edge); the other tiles append every composite at or above it
// while they are scored (then writing no score rows for them and not counting
// them in the histogram), and step 4 scans only the seed tiles.
// k_select_first falls back to the full row (no bound, too many appended, or a
// refinement needed); such a query is listed, its other tiles are scored and
// counted again, and a second k_select_first pass redoes its step 2 from the
// complete histogram before steps 3 and 4.
//
// Wide-range check (fixed-point sums of the doc-tiled kernels, fp32 and bf16
// weights): a fixed-point sum is within an absolute bound E of the exact score,
// so a score far below the query's scale can miss the relative error budget. At
// step 2 the lower edge of the k-th composite's bucket (a lower bound of the
// k-th approximate score, also with fused filtering) is compared with the
// query's limit (E over the budget). Below it, the query is listed as wide
// range: every tile is scored again with fp64 accumulation of exact fp64
// products (its histogram counted anew), and the second k_select_first pass
// selects from those rows.
#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ unsigned long long comp_key(uint32_t key, uint32_t id) {
    return ((unsigned long long)key << 32) | (unsigned long long)(~id);
}

// One wavefront walks a kHistBins histogram from the top bin down and finds
// the bin d holding the need-th largest element: above(d) < need <= above(d)+h[d].
// Returns d; *above receives the count of elements in bins above d.
__device__ int hist_walk(const uint32_t* h, uint32_t need, uint32_t* above) {
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int PER = kHistBins / kWave;
    const int top = kHistBins - 1 - lane * PER;
    uint32_t s = 0;
    for (int j = 0; j < PER; j++) s += h[top - j];
    uint32_t incl = s;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += v;
    }
    const uint32_t excl = incl - s;
    const unsigned long long m = __ballot(excl < need && need <= incl);
    const int owner = m ? __ffsll((long long)m) - 1 : kWave - 1;
    int dsel = 0;
    uint32_t ab = 0;
    if (lane == owner) {
        uint32_t run = excl;
        dsel = top - (PER - 1);
        ab = run;
        for (int j = 0; j < PER; j++) {
            const uint32_t c = h[top - j];
            if (run + c >= need) { dsel = top - j; ab = run; break; }
            run += c;
        }
    }
    dsel = __shfl(dsel, owner, kWave);
    *above = __shfl(ab, owner, kWave);
    return dsel;
}

__device__ __forceinline__ int64_t kq_of(const DevBatch& qb, int q, int64_t N) {
    return min((int64_t)qb.k[q], N);
}

// pass 0 runs once every tile is scored; pass 1 runs after phase 3 for the queries that
// fell back, whose histograms are complete only then (phase 2 counts the seed tiles of a
// fused fp32/uint8 query only).
__global__ __launch_bounds__(64) void k_select_first(DevBatch qb, int32_t q0, int64_t N, int precision,
                                                     uint32_t* __restrict__ hist1, SelState* __restrict__ state,
                                                     uint32_t* __restrict__ counters, int32_t* __restrict__ rescore_list,
                                                     int pass, int wide_check) {
    const int ql = blockIdx.x, q = q0 + ql;
    SelState* st = state + ql;
    if (pass == 1 && st->rescore == 0) return;
    const int64_t kq = kq_of(qb, q, N);
    if (kq == 0) {
        if (threadIdx.x == 0) st->resolved = 2;
        return;
    }
    uint32_t* h = hist1 + (int64_t)ql * kHistBins;
    uint32_t above;
    const int d = hist_walk(h, (uint32_t)kq, &above);
    const int fs = qb.first_shift[q];
    if (pass == 0 && wide_check) {
        // lower edge of the k-th composite's bucket: its score bits with the low ones cleared
        const float s_lo = __uint_as_float((uint32_t)(((unsigned long long)d << fs) >> 32));
        if ((double)s_lo < qb.q_wide_lim[q]) {
            __syncthreads();  // every lane is done reading the histogram
            for (int i = threadIdx.x; i < kHistBins; i += 64) h[i] = 0u;  // the fp64 pass counts anew
            if (threadIdx.x == 0) {
                st->fused = 0;
                st->n_cand = 0;
                st->resolved = 0;
                st->rescore = 2;
                rescore_list[atomicAdd(&counters[8], 1u)] = ql;
            }
            return;
        }
    }
    if (threadIdx.x != 0) return;
    const int64_t ge = (int64_t)above + h[d];
    int64_t kept;  // composites at or above the filter threshold
    if (precision == kBF16 && d > 0 && ge + h[d - 1] <= kCandCap) {
        // one bin lower: the bf16 error band below the k-th score then lies inside the candidates
        st->resolved = 1;
        st->lo = (unsigned long long)(d - 1) << fs;
        kept = ge + h[d - 1];
    } else if (ge <= kCandCap) {
        st->resolved = 1;
        st->lo = (unsigned long long)d << fs;
        kept = ge;
    } else {
        st->resolved = 0;
        st->prefix = (unsigned long long)d << fs;
        st->shift = fs;
        st->k_rem = (int32_t)(kq - above);
        kept = 0;
    }
    // Fused filtering holds the appended candidates (every composite >= the seed bound
    // of the non-seed tiles; the bound is at most the threshold) and the filter then
    // scans the seed tiles only. Otherwise the appended ones are dropped and the whole
    // row is scanned: no bound, too many appended, or a refinement is needed.
    if (st->fused == 1 && (st->resolved != 1 || st->fused_over || (int64_t)st->n_cand + kept > kCandCap)) {
        st->fused = 0;
        st->n_cand = 0;
        st->rescore = 1;  // its non-seed rows were not written: score them again
        rescore_list[atomicAdd(&counters[8], 1u)] = ql;
    }
}

// Fused filtering, after the seed tiles are scored. The bound of a query is the
// lower edge of a two-digit bucket (22 bits of the composite key) that holds the
// k-th largest composite among the seed tiles' documents: k_seed_bound finds the
// first-digit bin from the histogram the seed tiles built, k_seed_hist counts the
// next digit within that bin over the seed tiles' scores, and k_seed_refine picks
// the sub-bin. The k-th largest over all documents is at least as large, so the
// bound never exceeds it. With fewer than k seed documents there is no bound.
__global__ __launch_bounds__(64) void k_seed_bound(DevBatch qb, int32_t q0, int64_t N,
                                                   const uint32_t* __restrict__ hist1, SelState* __restrict__ state) {
    const int ql = blockIdx.x, q = q0 + ql;
    SelState* st = state + ql;
    const int64_t kq = kq_of(qb, q, N);
    if (kq == 0) {
        if (threadIdx.x == 0) st->fused = 0;
        return;
    }
    const uint32_t* h = hist1 + (int64_t)ql * kHistBins;
    uint32_t above;
    const int d = hist_walk(h, (uint32_t)kq, &above);
    if (threadIdx.x != 0) return;
    if ((int64_t)above + h[d] < kq) {
        st->fused = 0;
        return;
    }
    const int fs = qb.first_shift[q];
    st->prefix = (unsigned long long)d << fs;
    st->shift = fs;
    st->k_rem = (int32_t)(kq - above);
    st->fused = 2;  // refining
}

__global__ __launch_bounds__(512) void k_seed_hist(int64_t N, const uint32_t* __restrict__ S, int64_t ld,
                                                   int tile_shift, int stride, const SelState* __restrict__ state,
                                                   uint32_t* __restrict__ hist_ref) {
    __shared__ uint32_t hist[kHistBins];
    const int ql = blockIdx.y;
    const SelState st = state[ql];
    if (st.fused != 2) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < kHistBins; i += 512) hist[i] = 0u;
    __syncthreads();
    const int shift = st.shift, nshift = max(shift - kHistBits, 0);
    const unsigned long long want = st.prefix >> shift;
    const unsigned long long mask = (1ull << (shift - nshift)) - 1ull;
    const int64_t d0 = ((int64_t)blockIdx.x * stride) << tile_shift, d1 = min(N, d0 + (1ll << tile_shift));
    const uint32_t* Sq = S + (int64_t)ql * ld;
    // four rounds of 16-byte loads before the first count (a lane past the tile reads its last
    // aligned four scores and counts nothing)
    constexpr int R = 4;
    const int64_t last = (d1 - 1) & ~3ll;  // d + 3 < ld: rows are padded to 64
    for (int64_t d0r = d0 + 4 * tid; d0r < d1; d0r += 4 * 512 * R) {
        uint4 v[R];
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = *reinterpret_cast<const uint4*>(Sq + min(d0r + r * 2048, last));
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int64_t d = d0r + r * 2048;
            const uint32_t vs[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const unsigned long long c = comp_key(vs[j], (uint32_t)(d + j));
                if (d + j < d1 && (c >> shift) == want) atomicAdd(&hist[(c >> nshift) & mask], 1u);
            }
        }
    }
    __syncthreads();
    for (int b = tid; b < kHistBins; b += 512)
        if (hist[b]) atomicAdd(&hist_ref[(int64_t)ql * kHistBins + b], hist[b]);
}

__global__ __launch_bounds__(64) void k_seed_refine(uint32_t* __restrict__ hist_ref, SelState* __restrict__ state) {
    const int ql = blockIdx.x;
    SelState* st = state + ql;
    if (st->fused != 2) return;
    uint32_t* h = hist_ref + (int64_t)ql * kHistBins;
    uint32_t above;
    const int e = hist_walk(h, (uint32_t)st->k_rem, &above);
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += 64) h[i] = 0u;  // the refinement passes reuse the rows
    if (threadIdx.x != 0) return;
    const int nshift = max(st->shift - kHistBits, 0);
    st->bound = st->prefix | ((unsigned long long)e << nshift);
    st->prefix = 0;
    st->shift = 0;
    st->k_rem = 0;
    st->fused = 1;
}

__global__ __launch_bounds__(512) void k_refine_hist(int32_t q0, int64_t N, const uint32_t* __restrict__ S, int64_t ld,
                                                     const SelState* __restrict__ state, uint32_t* __restrict__ hist_ref) {
    __shared__ uint32_t hist[kHistBins];
    const int ql = blockIdx.y;
    const SelState st = state[ql];
    if (st.resolved != 0) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < kHistBins; i += 512) hist[i] = 0u;
    __syncthreads();
    const int shift = st.shift, nshift = max(shift - kHistBits, 0);
    const unsigned long long want = st.prefix >> shift;
    const unsigned long long mask = (1ull << (shift - nshift)) - 1ull;
    // a few workgroups per query stride over the row: the launch stays cheap when
    // no query needs a refinement (the usual case)
    const uint32_t* Sq = S + (int64_t)ql * ld;
    for (int64_t d = (int64_t)blockIdx.x * 512 + tid; d < N; d += (int64_t)gridDim.x * 512) {
        const unsigned long long c = comp_key(Sq[d], (uint32_t)d);
        if ((c >> shift) == want) atomicAdd(&hist[(c >> nshift) & mask], 1u);
    }
    __syncthreads();
    for (int b = tid; b < kHistBins; b += 512)
        if (hist[b]) atomicAdd(&hist_ref[(int64_t)ql * kHistBins + b], hist[b]);
}

__global__ __launch_bounds__(64) void k_refine_select(DevBatch qb, int32_t q0, int64_t N,
                                                      uint32_t* __restrict__ hist_ref, SelState* __restrict__ state) {
    const int ql = blockIdx.x, q = q0 + ql;
    SelState* st = state + ql;
    if (st->resolved != 0) return;
    uint32_t* h = hist_ref + (int64_t)ql * kHistBins;
    const int64_t kq = kq_of(qb, q, N);
    uint32_t above;
    const int d = hist_walk(h, (uint32_t)st->k_rem, &above);
    const uint32_t hd = h[d];
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += 64) h[i] = 0u;
    if (threadIdx.x != 0) return;
    const int nshift = max(st->shift - kHistBits, 0);
    const unsigned long long prefix = st->prefix | ((unsigned long long)d << nshift);
    const int32_t k_rem = st->k_rem - (int32_t)above;
    st->passes += 1;
    if ((kq - k_rem) + (int64_t)hd <= kCandCap) {
        st->resolved = 1;
        st->lo = prefix;
    } else {
        st->prefix = prefix;
        st->shift = nshift;
        st->k_rem = k_rem;
    }
}

// Append every composite >= the query's threshold to its candidate buffer.
// Each lane reads four consecutive scores with one 16-byte load (rows are
// 64-aligned). A wavefront reserves slots for its hits (ballot + popcount) in
// a workgroup-local LDS stage, so the scan never waits on a global atomic; at
// the end the workgroup takes one range of the query's buffer and copies the
// stage out. Hits that find the stage full are appended to the global buffer
// directly (slot from a global atomic), so any number of hits is handled.
constexpr int kFilterStage = 4096;

__device__ __forceinline__ void append_global(SelState* st, unsigned long long* C, bool take,
                                              unsigned long long c, int lane) {
    const unsigned long long m = __ballot(take);
    if (m == 0) return;
    int slot = 0;
    if (lane == 0) slot = atomicAdd(&st->n_cand, __popcll(m));
    slot = __shfl(slot, 0, kWave) + __popcll(m & ((1ull << lane) - 1ull));
    if (take) {
        if (slot < kCandCap) C[slot] = c;
        else st->overflow = 1;
    }
}

__global__ __launch_bounds__(512) void k_filter(int32_t q0, int64_t N, const uint32_t* __restrict__ S, int64_t ld,
                                                int per_block, SelState* __restrict__ state,
                                                unsigned long long* __restrict__ cand, int tile_shift,
                                                int seed_stride) {
    __shared__ unsigned long long stage[kFilterStage];
    __shared__ int n_stage, g_base;
    const int ql = blockIdx.y;
    SelState* st = state + ql;
    if (st->resolved != 1) return;
    const unsigned long long lo = st->lo;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    if (tid == 0) n_stage = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per_block, b1 = min(N, b0 + per_block);  // per_block % 256 == 0
    const uint32_t* Sq = S + (int64_t)ql * ld;
    unsigned long long* C = cand + (int64_t)ql * kCandCap;
    // Four rounds of 16-byte loads are issued before the first test (a single load in flight
    // per lane left the scan at about half the HBM rate). A lane past the range reads the
    // range's last aligned four scores instead (no branch around the load) and tests nothing.
    auto scan = [&](int64_t d0, int64_t d1) {  // d0 % 256 == 0
        constexpr int R = 4;
        const int64_t last = (d1 - 1) & ~3ll;  // d + 3 < ld: rows are padded to 64
        for (int64_t wb = d0 + (int64_t)wave * kWave * 4; wb < d1; wb += 512 * 4 * R) {
            uint4 v[R];
#pragma unroll
            for (int r = 0; r < R; r++)
                v[r] = *reinterpret_cast<const uint4*>(Sq + min(wb + r * 2048 + (int64_t)lane * 4, last));
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int64_t d = wb + r * 2048 + (int64_t)lane * 4;
                const uint32_t vs[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const unsigned long long c = comp_key(vs[j], (uint32_t)(d + j));
                    const bool take = d + j < d1 && c >= lo;
                    const unsigned long long m = __ballot(take);
                    if (m == 0) continue;
                    int slot = 0;
                    if (lane == 0) slot = atomicAdd(&n_stage, __popcll(m));
                    slot = __shfl(slot, 0, kWave) + __popcll(m & ((1ull << lane) - 1ull));
                    if (take && slot < kFilterStage) stage[slot] = c;
                    append_global(st, C, take && slot >= kFilterStage, c, lane);
                }
            }
        }
    };
    if (st->fused == 1 && seed_stride > 0) {
        // fused filtering: the other tiles' candidates were appended while they were
        // scored; only the seed tiles' documents are scanned here
        for (int64_t t = b0 >> tile_shift; (t << tile_shift) < b1; t++)
            if (t % seed_stride == 0) scan(max(b0, t << tile_shift), min(b1, (t + 1) << tile_shift));
    } else {
        scan(b0, b1);
    }
    __syncthreads();
    const int n = min(n_stage, kFilterStage);
    if (tid == 0) g_base = n ? atomicAdd(&st->n_cand, n) : 0;
    __syncthreads();
    const int base = g_base;
    for (int i = tid; i < n; i += 512) {
        if (base + i < kCandCap) C[base + i] = stage[i];
        else st->overflow = 1;
    }
}

// fp64 rescoring of the docs bid[0..nb) against the query held in LDS (terms
// ascending), by the whole workgroup: a wavefront takes 4 docs, 16 lanes each.
// Lane `sub` walks entries sub, sub+16, ... of the doc's forward row (sorted by
// term) and merges them with the query terms; each step's nonzero products are
// then added in row order (ascending term), one shuffle at a time, so the sum
// is the same sequence of fp64 additions as a serial walk of the row.
__device__ void rescore_band(const DevIndex& ix, const int32_t* bid, double* bs, int nb, const int32_t* qt,
                             const float* qw, int nq) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int grp = lane >> 4, sub = lane & 15;
    for (int base = wave * 4; base < nb; base += nw * 4) {
        const int i = base + grp;
        int64_t a = 0;
        int len = 0;
        if (i < nb) {
            const int64_t doc = bid[i];
            a = ix.fwd_row_ptr[doc];
            len = (int)(ix.fwd_row_ptr[doc + 1] - a);
        }
        int maxlen = len;
        maxlen = max(maxlen, __shfl_xor(maxlen, 16, kWave));
        maxlen = max(maxlen, __shfl_xor(maxlen, 32, kWave));
        double s = 0.0;
        int j = 0;
        for (int off = 0; off < maxlen; off += 16) {
            const int e = off + sub;
            double pr = 0.0;
            if (e < len) {
                const int t = ix.fwd_term[a + e];
                while (j < nq && qt[j] < t) j++;
                if (j < nq && qt[j] == t) pr = (double)qw[j] * (double)ix.fwd_w[a + e];
            }
            uint32_t mm = (uint32_t)(__ballot(pr != 0.0) >> (grp * 16)) & 0xFFFFu;
            while (__any(mm != 0u)) {
                const int src = grp * 16 + (mm ? __ffs(mm) - 1 : 0);
                const double v = __shfl(pr, src, kWave);
                if (mm) {
                    s += v;
                    mm &= mm - 1u;
                }
            }
        }
        if (sub == 0 && i < nb) bs[i] = s;
    }
}

// One wavefront walks a 256-bin histogram from the top bin down for the bin
// holding the need-th largest element; writes it and the count above it.
__device__ void walk256(const uint32_t* hist, uint32_t need, int* d_out, uint32_t* above_out) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t s = 0;
    for (int j = 0; j < 4; j++) s += hist[255 - lane * 4 - j];
    uint32_t incl = s;
    for (int dd = 1; dd < kWave; dd <<= 1) {
        const uint32_t v = __shfl_up(incl, dd, kWave);
        if (lane >= dd) incl += v;
    }
    const uint32_t excl = incl - s;
    const unsigned long long m = __ballot(excl < need && need <= incl);
    const int owner = m ? __ffsll((long long)m) - 1 : kWave - 1;
    if (lane == owner) {
        uint32_t run = excl;
        int dsel = 255 - lane * 4 - 3;
        uint32_t ab = run;
        for (int j = 0; j < 4; j++) {
            const uint32_t c = hist[255 - lane * 4 - j];
            if (run + c >= need) {
                dsel = 255 - lane * 4 - j;
                ab = run;
                break;
            }
            run += c;
        }
        *d_out = dsel;
        *above_out = ab;
    }
}

// The first kq band members by (fp64 score desc, doc id asc), written to ids /
// sc. Keys (score bits, ~doc id) are distinct and ordered like that pair (scores
// are >= 0, so their bits are monotone): a radix select with 8-bit digits (8 of
// the score, then 4 of ~id) finds the kq-th largest key, the kq keys at or above
// it are gathered into LDS, and each is placed by its rank among them.
// LDS used by band_topk: hist[256], wsc[kMaxK], wid[kMaxK] and three scalars
// (the caller may hand in arrays it no longer needs).
struct BandLds {
    uint32_t* hist;
    unsigned long long* wsc;
    int32_t* wid;
    int* d;
    uint32_t* above;
    int* cnt;
};

__device__ void band_topk(const double* bs, const int32_t* bid, int nb, int64_t kq, int32_t* ids, double* sc,
                          const BandLds& L) {
    const int tid = threadIdx.x, nt = blockDim.x;
    unsigned long long ph = 0, mh = 0;
    uint32_t pl = 0, ml = 0;
    uint32_t need = (uint32_t)min<int64_t>(kq, nb);
    if ((uint32_t)nb > need) {
        for (int d = 0; d < 12; d++) {
            for (int i = tid; i < 256; i += nt) L.hist[i] = 0u;
            __syncthreads();
            for (int i = tid; i < nb; i += nt) {
                const unsigned long long h = (unsigned long long)__double_as_longlong(bs[i]);
                const uint32_t l = ~(uint32_t)bid[i];
                if ((h & mh) == ph && (l & ml) == pl) {
                    const uint32_t dig = d < 8 ? (uint32_t)(h >> (56 - 8 * d)) & 255u : (l >> (88 - 8 * d)) & 255u;
                    atomicAdd(&L.hist[dig], 1u);
                }
            }
            __syncthreads();
            if (tid < kWave) walk256(L.hist, need, L.d, L.above);
            __syncthreads();
            const int dsel = *L.d;
            need -= *L.above;
            const uint32_t hd = L.hist[dsel];
            __syncthreads();
            if (d < 8) {
                ph |= (unsigned long long)dsel << (56 - 8 * d);
                mh |= 255ull << (56 - 8 * d);
            } else {
                pl |= (uint32_t)dsel << (88 - 8 * d);  // id digits: bits 31..24, ..., 7..0
                ml |= 255u << (88 - 8 * d);
            }
            if (hd == need) break;
        }
    }
    if (tid == 0) *L.cnt = 0;
    __syncthreads();
    for (int i = tid; i < nb; i += nt) {
        const unsigned long long h = (unsigned long long)__double_as_longlong(bs[i]);
        const uint32_t l = ~(uint32_t)bid[i];
        if (h > ph || (h == ph && l >= pl)) {
            const int pos = atomicAdd(L.cnt, 1);
            if (pos < kMaxK) {
                L.wsc[pos] = h;
                L.wid[pos] = bid[i];
            }
        }
    }
    __syncthreads();
    const int m = min(*L.cnt, kMaxK);
    for (int i = tid; i < m; i += nt) {
        const unsigned long long si = L.wsc[i];
        const int32_t di = L.wid[i];
        int r = 0;
        for (int j = 0; j < m; j++) {
            const unsigned long long sj = L.wsc[j];
            r += (sj > si) || (sj == si && L.wid[j] < di);
        }
        if (r < kq) {
            ids[r] = di;
            sc[r] = __longlong_as_double((long long)si);
        }
    }
}

// Band of the bf16 form. Every doc's approximate score satisfies
//   s(1-delta) - E <= approx <= s(1+delta) + E
// (delta: relative error of the stored bf16 weights and of the score's
// arithmetic; E: the fixed-point error bound). Then approx_k <= (1+delta) s_k + E,
// and every true top-k doc has
// approx >= s(1-delta) - E >= (approx_k - E)(1-delta)/(1+delta) - E = tau.
__device__ __forceinline__ double band_tau(float sk, double delta, double abs_err) {
    const double d = delta;
    const double t = ((double)sk - abs_err) * (1.0 - d) / (1.0 + d) - abs_err;
    return t > 0.0 ? t * (1.0 - 1e-12) : 0.0;
}

// Error terms of the bf16 band for a query: relative (delta) and absolute (E).
// Fixed-point sums: the stored-weight and final fp32 roundings, plus E. The fp64
// pass (wide range): exact products, an fp64 sum (relative error below 1e-13 for
// 256 terms) rounded once to fp32, no E. fp32 sums (global-atomic and
// document-parallel kernels): each product and addition rounds, so delta also
// covers gamma_m = m u / (1 - m u) with u = 2^-24 for m query terms; no E.
__device__ __forceinline__ void band_error(const DevBatch& qb, int q, int acc, int rescore, int m, double* rel,
                                           double* abs_err) {
    const double d = (double)qb.delta[q];
    if (rescore == 2) {
        *rel = d + 1e-12;
        *abs_err = 0.0;
    } else if (acc == kAccFloat) {
        const double mu = (double)(m + 1) * 0x1p-24;
        *rel = (1.0 + d) * (1.0 + mu / (1.0 - mu)) - 1.0;
        *abs_err = 0.0;
    } else {
        *rel = d;
        *abs_err = qb.q_abs_err[q];
    }
}

template <int P>
__global__ __launch_bounds__(1024) void k_final(DevIndex ix, DevBatch qb, int32_t q0, SelState* __restrict__ state,
                                                const unsigned long long* __restrict__ cand,
                                                double* __restrict__ band_s, int32_t* __restrict__ band_id,
                                                int32_t* __restrict__ out_ids, void* __restrict__ out_scores, int acc,
                                                uint32_t* __restrict__ counters, int32_t* __restrict__ rescore_list) {
    __shared__ unsigned long long sel[kMaxK];
    __shared__ uint32_t hist[256];
    __shared__ int sh_d, sh_cnt;
    __shared__ uint32_t sh_above;
    __shared__ int32_t sq_t[kMaxQueryNnz];
    __shared__ float sq_w[kMaxQueryNnz];
    __shared__ int32_t band_wid[P == kBF16 ? kMaxK : 1];
    const int tid = threadIdx.x;
    const int ql = blockIdx.x, q = q0 + ql;
    SelState* st = state + ql;
    const int64_t kq = kq_of(qb, q, ix.n_docs);
    const int kmax = qb.k_max;
    int32_t* ids = out_ids + (int64_t)q * kmax;
    for (int i = tid; i < kmax; i += 1024) {
        if (i >= kq) {
            ids[i] = -1;
            if (P == kBF16) ((double*)out_scores)[(int64_t)q * kmax + i] = 0.0;
            else ((uint32_t*)out_scores)[(int64_t)q * kmax + i] = 0u;
        }
    }
    if (kq == 0) return;
    const int n = min(st->n_cand, kCandCap);
    const unsigned long long* C = cand + (int64_t)ql * kCandCap;

    // radix select of the kq-th largest composite among the n candidates
    unsigned long long prefix = 0;
    int shift = 64;
    uint32_t need = (uint32_t)kq;
    if (n > kq) {
        while (shift > 0) {
            const int nshift = shift - 8;
            for (int i = tid; i < 256; i += 1024) hist[i] = 0u;
            __syncthreads();
            for (int i = tid; i < n; i += 1024) {
                const unsigned long long c = C[i];
                if (shift == 64 || (c >> shift) == (prefix >> shift)) atomicAdd(&hist[(c >> nshift) & 255ull], 1u);
            }
            __syncthreads();
            if (tid < kWave) {
                // 256 bins, 4 per lane, walked from the top
                const int lane = tid;
                uint32_t s = 0;
                for (int j = 0; j < 4; j++) s += hist[255 - lane * 4 - j];
                uint32_t incl = s;
                for (int dd = 1; dd < kWave; dd <<= 1) {
                    const uint32_t v = __shfl_up(incl, dd, kWave);
                    if (lane >= dd) incl += v;
                }
                const uint32_t excl = incl - s;
                const unsigned long long m = __ballot(excl < need && need <= incl);
                const int owner = m ? __ffsll((long long)m) - 1 : kWave - 1;
                if (lane == owner) {
                    uint32_t run = excl;
                    int dsel = 255 - lane * 4 - 3;
                    uint32_t ab = run;
                    for (int j = 0; j < 4; j++) {
                        const uint32_t c = hist[255 - lane * 4 - j];
                        if (run + c >= need) { dsel = 255 - lane * 4 - j; ab = run; break; }
                        run += c;
                    }
                    sh_d = dsel;
                    sh_above = ab;
                }
            }
            __syncthreads();
            const int d = sh_d;
            need -= sh_above;
            prefix |= (unsigned long long)d << nshift;
            shift = nshift;
            const uint32_t hd = hist[d];
            __syncthreads();
            if (hd == need) break;
        }
    }
    // gather the kq winners: composites whose bits above `shift` are >= the prefix's
    if (tid == 0) sh_cnt = 0;
    __syncthreads();
    for (int i = tid; i < n; i += 1024) {
        const unsigned long long c = C[i];
        const bool win = (shift == 64) || (shift == 0 ? c >= prefix : (c >> shift) >= (prefix >> shift));
        if (win) {
            const int pos = atomicAdd(&sh_cnt, 1);
            if (pos < kMaxK) sel[pos] = c;
        }
    }
    __syncthreads();
    const int m = min(sh_cnt, kMaxK);
    if (P != kBF16) {
        for (int i = tid; i < m; i += 1024) {
            const unsigned long long c = sel[i];
            int r = 0;
            for (int j = 0; j < m; j++) r += sel[j] > c;
            if (r < kq) {
                ids[r] = (int32_t)(~(uint32_t)c);
                ((uint32_t*)out_scores)[(int64_t)q * kmax + r] = (uint32_t)(c >> 32);
            }
        }
        return;
    }
    // bf16: exact k-th approximate score, then the error band and fp64 rescoring
    __shared__ unsigned long long sh_min;
    if (tid == 0) sh_min = ~0ull;
    __syncthreads();
    for (int i = tid; i < m; i += 1024) atomicMin(&sh_min, sel[i]);
    const int64_t qa = qb.q_row_ptr[q];
    const int nq = (int)(qb.q_row_ptr[q + 1] - qa);
    for (int i = tid; i < nq; i += 1024) {
        sq_t[i] = qb.q_term[qa + i];
        sq_w[i] = qb.q_w[qa + i];
    }
    __syncthreads();
    const float sk = __uint_as_float((uint32_t)(sh_min >> 32));
    double rel_err, abs_err;
    band_error(qb, q, acc, st->rescore, nq, &rel_err, &abs_err);
    double* bs = band_s + (int64_t)ql * kCandCap;
    int32_t* bid = band_id + (int64_t)ql * kCandCap;
    int nb = 0;
    if (sk == 0.0f) {
        // fewer than k docs share a term with the query: the k winners are every doc with a
        // positive score plus the lowest-id zero-score docs. A zero approximate score is exact
        // here: from fp32 or fp64 sums (no product of admissible weights underflows to 0), or
        // from fixed point only if no positive product can round to 0 units (otherwise the
        // wide-range check sent the query to the fp64 pass: its k-th bucket starts at 0).
        for (int i = tid; i < m; i += 1024) bid[i] = (int32_t)(~(uint32_t)sel[i]);
        nb = m;
    } else {
        const double tau = band_tau(sk, rel_err, abs_err);
        // with fused filtering the other tiles' candidates start at the bound, the seed tiles' at lo
        const unsigned long long lo = st->fused == 1 ? max(st->lo, st->bound) : st->lo;
        const double lo_val = (double)__uint_as_float((uint32_t)(lo >> 32));
        const bool inside = tau > 0.0 && (((uint32_t)lo == 0u) ? (lo_val <= tau) : (lo_val < tau));
        if (!inside) {
            if (tid == 0) {
                st->need_band_pass = 1;
                st->tau = tau;
                if (st->fused == 1) {  // its other tiles wrote no rows: score them for the band pass
                    st->rescore = 3;
                    rescore_list[atomicAdd(&counters[8], 1u)] = ql;
                }
            }
            return;
        }
        if (tid == 0) sh_cnt = 0;
        __syncthreads();
        for (int i = tid; i < n; i += 1024) {
            const unsigned long long c = C[i];
            const double v = (double)__uint_as_float((uint32_t)(c >> 32));
            if (v > 0.0 && v >= tau) bid[atomicAdd(&sh_cnt, 1)] = (int32_t)(~(uint32_t)c);
        }
        __syncthreads();
        nb = sh_cnt;
    }
    __threadfence_block();
    __syncthreads();
    rescore_band(ix, bid, bs, nb, sq_t, sq_w, nq);
    if (tid == 0) st->band = nb;
    __threadfence_block();
    __syncthreads();
    // sel (the approximate winners) is no longer needed: it holds the exact winners' scores
    band_topk(bs, bid, nb, kq, ids, (double*)out_scores + (int64_t)q * kmax,
              BandLds{hist, sel, band_wid, &sh_d, &sh_above, &sh_cnt});
}

__global__ __launch_bounds__(512) void k_band_filter(int32_t q0, int64_t N, const uint32_t* __restrict__ S,
                                                     int64_t ld, int per_block, SelState* __restrict__ state,
                                                     int32_t* __restrict__ band_id) {
    const int ql = blockIdx.y;
    SelState* st = state + ql;
    if (st->need_band_pass != 1) return;
    const double tau = st->tau;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int64_t d0 = (int64_t)blockIdx.x * per_block, d1 = min(N, d0 + per_block);
    const uint32_t* Sq = S + (int64_t)ql * ld;
    int32_t* B = band_id + (int64_t)ql * kCandCap;
    for (int64_t wb = d0 + wave * kWave; wb < d1; wb += 512) {
        const int64_t d = wb + lane;
        const double v = d < d1 ? (double)__uint_as_float(Sq[d]) : 0.0;
        const bool take = v > 0.0 && v >= tau;
        const unsigned long long m = __ballot(take);
        if (m == 0) continue;
        int slot = 0;
        if (lane == 0) slot = atomicAdd(&st->band, __popcll(m));
        slot = __shfl(slot, 0, kWave) + __popcll(m & ((1ull << lane) - 1ull));
        if (take) {
            if (slot < kCandCap) B[slot] = (int32_t)d;
            else st->overflow = 1;
        }
    }
}

__global__ __launch_bounds__(1024) void k_band_final(DevIndex ix, DevBatch qb, int32_t q0, SelState* __restrict__ state,
                                                     double* __restrict__ band_s, int32_t* __restrict__ band_id,
                                                     int32_t* __restrict__ out_ids, double* __restrict__ out_scores) {
    __shared__ int32_t sq_t[kMaxQueryNnz];
    __shared__ float sq_w[kMaxQueryNnz];
    __shared__ uint32_t hist[256];
    __shared__ unsigned long long wsc[kMaxK];
    __shared__ int32_t wid[kMaxK];
    __shared__ int sh_d, sh_cnt;
    __shared__ uint32_t sh_above;
    const int ql = blockIdx.x, q = q0 + ql;
    SelState* st = state + ql;
    if (st->need_band_pass != 1) return;
    const int tid = threadIdx.x;
    const int64_t qa = qb.q_row_ptr[q];
    const int nq = (int)(qb.q_row_ptr[q + 1] - qa);
    for (int i = tid; i < nq; i += 1024) {
        sq_t[i] = qb.q_term[qa + i];
        sq_w[i] = qb.q_w[qa + i];
    }
    __syncthreads();
    const int64_t kq = kq_of(qb, q, ix.n_docs);
    if (st->overflow) {
        // the band does not fit the buffer: the row is left as padding and flagged
        for (int i = tid; i < kq; i += 1024) {
            out_ids[(int64_t)q * qb.k_max + i] = -1;
            out_scores[(int64_t)q * qb.k_max + i] = 0.0;
        }
        return;
    }
    const int nb = min(st->band, kCandCap);
    double* bs = band_s + (int64_t)ql * kCandCap;
    int32_t* bid = band_id + (int64_t)ql * kCandCap;
    rescore_band(ix, bid, bs, nb, sq_t, sq_w, nq);
    __threadfence_block();
    __syncthreads();
    band_topk(bs, bid, nb, kq, out_ids + (int64_t)q * qb.k_max, out_scores + (int64_t)q * qb.k_max,
              BandLds{hist, wsc, wid, &sh_d, &sh_above, &sh_cnt});
}

__global__ void k_diag(int32_t q0, int32_t qt, const SelState* __restrict__ state, int32_t* __restrict__ diag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= qt) return;
    const SelState st = state[i];
    int32_t* o = diag + (int64_t)(q0 + i) * kDiagWords;
    o[0] = st.n_cand;
    o[1] = st.passes;
    o[2] = st.band;
    o[3] = st.overflow;
    o[4] = st.rescore;
    o[5] = st.fused == 1 ? 1 : 0;
    o[6] = st.pruned;
    o[7] = 0;
}

}  // namespace

hipError_t launch_seed_bound(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const Workspace& ws,
                             hipStream_t s, int tile_shift, int stride) {
    hipLaunchKernelGGL(k_seed_bound, dim3(qt), dim3(64), 0, s, qb, q0, ix.n_docs, (const uint32_t*)ws.hist1,
                       ws.state);
    GS_CHECK_LAUNCH("k_seed_bound");
    const int64_t n_tiles = (ix.n_docs + (1ll << tile_shift) - 1) >> tile_shift;
    const int64_t seeds = (n_tiles + stride - 1) / stride;
    hipLaunchKernelGGL(k_seed_hist, dim3((unsigned)seeds, (unsigned)qt), dim3(512), 0, s, ix.n_docs,
                       (const uint32_t*)ws.scores, ws.ld, tile_shift, stride, (const SelState*)ws.state, ws.hist_ref);
    GS_CHECK_LAUNCH("k_seed_hist");
    hipLaunchKernelGGL(k_seed_refine, dim3(qt), dim3(64), 0, s, ws.hist_ref, ws.state);
    GS_CHECK_LAUNCH("k_seed_refine");
    return hipSuccess;
}

hipError_t launch_select(const DevIndex& ix, const DevBatch& qb, int32_t q0, int32_t qt, const Workspace& ws,
                         int32_t* out_ids, void* out_scores, int32_t* diag, hipStream_t s, int acc, int tile_shift,
                         int seed_stride, const ScoreOpts* phase3, bool wide) {
    const int64_t N = ix.n_docs;
    const int per = 65536;
    const dim3 grid_scan((unsigned)((N + per - 1) / per), (unsigned)qt);
    const int wide_check = acc == kAccFixed ? 1 : 0;
    hipLaunchKernelGGL(k_select_first, dim3(qt), dim3(64), 0, s, qb, q0, N, ix.precision, ws.hist1, ws.state,
                       ws.counters, ws.rescore_list, 0, wide_check);
    GS_CHECK_LAUNCH("k_select_first");
    if (phase3 || wide) {  // rows (and counts) of the listed queries: fused fallback, wide range
        hipError_t e = hipSuccess;
        if (phase3) e = launch_score_tiled(ix, qb, q0, qt, *phase3, ws, s, 3);
        if (e == hipSuccess && wide) e = launch_score_wide(ix, qb, q0, ws, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_select_first, dim3(qt), dim3(64), 0, s, qb, q0, N, ix.precision, ws.hist1, ws.state,
                           ws.counters, ws.rescore_list, 1, 0);
        GS_CHECK_LAUNCH("k_select_first");
    }
    auto final_pass = [&]() -> hipError_t {
        switch (ix.precision) {
            case kFP32:
                hipLaunchKernelGGL(k_final<kFP32>, dim3(qt), dim3(1024), 0, s, ix, qb, q0, ws.state,
                                   (const unsigned long long*)ws.cand, ws.band_s, ws.band_id, out_ids, out_scores,
                                   acc, ws.counters, ws.rescore_list);
                break;
            case kU8:
                hipLaunchKernelGGL(k_final<kU8>, dim3(qt), dim3(1024), 0, s, ix, qb, q0, ws.state,
                                   (const unsigned long long*)ws.cand, ws.band_s, ws.band_id, out_ids, out_scores,
                                   acc, ws.counters, ws.rescore_list);
                break;
            default:
                hipLaunchKernelGGL(k_final<kBF16>, dim3(qt), dim3(1024), 0, s, ix, qb, q0, ws.state,
                                   (const unsigned long long*)ws.cand, ws.band_s, ws.band_id, out_ids, out_scores,
                                   acc, ws.counters, ws.rescore_list);
                break;
        }
        GS_CHECK_LAUNCH("k_final");
        return hipSuccess;
    };
    if (N == 0) return final_pass();  // empty collection: padding only
    for (int p = 0; p < kRefinePasses; p++) {
        hipLaunchKernelGGL(k_refine_hist, dim3(8, (unsigned)qt), dim3(512), 0, s, q0, N, (const uint32_t*)ws.scores,
                           ws.ld, (const SelState*)ws.state, ws.hist_ref);
        GS_CHECK_LAUNCH("k_refine_hist");
        hipLaunchKernelGGL(k_refine_select, dim3(qt), dim3(64), 0, s, qb, q0, N, ws.hist_ref, ws.state);
        GS_CHECK_LAUNCH("k_refine_select");
    }
    hipLaunchKernelGGL(k_filter, grid_scan, dim3(512), 0, s, q0, N, (const uint32_t*)ws.scores, ws.ld, per, ws.state,
                       ws.cand, seed_stride > 0 ? tile_shift : 16, seed_stride);
    GS_CHECK_LAUNCH("k_filter");
    hipError_t e = final_pass();
    if (e != hipSuccess) return e;
    if (ix.precision == kBF16) {
        if (phase3) {  // fused queries whose band reaches below their candidates: the other tiles' rows
            e = launch_score_tiled(ix, qb, q0, qt, *phase3, ws, s, 5);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_band_filter, grid_scan, dim3(512), 0, s, q0, N, (const uint32_t*)ws.scores, ws.ld, per,
                           ws.state, ws.band_id);
        GS_CHECK_LAUNCH("k_band_filter");
        hipLaunchKernelGGL(k_band_final, dim3(qt), dim3(1024), 0, s, ix, qb, q0, ws.state, ws.band_s, ws.band_id,
                           out_ids, (double*)out_scores);
        GS_CHECK_LAUNCH("k_band_final");
    }
    if (diag) {
        hipLaunchKernelGGL(k_diag, dim3((qt + 255) / 256), dim3(256), 0, s, q0, qt, (const SelState*)ws.state, diag);
        GS_CHECK_LAUNCH("k_diag");
    }
    return hipSuccess;
}

}  // namespace gs
