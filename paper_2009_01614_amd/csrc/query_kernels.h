// Query-side kernels (query_kernels.hip, filter_kernels.hip) and their arguments.
#pragma once
#include "internal.h"

namespace isax {

// Per-query statistics slots (unsigned long long each).
enum { ST_LEAVES = 0, ST_LEAVES_KEPT, ST_SERIES_LB, ST_REFINED, ST_REFINE_BYTES, ST_CANDS, ST_DTW, ST_DTW_CELLS,
       ST_PRECHECKED /* series bounded with their BF16 row before refinement */, ST_N };

// Everything one batch of queries needs on the device.  Passed by value.
struct QueryArgs {
    // index (read only)
    const float* data;
    const float* xs;            // rows in leaf order (position p = sorted position), or null
    int64_t n;
    int len, w, c, m_seg, ws, ns;
    int leaf_size;
    int64_t n_leaves;
    const uint8_t* words_sorted;
    const int32_t* ids_sorted;
    const uint8_t* env_lo;
    const uint8_t* env_hi;
    const uint8_t* node_lo;     // [n_nodes][ws] envelopes of kNodeLeaves consecutive leaves
    const uint8_t* node_hi;
    int64_t n_nodes;
    const uint64_t* leaf_key;
    const float* beta;
    float delta_x;
    // batch
    int mq;           // queries in this batch
    const float* Q;   // [mq][len]
    const int32_t* kq;// [mq] k per query
    int kmax;         // row stride of bestk and of the outputs
    int cap;          // candidate slots per query
    float tau_scale;  // 1 + eps: slack on every comparison with the best-so-far
    float lb_scale;   // 1 - 2^-16: slack on every lower bound
    int flags;        // ISAX_QF_*
    int rerun;        // 1: frozen best-so-far, no best-k insertion, skip finished queries
    int skip_done;    // 1: rows whose done flag is set take no part in the filter and its refinement
                      //    (the free slots of a serving table)
    int home_leaves;  // leaves the approximate answer covers at least (0: the default, 4)
    int leaf_stride;  // leaf pass: every leaf_stride-th block of leaves only (0 or 1: every leaf)
    const int32_t* qsel;  // leaf pass: the queries it bounds leaves for, [nsel] (null: all mq)
    int nsel;
    float* paa;       // [mq][w]
    uint8_t* sym;     // [mq][ws]
    uint64_t* qkey;   // [mq]
    float4* qinfo;    // [mq] {|q|^2, max|q|, delta, tau after the approximate answer}
    float* edges;     // [mq][2][ns]  widened region edges: lower then upper
    float* T;         // [mq][w][ns]  per-segment squared lower-bound table
    float* tau0;      // [mq] extra upper bound on the k-th squared distance (+inf if none)
    unsigned long long* bestk;  // [mq][kmax] k smallest (d2 bits << 32 | id) seen so far
    unsigned long long* cand;   // [mq][cap]
    unsigned* cand_count;       // [mq]
    int64_t* home;              // [mq][2] leaf range of the approximate answer
    unsigned long long* stats;  // [mq][ST_N]
    int* done;                  // [mq] 1 once the query's answer is written
    int* status;                // [mq] 0 ok, 1 candidate overflow (re-run), 2 fewer than k candidates,
                                //      3 window wider than the top-k block's LDS
    int64_t* out_ids;           // [mq][kmax]
    float* out_dists;           // [mq][kmax]
    // best-first rounds: round 0 = one pass over every leaf; round 1 = leaves
    // whose bound is below theta[q]; round 2 = the others
    int round;
    float* theta;               // [mq]
    unsigned* leaf_hist;        // [mq][kLeafBins]
    uint2* leaf_list;           // [mq][leaf_cap] {leaf, bound bits} of leaves within the first bound
    unsigned* leaf_count;       // [mq] leaves within the first bound (also those past leaf_cap)
    int64_t leaf_cap;
    int64_t grid_leaves;        // rounds 1 and 2: blocks per query (0: one per 256 leaves)
    unsigned* list_rest;        // [mq] listed leaves round 2 would still bound (after round 1)
    // distance measure
    int metric;                 // ISAX_METRIC_*
    int window;                 // DTW band half-width r
    float lbk_scale;            // DTW: 1 - eps, slack on LB_Keogh
    int all_leaves;             // 1: no leaf or series bound (the plain scan under DTW)
    float* env_paa;             // [mq][2][w] PAA of the upper then lower query envelope (ED: the query PAA twice)
    float* qenv;                // [mq][2][len] DTW: upper then lower envelope of the query
    // refinement precheck (ED, an index with the full-row BF16 copy): each series is first
    // bounded from below with the copy, and only series whose bound is within the
    // best-so-far have their rows read
    const uint16_t* pc_x;       // [n][pc_stride] BF16 rows in leaf order, or null (no precheck)
    const float4* pc_meta;      // [n] {|x|^2, |e_x| (up), |x~| (up), 1}
    int pc_stride;
    int pc_home;                // 1: the approximate answer prechecks its series too (rows in host memory)
    float pc_gamma, pc_kappa;   // FP32 dot of len terms; slack on |q|^2 + |x|^2
};
constexpr int kDtwMaxLen = 2048;  // longest series the DTW path takes (its LDS plan)
// The filter's first phase reads one tile in kFilterSub (an even sample of the
// collection) whose candidates tighten the bound before the other tiles.
constexpr int kFilterSub = 64;
// Row of the series at sorted position p (id = ids_sorted[p]): the leaf-order
// copy when the index keeps one, else the borrowed collection.
__device__ inline const float* series_row(const QueryArgs& a, int64_t p, int32_t id) {
    return a.xs ? a.xs + p * a.len : a.data + (int64_t)id * a.len;
}
constexpr int kLeafBins = 64;
constexpr int kFirstLeaves = 64;  // leaves refined first, by smallest lower bound
constexpr int kHistQueries = 4;   // queries per block of the leaf pass
constexpr int kHistLeafRounds = 4; // leaves per thread of the leaf pass

void launch_check_finite(const float* x, int64_t count, int* flag, hipStream_t s);
void launch_qprep(const QueryArgs& a, hipStream_t s);
void launch_homeleaf(const QueryArgs& a, hipStream_t s);
void launch_index_scan(const QueryArgs& a, hipStream_t s);
void launch_leaf_order(const QueryArgs& a, hipStream_t s);  // histogram of leaf bounds -> theta
// dst.tau0[map[i].y] = min(itself, the k-th best of src row map[i].x): a bound
// found by one batch handed to the rows of another.
void launch_carry_bound(const QueryArgs& src, const QueryArgs& dst, const int2* map, int n, hipStream_t s);
// list_rest[q] = list entries at or above theta still within the best-so-far
// (queries not done, whose list holds every leaf within the first bound).
void launch_list_recount(const QueryArgs& a, int64_t grid_x, hipStream_t s);
void launch_seed(const QueryArgs& a, hipStream_t s);
void launch_brute_scan(const QueryArgs& a, hipStream_t s);
void launch_topk(const QueryArgs& a, hipStream_t s);
// Queries wq[0..n_wide) whose window exceeded the top-k block's LDS (status 3):
// their answers from vals [n_wide][cap] (8 bytes per candidate) of scratch.
void launch_topk_wide(const QueryArgs& a, const int* wq, int n_wide, double* vals, hipStream_t s);
void launch_rerun_reset(const QueryArgs& a, hipStream_t s);
void launch_lower_bounds(const QueryArgs& a, float* out, hipStream_t s);
// Hybrid batches: rows pos[0..mf) of (Q, kq) into (Qf, kqf); answer rows back to pos.
void launch_gather_queries(const float* Q, const int32_t* kq, const int32_t* pos, int mf, int len, float* Qf,
                           int32_t* kqf, hipStream_t s);
void launch_scatter_answers(const int64_t* ids, const float* dists, const int32_t* pos, int mf, int kmax,
                            int64_t* out_ids, float* out_dists, hipStream_t s);

// Reduced-precision filter (filter_kernels.hip).
struct FilterArgs {
    int kind;                 // 0 BF16, 1 FP8
    int dim;                  // codes per row: the padded length, or D of the spectral copy
    const double* spec;       // spectral copy: the transform [len][dim] (FP64), else null
    const void* xq;           // collection codes [n][dim] (uint16 BF16 bits or uint8 E4M3)
    const float4* xmeta;      // [n] {|x|^2, |e_x|, |x~|, scale}
    void* qq;                 // query codes [mq_pad][dim]
    int mq_pad;               // rows of qq and qmeta
    float4* qmeta;            // [mq_pad] {|q|^2, |e_q|, |q~|, scale}
    float gamma;              // accumulation error factor
    float kappa;              // relative slack on |q|^2 + |x|^2
    unsigned* fcand;          // [mq][fcap] candidate ids from the filter
    unsigned* fcount;         // [mq]
    int fcap;
    float* out_approx;        // optional [mq][n] (inspection)
    float* out_margin;        // optional [mq][n]
    int phase;                // 0: every tile; 1: the sample tiles; 2: the other tiles;
                              // 3: the other tiles among sorted positions [range_lo, range_hi);
                              // 4 and 5: phase 2 split into a second sample and the rest
    int64_t range_lo, range_hi;  // phase 3; range_lo a multiple of kFilterAlign
};
// The sample of the first phase: units of kFilterAlign consecutive sorted
// positions, every kFilterSub-th unit (the same series for every tile size of
// the filter's configurations).  With R = kFilterAlign / TS tiles per unit:
constexpr int kFilterAlign = 128;  // the largest tile of any filter configuration
// sample tiles among tiles [0, t)
__host__ __device__ inline int64_t filter_samples_before(int64_t t, int R) {
    const int64_t g = (int64_t)kFilterSub * R;
    return t / g * R + (t % g < R ? t % g : R);
}
// tile of the v-th sample tile (phase 1) or of the v-th other tile (phases 2 and 3)
__host__ __device__ inline int64_t filter_sample_tile(int64_t v, int R) { return v / R * kFilterSub * R + v % R; }
__host__ __device__ inline int64_t filter_other_tile(int64_t v, int R) {
    const int64_t g = (int64_t)(kFilterSub - 1) * R;
    return v / g * kFilterSub * R + R + v % g;
}
// Phases 4 and 5 split the other units (phase 2) in two: phase 4 takes the unit
// kFilterSub / 2 past each sample unit (a second even sample of the
// collection), phase 5 the rest.  Tiles of phase 4 among tiles [0, t):
__host__ __device__ inline int64_t filter_seconds_before(int64_t t, int R) {
    const int64_t g = (int64_t)kFilterSub * R, o = (int64_t)(kFilterSub / 2) * R, r = t % g;
    return t / g * R + (r <= o ? 0 : (r - o < R ? r - o : R));
}
__host__ __device__ inline int64_t filter_second_tile(int64_t v, int R) {
    return v / R * kFilterSub * R + (int64_t)(kFilterSub / 2) * R + v % R;
}
__host__ __device__ inline int64_t filter_rest_tile(int64_t v, int R) {
    const int64_t g = (int64_t)(kFilterSub - 2) * R, w = v % g;
    int64_t u = w / R + 1;
    if (u >= kFilterSub / 2) ++u;
    return v / g * kFilterSub * R + u * R + w % R;
}
// Sum over a group of 16 lanes (the same value in all of them).
__device__ inline float sum16(float v) {
    v += __shfl_xor(v, 1, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 8, 16);
    return v;
}

// Lower bound on ED^2 of the query (qrow, FP32, in LDS) to the series at sorted
// position p from its BF16 copy, by a group of 16 lanes (the same value in all
// of them): approx - M with approx = |q|^2 + |x|^2 - 2 fl(q.x~) and
// M = 2 (|q| |e_x| + gamma |q| |x~|) + kappa (|q|^2 + |x|^2), since
// q.x - q.x~ = q.e_x, the FP32 dot of len terms is within gamma |q| |x~| of
// q.x~, and kappa covers the FP32 norms and this sum.  qn = |q|^2 (FP32), nq >= |q|.
__device__ inline float precheck16(const QueryArgs& a, int64_t p, const float* qrow, int gl, float qn, float nq) {
    const uint16_t* xr = a.pc_x + p * a.pc_stride;
    float s = 0.f;
    for (int j0 = gl * 8; j0 < a.len; j0 += 128) {
        const uint4 v = *reinterpret_cast<const uint4*>(xr + j0);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (j0 + e < a.len)
                s = fmaf(qrow[j0 + e], __uint_as_float((e & 1) ? (w[e >> 1] & 0xFFFF0000u) : (w[e >> 1] << 16)), s);
    }
    s = sum16(s);
    const float4 m = a.pc_meta[p];
    const float approx = qn + m.x - 2.f * s;
    const float M = (2.f * (nq * m.y + a.pc_gamma * nq * m.z) + a.pc_kappa * (qn + m.x)) * (1.f + 0x1p-20f);
    return approx - M;
}

int filter_len_pad(int len);              // rows of the reduced-precision copies are padded to this
int filter_queries_per_block(int len);    // query codes are padded to a multiple of this
int filter_rows_bf16(int dim, int mq);    // query rows the BF16 filter computes for mq queries (dim codes per row)
void launch_quantise_queries(const QueryArgs& a, const FilterArgs& f, int mq_pad, unsigned* qmax, hipStream_t s);
void launch_filter(const QueryArgs& a, const FilterArgs& f, const unsigned* qmax, hipStream_t s);
void launch_refine_filtered(const QueryArgs& a, const FilterArgs& f, hipStream_t s);
// Serving tables: ovf[q] = fcount[q] > fcap, then fcount[q] = 0, for q < a.mq.
void launch_note_overflow(const QueryArgs& a, const FilterArgs& f, int* ovf, hipStream_t s);
// Per-query state of rows map[i].x of (sa, sf) into rows map[i].y of (da, df): key, norms,
// bounds, best-k list, candidate list, approximate-answer range, statistics, status, the
// filter's query codes and factors (where both have them), and with rows_too the query row
// and k.  done of the destination row is set to 0 and, when free_src, that of the source
// row to 1.
void launch_copy_rows(const QueryArgs& sa, const FilterArgs& sf, const QueryArgs& da, const FilterArgs& df,
                      const int2* map, int n, bool free_src, hipStream_t s, bool rows_too = true);
void launch_filter_tighten(const QueryArgs& a, const FilterArgs& f, hipStream_t s);

}  // namespace isax
