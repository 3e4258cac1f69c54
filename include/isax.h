/*
 * isax.h -- exact k-nearest-neighbour Euclidean search over an in-memory
 * collection of data series with an iSAX index, on one AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no C++ or PyTorch types.
 *
 * Paper: B. Peng, P. Fatourou, T. Palpanas, "Data Series Indexing Gone
 * Parallel".  The method summarises every series with PAA and an iSAX word
 * (Sec. II, iSAX Representation), groups the words into leaves of an index
 * whose root subtrees are selected by the first bit of every segment (Sec. II,
 * ADS+ Index; Sec. III, ParIS/ParIS+ approach), and answers an exact
 * nearest-neighbour query (Sec. II, Similarity Search) by (1) an approximate
 * answer that sets the best-so-far distance, (2) lower-bound distances
 * between the query and the leaves / iSAX summaries, pruning those above the
 * best-so-far, and (3) real distances for the survivors, updating the
 * best-so-far (Sec. III, ParIS/ParIS+ and MESSI query answering).
 *
 * Conventions shared by every entry point
 *   - Pointers documented "device" are HIP device pointers on the current
 *     device; "host" pointers are ordinary host memory.
 *   - Series are FP32, row-major, `len` contiguous values per series.
 *   - Distances are Euclidean (not squared); returned lists are ascending by
 *     (distance, series id): ties go to the lower id.
 *   - The library never normalises: it measures the values it is given.
 *   - Every call validates its arguments before any device work and returns
 *     ISAX_EINVAL (or NULL) on a bad argument, writing nothing to outputs.
 *     The text of the last error of the calling thread is returned by
 *     isax_last_error().  HIP failures give ISAX_EDEVICE with HIP's message.
 *   - Calls run on the stream given in their options (NULL: the null stream)
 *     and return after the results are in the output buffers.
 *   - Query scratch blocks of 1 MiB to 1 GiB stay allocated after a call for
 *     reuse (at most 4 GiB idle per device); they are freed when a device
 *     allocation of the library would otherwise fail.
 */
#ifndef ISAX_H
#define ISAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
    ISAX_OK = 0,
    ISAX_EINVAL = -1,    /* bad argument, or a non-finite value in data or queries */
    ISAX_ENOMEM = -2,    /* device allocation failed */
    ISAX_EDEVICE = -3,   /* a HIP call failed */
    ISAX_EOVERFLOW = -4  /* a query's candidate list still overflowed after 8 re-runs (see candidate_capacity) */
};

/* Query execution modes (isax_query_options.mode). All return the same exact answer. */
enum {
    ISAX_MODE_INDEX = 0, /* iSAX path: home leaf, leaf and series lower bounds, refinement (Sec. III) */
    ISAX_MODE_SCAN = 1,  /* plain FP32 scan of every series (the sequential-scan baseline, Sec. I) */
    ISAX_MODE_BF16 = 2,  /* BF16 matrix-core dot-product filter with a proven error margin, FP32 refinement */
    ISAX_MODE_FP8 = 3,   /* FP8 E4M3 (power-of-two scale per series) filter, same margin rule */
    ISAX_MODE_HYBRID = 4 /* per query, the iSAX path or the BF16 filter, by the leaves the iSAX path would
                            still have to bound after its first best-first round (Sec. III pruning)
                            against the filter's cost (hybrid_leaves); needs the BF16 copy, ED only */
};

/* Query flags (isax_query_options.flags): switches for testing; the answer never changes. */
enum {
    ISAX_QF_NO_SHARING = 1,       /* do not lower the best-so-far during the scan */
    ISAX_QF_NO_EARLY_ABANDON = 2, /* refine every surviving series to the end */
    ISAX_QF_NO_BEST_FIRST = 4,    /* index mode: visit leaves in layout order in one pass, instead of the
                                     leaves of smallest lower bound first (MESSI's priority order, Sec. III) */
    ISAX_QF_NO_SHORTCUT = 8,      /* hybrid mode: price every query with the cost model even when the whole
                                     batch is cheap enough for the filter alone */
    ISAX_QF_FILTER_CHEAP = 16,    /* hybrid mode: price the filter at 1/1000 of its model, or */
    ISAX_QF_FILTER_DEAR = 32,     /* at 1000 times it, so that small collections exercise each of the
                                     planner's routes (testing) */
    ISAX_QF_FULL_ROWS = 64,       /* BF16 filter: read the full-length BF16 copy even when the index also
                                     holds the spectral copy (precision bit 3) */
    ISAX_QF_NO_PRECHECK = 128     /* read rows directly.  By default (ED, an index with the full-row BF16
                                     copy) a series that survives the iSAX bounds is first bounded from
                                     below with its BF16 row, approx - M as in the filter, and its row is
                                     read only if that bound is within the best-so-far (in device memory
                                     where sampled refinements show early abandoning reading more FP32
                                     bytes per series than the BF16 row holds; in host memory always); for
                                     a collection in pinned host memory the approximate answer does the
                                     same, reading only the series whose bound is within the k-th smallest
                                     upper bound approx + M of its leaves.  Answers are the same either
                                     way */
};

/* Distance measures (isax_query_options.metric). */
enum {
    ISAX_METRIC_ED = 0, /* Euclidean distance (Sec. II, Similarity Search) */
    ISAX_METRIC_DTW = 1 /* dynamic time warping (Sec. II names it; Sec. V answers it on the same index):
                           D(i,j) = (q_i - x_j)^2 + min(D(i-1,j-1), D(i-1,j), D(i,j-1)) over the
                           Sakoe-Chiba band |i - j| <= window, D(-1,-1) = 0, +inf outside;
                           distance = sqrt(D(len-1, len-1)) */
};

#define ISAX_MAX_K 1024
#define ISAX_MAX_WINDOW 31 /* largest DTW band half-width */
#define ISAX_MAX_LEN 4096
#define ISAX_MAX_SEGMENTS 64

typedef struct isax_index isax_index; /* opaque, owned by the library */

/* Region edges of the iSAX symbols (isax_build_options.edges). */
enum {
    ISAX_EDGES_NORMAL = 0,   /* Phi^-1(j / 2^c): equiprobable regions for N(0,1) segment means (z-normalised
                                series) */
    ISAX_EDGES_EMPIRICAL = 1 /* the collection's own quantiles, for data that is not z-normalised (embedding
                                vectors, Sec. V): the FP32 segment means of every segment of
                                S = min(n, ceil(65536 / segments)) series at ids floor(t n / S), t < S, and
                                edge j = the ceil(j V / 2^c)-th smallest of those V = S * segments values (the
                                inverted-CDF quantile at j / 2^c).  Nested across c like the normal edges;
                                every bound stays a lower bound (it holds for any ordered edges). */
};

typedef struct isax_build_options {
    int32_t leaf_size; /* series per leaf (consecutive runs of the sorted order); 0 = 256; 16..1024 */
    int32_t key_bits;  /* leading bits of the interleaved key that are sorted; 0 = min(64, w*c); 8..64, multiple of 8 */
    int32_t precision; /* bit 0: also keep a BF16 copy, bit 1: also keep an FP8 E4M3 copy (needed by those modes);
                          bit 2: also keep the FP32 rows in leaf order (n x len x 4 bytes more), read by
                          refinement instead of the borrowed data: the series of a leaf are then
                          consecutive in memory. Answers are the same either way.
                          bit 3: also keep the spectral copy, a reduced representation for the BF16
                          filter (lower-bound pruning on a reduced representation before real
                          distances, Sec. II-III): with y = T x, T the orthonormal DCT-II of length
                          len, the series is summarised by ext(x) = (y_0 .. y_{D-2}, |(y_{D-1} ..
                          y_{len-1})|), D = spectral_dim coordinates in BF16 (n x D x 2 bytes), computed
                          in FP64.  |ext(x)| = |x| and q.x <= ext(q).ext(x), so the filter's margin
                          rule holds with ext in place of the rows: the BF16 filter (modes BF16 and
                          HYBRID, and the server's filter modes) then reads this copy, D / len of the
                          matrix work, and refines more candidates where the dropped coefficients
                          carry energy.  Answers are the same. */
    int32_t edges;     /* ISAX_EDGES_*: how the 2^c - 1 region edges are chosen */
    void* stream;      /* hipStream_t the build runs on; NULL = null stream */
    int32_t spectral_dim; /* D of the spectral copy: 0 = three quarters of the padded length (len rounded up
                             to a multiple of 64), rounded down to a multiple of 64, within 64..256 (192
                             for len 256); else a multiple of 64 in 64..256, below len */
    int32_t reserved;     /* must be 0 */
} isax_build_options;

typedef struct isax_query_stats { /* per query, filled when requested */
    int64_t leaves_scanned;  /* leaves whose lower bound was computed */
    int64_t leaves_kept;     /* leaves that survived the leaf bound */
    int64_t series_bounded;  /* series whose iSAX lower bound was computed */
    int64_t series_refined;  /* series whose real distance was (partly) computed */
    int64_t refine_bytes;    /* raw-data bytes read by refinement */
    int64_t candidates;      /* entries appended to the candidate list */
    float tau_initial;       /* squared best-so-far after the approximate answer */
    float tau_final;         /* squared k-th distance found, FP32 */
    int64_t dtw_series;      /* DTW only: series whose warping distance was (partly) computed */
    int64_t dtw_cells;       /* DTW only: band cells computed (columns x (2 window + 1)) */
    int64_t leaves_initial;  /* index and hybrid modes (best-first order): leaves other than the home leaf
                                whose lower bound is within the best-so-far of the approximate answer;
                                -1 where not computed */
    int32_t path;            /* the mode that answered this query (ISAX_MODE_INDEX or _BF16 under hybrid) */
    int32_t candidate_capacity; /* candidate slots per query of the pass that answered it (the option's value,
                                   16384 by default, or more after growth) */
} isax_query_stats;

typedef struct isax_query_options {
    int32_t mode;               /* ISAX_MODE_* */
    int32_t candidate_capacity; /* candidate slots per query; 0 = 16384 (at least k).  A query whose list
                                   overflows is run again with its bound frozen at the k-th smallest stored
                                   distance, after the lists of its batch have grown to 1.25x the count
                                   the last pass emitted (at most 8 re-runs, else ISAX_EOVERFLOW; ISAX_ENOMEM
                                   if the grown lists of one batch would exceed 16 GiB).  The filter modes
                                   keep a separate list of filter survivors that also grows on overflow. */
    int32_t flags;              /* ISAX_QF_* */
    int32_t batch;              /* queries per internal pass; 0 = 1024 */
    const int32_t* k_per_query; /* device, m values in 1..k (row i keeps k_i results, the rest
                                   of the row is filled with id -1 and +inf); NULL = k for all */
    void* stream;               /* hipStream_t; NULL = null stream */
    isax_query_stats* stats;    /* host, m entries, or NULL */
    int32_t metric;             /* ISAX_METRIC_*; DTW runs in ISAX_MODE_INDEX and ISAX_MODE_SCAN only */
    int32_t window;             /* DTW band half-width, 0..min(ISAX_MAX_WINDOW, len-1); must be 0 for ED */
    int64_t hybrid_leaves;      /* ISAX_MODE_HYBRID, >= 0.  est = leaves left for the second round (bound at
                                   least the first round's threshold, within the best-so-far after it; for a
                                   query with more than 32768 leaves within the first bound, that count).
                                   > 0: queries with est above it take the filter.  0: a cost model chooses
                                   the queries of largest est for the filter when its pass over the whole
                                   collection costs less than the index work they would leave. */
} isax_query_options;

/* Last error message of the calling thread ("" if none). Static storage, thread-local. */
const char* isax_last_error(void);

/*
 * Build an index over `data` (n x len FP32: device memory, or pinned host
 * memory mapped at the same address on the device, which refinement then
 * reads across the bus).  `segments` (w) is the
 * number of PAA segments and must divide len (segments of equal length, Sec.
 * II); `card_bits` (c, 1..8) is the number of bits of every iSAX symbol.
 * Regions are cut at the standard-normal quantiles Phi^-1(j / 2^c).
 * The index BORROWS `data`: the caller keeps it allocated and unmodified until
 * isax_free().  Returns NULL on error (see isax_last_error()); EINVAL if data
 * holds a non-finite value.  n < 2^31, len <= ISAX_MAX_LEN,
 * segments <= ISAX_MAX_SEGMENTS; the BF16 / FP8 copies need len <= 512.
 */
isax_index* isax_build(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits);
isax_index* isax_build_ex(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                          const isax_build_options* opt);

/* Release an index and everything it owns (not the borrowed data). NULL is a no-op. */
void isax_free(isax_index* idx);

/*
 * Page-locked host memory for a collection kept in host memory (the paper's
 * plan for raw data that does not fit in GPU memory, Sec. V): `bytes` bytes
 * mapped at the same address on the current device (hipHostMalloc), to pass
 * to isax_build as `data`.  Returns NULL on failure (see isax_last_error());
 * the caller owns the memory and releases it with isax_host_free (NULL is a
 * no-op) after the last index over it is freed.
 */
void* isax_host_alloc(int64_t bytes);
void isax_host_free(void* p);

/*
 * Exact k-NN of m queries (device, m x len FP32).  Writes out_ids (device,
 * m x k int64) and out_dists (device, m x k FP32): for each query the k
 * series of smallest Euclidean distance, ascending, ties by lower id (Sec. II,
 * Similarity Search, generalised from 1 to k neighbours).  m = 0 succeeds with
 * no work.  1 <= k <= min(n, ISAX_MAX_K).  EINVAL if a query value is not
 * finite.  Answers are staged in library scratch and copied to out_ids /
 * out_dists (and opt->stats) only when every batch has succeeded: on any error
 * return the outputs are untouched.  Any number of series may tie at the k-th
 * distance (the lowest ids are returned).
 * With opt->metric = ISAX_METRIC_DTW the same index answers the k nearest
 * series under banded DTW (ISAX_METRIC_DTW above): the leaf and series
 * bounds use the PAA of the query's envelope, then LB_Keogh, then the DTW
 * recurrence in FP32 with early abandoning; the final order is decided by
 * the recurrence recomputed in FP64 (the returned distance is that value's
 * square root rounded to FP32).
 */
int isax_query(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids, float* out_dists);
int isax_query_ex(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids, float* out_dists,
                  const isax_query_options* opt);

/*
 * isax_query_ex without any device allocation, for callers that cannot
 * allocate device memory during a query: request loops that must keep a fixed
 * memory footprint, code that may not call hipMalloc / hipFree or a caching
 * allocator, harnesses that forbid allocation.  Same arguments, options,
 * answers (ids, and distances bit for bit) and error behaviour as
 * isax_query_ex.  Every device buffer of the call is carved from a fixed
 * array of 256 MiB compiled into the library: each device holds its own copy
 * from the library's load on it until the process ends.
 *   - Sizes: the queries run in batches of opt->batch, or (batch 0) of the
 *     largest size whose scratch fits, at most 1024.  If the staged answers
 *     (m x k x 12 bytes) and one batch do not fit, the call returns
 *     ISAX_EINVAL before any device work, naming the sizes.
 *   - Data-dependent growth (candidate lists that grow for a re-run, a tie
 *     window wider than 2048 entries) takes what is left of the array; if that
 *     is not enough the call returns ISAX_ENOMEM and the outputs are untouched.
 *   - The array keeps the last call's contents; every call initialises what
 *     it reads.  Calls on one device are serialised by a lock held for the
 *     whole call (including the wait for its stream), so they never overlap.
 *   - Host-side bookkeeping (status read-back, the hybrid planner) uses
 *     ordinary host memory.
 */
int isax_query_noalloc(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids,
                       float* out_dists, const isax_query_options* opt);

/* ---------------------------------------------------------- inspection */

/* The 2^c - 1 region edges used for c-bit symbols, FP32, ascending (host out): Phi^-1(j / 2^c). */
int isax_breakpoints(int32_t card_bits, float* out);
/* The 2^c - 1 region edges of an index (host out, FP32, ascending), normal or empirical. */
int isax_index_breakpoints(const isax_index* idx, float* out);

/*
 * iSAX words of n series without building an index (Sec. II, iSAX
 * Representation): out_words (device, n x segments uint8) receives the
 * symbol of every segment.  max_abs (host, may be NULL) receives max |x|.
 */
int isax_summarize(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                   uint8_t* out_words, float* max_abs, void* stream);

typedef struct isax_index_info {
    int64_t n;
    int32_t len, segments, card_bits, leaf_size, key_bits;
    int32_t has_bf16, has_fp8;
    int64_t n_leaves;
    float max_abs;       /* max |x| over the collection */
    float delta;         /* bound on |FP32 PAA - exact PAA| of any series */
    int64_t device_bytes;/* bytes the index owns on the device */
    int32_t has_sorted_rows; /* 1 if the index keeps the FP32 rows in leaf order (precision bit 2) */
    int32_t edges;           /* ISAX_EDGES_* of the build */
    int32_t spectral_dim;    /* D of the spectral copy (precision bit 3), 0 if none */
    int32_t reserved;
} isax_index_info;

int isax_index_get_info(const isax_index* idx, isax_index_info* out);

/*
 * Copy the index layout out (all device, any may be NULL): ids_sorted
 * (n int32, series ids in leaf order), words_sorted (n x segments uint8),
 * env_lo / env_hi (n_leaves x segments uint8, per-leaf per-segment min / max
 * symbol).  Leaf i holds sorted positions [i*leaf_size, (i+1)*leaf_size).
 */
int isax_index_export(const isax_index* idx, int32_t* ids_sorted, uint8_t* words_sorted,
                      uint8_t* env_lo, uint8_t* env_hi);

/*
 * Squared iSAX lower bounds used for pruning (Sec. III, lower-bound distance
 * calculations): out_lb (device, m x n FP32, column = original series id)
 * receives the bound of every (query, series) pair.  Each value is at most
 * the squared Euclidean distance of the pair.
 */
int isax_lower_bounds(isax_index* idx, const float* queries, int64_t m, float* out_lb);

/*
 * Scores of the reduced-precision filter (mode ISAX_MODE_BF16 or _FP8), for
 * testing its margin: out_approx (device, m x n) = |q|^2 + |x|^2 - 2 q~.x~
 * accumulated on the matrix cores, out_margin (device, m x n) = the bound M
 * with |ED^2 - approx| <= M.  m <= 1024.  Where the index holds the spectral
 * copy, BF16 scores are those of that copy (q~, x~ the BF16 copies of ext(q),
 * ext(x)): then |ext-distance^2 - approx| <= M, and approx - M <= ED^2.
 */
int isax_filter_scores(isax_index* idx, const float* queries, int64_t m, int32_t mode,
                       float* out_approx, float* out_margin);

/* ------------------------------------------------------- kernel timing */
/* When enabled, every library kernel launch is bracketed by HIP events on its
 * own stream; isax_profile_read() returns per-kernel totals (host out).  One
 * entry is a count, not a kernel: "filter_full_rows_switch" (in
 * algorithmic_bytes) counts the filter passes that moved from the spectral
 * copy to the full rows after their second sample (both copies present: the
 * sample's candidates, extrapolated to the rest of the collection, would cost
 * more to refine than the spectral copy saves). */
typedef struct isax_profile_entry {
    char name[48];
    int64_t launches;
    double total_ms;
    double algorithmic_bytes; /* bytes the method must move in those launches (where defined) */
} isax_profile_entry;

int isax_profile_enable(int32_t on);
int isax_profile_read(isax_profile_entry* out, int32_t max_entries, int32_t* n_entries);
int isax_profile_reset(void);

/* ------------------------------------------------------------- testing */
/*
 * Fault injection for tests of the error paths: the `countdown`-th device
 * allocation the library requests from now on (query scratch and index
 * arrays; blocks reused from the cache count too) fails as if the device were
 * out of memory, and the call reports ISAX_ENOMEM.  0 switches it off.
 * Process-wide.
 */
int isax_debug_fail_allocation(int64_t countdown);

/* ------------------------------------------------------------- serving */
/*
 * A request loop over resident indexes.  submit() copies the host query and
 * returns at once; poll() returns results as they complete.  Two admission
 * policies:
 *   - step level (the default of ISAX_MODE_BF16 / _FP8): per collection, a
 *     table of max_batch query rows stays on the device and the collection is
 *     swept in `chunks` steps, each running the reduced-precision filter over
 *     one chunk for every occupied row and refining its candidates.  A waiting
 *     request takes a free row between two steps, at whatever chunk the sweep
 *     has reached, and leaves after one full sweep (wrapping around), so it
 *     never waits for another batch to end; collections run on their own
 *     streams.  A row that lost filter candidates to a full buffer is answered
 *     again by itself.
 *   - batch level (every other mode, or ISAX_SERVE_BATCHES): a free worker takes
 *     the oldest waiting request and the other waiting requests of its
 *     collection while the batch's device scratch fits the memory budget, and
 *     answers them with one isax_query_ex call on its own stream; `streams`
 *     workers overlap on the device.
 * Every result equals the result of the same query run alone (ids, and
 * distances bit for bit).
 */
typedef struct isax_server isax_server;

enum {
    ISAX_SERVE_BATCHES = 1 /* batch-level admission also in the filter modes */
};

typedef struct isax_server_options {
    int32_t max_batch;       /* batch level: requests per batch (0 = 256); step level: rows of each
                                collection's table (0 = 512); 1..4096 */
    int32_t streams;         /* batch level: batches in flight (workers); 0 = 4 */
    int64_t memory_budget;   /* batch level: bytes of per-batch scratch allowed in flight; 0 = 4 GiB */
    int32_t mode;            /* ISAX_MODE_* used for every request (hybrid with its cost model); the
                                server answers Euclidean k-NN */
    int32_t flags;           /* ISAX_SERVE_* */
    int32_t chunks;          /* step level: steps per sweep of a collection; 0 = 8; 1..1024 */
    int32_t reserved;        /* must be 0 */
} isax_server_options;

typedef struct isax_result {
    uint64_t tag;            /* the caller's tag from submit() */
    int32_t status;          /* ISAX_OK or an error code */
    int32_t k;
    int32_t collection;
    int32_t batch_size;      /* batch level: requests in its batch; step level: occupied rows of the
                                table when it joined */
    double t_submit, t_start, t_done; /* seconds, steady clock: submitted, taken into a batch or a
                                         table row, answered */
    int64_t ids[ISAX_MAX_K];
    float dists[ISAX_MAX_K];
    char message[120];       /* status != ISAX_OK: the error text of the batch that failed ("" otherwise) */
} isax_result;

isax_server* isax_server_create(isax_index* const* collections, int32_t n_collections,
                                const isax_server_options* opt);
/* query: host, len floats of that collection; 1 <= k <= min(n, ISAX_MAX_K). */
int isax_server_submit(isax_server* s, int32_t collection, const float* query, int32_t k, uint64_t tag);
/* Wait up to timeout_ms for results; returns how many were written to out (0..max). */
int isax_server_poll(isax_server* s, isax_result* out, int32_t max_results, int32_t timeout_ms);
/* Requests submitted and not yet returned by poll(). */
int64_t isax_server_pending(isax_server* s);
void isax_server_destroy(isax_server* s);
/* Seconds on the steady clock the server stamps results with. */
double isax_clock(void);

#ifdef __cplusplus
}
#endif
#endif /* ISAX_H */
