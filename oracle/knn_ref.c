/*
 * Brute-force exact k-NN under Euclidean distance, FP64 (CPU oracle, plain C).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests and by the benchmark's
 * CPU-baseline leg through ctypes; never linked into the product library.
 *
 * Definition (Sec. II, Similarity Search): for a query q and every series x_i
 * of the collection, D_i = sum over t = 0..len-1 of (q_t - x_{i,t})^2, the
 * FP32 inputs promoted to FP64, accumulated in index order t = 0, 1, 2, ...
 * with no fused multiply-add (built with -ffp-contract=off).  The answer is
 * the first k entries of the collection ordered by (D_i, i) ascending; the
 * distance reported is sqrt(D_i).  This is the same arithmetic, in the same
 * order, as knn_ref.knn_exact in numpy, so the two agree bit for bit.
 *
 * oracle_knn_merge() folds a block of series with global ids id_offset..
 * into running per-query top-k lists, so a collection larger than host memory
 * can be streamed through in chunks.  The lists are kept sorted by (D, id);
 * entries with D = +inf and id = -1 are empty.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int precedes(double da, int64_t ia, double db, int64_t ib) {
    return da < db || (da == db && ia < ib);
}

/* insert (d, id) into the ascending list (bd, bi) of length k, if it belongs */
static void insert_sorted(double* bd, int64_t* bi, int k, double d, int64_t id) {
    if (!precedes(d, id, bd[k - 1], bi[k - 1])) return;
    int p = k - 1;
    while (p > 0 && precedes(d, id, bd[p - 1], bi[p - 1])) {
        bd[p] = bd[p - 1];
        bi[p] = bi[p - 1];
        --p;
    }
    bd[p] = d;
    bi[p] = id;
}

static double sq_dist(const float* q, const float* x, int len) {
    double D = 0.0;
    for (int t = 0; t < len; ++t) {
        double d = (double)q[t] - (double)x[t];
        D += d * d;
    }
    return D;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D_i for one query against n series (row-major X). */
void oracle_sq_dists(const float* X, int64_t n, int32_t len, const float* q, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = sq_dist(q, X + i * (int64_t)len, len);
}

void oracle_knn_init(double* best_d, int64_t* best_id, int64_t count) {
    for (int64_t i = 0; i < count; ++i) {
        best_d[i] = INFINITY;
        best_id[i] = -1;
    }
}

void oracle_knn_merge(const float* X, int64_t n, int32_t len, int64_t id_offset,
                      const float* Q, int32_t m, int32_t k,
                      double* best_d, int64_t* best_id) {
    int nt = oracle_num_threads();
    double* td = (double*)malloc(sizeof(double) * (size_t)nt * k);
    int64_t* ti = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt * k);
    for (int32_t j = 0; j < m; ++j) {
        const float* q = Q + (int64_t)j * len;
        oracle_knn_init(td, ti, (int64_t)nt * k);
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* md = td + (int64_t)tid * k;
            int64_t* mi = ti + (int64_t)tid * k;
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i)
                insert_sorted(md, mi, k, sq_dist(q, X + i * (int64_t)len, len), id_offset + i);
        }
        double* bd = best_d + (int64_t)j * k;
        int64_t* bi = best_id + (int64_t)j * k;
        for (int t = 0; t < nt; ++t)
            for (int r = 0; r < k; ++r)
                if (ti[(int64_t)t * k + r] >= 0)
                    insert_sorted(bd, bi, k, td[(int64_t)t * k + r], ti[(int64_t)t * k + r]);
    }
    free(td);
    free(ti);
}

/*
 * Dynamic time warping with a Sakoe-Chiba band of half-width r (the usual
 * definition; the paper names DTW as a similarity measure in Sec. II and
 * answers it on the same index, Sec. V):
 *   D(i, j) = (q_i - x_j)^2 + min(D(i-1, j-1), D(i-1, j), D(i, j-1)) for
 *   |i - j| <= r, D(-1, -1) = 0, +inf outside the band or the grid;
 *   DTW^2 = D(len-1, len-1).
 * Every cell: d = (double)q_i - (double)x_j, d * d rounded, + min rounded, the
 * same operations as dtw_ref.dtw_sq in numpy, so the two agree bit for bit.
 * The grid is filled row by row (i), keeping rows i-1 and i of length len.
 */
static double dtw_sq(const float* q, const float* x, int len, int r, double* prev, double* cur) {
    for (int j = 0; j < len; ++j) prev[j] = INFINITY;
    for (int i = 0; i < len; ++i) {
        for (int j = 0; j < len; ++j) cur[j] = INFINITY;
        int j0 = i - r < 0 ? 0 : i - r;
        int j1 = i + r + 1 > len ? len : i + r + 1;
        for (int j = j0; j < j1; ++j) {
            double d = (double)q[i] - (double)x[j];
            double c = d * d;
            double m;
            if (i == 0 && j == 0) {
                m = 0.0;
            } else {
                double diag = (i > 0 && j > 0) ? prev[j - 1] : INFINITY;
                double up = i > 0 ? prev[j] : INFINITY;
                double left = j > 0 ? cur[j - 1] : INFINITY;
                m = diag < up ? diag : up;
                m = left < m ? left : m;
            }
            cur[j] = c + m;
        }
        double* t = prev;
        prev = cur;
        cur = t;
    }
    return prev[len - 1];
}

/* DTW^2 of one query against n series. */
void oracle_dtw_sq(const float* X, int64_t n, int32_t len, const float* q, int32_t r, double* out) {
#pragma omp parallel
    {
        double* rows = (double*)malloc(sizeof(double) * 2 * (size_t)len);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) out[i] = dtw_sq(q, X + i * (int64_t)len, len, r, rows, rows + len);
        free(rows);
    }
}

/* As oracle_knn_merge, under DTW^2 with band half-width r. */
void oracle_dtw_knn_merge(const float* X, int64_t n, int32_t len, int64_t id_offset,
                          const float* Q, int32_t m, int32_t k, int32_t r,
                          double* best_d, int64_t* best_id) {
    int nt = oracle_num_threads();
    double* td = (double*)malloc(sizeof(double) * (size_t)nt * k);
    int64_t* ti = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt * k);
    for (int32_t j = 0; j < m; ++j) {
        const float* q = Q + (int64_t)j * len;
        oracle_knn_init(td, ti, (int64_t)nt * k);
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* md = td + (int64_t)tid * k;
            int64_t* mi = ti + (int64_t)tid * k;
            double* rows = (double*)malloc(sizeof(double) * 2 * (size_t)len);
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i)
                insert_sorted(md, mi, k, dtw_sq(q, X + i * (int64_t)len, len, r, rows, rows + len), id_offset + i);
            free(rows);
        }
        double* bd = best_d + (int64_t)j * k;
        int64_t* bi = best_id + (int64_t)j * k;
        for (int t = 0; t < nt; ++t)
            for (int s = 0; s < k; ++s)
                if (ti[(int64_t)t * k + s] >= 0)
                    insert_sorted(bd, bi, k, td[(int64_t)t * k + s], ti[(int64_t)t * k + s]);
    }
    free(td);
    free(ti);
}
