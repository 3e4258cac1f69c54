// Host check of the filter pass's phase enumeration (csrc/query_kernels.h):
// for every tile count and tiles-per-unit value R the filter configurations
// use, phases {1, 2} and {1, 4, 5} each meet every tile exactly once, phases
// 2, 4 and 5 list their tiles in increasing order, and the serving chunks'
// phase-3 tiles together with phase 1 meet every tile exactly once.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "query_kernels.h"

using namespace isax;

static int fail(const char* what, int R, long long n) {
    std::printf("FAIL %s R=%d tiles=%lld\n", what, R, n);
    return 1;
}

static int check(int R, long long n_tiles) {
    const long long ns = filter_samples_before(n_tiles, R), n2 = filter_seconds_before(n_tiles, R);
    std::vector<int> seen(n_tiles, 0), seen2(n_tiles, 0);
    for (long long v = 0; v < ns; ++v) {
        const long long t = filter_sample_tile(v, R);
        if (t < 0 || t >= n_tiles) return fail("sample tile out of range", R, n_tiles);
        ++seen[t];
        ++seen2[t];
    }
    long long prev = -1;
    for (long long v = 0; v < n_tiles - ns; ++v) {
        const long long t = filter_other_tile(v, R);
        if (t < 0 || t >= n_tiles || t <= prev) return fail("other tile", R, n_tiles);
        prev = t;
        ++seen[t];
    }
    prev = -1;
    for (long long v = 0; v < n2; ++v) {
        const long long t = filter_second_tile(v, R);
        if (t < 0 || t >= n_tiles || t <= prev) return fail("second tile", R, n_tiles);
        prev = t;
        ++seen2[t];
    }
    prev = -1;
    for (long long v = 0; v < n_tiles - ns - n2; ++v) {
        const long long t = filter_rest_tile(v, R);
        if (t < 0 || t >= n_tiles || t <= prev) return fail("rest tile", R, n_tiles);
        prev = t;
        ++seen2[t];
    }
    for (long long t = 0; t < n_tiles; ++t)
        if (seen[t] != 1 || seen2[t] != 1) return fail("tile not met exactly once", R, n_tiles);
    // serving: chunk boundaries on whole units; phase 3 of [lo, hi) is the other tiles in it
    const long long unit = R, chunk_units = 1 + (n_tiles / unit) / 5;
    std::vector<int> seen3(n_tiles, 0);
    for (long long v = 0; v < ns; ++v) ++seen3[filter_sample_tile(v, R)];
    for (long long lo = 0; lo < n_tiles; lo += chunk_units * unit) {
        const long long hi = lo + chunk_units * unit < n_tiles ? lo + chunk_units * unit : n_tiles;
        const long long g_lo = lo - filter_samples_before(lo, R), g_hi = hi - filter_samples_before(hi, R);
        for (long long v = 0; v < g_hi - g_lo; ++v) {
            const long long t = filter_other_tile(g_lo + v, R);
            if (t < lo || t >= hi) return fail("phase-3 tile outside its chunk", R, n_tiles);
            ++seen3[t];
        }
    }
    for (long long t = 0; t < n_tiles; ++t)
        if (seen3[t] != 1) return fail("serving chunks do not partition the other tiles", R, n_tiles);
    return 0;
}

int main() {
    std::srand(20090164);
    for (int R : {1, 2, 4, 8, 16, 32}) {
        for (long long n = 1; n <= 3LL * kFilterSub * R + 5; ++n)
            if (check(R, n)) return 1;
        for (int i = 0; i < 60; ++i)
            if (check(R, 1 + std::rand() % 200000)) return 1;
    }
    std::printf("ok\n");
    return 0;
}
