// CPU harness of the request loop's scheduling core (serve_sched.cpp) with
// stub runners: no device, built under ThreadSanitizer or Address/Undefined
// sanitizers by tests/test_serve_sched_cpu.py.
//
// The stub step runner keeps what the device table would hold and checks the
// engine's use of it: a row is admitted only when free, every occupied row
// sees every chunk of the sweep exactly once before it is finished, and a
// finished row is answered from its own query.  Some steps lose candidates
// (the row must then be answered alone), some final orderings ask for that
// too, and some device calls fail (every occupied row then reports the
// error).  Producers submit from several threads while a consumer polls; every
// request must come back exactly once with the answer its query implies.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <random>
#include <thread>

#include "serve_sched.h"

using namespace isax::serve;

static int g_errors = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_errors;                                                   \
        }                                                                 \
    } while (0)

// The answer the stubs give for a query: id j of it is base(q) + j.
static int64_t base_of(const float* q) { return (int64_t)q[0] * 1000; }

struct StubStep : StepRunner {
    int S, C, L;
    std::vector<std::vector<float>> q;
    std::vector<int> k, busy;
    std::vector<std::vector<int>> seen;
    struct Out {  // what a queued step hands back
        std::vector<int> ovf, status, fin_k;
        std::vector<int64_t> base;
    };
    std::deque<Out> queued;
    std::mt19937 rng;
    int fail_every, calls = 0;
    StubStep(int slots, int chunks, int len, int seed, int fail_every_)
        : S(slots), C(chunks), L(len), q(slots), k(slots, 0), busy(slots, 0), seen(slots), rng(seed),
          fail_every(fail_every_) {}
    int slots() const override { return S; }
    int chunks() const override { return C; }
    int len() const override { return L; }
    void launch(const float* hq, const int32_t* hk, const int* adm, int n_adm, int chunk, int hi, const int* fin,
                int n_fin) override {
        CHECK(queued.size() < 2);
        if (fail_every && ++calls % fail_every == 0) throw Failure{ISAX_EDEVICE, "injected device failure"};
        // in device order: admissions, the sweep of the chunk, the final ordering
        Out o;
        for (int i = 0; i < n_adm; ++i) {
            const int r = adm[i];
            CHECK(r >= 0 && r < S);
            CHECK(!busy[r]);
            busy[r] = 1;
            q[r].assign(hq + (size_t)i * L, hq + (size_t)(i + 1) * L);
            k[r] = hk[i];
            seen[r].assign(C, 0);
        }
        CHECK(chunk >= 0 && chunk < C);
        o.ovf.assign(hi, 0);
        for (int r = 0; r < S; ++r) {
            CHECK(r < hi || !busy[r]);
            if (r < hi && busy[r]) {
                ++seen[r][chunk];
                o.ovf[r] = std::uniform_int_distribution<int>(0, 199)(rng) == 0;
            }
        }
        for (int i = 0; i < n_fin; ++i) {
            const int r = fin[i];
            CHECK(r >= 0 && r < hi && busy[r]);
            for (int c = 0; c < C; ++c) CHECK(seen[r][c] == 1);
            o.status.push_back(std::uniform_int_distribution<int>(0, 99)(rng) == 0 ? 3 : 0);
            o.fin_k.push_back(k[r]);
            o.base.push_back(base_of(q[r].data()));
            busy[r] = 0;
        }
        queued.push_back(std::move(o));
    }
    void collect(int* ovf, int kout, int64_t* ids, float* dists, int* status) override {
        CHECK(!queued.empty());
        if (queued.empty()) return;
        Out o = std::move(queued.front());
        queued.pop_front();
        std::copy(o.ovf.begin(), o.ovf.end(), ovf);
        for (size_t i = 0; i < o.status.size(); ++i) {
            CHECK(o.fin_k[i] <= kout);
            for (int j = 0; j < o.fin_k[i]; ++j) {
                ids[i * kout + j] = o.base[i] + j;
                dists[i * kout + j] = (float)j;
            }
            status[i] = o.status[i];
        }
    }
    void reset() override {
        queued.clear();
        std::fill(busy.begin(), busy.end(), 0);
    }
    int run_alone(const float* hq, int kk, int64_t* ids, float* dists, std::string&) override {
        for (int j = 0; j < kk; ++j) {
            ids[j] = base_of(hq) + j;
            dists[j] = (float)j;
        }
        return ISAX_OK;
    }
};

struct StubBatch : BatchRunner {
    int fail_every;
    std::atomic<int> calls{0};
    explicit StubBatch(int f) : fail_every(f) {}
    int64_t scratch_bytes(int, int m, int kmax) override { return (int64_t)m * (64 + kmax); }
    int run(int, const float* q, const int32_t* k, int m, int kmax, int64_t* ids, float* dists,
            std::string& err) override {
        if (fail_every && ++calls % fail_every == 0) {
            err = "injected device failure";
            return ISAX_EDEVICE;
        }
        for (int i = 0; i < m; ++i) {
            CHECK(k[i] <= kmax);
            for (int j = 0; j < k[i]; ++j) {
                ids[(size_t)i * kmax + j] = base_of(q + (size_t)i * 8) + j;
                dists[(size_t)i * kmax + j] = (float)j;
            }
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        return ISAX_OK;
    }
};

// Submits n_req requests from n_prod threads over n_coll collections (query
// length 8, q[0] = the tag, so the expected answer follows from the tag), polls
// until every one came back, then stops the workers.
static void drive(Core& core, int n_coll, int n_req, int n_prod, std::vector<std::thread>& workers) {
    std::vector<std::thread> prod;
    for (int p = 0; p < n_prod; ++p)
        prod.emplace_back([&, p] {
            std::mt19937 rng(1000 + p);
            for (int t = p; t < n_req; t += n_prod) {
                Request r;
                r.tag = (uint64_t)t;
                r.coll = t % n_coll;
                r.k = 1 + (int)(rng() % 20);
                r.q.assign(8, 0.f);
                r.q[0] = (float)t;
                r.t_submit = now();
                {
                    std::lock_guard<std::mutex> lk(core.mu);
                    core.queue.push_back(std::move(r));
                    ++core.pending;
                }
                core.cv_work.notify_all();
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
            }
        });
    std::map<uint64_t, isax_result> got;
    const double deadline = now() + 60;
    // polls without a timed wait: libstdc++ implements wait_for with pthread_cond_clockwait,
    // which this toolchain's ThreadSanitizer does not intercept (it would report the mutex as
    // never released)
    while ((int)got.size() < n_req && now() < deadline) {
        std::this_thread::sleep_for(std::chrono::microseconds(200));
        std::unique_lock<std::mutex> lk(core.mu);
        while (!core.results.empty()) {
            const isax_result r = core.results.front();
            core.results.pop_front();
            --core.pending;
            CHECK(got.count(r.tag) == 0);
            got[r.tag] = r;
        }
    }
    for (auto& t : prod) t.join();
    {
        std::lock_guard<std::mutex> lk(core.mu);
        core.stop = true;
    }
    core.cv_work.notify_all();
    for (auto& t : workers) t.join();
    CHECK((int)got.size() == n_req);
    int failed = 0;
    for (auto& kv : got) {
        const isax_result& r = kv.second;
        CHECK(r.collection == (int)(kv.first % n_coll));
        CHECK(r.t_submit <= r.t_start && r.t_start <= r.t_done);
        if (r.status != ISAX_OK) {
            CHECK(std::strlen(r.message) > 0);
            ++failed;
            continue;
        }
        for (int j = 0; j < r.k; ++j) {
            CHECK(r.ids[j] == (int64_t)kv.first * 1000 + j);
            CHECK(r.dists[j] == (float)j);
        }
    }
    CHECK(core.pending == 0);
    std::printf("requests %d, failed %d\n", n_req, failed);
}

int main() {
    {
        // step level: two collections, small tables so rows are reused many times
        Core core;
        StubStep a(5, 4, 8, 1, 0), b(3, 7, 8, 2, 97);
        std::vector<std::thread> w;
        w.emplace_back([&] { step_engine(core, 0, a); });
        w.emplace_back([&] { step_engine(core, 1, b); });
        drive(core, 2, 3000, 4, w);
    }
    {
        // batch level: three workers, a memory budget that admits a few requests at a time
        Core core;
        StubBatch r1(0), r2(0), r3(53);
        std::vector<std::thread> w;
        w.emplace_back([&] { batch_worker(core, r1, 16, 4000); });
        w.emplace_back([&] { batch_worker(core, r2, 16, 4000); });
        w.emplace_back([&] { batch_worker(core, r3, 16, 4000); });
        drive(core, 2, 3000, 4, w);
    }
    if (g_errors) {
        std::printf("FAILED: %d checks\n", g_errors);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
