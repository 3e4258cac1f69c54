// Request loop over resident indexes: the C ABI and the device runners of the
// scheduling core (serve_sched.h, which describes both admission policies).
//
// Batch level: each worker thread owns a HIP stream and pinned staging, and
// answers a batch with isax_query_ex on its stream.  Step level (BF16 / FP8
// modes): one engine thread per collection owns a stream and a serving table
// (runtime.hip), which keeps the admitted queries resident and sweeps the
// collection chunk by chunk.  Every answer is exact, and its distances come
// from one fixed-order computation per (query, series) pair, so a request's
// result is the same alone and in any mix.
#include <algorithm>
#include <cstring>
#include <memory>
#include <thread>

#include "internal.h"
#include "serve_sched.h"

using isax::serve::Core;
using isax::serve::Failure;

namespace {

// Batch level: one stream, pinned host staging and device buffers per worker.
struct HipBatchRunner : isax::serve::BatchRunner {
    const std::vector<isax_index*>& colls;
    int mode;
    int B, max_len;
    hipStream_t stream = nullptr;
    float *hq = nullptr, *dq = nullptr, *hd = nullptr, *dd = nullptr;
    int64_t *hi = nullptr, *di = nullptr;
    int32_t *hk = nullptr, *dk = nullptr;
    bool ok = false;
    std::string why;
    HipBatchRunner(const std::vector<isax_index*>& c, int mode_, int B_, int max_len_)
        : colls(c), mode(mode_), B(B_), max_len(max_len_) {
        (void)hipSetDevice(colls[0]->device);
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            stream = nullptr;
            why = "server stream creation failed";
            return;
        }
        ok = hipHostMalloc((void**)&hq, (size_t)B * max_len * 4, 0) == hipSuccess &&
             hipHostMalloc((void**)&hd, (size_t)B * ISAX_MAX_K * 4, 0) == hipSuccess &&
             hipHostMalloc((void**)&hi, (size_t)B * ISAX_MAX_K * 8, 0) == hipSuccess &&
             hipHostMalloc((void**)&hk, (size_t)B * 4, 0) == hipSuccess &&
             hipMalloc((void**)&dq, (size_t)B * max_len * 4) == hipSuccess &&
             hipMalloc((void**)&dd, (size_t)B * ISAX_MAX_K * 4) == hipSuccess &&
             hipMalloc((void**)&di, (size_t)B * ISAX_MAX_K * 8) == hipSuccess &&
             hipMalloc((void**)&dk, (size_t)B * 4) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            why = "server staging allocation failed";
        }
    }
    ~HipBatchRunner() override {
        (void)hipFree(dq);
        (void)hipFree(dd);
        (void)hipFree(di);
        (void)hipFree(dk);
        (void)hipHostFree(hq);
        (void)hipHostFree(hd);
        (void)hipHostFree(hi);
        (void)hipHostFree(hk);
        if (stream) (void)hipStreamDestroy(stream);
    }
    int64_t scratch_bytes(int coll, int m, int kmax) override {
        return isax::query_scratch_bytes(colls[coll], m, kmax, mode);
    }
    int run(int coll, const float* q, const int32_t* k, int m, int kmax, int64_t* ids, float* dists,
            std::string& err) override {
        // without its own stream or staging the worker answers with an error instead of
        // running on the null stream
        if (!ok) {
            err = why;
            return ISAX_ENOMEM;
        }
        isax_index* idx = colls[coll];
        const int len = idx->len;
        std::memcpy(hq, q, (size_t)m * len * 4);
        std::memcpy(hk, k, (size_t)m * 4);
        (void)hipMemcpyAsync(dq, hq, (size_t)m * len * 4, hipMemcpyHostToDevice, stream);
        (void)hipMemcpyAsync(dk, hk, (size_t)m * 4, hipMemcpyHostToDevice, stream);
        isax_query_options qo{};
        qo.mode = mode;
        qo.k_per_query = dk;
        qo.stream = stream;
        int rc = isax_query_ex(idx, dq, m, kmax, di, dd, &qo);
        if (rc != ISAX_OK) {
            err = isax_last_error();
            return rc;
        }
        (void)hipMemcpyAsync(hi, di, (size_t)m * kmax * 8, hipMemcpyDeviceToHost, stream);
        (void)hipMemcpyAsync(hd, dd, (size_t)m * kmax * 4, hipMemcpyDeviceToHost, stream);
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return ISAX_EDEVICE;
        }
        std::memcpy(ids, hi, (size_t)m * kmax * 8);
        std::memcpy(dists, hd, (size_t)m * kmax * 4);
        return ISAX_OK;
    }
};

// Step level: the serving table of one collection on the engine's stream.
struct HipStepRunner : isax::serve::StepRunner {
    isax_index* idx;
    int mode;
    hipStream_t stream = nullptr;
    isax::StepTable* table = nullptr;
    float *dq = nullptr, *dd = nullptr;
    int64_t* di = nullptr;
    HipStepRunner(isax_index* idx_, int mode_, int slots, int chunks) : idx(idx_), mode(mode_) {
        (void)hipSetDevice(idx->device);
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            throw isax::Error{ISAX_EDEVICE, "server stream creation failed"};
        }
        try {
            table = isax::step_table_create(idx, mode, slots, chunks, stream);
            if (hipMalloc((void**)&dq, (size_t)idx->len * 4) != hipSuccess ||
                hipMalloc((void**)&dd, (size_t)ISAX_MAX_K * 4) != hipSuccess ||
                hipMalloc((void**)&di, (size_t)ISAX_MAX_K * 8) != hipSuccess) {
                (void)hipGetLastError();
                throw isax::Error{ISAX_ENOMEM, "server staging allocation failed"};
            }
        } catch (...) {
            release();
            throw;
        }
        slots_ = slots;
        chunks_ = isax::step_table_chunks(table);
    }
    void release() {
        isax::step_table_destroy(table);
        table = nullptr;
        (void)hipFree(dq);
        (void)hipFree(dd);
        (void)hipFree(di);
        if (stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
    ~HipStepRunner() override { release(); }
    int slots_ = 0, chunks_ = 0;
    int slots() const override { return slots_; }
    int chunks() const override { return chunks_; }
    int len() const override { return idx->len; }
    template <class F>
    void guard(F&& f) {
        try {
            f();
        } catch (const isax::Error& e) {
            throw Failure{e.code, e.msg};
        }
    }
    void launch(const float* q, const int32_t* k, const int* adm, int n_adm, int chunk, int hi, const int* fin,
                int n_fin) override {
        guard([&] { isax::step_table_launch(table, q, k, adm, n_adm, chunk, hi, fin, n_fin); });
    }
    void collect(int* ovf, int kout, int64_t* ids, float* dists, int* status) override {
        guard([&] { isax::step_table_collect(table, ovf, kout, ids, dists, status); });
    }
    void reset() override {
        guard([&] { isax::step_table_reset(table); });
    }
    int run_alone(const float* q, int k, int64_t* ids, float* dists, std::string& err) override {
        isax_query_options qo{};
        qo.mode = mode;
        qo.stream = stream;
        if (hipMemcpyAsync(dq, q, (size_t)idx->len * 4, hipMemcpyHostToDevice, stream) != hipSuccess) {
            err = "query upload failed";
            return ISAX_EDEVICE;
        }
        int rc = isax_query_ex(idx, dq, 1, k, di, dd, &qo);
        if (rc != ISAX_OK) {
            err = isax_last_error();
            return rc;
        }
        if (hipMemcpyAsync(ids, di, (size_t)k * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipMemcpyAsync(dists, dd, (size_t)k * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            err = "answer download failed";
            return ISAX_EDEVICE;
        }
        return ISAX_OK;
    }
};

}  // namespace

struct isax_server {
    std::vector<isax_index*> colls;
    isax_server_options opt{};
    Core core;
    std::vector<std::unique_ptr<isax::serve::BatchRunner>> batch_runners;
    std::vector<std::unique_ptr<isax::serve::StepRunner>> step_runners;
    std::vector<std::thread> threads;
};

extern "C" {

isax_server* isax_server_create(isax_index* const* collections, int32_t n_collections, const isax_server_options* o) {
    isax::clear_error();
    if (!collections || n_collections < 1) {
        isax::set_error(ISAX_EINVAL, "at least one collection is needed");
        return nullptr;
    }
    isax_server_options opt{};
    if (o) opt = *o;
    const bool filter_mode = opt.mode == ISAX_MODE_BF16 || opt.mode == ISAX_MODE_FP8;
    const bool step = filter_mode && !(opt.flags & ISAX_SERVE_BATCHES);
    if (opt.max_batch == 0) opt.max_batch = step ? 512 : 256;
    if (opt.streams == 0) opt.streams = 4;
    if (opt.memory_budget == 0) opt.memory_budget = int64_t(4) << 30;
    if (opt.chunks == 0) opt.chunks = 8;
    if (opt.max_batch < 1 || opt.max_batch > 4096 || opt.streams < 1 || opt.streams > 16 || opt.memory_budget < 0 ||
        opt.mode < ISAX_MODE_INDEX || opt.mode > ISAX_MODE_HYBRID || (opt.flags & ~ISAX_SERVE_BATCHES) != 0 ||
        opt.chunks < 1 || opt.chunks > 1024 || opt.reserved != 0) {
        isax::set_error(ISAX_EINVAL, "bad server options (max_batch 1..4096, streams 1..16, mode, flags, "
                                     "chunks 1..1024, reserved = 0)");
        return nullptr;
    }
    std::unique_ptr<isax_server> s(new isax_server());
    s->opt = opt;
    int max_len = 0;
    for (int i = 0; i < n_collections; ++i) {
        isax_index* idx = collections[i];
        if (!idx || idx->device != collections[0]->device) {
            isax::set_error(ISAX_EINVAL, "collections must be non-NULL indexes on one device");
            return nullptr;
        }
        if (((opt.mode == ISAX_MODE_BF16 || opt.mode == ISAX_MODE_HYBRID) && !idx->x_bf16 && !idx->x_spec) ||
            (opt.mode == ISAX_MODE_FP8 && !idx->x_fp8)) {
            isax::set_error(ISAX_EINVAL, "a collection lacks the reduced-precision copy the mode needs");
            return nullptr;
        }
        s->colls.push_back(idx);
        max_len = std::max(max_len, idx->len);
    }
    isax_server* raw = s.get();
    if (step) {
        try {
            for (int c = 0; c < n_collections; ++c)
                s->step_runners.emplace_back(new HipStepRunner(s->colls[c], opt.mode, opt.max_batch, opt.chunks));
        } catch (const isax::Error& e) {
            isax::set_error(e.code, e.msg);
            return nullptr;
        } catch (const std::bad_alloc&) {
            isax::set_error(ISAX_ENOMEM, "host allocation failed");
            return nullptr;
        }
        for (int c = 0; c < n_collections; ++c)
            s->threads.emplace_back([raw, c] { isax::serve::step_engine(raw->core, c, *raw->step_runners[c]); });
    } else {
        for (int w = 0; w < opt.streams; ++w)
            s->batch_runners.emplace_back(new HipBatchRunner(s->colls, opt.mode, opt.max_batch, max_len));
        for (int w = 0; w < opt.streams; ++w)
            s->threads.emplace_back([raw, w] {
                isax::serve::batch_worker(raw->core, *raw->batch_runners[w], raw->opt.max_batch,
                                          raw->opt.memory_budget);
            });
    }
    return s.release();
}

int isax_server_submit(isax_server* s, int32_t collection, const float* query, int32_t k, uint64_t tag) {
    isax::clear_error();
    if (!s || !query || collection < 0 || collection >= (int32_t)s->colls.size()) {
        isax::set_error(ISAX_EINVAL, "bad server, query or collection");
        return ISAX_EINVAL;
    }
    const isax_index* idx = s->colls[collection];
    if (k < 1 || k > ISAX_MAX_K || k > idx->n) {
        isax::set_error(ISAX_EINVAL, "k must be in 1..min(n, 1024)");
        return ISAX_EINVAL;
    }
    for (int t = 0; t < idx->len; ++t)
        if (!(std::fabs(query[t]) <= 3.4028235e38f)) {
            isax::set_error(ISAX_EINVAL, "query holds a non-finite value");
            return ISAX_EINVAL;
        }
    isax::serve::Request r{tag, collection, k, std::vector<float>(query, query + idx->len), isax::serve::now()};
    {
        std::lock_guard<std::mutex> lk(s->core.mu);
        if (s->core.stop) {
            isax::set_error(ISAX_EINVAL, "server is shutting down");
            return ISAX_EINVAL;
        }
        s->core.queue.push_back(std::move(r));
        ++s->core.pending;
    }
    // every waiter: step engines serve one collection each
    s->core.cv_work.notify_all();
    return ISAX_OK;
}

int isax_server_poll(isax_server* s, isax_result* out, int32_t max_results, int32_t timeout_ms) {
    if (!s || !out || max_results < 0) return ISAX_EINVAL;
    std::unique_lock<std::mutex> lk(s->core.mu);
    if (s->core.results.empty() && timeout_ms > 0)
        s->core.cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !s->core.results.empty(); });
    int n = 0;
    while (n < max_results && !s->core.results.empty()) {
        out[n++] = s->core.results.front();
        s->core.results.pop_front();
        --s->core.pending;
    }
    return n;
}

int64_t isax_server_pending(isax_server* s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lk(s->core.mu);
    return s->core.pending;
}

void isax_server_destroy(isax_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->core.mu);
        s->core.stop = true;
    }
    s->core.cv_work.notify_all();
    for (auto& t : s->threads) t.join();
    delete s;
}

}  // extern "C"
