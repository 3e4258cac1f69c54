// Serving loop: continuous batching of exact k-NN requests over resident indexes.
//
// The paper motivates fast exact search with interactive exploration of large
// collections (Sec. I; Sec. V); this loop keeps the indexes resident and
// serves requests as they arrive.  Each of `streams` worker threads owns one
// HIP stream and pinned staging buffers.  A free worker takes the oldest
// waiting request and every other waiting request of the same collection (up
// to max_batch), provided the batch's device scratch fits in what is left of
// the memory budget, and runs it with isax_query_ex on its own stream; so
// requests that arrive while other batches run are admitted as soon as a
// worker and memory are free, and batches on different streams overlap on the
// device.  Every request's answer is exact and its distances come from one
// fixed-order computation per (query, series) pair, so it is the same alone
// and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "internal.h"

namespace {

struct Request {
    uint64_t tag;
    int32_t coll;
    int32_t k;
    std::vector<float> q;
    double t_submit;
};

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

}  // namespace

struct isax_server {
    std::vector<isax_index*> colls;
    isax_server_options opt{};
    int max_len = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<isax_result> results;
    int64_t pending = 0;
    int64_t mem_in_use = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    void worker_main(int wid);
};

void isax_server::worker_main(int wid) {
    (void)wid;
    int dev = colls[0]->device;
    (void)hipSetDevice(dev);
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    const int B = opt.max_batch;
    float *hq = nullptr, *dq = nullptr, *hd = nullptr, *dd = nullptr;
    int64_t *hi = nullptr, *di = nullptr;
    int32_t *hk = nullptr, *dk = nullptr;
    bool ok = hipHostMalloc((void**)&hq, (size_t)B * max_len * 4, 0) == hipSuccess &&
              hipHostMalloc((void**)&hd, (size_t)B * ISAX_MAX_K * 4, 0) == hipSuccess &&
              hipHostMalloc((void**)&hi, (size_t)B * ISAX_MAX_K * 8, 0) == hipSuccess &&
              hipHostMalloc((void**)&hk, (size_t)B * 4, 0) == hipSuccess &&
              hipMalloc((void**)&dq, (size_t)B * max_len * 4) == hipSuccess &&
              hipMalloc((void**)&dd, (size_t)B * ISAX_MAX_K * 4) == hipSuccess &&
              hipMalloc((void**)&di, (size_t)B * ISAX_MAX_K * 8) == hipSuccess &&
              hipMalloc((void**)&dk, (size_t)B * 4) == hipSuccess;
    while (true) {
        std::vector<Request> batch;
        int64_t mem = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            while (true) {
                if (stop && queue.empty()) break;
                if (!queue.empty()) {
                    // oldest request's collection; admit while the scratch estimate fits the budget
                    const int coll = queue.front().coll;
                    const isax_index* idx = colls[coll];
                    int kmax = 0;
                    std::vector<size_t> take;
                    for (size_t i = 0; i < queue.size() && (int)take.size() < B; ++i) {
                        if (queue[i].coll != coll) continue;
                        const int km = std::max(kmax, queue[i].k);
                        const int64_t need = isax::query_scratch_bytes(idx, (int)take.size() + 1, km, opt.mode);
                        if (mem_in_use + need > opt.memory_budget && !take.empty()) break;
                        if (mem_in_use + need > opt.memory_budget && mem_in_use > 0) break;
                        take.push_back(i);
                        kmax = km;
                        mem = need;
                    }
                    if (!take.empty()) {
                        for (size_t j = take.size(); j-- > 0;) {
                            batch.push_back(std::move(queue[take[j]]));
                            queue.erase(queue.begin() + (std::ptrdiff_t)take[j]);
                        }
                        std::reverse(batch.begin(), batch.end());
                        mem_in_use += mem;
                        break;
                    }
                }
                cv_work.wait(lk);
            }
        }
        if (batch.empty()) break;
        const double t_start = now();
        const int m = (int)batch.size();
        isax_index* idx = colls[batch[0].coll];
        const int len = idx->len;
        int kmax = 0;
        for (int i = 0; i < m; ++i) {
            std::memcpy(hq + (size_t)i * len, batch[i].q.data(), (size_t)len * 4);
            hk[i] = batch[i].k;
            kmax = std::max(kmax, batch[i].k);
        }
        int rc = ok ? ISAX_OK : ISAX_ENOMEM;
        std::string err = ok ? "" : "server staging allocation failed";
        if (ok) {
            (void)hipMemcpyAsync(dq, hq, (size_t)m * len * 4, hipMemcpyHostToDevice, stream);
            (void)hipMemcpyAsync(dk, hk, (size_t)m * 4, hipMemcpyHostToDevice, stream);
            isax_query_options qo{};
            qo.mode = opt.mode;
            qo.k_per_query = dk;
            qo.stream = stream;
            rc = isax_query_ex(idx, dq, m, kmax, di, dd, &qo);
            if (rc == ISAX_OK) {
                (void)hipMemcpyAsync(hi, di, (size_t)m * kmax * 8, hipMemcpyDeviceToHost, stream);
                (void)hipMemcpyAsync(hd, dd, (size_t)m * kmax * 4, hipMemcpyDeviceToHost, stream);
                if (hipStreamSynchronize(stream) != hipSuccess) rc = ISAX_EDEVICE;
            } else {
                err = isax_last_error();
            }
        }
        const double t_done = now();
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int i = 0; i < m; ++i) {
                isax_result r;
                std::memset(&r, 0, sizeof(r));
                r.tag = batch[i].tag;
                r.status = rc;
                r.k = batch[i].k;
                r.collection = batch[i].coll;
                r.batch_size = m;
                r.t_submit = batch[i].t_submit;
                r.t_start = t_start;
                r.t_done = t_done;
                if (rc == ISAX_OK) {
                    std::memcpy(r.ids, hi + (size_t)i * kmax, (size_t)r.k * 8);
                    std::memcpy(r.dists, hd + (size_t)i * kmax, (size_t)r.k * 4);
                }
                results.push_back(r);
            }
            mem_in_use -= mem;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    (void)hipFree(dq);
    (void)hipFree(dd);
    (void)hipFree(di);
    (void)hipFree(dk);
    (void)hipHostFree(hq);
    (void)hipHostFree(hd);
    (void)hipHostFree(hi);
    (void)hipHostFree(hk);
    (void)hipStreamDestroy(stream);
}

extern "C" {

isax_server* isax_server_create(isax_index* const* collections, int32_t n_collections, const isax_server_options* o) {
    isax::clear_error();
    if (!collections || n_collections < 1) {
        isax::set_error(ISAX_EINVAL, "at least one collection is needed");
        return nullptr;
    }
    isax_server_options opt{};
    if (o) opt = *o;
    if (opt.max_batch == 0) opt.max_batch = 256;
    if (opt.streams == 0) opt.streams = 4;
    if (opt.memory_budget == 0) opt.memory_budget = int64_t(4) << 30;
    if (opt.max_batch < 1 || opt.max_batch > 4096 || opt.streams < 1 || opt.streams > 16 || opt.memory_budget < 0 ||
        opt.mode < ISAX_MODE_INDEX || opt.mode > ISAX_MODE_HYBRID || opt.reserved != 0) {
        isax::set_error(ISAX_EINVAL, "bad server options (max_batch 1..4096, streams 1..16, mode, reserved = 0)");
        return nullptr;
    }
    auto* s = new isax_server();
    s->opt = opt;
    for (int i = 0; i < n_collections; ++i) {
        isax_index* idx = collections[i];
        if (!idx || idx->device != collections[0]->device) {
            isax::set_error(ISAX_EINVAL, "collections must be non-NULL indexes on one device");
            delete s;
            return nullptr;
        }
        if (((opt.mode == ISAX_MODE_BF16 || opt.mode == ISAX_MODE_HYBRID) && !idx->x_bf16) || (opt.mode == ISAX_MODE_FP8 && !idx->x_fp8)) {
            isax::set_error(ISAX_EINVAL, "a collection lacks the reduced-precision copy the mode needs");
            delete s;
            return nullptr;
        }
        s->colls.push_back(idx);
        s->max_len = std::max(s->max_len, idx->len);
    }
    for (int w = 0; w < opt.streams; ++w) s->workers.emplace_back(&isax_server::worker_main, s, w);
    return s;
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
    Request r{tag, collection, k, std::vector<float>(query, query + idx->len), now()};
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            isax::set_error(ISAX_EINVAL, "server is shutting down");
            return ISAX_EINVAL;
        }
        s->queue.push_back(std::move(r));
        ++s->pending;
    }
    s->cv_work.notify_one();
    return ISAX_OK;
}

int isax_server_poll(isax_server* s, isax_result* out, int32_t max_results, int32_t timeout_ms) {
    if (!s || !out || max_results < 0) return ISAX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !s->results.empty(); });
    int n = 0;
    while (n < max_results && !s->results.empty()) {
        out[n++] = s->results.front();
        s->results.pop_front();
        --s->pending;
    }
    return n;
}

int64_t isax_server_pending(isax_server* s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->pending;
}

void isax_server_destroy(isax_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
}

}  // extern "C"
