// Scheduling core of the request loop: batch-level workers and step-level
// engines over the runner interfaces of serve_sched.h (no HIP here).
#include "serve_sched.h"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace isax {
namespace serve {

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

void Core::publish(const Request& r, int status, const std::string& msg, int batch_size, double t_start,
                   const int64_t* ids, const float* dists) {
    isax_result res;
    std::memset(&res, 0, sizeof(res));
    res.tag = r.tag;
    res.status = status;
    res.k = r.k;
    res.collection = r.coll;
    res.batch_size = batch_size;
    res.t_submit = r.t_submit;
    res.t_start = t_start;
    res.t_done = now();
    if (status == ISAX_OK) {
        std::memcpy(res.ids, ids, (size_t)r.k * sizeof(int64_t));
        std::memcpy(res.dists, dists, (size_t)r.k * sizeof(float));
    } else {
        std::strncpy(res.message, msg.c_str(), sizeof(res.message) - 1);
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        results.push_back(res);
    }
    cv_done.notify_all();
}

// ------------------------------------------------------------------ batch level
void batch_worker(Core& core, BatchRunner& runner, int max_batch, int64_t memory_budget) {
    std::vector<float> hq;
    std::vector<int32_t> hk;
    std::vector<int64_t> ids;
    std::vector<float> dists;
    for (;;) {
        std::vector<Request> batch;
        int64_t mem = 0;
        {
            std::unique_lock<std::mutex> lk(core.mu);
            for (;;) {
                if (!core.queue.empty()) {
                    // the oldest request's collection; admit while the scratch estimate fits the budget
                    const int coll = core.queue.front().coll;
                    int kmax = 0;
                    std::vector<size_t> take;
                    for (size_t i = 0; i < core.queue.size() && (int)take.size() < max_batch; ++i) {
                        if (core.queue[i].coll != coll) continue;
                        const int km = std::max(kmax, core.queue[i].k);
                        const int64_t need = runner.scratch_bytes(coll, (int)take.size() + 1, km);
                        if (core.mem_in_use + need > memory_budget && !take.empty()) break;
                        if (core.mem_in_use + need > memory_budget && core.mem_in_use > 0) break;
                        take.push_back(i);
                        kmax = km;
                        mem = need;
                    }
                    if (!take.empty()) {
                        for (size_t j = take.size(); j-- > 0;) {
                            batch.push_back(std::move(core.queue[take[j]]));
                            core.queue.erase(core.queue.begin() + (std::ptrdiff_t)take[j]);
                        }
                        std::reverse(batch.begin(), batch.end());
                        core.mem_in_use += mem;
                        break;
                    }
                }
                if (core.stop && core.queue.empty()) return;
                core.cv_work.wait(lk);
            }
        }
        const double t_start = now();
        const int m = (int)batch.size();
        const int coll = batch[0].coll;
        const int len = (int)batch[0].q.size();
        int kmax = 0;
        hq.resize((size_t)m * len);
        hk.resize(m);
        for (int i = 0; i < m; ++i) {
            std::memcpy(hq.data() + (size_t)i * len, batch[i].q.data(), (size_t)len * sizeof(float));
            hk[i] = batch[i].k;
            kmax = std::max(kmax, batch[i].k);
        }
        ids.assign((size_t)m * kmax, -1);
        dists.assign((size_t)m * kmax, 0.f);
        std::string err;
        const int rc = runner.run(coll, hq.data(), hk.data(), m, kmax, ids.data(), dists.data(), err);
        for (int i = 0; i < m; ++i)
            core.publish(batch[i], rc, err, m, t_start, ids.data() + (size_t)i * kmax, dists.data() + (size_t)i * kmax);
        {
            std::lock_guard<std::mutex> lk(core.mu);
            core.mem_in_use -= mem;
        }
        core.cv_work.notify_all();
    }
}

// ------------------------------------------------------------------ step level
void step_engine(Core& core, int coll, StepRunner& runner) {
    struct Row {
        bool busy = false;
        bool ovf = false;  // lost filter candidates in some step: answered alone
        int left = 0;      // steps until the row has swept the collection
        int occupancy = 0; // occupied rows when it joined
        double t_start = 0;
        Request req;
    };
    const int S = runner.slots(), C = runner.chunks(), len = runner.len();
    std::vector<Row> rows(S);
    std::vector<float> hq;
    std::vector<int32_t> hk;
    std::vector<int> rid, fin, ovf(S), status(S);
    std::vector<int64_t> ids, one_ids(ISAX_MAX_K);
    std::vector<float> dists, one_d(ISAX_MAX_K);
    int chunk = 0, busy = 0;
    auto release = [&](int r) {
        rows[r].busy = false;
        rows[r].req.q.clear();
        --busy;
    };
    for (;;) {
        std::vector<Request> admitted;
        {
            std::unique_lock<std::mutex> lk(core.mu);
            for (;;) {
                const int room = S - busy;
                for (auto it = core.queue.begin(); it != core.queue.end() && (int)admitted.size() < room;) {
                    if (it->coll == coll) {
                        admitted.push_back(std::move(*it));
                        it = core.queue.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (!admitted.empty() || busy > 0) break;
                if (core.stop) return;
                core.cv_work.wait(lk);
            }
        }
        // free rows, lowest first, for the new requests
        const int n = (int)admitted.size();
        const double t_adm = now();
        rid.clear();
        hq.resize((size_t)n * len);
        hk.resize(n);
        for (int i = 0, r = 0; i < n; ++i, ++r) {
            while (rows[r].busy) ++r;
            Row& row = rows[r];
            row.busy = true;
            row.ovf = false;
            row.left = C;
            row.t_start = t_adm;
            row.req = std::move(admitted[i]);
            std::memcpy(hq.data() + (size_t)i * len, row.req.q.data(), (size_t)len * sizeof(float));
            hk[i] = row.req.k;
            rid.push_back(r);
        }
        busy += n;
        for (int r : rid) rows[r].occupancy = busy;
        int hi = 0;
        for (int r = 0; r < S; ++r)
            if (rows[r].busy) hi = r + 1;
        fin.clear();
        int kout = 1;
        for (int r = 0; r < hi; ++r)
            if (rows[r].busy && rows[r].left == 1) {
                fin.push_back(r);
                kout = std::max(kout, rows[r].req.k);
            }
        ids.assign(fin.size() * kout, -1);
        dists.assign(fin.size() * kout, 0.f);
        try {
            runner.admit(hq.data(), hk.data(), rid.data(), n);
            runner.step(chunk, hi);
            runner.finish(fin.data(), (int)fin.size());
            runner.sync(ovf.data(), kout, ids.data(), dists.data(), status.data());
        } catch (const Failure& f) {
            // the table's state is unknown: every occupied row fails with the error
            for (int r = 0; r < S; ++r)
                if (rows[r].busy) {
                    core.publish(rows[r].req, f.code, f.msg, rows[r].occupancy, rows[r].t_start, nullptr, nullptr);
                    release(r);
                }
            continue;
        }
        for (int r = 0; r < hi; ++r)
            if (rows[r].busy) {
                rows[r].ovf |= ovf[r] != 0;
                --rows[r].left;
            }
        for (size_t j = 0; j < fin.size(); ++j) {
            Row& row = rows[fin[j]];
            if (status[j] != 0 || row.ovf) {
                std::string err;
                int rc = ISAX_EDEVICE;
                try {
                    rc = runner.run_alone(row.req.q.data(), row.req.k, one_ids.data(), one_d.data(), err);
                } catch (const Failure& f) {
                    rc = f.code;
                    err = f.msg;
                }
                core.publish(row.req, rc, err, row.occupancy, row.t_start, one_ids.data(), one_d.data());
            } else {
                core.publish(row.req, ISAX_OK, "", row.occupancy, row.t_start, ids.data() + j * kout,
                             dists.data() + j * kout);
            }
            release(fin[j]);
        }
        chunk = (chunk + 1) % C;
    }
}

}  // namespace serve
}  // namespace isax
