// Scheduling core of the request loop: batch-level workers and step-level
// engines over the runner interfaces of serve_sched.h (no HIP here).
#include "serve_sched.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>

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
// Two steps are in flight: step j+1 is queued before the answers of step j are
// read, so the device does not wait for the host between steps.  A request
// holds its row from the step that admits it to the step that finishes it (a
// finished row is free for the next step, since the device copies it out
// first); the lost-candidate flags of a step belong to the requests that held
// the rows in that step.
void step_engine(Core& core, int coll, StepRunner& runner) {
    struct Entry {
        Request req;
        bool ovf = false;   // lost filter candidates in some step: answered alone
        int left = 0;       // steps until it has swept the collection
        int occupancy = 0;  // occupied rows when it joined
        double t_start = 0;
    };
    using EntryP = std::shared_ptr<Entry>;
    struct Launched {
        std::vector<EntryP> held;  // the row holders of the step, [hi]
        std::vector<EntryP> fin;   // finished in the step, in the order of its answers
        int kout = 1;
    };
    const int S = runner.slots(), C = runner.chunks(), len = runner.len();
    std::vector<EntryP> rows(S);
    std::deque<Launched> flight;
    std::vector<float> hq;
    std::vector<int32_t> hk;
    std::vector<int> adm, fin, ovf(S), status(S);
    std::vector<int64_t> ids, one_ids(ISAX_MAX_K);
    std::vector<float> dists, one_d(ISAX_MAX_K);
    int chunk = 0, busy = 0;
    auto fail_all = [&](const Failure& f) {
        // the table's state is unknown: every request in it or in flight fails with the error
        for (Launched& l : flight)
            for (EntryP& e : l.fin) core.publish(e->req, f.code, f.msg, e->occupancy, e->t_start, nullptr, nullptr);
        flight.clear();
        for (EntryP& e : rows)
            if (e) {
                core.publish(e->req, f.code, f.msg, e->occupancy, e->t_start, nullptr, nullptr);
                e.reset();
            }
        busy = 0;
        try {
            runner.reset();
        } catch (const Failure&) {
        }
    };
    auto collect = [&]() {
        Launched l = std::move(flight.front());
        flight.pop_front();
        ids.assign(l.fin.size() * l.kout, -1);
        dists.assign(l.fin.size() * l.kout, 0.f);
        runner.collect(ovf.data(), l.kout, ids.data(), dists.data(), status.data());
        for (size_t r = 0; r < l.held.size(); ++r)
            if (l.held[r] && ovf[r]) l.held[r]->ovf = true;
        for (size_t j = 0; j < l.fin.size(); ++j) {
            Entry& e = *l.fin[j];
            if (status[j] != 0 || e.ovf) {
                std::string err;
                int rc = ISAX_EDEVICE;
                try {
                    rc = runner.run_alone(e.req.q.data(), e.req.k, one_ids.data(), one_d.data(), err);
                } catch (const Failure& f) {
                    rc = f.code;
                    err = f.msg;
                }
                core.publish(e.req, rc, err, e.occupancy, e.t_start, one_ids.data(), one_d.data());
            } else {
                core.publish(e.req, ISAX_OK, "", e.occupancy, e.t_start, ids.data() + j * l.kout,
                             dists.data() + j * l.kout);
            }
        }
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
                if (!admitted.empty() || busy > 0 || !flight.empty()) break;
                if (core.stop) return;
                core.cv_work.wait(lk);
            }
        }
        if (!admitted.empty() || busy > 0) {
            // free rows, lowest first, for the new requests
            const int n = (int)admitted.size();
            const double t_adm = now();
            adm.clear();
            hq.resize((size_t)n * len);
            hk.resize(n);
            for (int i = 0, r = 0; i < n; ++i, ++r) {
                while (rows[r]) ++r;
                EntryP e = std::make_shared<Entry>();
                e->req = std::move(admitted[i]);
                e->left = C;
                e->t_start = t_adm;
                std::memcpy(hq.data() + (size_t)i * len, e->req.q.data(), (size_t)len * sizeof(float));
                hk[i] = e->req.k;
                rows[r] = std::move(e);
                adm.push_back(r);
            }
            busy += n;
            for (int r : adm) rows[r]->occupancy = busy;
            Launched l;
            int hi = 0;
            for (int r = 0; r < S; ++r)
                if (rows[r]) hi = r + 1;
            l.held.assign(rows.begin(), rows.begin() + hi);
            fin.clear();
            for (int r = 0; r < hi; ++r)
                if (rows[r] && --rows[r]->left == 0) {
                    fin.push_back(r);
                    l.kout = std::max(l.kout, rows[r]->req.k);
                    l.fin.push_back(std::move(rows[r]));
                    --busy;
                }
            try {
                runner.launch(hq.data(), hk.data(), adm.data(), n, chunk, hi, fin.data(), (int)fin.size());
            } catch (const Failure& f) {
                for (EntryP& e : l.fin) core.publish(e->req, f.code, f.msg, e->occupancy, e->t_start, nullptr, nullptr);
                fail_all(f);
                continue;
            }
            flight.push_back(std::move(l));
            chunk = (chunk + 1) % C;
            if (flight.size() < 2) continue;
        }
        try {
            collect();
        } catch (const Failure& f) {
            fail_all(f);
        }
    }
}

}  // namespace serve
}  // namespace isax
