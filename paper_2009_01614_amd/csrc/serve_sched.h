// Scheduling core of the request loop (no HIP: it drives the device through
// the runner interfaces below, so it also builds on the CPU against stub
// runners for the sanitizer tests).
//
// The paper motivates fast exact search with interactive exploration of large
// collections (Sec. I; Sec. V).  Two admission policies:
//   - batch level: a worker takes the oldest waiting request and every other
//     waiting request of its collection (up to max_batch) while the batch's
//     device scratch fits the memory budget, and answers the batch with one
//     call; workers run on their own streams, so batches overlap.
//   - step level (the reduced-precision filter modes): per collection, a table
//     of rows stays resident and the collection is swept in chunks; every step
//     runs one chunk for every occupied row.  Waiting requests join free rows
//     between steps, at whatever chunk the sweep has reached, and leave after
//     one full sweep (the sweep wraps around), so a request never waits for a
//     batch to finish.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/isax.h"

namespace isax {
namespace serve {

double now();  // seconds on the steady clock

struct Request {
    uint64_t tag;
    int32_t coll;
    int32_t k;
    std::vector<float> q;
    double t_submit;
};

// A failed device call of a runner.
struct Failure {
    int code;
    std::string msg;
};

// The state every worker of a server shares.
struct Core {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<isax_result> results;
    int64_t pending = 0;     // submitted, not yet returned by poll
    int64_t mem_in_use = 0;  // batch level: scratch of the batches in flight
    bool stop = false;
    // Appends one result (caller does not hold mu).
    void publish(const Request& r, int status, const std::string& msg, int batch_size, double t_start,
                 const int64_t* ids, const float* dists);
};

// Answers one batch of one collection (batch-level admission).
struct BatchRunner {
    virtual ~BatchRunner() = default;
    // Device scratch a batch of m queries with largest k kmax would hold.
    virtual int64_t scratch_bytes(int coll, int m, int kmax) = 0;
    // queries q [m][len of coll] (host), k[m]; ids / dists (host) [m][kmax].
    // Returns ISAX_OK or an error code with its text in err.
    virtual int run(int coll, const float* q, const int32_t* k, int m, int kmax, int64_t* ids, float* dists,
                    std::string& err) = 0;
};

// The device side of a step-level table of one collection.  Calls may throw Failure.
struct StepRunner {
    virtual ~StepRunner() = default;
    virtual int slots() const = 0;
    virtual int chunks() const = 0;  // steps per sweep
    virtual int len() const = 0;
    // Queues one step (at most two are queued and not yet collected): queries
    // q [n_adm][len] with k into the free rows adm[], chunk `chunk` of the sweep
    // for the occupied rows among [0, hi), then the final ordering of rows
    // fin[] (they are free for the next step).
    virtual void launch(const float* q, const int32_t* k, const int* adm, int n_adm, int chunk, int hi,
                        const int* fin, int n_fin) = 0;
    // Waits for the oldest queued step: ovf [its hi], the answers [n_fin][kout]
    // and status of its final ordering (status != 0: answer that row alone).
    virtual void collect(int* ovf, int kout, int64_t* ids, float* dists, int* status) = 0;
    // After a failure: nothing queued, every row free.
    virtual void reset() = 0;
    // One query answered by itself (rows that lost candidates).
    virtual int run_alone(const float* q, int k, int64_t* ids, float* dists, std::string& err) = 0;
};

// Worker loop of batch-level admission; returns once stop is set and the queue
// is empty.  max_batch >= 1; runner.run is called without mu held.
void batch_worker(Core& core, BatchRunner& runner, int max_batch, int64_t memory_budget);

// Engine loop of step-level admission for collection `coll`; returns once stop
// is set, no request of the collection waits and no row is occupied.
void step_engine(Core& core, int coll, StepRunner& runner);

}  // namespace serve
}  // namespace isax
