// Serving core: admission by device-memory footprint and continuous batching
// of queued traversal queries, independent of the device (an Executor runs
// the batches), so the scheduling policy is testable on a CPU.
//
// Policy. A query whose single-query footprint exceeds the budget is refused
// at submission. Worker threads (one per device stream) repeatedly take the
// oldest pending query and add every other pending query for the same graph
// and algorithm, up to the executor's batch limit and the memory still free
// (budget minus running batches, results not yet collected and the bytes the
// executor holds between batches). Idle bytes in the way of a batch are
// trimmed first; a batch that still does not fit waits until memory frees
// up. Queries that arrive while others run are picked up by the next free
// worker, so batches of different sizes run concurrently on different
// streams. A result stays charged to the budget until the client collects
// it. Invariant: device bytes held <= in_use + idle <= budget, given that
// work_bytes() bounds what a batch allocates beyond idle memory it reuses.
// A query that cannot fit even alone while nothing runs and nothing is
// charged (idle memory that trim() cannot free fills the budget) fails with
// an admission status instead of waiting forever.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

namespace gg {
namespace serve {

using Clock = std::chrono::steady_clock;

// status of a query refused because it can never fit (the C ABI's GG_ERR_ADMISSION)
constexpr int kAdmissionStatus = 6;

// thrown by submit() when a single query can never fit the memory budget
struct AdmissionError : std::runtime_error {
    explicit AdmissionError(const std::string &m) : std::runtime_error(m) {}
};

struct Req {
    int64_t ticket = 0;
    int gid = 0, algo = 0, src = 0;
    Clock::time_point t_arrive, t_start, t_done;
    int status = 0;          // 0 ok, else a gg_status code
    int batch_size = 0;
    size_t result_bytes = 0;
    void *result = nullptr;  // executor-owned result storage
    bool done = false;
};

struct Batch {
    int gid = 0, algo = 0;
    std::vector<Req *> reqs;
    size_t work_bytes = 0;  // transient footprint while the batch runs
};

class Executor {
public:
    virtual ~Executor() = default;
    // most queries of (graph, algorithm) one batch may hold
    virtual int max_batch(int gid, int algo) const = 0;
    // device bytes a batch of k queries needs while it runs (results excluded)
    virtual size_t work_bytes(int gid, int algo, int k) const = 0;
    // device bytes one query's result occupies until collected
    virtual size_t result_bytes(int gid, int algo) const = 0;
    // run the batch on the worker's stream; fill each Req's status / result
    virtual void run(int worker, Batch &b) = 0;
    // free one collected result
    virtual void release(Req &r) = 0;
    // device bytes held between batches (pooled workspaces, derived layouts
    // of the served graphs): charged to the budget beside running batches
    // and uncollected results
    virtual size_t idle_bytes() { return 0; }
    // free idle bytes (best effort) until idle_bytes() <= target
    virtual void trim(size_t target) { (void)target; }
    // the part of idle_bytes() that trim() cannot free (derived layouts)
    virtual size_t pinned_bytes() { return 0; }
};

struct Stats {
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, collected = 0;
    int32_t max_batch_seen = 0;
    size_t bytes_in_use = 0, bytes_peak = 0;  // running batches + uncollected results
    size_t bytes_idle = 0;                    // held by the executor between batches
    int64_t trims = 0;                        // batches that had idle memory freed first
    double busy_ms = 0;
};

class Core {
public:
    Core(Executor *ex, size_t budget, int workers);
    ~Core();
    // returns the ticket; throws AdmissionError if a single query can never fit
    int64_t submit(int gid, int algo, int src);
    // true when the query is done; copies its record (result stays charged until collect)
    bool peek(int64_t ticket, Req &out);
    // block until done or timeout (seconds, < 0 = forever); true when done
    bool wait(int64_t ticket, double timeout_s, Req &out);
    // release a done query's result (after the caller copied it); false if unknown
    bool collect(int64_t ticket);
    bool known(int64_t ticket);
    Stats stats();
    void shutdown();

private:
    void worker(int id);
    bool form_batch(Batch &b);  // called with mu held
    bool try_batch(Batch &b);   // the head query's batch, if it fits now (mu held)

    Executor *ex_;
    size_t budget_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Req *> pending_;
    std::map<int64_t, std::unique_ptr<Req>> reqs_;
    std::vector<std::thread> threads_;
    int64_t next_ticket_ = 1;
    size_t in_use_ = 0;
    int running_ = 0;  // batches on the device now
    bool stop_ = false;
    Stats st_;
};

}  // namespace serve
}  // namespace gg
