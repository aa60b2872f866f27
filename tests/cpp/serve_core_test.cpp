// CPU test of the serving core's policy with a fake executor (no device):
// admission refusal, continuous batching per (graph, algorithm), the memory
// budget (including uncollected results) and result delivery.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "../../paper_2012_07990_amd/csrc/serve_core.hpp"

using namespace gg::serve;

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                      \
        }                                                                      \
    } while (0)

struct Fake : Executor {
    size_t work_per = 100, result_per = 10;
    int sleep_ms = 2;
    std::atomic<int> running{0}, max_running{0};
    std::atomic<int> mixed{0};
    int max_batch(int, int algo) const override { return algo == 0 ? 64 : algo == 4 ? 16 : 1; }
    size_t work_bytes(int, int, int k) const override { return work_per * (size_t)k; }
    size_t result_bytes(int, int) const override { return result_per; }
    void run(int, Batch &b) override {
        int r = ++running;
        int m = max_running.load();
        while (r > m && !max_running.compare_exchange_weak(m, r)) {}
        for (Req *q : b.reqs)
            if (q->gid != b.gid || q->algo != b.algo) mixed++;
        std::this_thread::sleep_for(std::chrono::milliseconds(sleep_ms));
        for (Req *q : b.reqs) {
            int *v = (int *)std::malloc(sizeof(int));
            *v = q->src * 3 + q->algo;
            q->result = v;
            q->status = q->src < 0 ? 5 : 0;
        }
        --running;
    }
    void release(Req &r) override {
        std::free(r.result);
        r.result = nullptr;
    }
};

static void test_admission() {
    Fake f;
    Core c(&f, 50, 1);
    bool threw = false;
    try {
        c.submit(0, 0, 1);
    } catch (const AdmissionError &) {
        threw = true;
    }
    CHECK(threw);
    CHECK(c.stats().rejected == 1);
    std::puts("ok admission");
}

static void test_batching_and_results() {
    Fake f;
    f.sleep_ms = 20;
    Core c(&f, 1 << 30, 1);
    std::vector<int64_t> t;
    for (int i = 0; i < 200; i++) t.push_back(c.submit(i % 2, 0, i));  // two graphs, BFS
    for (int i = 0; i < 200; i++) {
        Req r;
        CHECK(c.wait(t[i], 10.0, r));
        CHECK(r.status == 0 && *(int *)r.result == i * 3);
        CHECK(r.batch_size >= 1 && r.batch_size <= 64);
        CHECK(c.collect(t[i]));
    }
    const Stats s = c.stats();
    CHECK(s.completed == 200 && s.collected == 200);
    CHECK(s.max_batch_seen > 1);       // queued queries were batched
    CHECK(s.batches < 200);
    CHECK(f.mixed.load() == 0);        // a batch never mixes graphs or algorithms
    CHECK(s.bytes_in_use == 0);
    std::puts("ok batching");
}

static void test_budget_limits_batch_and_concurrency() {
    Fake f;
    f.sleep_ms = 5;
    Core c(&f, 400, 4);  // at most 3 queries (3 * 110) in flight
    std::vector<int64_t> t;
    for (int i = 0; i < 60; i++) t.push_back(c.submit(0, 0, i));
    for (auto x : t) {
        Req r;
        CHECK(c.wait(x, 10.0, r));
        CHECK(r.batch_size <= 3);
        CHECK(c.collect(x));
    }
    CHECK(c.stats().bytes_peak <= 400);
    std::puts("ok budget");
}

static void test_uncollected_results_hold_memory() {
    Fake f;
    f.sleep_ms = 1;
    f.work_per = 10;
    f.result_per = 100;
    Core c(&f, 230, 2);  // two queries fit (2 * 110); their results (2 * 100) stay charged
    int64_t a = c.submit(0, 1, 1), b = c.submit(0, 1, 2);  // SSSP: no batching
    Req r;
    CHECK(c.wait(a, 5.0, r));
    CHECK(c.wait(b, 5.0, r));
    int64_t d = c.submit(0, 1, 3);
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    CHECK(!c.peek(d, r));            // blocked: both results still held
    CHECK(c.collect(a));
    CHECK(c.wait(d, 5.0, r));        // runs once memory was released
    CHECK(*(int *)r.result == 3 * 3 + 1);
    std::puts("ok hold");
}

static void test_failed_query_frees_memory() {
    Fake f;
    Core c(&f, 1000, 1);
    int64_t a = c.submit(0, 1, -1);
    Req r;
    CHECK(c.wait(a, 5.0, r));
    CHECK(r.status == 5);
    CHECK(c.collect(a));
    CHECK(c.stats().bytes_in_use == 0);
    std::puts("ok failure");
}

static void test_concurrent_workers_overlap() {
    Fake f;
    f.sleep_ms = 30;
    Core c(&f, 1 << 30, 4);
    std::vector<int64_t> t;
    for (int g = 0; g < 4; g++) t.push_back(c.submit(g, 1, g));  // four independent SSSP queries
    for (auto x : t) {
        Req r;
        CHECK(c.wait(x, 5.0, r));
        c.collect(x);
    }
    CHECK(f.max_running.load() >= 2);
    std::puts("ok overlap");
}

// An executor that keeps one workspace per finished batch (like a pool):
// the core charges those idle bytes, trims them when a batch needs the room,
// and held bytes (running + results + idle) never pass the budget.
struct Pooling : Fake {
    std::mutex mu;
    size_t pooled = 0, held_peak = 0, running_bytes = 0;
    std::atomic<int> trims{0};
    size_t idle_bytes() override {
        std::lock_guard<std::mutex> lk(mu);
        return pooled;
    }
    void trim(size_t target) override {
        std::lock_guard<std::mutex> lk(mu);
        while (pooled > target && pooled >= work_per) pooled -= work_per;
        if (pooled > target) pooled = 0;
        trims++;
    }
    size_t outstanding = 0;  // results not yet released
    void run(int w, Batch &b) override {
        {
            std::lock_guard<std::mutex> lk(mu);
            // reuse a pooled workspace when there is one
            const size_t reuse = pooled >= work_per ? work_per : 0;
            pooled -= reuse;
            running_bytes += work_per * b.reqs.size();
            outstanding += result_per * b.reqs.size();
            held_peak = std::max(held_peak, running_bytes + pooled + outstanding);
        }
        Fake::run(w, b);
        std::lock_guard<std::mutex> lk(mu);
        running_bytes -= work_per * b.reqs.size();
        pooled += work_per * b.reqs.size();  // the workspace goes back to the pool
    }
    void release(Req &r) override {
        {
            std::lock_guard<std::mutex> lk(mu);
            outstanding -= result_per;
        }
        Fake::release(r);
    }
};

static void test_idle_bytes_charged_and_trimmed() {
    Pooling f;
    f.sleep_ms = 2;
    Core c(&f, 400, 3);  // 3 single queries of 110 fit; a pool of 300 idle bytes must be trimmed to admit more
    std::vector<int64_t> t;
    for (int i = 0; i < 40; i++) t.push_back(c.submit(i % 4, 1, i));  // SSSP: one per batch
    for (auto x : t) {
        Req r;
        CHECK(c.wait(x, 10.0, r));
        CHECK(r.status == 0);
        CHECK(c.collect(x));
    }
    const Stats s = c.stats();
    CHECK(s.bytes_peak <= 400);
    CHECK(f.held_peak <= 400);
    CHECK(s.trims > 0 && f.trims.load() > 0);
    CHECK(s.bytes_idle == f.idle_bytes());
    std::puts("ok idle bytes");
}

// Idle memory that cannot be trimmed (derived layouts) larger than what a
// query needs: the query fails with the admission status instead of waiting
// forever, at submission when the pinned bytes are known, else when nothing
// runs and nothing is charged.
struct Pinned : Fake {
    std::atomic<size_t> pinned{0};
    size_t idle_bytes() override { return pinned; }
    size_t pinned_bytes() override { return pinned; }
};

static void test_untrimmable_idle_bytes_fail_instead_of_hanging() {
    Pinned f;
    Core c(&f, 300, 2);
    f.pinned = 250;  // 110 per query no longer fits beside 250
    bool threw = false;
    try {
        c.submit(0, 1, 1);
    } catch (const AdmissionError &) {
        threw = true;
    }
    CHECK(threw);
    f.pinned = 0;
    int64_t a = c.submit(0, 1, 2);
    Req r;
    CHECK(c.wait(a, 5.0, r) && r.status == 0);
    CHECK(c.collect(a));
    // layouts that appear after submission: the queued queries fail, later ones run
    Pinned g;
    g.sleep_ms = 50;
    Core d(&g, 300, 1);
    int64_t q1 = d.submit(0, 1, 1);
    int64_t q2 = d.submit(0, 0, 2), q3 = d.submit(0, 0, 3);
    std::this_thread::sleep_for(std::chrono::milliseconds(10));
    g.pinned = 250;  // built while q1 runs
    CHECK(d.wait(q1, 5.0, r) && r.status == 0);
    CHECK(d.collect(q1));
    CHECK(d.wait(q2, 5.0, r) && r.status == kAdmissionStatus);
    CHECK(d.wait(q3, 5.0, r) && r.status == kAdmissionStatus);
    CHECK(d.collect(q2) && d.collect(q3));
    std::puts("ok pinned idle bytes");
}

int main() {
    test_admission();
    test_batching_and_results();
    test_budget_limits_batch_and_concurrency();
    test_uncollected_results_hold_memory();
    test_failed_query_frees_memory();
    test_concurrent_workers_overlap();
    test_idle_bytes_charged_and_trimmed();
    test_untrimmable_idle_bytes_fail_instead_of_hanging();
    std::puts("ALL OK");
    return 0;
}
