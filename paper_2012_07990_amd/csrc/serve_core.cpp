// Serving core (see serve_core.hpp): admission and continuous batching.
// Plain C++ with no device code, so the policy is tested on a CPU with a
// fake executor.
#include "serve_core.hpp"

#include <algorithm>

namespace gg {
namespace serve {

static double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

Core::Core(Executor *ex, size_t budget, int workers) : ex_(ex), budget_(budget) {
    if (workers < 1) workers = 1;
    for (int i = 0; i < workers; i++) threads_.emplace_back([this, i] { worker(i); });
}

Core::~Core() { shutdown(); }

void Core::shutdown() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    for (auto &t : threads_)
        if (t.joinable()) t.join();
    threads_.clear();
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : reqs_) {
        Req &r = *kv.second;
        if (r.done && r.result) ex_->release(r);
    }
    reqs_.clear();
    pending_.clear();
}

int64_t Core::submit(int gid, int algo, int src) {
    const size_t one = ex_->work_bytes(gid, algo, 1) + ex_->result_bytes(gid, algo);
    std::lock_guard<std::mutex> lk(mu_);
    const size_t pinned = ex_->pinned_bytes();
    if (one > budget_ || pinned > budget_ - one) {
        st_.rejected++;
        throw AdmissionError("query footprint " + std::to_string(one) + " B plus " + std::to_string(pinned) +
                             " B of derived layouts exceeds the serving budget " + std::to_string(budget_) + " B");
    }
    auto r = std::make_unique<Req>();
    r->ticket = next_ticket_++;
    r->gid = gid;
    r->algo = algo;
    r->src = src;
    r->t_arrive = Clock::now();
    r->result_bytes = ex_->result_bytes(gid, algo);
    pending_.push_back(r.get());
    const int64_t t = r->ticket;
    reqs_[t] = std::move(r);
    st_.submitted++;
    cv_work_.notify_one();
    return t;
}

// Oldest pending query first; then every pending query of the same graph and
// algorithm, up to the batch limit and the memory that is free now.
bool Core::form_batch(Batch &b) {
    while (!pending_.empty()) {
        if (try_batch(b)) return true;
        if (running_ != 0 || in_use_ != 0) return false;  // wait for memory
        // nothing can free memory any more: the head query can never run
        Req *head = pending_.front();
        pending_.pop_front();
        head->status = kAdmissionStatus;
        head->result_bytes = 0;
        head->t_start = head->t_done = Clock::now();
        head->done = true;
        st_.rejected++;
        cv_done_.notify_all();
    }
    return false;
}

bool Core::try_batch(Batch &b) {
    Req *head = pending_.front();
    const int lim = std::max(1, ex_->max_batch(head->gid, head->algo));
    const size_t free_bytes = budget_ > in_use_ ? budget_ - in_use_ : 0;
    std::vector<Req *> pick{head};
    for (auto it = pending_.begin() + 1; it != pending_.end() && (int)pick.size() < lim; ++it)
        if ((*it)->gid == head->gid && (*it)->algo == head->algo) pick.push_back(*it);
    // shrink until the batch (work + results) fits beside the idle bytes,
    // trimming idle memory that is in the way
    size_t idle = ex_->idle_bytes();
    while (!pick.empty()) {
        const size_t need = ex_->work_bytes(head->gid, head->algo, (int)pick.size()) + pick.size() * head->result_bytes;
        if (need <= free_bytes && idle > free_bytes - need) {
            ex_->trim(free_bytes - need);
            idle = ex_->idle_bytes();
            st_.trims++;
        }
        if (need <= free_bytes && idle <= free_bytes - need) {
            b.gid = head->gid;
            b.algo = head->algo;
            b.reqs = pick;
            b.work_bytes = ex_->work_bytes(head->gid, head->algo, (int)pick.size());
            in_use_ += need;
            running_++;
            st_.bytes_peak = std::max(st_.bytes_peak, in_use_ + idle);
            for (Req *r : pick) pending_.erase(std::find(pending_.begin(), pending_.end(), r));
            return true;
        }
        pick.pop_back();
    }
    return false;  // not even one query fits
}

void Core::worker(int id) {
    for (;;) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(mu_);
            // pending work is still drained while stopping
            cv_work_.wait(lk, [&] { return form_batch(b) || stop_; });
            if (b.reqs.empty()) return;
        }
        const auto t0 = Clock::now();
        for (Req *r : b.reqs) {
            r->t_start = t0;
            r->batch_size = (int)b.reqs.size();
        }
        ex_->run(id, b);
        const auto t1 = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu_);
            in_use_ -= b.work_bytes;
            running_--;
            for (Req *r : b.reqs) {
                r->t_done = t1;
                r->done = true;
                if (r->status != 0) {  // failed queries keep no result
                    in_use_ -= r->result_bytes;
                    r->result_bytes = 0;
                }
            }
            st_.completed += (int64_t)b.reqs.size();
            st_.batches++;
            st_.max_batch_seen = std::max<int32_t>(st_.max_batch_seen, (int32_t)b.reqs.size());
            st_.busy_ms += ms_between(t0, t1);
        }
        cv_done_.notify_all();
        cv_work_.notify_all();  // memory freed / more work may fit
    }
}

bool Core::peek(int64_t ticket, Req &out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end() || !it->second->done) return false;
    out = *it->second;
    return true;
}

bool Core::wait(int64_t ticket, double timeout_s, Req &out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto ready = [&] {
        auto it = reqs_.find(ticket);
        return it == reqs_.end() || it->second->done;
    };
    if (timeout_s < 0) {
        cv_done_.wait(lk, ready);
    } else {
        // system-clock deadline: waits through pthread_cond_timedwait
        const auto deadline = std::chrono::system_clock::now() +
                              std::chrono::duration_cast<std::chrono::system_clock::duration>(
                                  std::chrono::duration<double>(timeout_s));
        if (!cv_done_.wait_until(lk, deadline, ready)) return false;
    }
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return false;
    out = *it->second;
    return true;
}

bool Core::collect(int64_t ticket) {
    std::unique_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end() || !it->second->done) return false;
        r = std::move(it->second);
        reqs_.erase(it);
        in_use_ -= r->result_bytes;
        st_.collected++;
    }
    if (r->result) ex_->release(*r);
    cv_work_.notify_all();
    return true;
}

bool Core::known(int64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    return reqs_.count(ticket) != 0;
}

Stats Core::stats() {
    std::lock_guard<std::mutex> lk(mu_);
    Stats s = st_;
    s.bytes_in_use = in_use_;
    s.bytes_idle = ex_->idle_bytes();
    return s;
}

}  // namespace serve
}  // namespace gg
