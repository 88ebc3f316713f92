// Continuous-batching request scheduler (host only, no HIP dependency).
//
// Requests enter a FIFO queue.  A batcher thread admits queued requests in
// order while (a) fewer than max_inflight batches are on the device, (b) the
// head request's bytes fit in the device arena (first-fit allocator), and
// (c) the batch limits allow: requests of more than small_cells cells run
// alone (their copies dwarf a launch, so fusing them would only delay the
// others), smaller ones are fused up to max_batch_requests and
// max_batch_cells.  The executor enqueues copies in, one fused launch per
// precision and copies out, and returns at once.  A completion thread waits
// for batches in submission order and, within a batch, for each request's
// own copy-out, then frees that request's arena range and completes it, which
// lets the batcher admit more.  Requests therefore join the device while
// earlier batches are still running (continuous batching).
//
// Executor interface (duck-typed):
//   void *launch(const std::vector<Request*> &batch);  // enqueue; returns a token
//   int   wait(void *token, size_t i);                 // block until request i's
//                                                      // result is out; 0 or error
//   void  release(void *token);
//   int64_t launches(void *token);
#pragma once
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace ak {

// First-fit allocator over [0, capacity) with 256-byte granules.
class Arena {
  public:
    explicit Arena(size_t cap = 0) { reset(cap); }
    void reset(size_t cap)
    {
        cap_ = cap & ~(size_t)255;
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = 0;
    }
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    // offset, or SIZE_MAX if no free range is large enough
    size_t alloc(size_t bytes)
    {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t ranges() const { return free_.size(); }

  private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

enum ReqState { kQueued = 0, kAdmitted = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Request {
    // what to compute (opaque to the scheduler)
    const void *mech = nullptr;
    int prec = 0;
    int ns = 0;
    const void *T = nullptr, *P = nullptr, *Y = nullptr;
    void *om = nullptr;
    int64_t ldY = 0, ldO = 0, n = 0;
    size_t bytes = 0;          // arena bytes
    size_t arena_off = SIZE_MAX;
    // state
    int state = kQueued;
    int rc = 0;
    std::string error;         // why the request failed (set with state, under mu)
    double t_submit = 0, t_done = 0;
    std::mutex mu;
    std::condition_variable cv;
};

inline double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SchedConfig {
    size_t arena_bytes = (size_t)1 << 30;
    int max_inflight = 3;
    int max_batch_requests = 64;
    int64_t max_batch_cells = (int64_t)1 << 16;
    int64_t small_cells = 4096;   // larger requests are never fused
    bool batching = true;     // false: one request per batch (one launch per request)
};

struct SchedStats {
    int64_t submitted = 0, completed = 0, cancelled = 0, failed = 0, launches = 0, batches = 0;
    int64_t cells = 0;
    double first_submit = 0, last_done = 0;
    std::vector<double> latency;   // seconds, completed requests
};

template <class Exec>
class Scheduler {
  public:
    Scheduler(const SchedConfig &c, Exec *exec) : cfg_(c), exec_(exec), arena_(c.arena_bytes)
    {
        batcher_ = std::thread([this] { batch_loop(); });
        completer_ = std::thread([this] { complete_loop(); });
    }
    ~Scheduler() { shutdown(); }

    // 0, or AK-style negative code (-4 too big for the arena)
    int submit(Request *r)
    {
        if (Arena::round(r->bytes) > arena_.capacity()) return -4;
        std::lock_guard<std::mutex> g(mu_);
        if (stop_) return -1;
        r->state = kQueued;
        r->t_submit = now_s();
        if (stats_.submitted == 0) stats_.first_submit = r->t_submit;
        stats_.submitted++;
        queue_.push_back(r);
        cv_.notify_all();
        return 0;
    }

    // 0 if cancelled; 1 if it was already admitted (too late)
    int cancel(Request *r)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = std::find(queue_.begin(), queue_.end(), r);
        if (it == queue_.end()) return 1;
        queue_.erase(it);
        stats_.cancelled++;
        finish(r, kCancelled, -6);
        return 0;
    }

    // 0 done, or the request's error, or -5 on timeout (timeout < 0: forever)
    static int wait(Request *r, double timeout_s)
    {
        std::unique_lock<std::mutex> l(r->mu);
        auto done = [r] { return r->state >= kDone; };
        if (timeout_s < 0) {
            r->cv.wait(l, done);
        } else {
            // system_clock deadline: a timed wait that thread sanitizers follow
            const auto deadline = std::chrono::system_clock::now() +
                                  std::chrono::duration_cast<std::chrono::system_clock::duration>(
                                      std::chrono::duration<double>(timeout_s));
            if (!r->cv.wait_until(l, deadline, done)) return -5;
        }
        return r->state == kDone ? 0 : r->rc;
    }

    void shutdown()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (stop_) return;
            stop_ = true;
            // queued requests are cancelled; admitted ones drain
            for (Request *r : queue_) {
                stats_.cancelled++;
                finish(r, kCancelled, -6);
            }
            queue_.clear();
            cv_.notify_all();
        }
        if (batcher_.joinable()) batcher_.join();
        {
            std::lock_guard<std::mutex> g(mu_);
            batcher_done_ = true;
            cv_.notify_all();
        }
        if (completer_.joinable()) completer_.join();
    }

    SchedStats stats()
    {
        std::lock_guard<std::mutex> g(mu_);
        return stats_;
    }
    void reset_stats()
    {
        std::lock_guard<std::mutex> g(mu_);
        stats_ = SchedStats{};
    }
    size_t queue_depth()
    {
        std::lock_guard<std::mutex> g(mu_);
        return queue_.size();
    }
    int inflight()
    {
        std::lock_guard<std::mutex> g(mu_);
        return (int)inflight_.size();
    }
    size_t arena_used()
    {
        std::lock_guard<std::mutex> g(mu_);
        return arena_.used();
    }
    size_t arena_capacity() const { return arena_.capacity(); }

  private:
    struct Batch {
        std::vector<Request *> reqs;
        void *token = nullptr;
    };

    static void finish(Request *r, int state, int rc, std::string err = std::string())
    {
        std::lock_guard<std::mutex> l(r->mu);
        r->state = state;
        r->rc = rc;
        r->error = std::move(err);
        r->t_done = now_s();
        r->cv.notify_all();
    }

    void batch_loop()
    {
        std::unique_lock<std::mutex> l(mu_);
        for (;;) {
            cv_.wait(l, [this] {
                return stop_ || (!queue_.empty() && (int)inflight_.size() < cfg_.max_inflight);
            });
            if (stop_) return;
            Batch b;
            int64_t cells = 0;
            while (!queue_.empty() && (int)b.reqs.size() < cfg_.max_batch_requests) {
                Request *r = queue_.front();
                const bool big = r->n > cfg_.small_cells;
                if (!b.reqs.empty() &&
                    (!cfg_.batching || big || cells + r->n > cfg_.max_batch_cells))
                    break;
                const size_t off = arena_.alloc(r->bytes);
                if (off == SIZE_MAX) break;   // head of line waits for memory
                r->arena_off = off;
                {
                    std::lock_guard<std::mutex> rl(r->mu);
                    r->state = kAdmitted;
                }
                queue_.pop_front();
                b.reqs.push_back(r);
                cells += r->n;
                if (!cfg_.batching || big) break;
            }
            if (b.reqs.empty()) {
                // nothing fits until a batch completes
                cv_.wait(l, [this] { return stop_ || arena_freed_; });
                arena_freed_ = false;
                continue;
            }
            l.unlock();
            b.token = exec_->launch(b.reqs);
            l.lock();
            stats_.batches++;
            inflight_.push_back(std::move(b));
            cv_.notify_all();
        }
    }

    void complete_loop()
    {
        std::unique_lock<std::mutex> l(mu_);
        for (;;) {
            cv_.wait(l, [this] { return !inflight_.empty() || (stop_ && batcher_done_); });
            if (inflight_.empty()) return;
            Batch b = inflight_.front();
            for (size_t i = 0; i < b.reqs.size(); ++i) {
                l.unlock();
                std::string err;
                const int rc = exec_->wait(b.token, i, &err);
                l.lock();
                Request *r = b.reqs[i];
                arena_.release(r->arena_off, r->bytes);
                r->arena_off = SIZE_MAX;
                arena_freed_ = true;
                const double t = now_s();
                if (rc == 0) {
                    stats_.completed++;
                    stats_.cells += r->n;
                    stats_.latency.push_back(t - r->t_submit);
                    stats_.last_done = t;
                } else {
                    stats_.failed++;
                }
                finish(r, rc == 0 ? kDone : kFailed, rc, std::move(err));
                cv_.notify_all();
            }
            // the executor's slot is free before the batch leaves inflight_, so
            // a batch the batcher admits next always finds a slot (the
            // executor's lock is never held while taking this one)
            stats_.launches += exec_launches(b.token);
            exec_->release(b.token);
            inflight_.pop_front();
            cv_.notify_all();
        }
    }

    int64_t exec_launches(void *token) { return exec_->launches(token); }

    SchedConfig cfg_;
    Exec *exec_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Request *> queue_;
    std::deque<Batch> inflight_;
    bool stop_ = false, batcher_done_ = false, arena_freed_ = false;
    SchedStats stats_;
    std::thread batcher_, completer_;
};

// p-th percentile (0..100) of a sample, linear interpolation
inline double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double x = p / 100.0 * (double)(v.size() - 1);
    const size_t i = (size_t)x;
    const double f = x - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace ak
