// Host-only tests of the continuous-batching scheduler with a mock executor
// (no GPU): arena allocation, FIFO admission by memory, continuous batching,
// in-flight limits, cancellation, timeouts, executor failure, shutdown, and a
// multi-threaded stress run.  Built and run by tests/test_serving_cpu.py
// under ThreadSanitizer and under AddressSanitizer/UBSan.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "ak_sched.h"

using namespace ak;

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

// Mock executor: each launch records its batch; wait() blocks until the test
// opens that batch's gate (or returns at once in auto mode).
struct MockExec {
    // slots like the GPU executor's: launch takes a free one (a null token if
    // none is free, which fails the batch), release frees it
    int nslots = 1 << 30;
    int used_slots = 0;
    struct Tok {
        std::vector<int> ids;
        bool open = false;
        int rc = 0;
    };
    std::mutex mu;
    std::condition_variable cv;
    std::vector<std::shared_ptr<Tok>> toks;
    std::atomic<int> outstanding{0}, max_outstanding{0};
    bool autoc = false;
    int fail_batch = -1;
    std::mt19937 rng{1};

    void *launch(const std::vector<Request *> &b)
    {
        auto t = std::make_shared<Tok>();
        for (Request *r : b) t->ids.push_back((int)r->n);
        std::lock_guard<std::mutex> g(mu);
        if (used_slots == nslots) return nullptr;
        ++used_slots;
        if ((int)toks.size() == fail_batch) t->rc = -2;
        toks.push_back(t);
        const int o = ++outstanding;
        int m = max_outstanding.load();
        while (o > m && !max_outstanding.compare_exchange_weak(m, o)) {
        }
        cv.notify_all();
        return t.get();
    }
    // request i of a batch; the batch counts as outstanding until its last
    // request has been waited for
    int wait(void *p, size_t i, std::string *err)
    {
        if (!p) {
            *err = "no slot";
            return -2;
        }
        Tok *t = (Tok *)p;
        std::unique_lock<std::mutex> l(mu);
        if (autoc) {
            l.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
            l.lock();
        } else {
            cv.wait(l, [t] { return t->open; });
        }
        if (i + 1 == t->ids.size()) --outstanding;
        if (t->rc) *err = "mock batch failure";
        return t->rc;
    }
    void release(void *p)
    {
        std::lock_guard<std::mutex> g(mu);
        if (p) --used_slots;
    }
    int64_t launches(void *) { return 1; }
    void open(size_t i)
    {
        std::lock_guard<std::mutex> g(mu);
        toks.at(i)->open = true;
        cv.notify_all();
    }
    size_t nbatches()
    {
        std::lock_guard<std::mutex> g(mu);
        return toks.size();
    }
    std::vector<int> batch(size_t i)
    {
        std::lock_guard<std::mutex> g(mu);
        return toks.at(i)->ids;
    }
    void wait_batches(size_t n)
    {
        std::unique_lock<std::mutex> l(mu);
        cv.wait_until(l, std::chrono::system_clock::now() + std::chrono::seconds(10),
                      [&] { return toks.size() >= n; });
        CHECK(toks.size() >= n);
    }
};

// request whose n is its id (unique per test) and whose size is `bytes`
static std::unique_ptr<Request> req(int id, size_t bytes)
{
    std::unique_ptr<Request> r(new Request());
    r->n = id;
    r->bytes = bytes;
    return r;
}

static void settle() { std::this_thread::sleep_for(std::chrono::milliseconds(30)); }

static void test_arena()
{
    Arena a(1000 * 256);
    CHECK(a.capacity() == 256000);
    const size_t x = a.alloc(100), y = a.alloc(300), z = a.alloc(256);
    CHECK(x == 0 && y == 256 && z == 768);
    CHECK(a.used() == 1024);
    a.release(y, 300);
    CHECK(a.alloc(600) == 1024);             // hole of 512 too small: first fit after z
    const size_t w = a.alloc(512);
    CHECK(w == 256);                         // reuses the hole exactly
    a.release(x, 100);
    a.release(w, 512);
    a.release(z, 256);
    a.release(1024, 600);
    CHECK(a.used() == 0 && a.ranges() == 1);  // everything coalesced
    CHECK(a.alloc(256000) == 0);
    CHECK(a.alloc(1) == SIZE_MAX);
}

static void test_continuous_batching()
{
    MockExec ex;
    SchedConfig c;
    c.arena_bytes = 1 << 20;
    c.max_inflight = 1;
    Scheduler<MockExec> s(c, &ex);
    auto r0 = req(100, 1000);
    CHECK(s.submit(r0.get()) == 0);
    ex.wait_batches(1);
    std::vector<std::unique_ptr<Request>> rs;
    for (int i = 1; i <= 4; ++i) {
        rs.push_back(req(100 + i, 1000));
        CHECK(s.submit(rs.back().get()) == 0);
    }
    settle();
    CHECK(ex.nbatches() == 1);               // slot busy: the four wait
    CHECK(s.queue_depth() == 4);
    ex.open(0);
    ex.wait_batches(2);
    auto b1 = ex.batch(1);
    CHECK(b1.size() == 4 && b1[0] == 101 && b1[3] == 104);   // admitted together, FIFO
    ex.open(1);
    for (auto &r : rs) CHECK(Scheduler<MockExec>::wait(r.get(), 5.0) == 0);
    CHECK(Scheduler<MockExec>::wait(r0.get(), 5.0) == 0);
    auto st = s.stats();
    CHECK(st.completed == 5 && st.batches == 2 && st.latency.size() == 5);
    CHECK(s.arena_used() == 0);
}

static void test_admission_by_memory_fifo()
{
    MockExec ex;
    SchedConfig c;
    c.arena_bytes = 10 * 256;
    c.max_inflight = 3;
    Scheduler<MockExec> s(c, &ex);
    auto a = req(1, 6 * 256), b = req(2, 6 * 256), d = req(3, 2 * 256);
    CHECK(s.submit(a.get()) == 0);
    ex.wait_batches(1);
    CHECK(s.submit(b.get()) == 0);
    CHECK(s.submit(d.get()) == 0);
    settle();
    CHECK(ex.nbatches() == 1);               // b does not fit; d must not overtake b
    CHECK(s.queue_depth() == 2);
    ex.open(0);
    ex.wait_batches(2);
    auto b1 = ex.batch(1);
    CHECK(b1.size() == 2 && b1[0] == 2 && b1[1] == 3);
    ex.open(1);
    CHECK(Scheduler<MockExec>::wait(d.get(), 5.0) == 0);
    auto big = req(9, 11 * 256);
    CHECK(s.submit(big.get()) == -4);        // larger than the arena
}

static void test_large_requests_run_alone()
{
    MockExec ex;
    SchedConfig c;
    c.arena_bytes = 1 << 20;
    c.max_inflight = 1;
    c.small_cells = 100;
    Scheduler<MockExec> s(c, &ex);
    auto g = req(1, 256);                     // occupies the only slot
    CHECK(s.submit(g.get()) == 0);
    ex.wait_batches(1);
    auto a = req(11, 256), big = req(500, 256), b = req(12, 256), d = req(13, 256);
    for (Request *r : {a.get(), big.get(), b.get(), d.get()}) CHECK(s.submit(r) == 0);
    settle();
    ex.open(0);
    ex.wait_batches(2);
    CHECK(ex.batch(1).size() == 1 && ex.batch(1)[0] == 11);   // stops before the large one
    ex.open(1);
    ex.wait_batches(3);
    CHECK(ex.batch(2).size() == 1 && ex.batch(2)[0] == 500);  // the large one alone
    ex.open(2);
    ex.wait_batches(4);
    auto b3 = ex.batch(3);
    CHECK(b3.size() == 2 && b3[0] == 12 && b3[1] == 13);      // small ones fused again
    ex.open(3);
    for (Request *r : {a.get(), big.get(), b.get(), d.get()})
        CHECK(Scheduler<MockExec>::wait(r, 5.0) == 0);
    CHECK(s.arena_used() == 0);
}

static void test_inflight_limit_one_launch_per_request()
{
    MockExec ex;
    ex.autoc = true;
    SchedConfig c;
    c.arena_bytes = 1 << 20;
    c.max_inflight = 2;
    c.batching = false;
    Scheduler<MockExec> s(c, &ex);
    std::vector<std::unique_ptr<Request>> rs;
    for (int i = 0; i < 40; ++i) {
        rs.push_back(req(i + 1, 512));
        CHECK(s.submit(rs.back().get()) == 0);
    }
    for (auto &r : rs) CHECK(Scheduler<MockExec>::wait(r.get(), 10.0) == 0);
    CHECK(ex.nbatches() == 40);              // one request per batch
    CHECK(ex.max_outstanding.load() <= 2);
}

static void test_cancel_timeout_failure()
{
    MockExec ex;
    ex.fail_batch = 0;
    SchedConfig c;
    c.arena_bytes = 1 << 20;
    c.max_inflight = 1;
    Scheduler<MockExec> s(c, &ex);
    auto a = req(1, 256), b = req(2, 256), d = req(3, 256);
    CHECK(s.submit(a.get()) == 0);
    ex.wait_batches(1);
    CHECK(s.submit(b.get()) == 0);
    CHECK(s.submit(d.get()) == 0);
    CHECK(Scheduler<MockExec>::wait(a.get(), 0.05) == -5);   // gated: times out
    CHECK(s.cancel(b.get()) == 0);                          // still queued
    CHECK(Scheduler<MockExec>::wait(b.get(), 1.0) == -6);
    CHECK(s.cancel(a.get()) == 1);                          // already on the device
    ex.open(0);                                             // batch 0 fails
    CHECK(Scheduler<MockExec>::wait(a.get(), 5.0) == -2);
    ex.wait_batches(2);
    ex.open(1);                                             // the server keeps serving
    CHECK(Scheduler<MockExec>::wait(d.get(), 5.0) == 0);
    auto st = s.stats();
    CHECK(st.failed == 1 && st.cancelled == 1 && st.completed == 1);
    // the failure's text travels with the request
    std::lock_guard<std::mutex> l(a->mu);
    CHECK(a->error == "mock batch failure");
}

// A failed request's error stays readable after its scheduler and executor
// are gone (the text is copied into the request at completion).
static void test_error_outlives_server()
{
    auto a = req(1, 256);
    {
        auto ex = std::make_unique<MockExec>();
        ex->fail_batch = 0;
        ex->autoc = true;
        SchedConfig c;
        c.arena_bytes = 1 << 20;
        auto s = std::make_unique<Scheduler<MockExec>>(c, ex.get());
        CHECK(s->submit(a.get()) == 0);
        CHECK(Scheduler<MockExec>::wait(a.get(), 5.0) == -2);
        s->shutdown();
        s.reset();
        ex.reset();
    }
    std::lock_guard<std::mutex> l(a->mu);
    CHECK(a->state == kFailed && a->error == "mock batch failure");
}

static void test_shutdown()
{
    MockExec ex;
    SchedConfig c;
    c.arena_bytes = 1 << 20;
    c.max_inflight = 1;
    auto s = std::make_unique<Scheduler<MockExec>>(c, &ex);
    auto a = req(1, 256), b = req(2, 256);
    CHECK(s->submit(a.get()) == 0);
    ex.wait_batches(1);
    CHECK(s->submit(b.get()) == 0);
    std::thread opener([&] {
        std::this_thread::sleep_for(std::chrono::milliseconds(50));
        ex.open(0);
    });
    s->shutdown();                           // b cancelled, a drained
    opener.join();
    CHECK(Scheduler<MockExec>::wait(a.get(), 1.0) == 0);
    CHECK(Scheduler<MockExec>::wait(b.get(), 1.0) == -6);
    auto c2 = req(3, 256);
    CHECK(s->submit(c2.get()) == -1);
}

static void test_stress()
{
    MockExec ex;
    ex.autoc = true;
    ex.nslots = 3;                 // exactly max_inflight slots, as on the GPU
    SchedConfig c;
    c.arena_bytes = 64 * 1024;
    c.max_inflight = 3;
    c.max_batch_requests = 16;
    Scheduler<MockExec> s(c, &ex);
    const int nthreads = 8, per = 200;
    std::vector<std::thread> th;
    std::atomic<int> done{0};
    for (int t = 0; t < nthreads; ++t) {
        th.emplace_back([&, t] {
            std::mt19937 rng(t + 7);
            for (int i = 0; i < per; ++i) {
                auto r = req(1000 * (t + 1) + i, 256 * (1 + rng() % 64));
                CHECK(s.submit(r.get()) == 0);
                CHECK(Scheduler<MockExec>::wait(r.get(), 30.0) == 0);
                done++;
            }
        });
    }
    for (auto &x : th) x.join();
    CHECK(done == nthreads * per);
    auto st = s.stats();
    CHECK(st.completed == nthreads * per && st.latency.size() == (size_t)(nthreads * per));
    CHECK(s.arena_used() == 0);
    CHECK(ex.max_outstanding.load() <= 3);
    CHECK(percentile({1, 2, 3, 4, 5}, 50) == 3.0);
    CHECK(percentile({1, 2}, 100) == 2.0);
}

int main()
{
    test_error_outlives_server();
    test_arena();
    test_continuous_batching();
    test_admission_by_memory_fifo();
    test_large_requests_run_alone();
    test_inflight_limit_one_launch_per_request();
    test_cancel_timeout_failure();
    test_shutdown();
    test_stress();
    std::printf("OK\n");
    return 0;
}
