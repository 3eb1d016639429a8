// Concurrency test of the served scheduler's threads (fsa_sched.hpp:
// Scheduler + Runner) with a fake device, built with ThreadSanitizer.
//
// The fake device runs each queue's requests in launch order, each taking a
// scripted service time on the host clock, and wakes the waiter of that
// queue when the oldest one has finished.  Client threads submit requests of
// several sizes under a budget that forces admission waits and evictions,
// poll, wait with and without timeouts, and cancel; a burst runs under a
// queue timeout shorter than its backlog; then the server shuts down with
// work in flight.  Checks: every request ends OK, cancelled or timed out,
// each exactly once; no request runs before its tensor is built; the budget
// is never exceeded; the statistics add up.  Exit status 0 = all passed.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_2504_19410_amd/csrc/fsa_sched.hpp"

using namespace fsa::sched;
using Clock = std::chrono::steady_clock;

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);  \
            ++g_fail;                                                 \
        }                                                             \
    } while (0)

static double now_s() {
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct FakeDevice : Backend, CompletionSource {
    struct Plan {
        int id;
        bool built = false;
        bool destroyed = false;
    };
    struct Job {
        uint64_t ticket;
        double t_done;
    };
    struct Queue {
        std::mutex mu;
        std::condition_variable cv;
        std::deque<Job> fifo;
        double busy_until = 0;
    };

    explicit FakeDevice(int nq) : queues(nq) {}
    std::mutex mu;  // plans and counters
    std::map<void*, Plan*> plans;
    std::vector<Queue> queues;
    std::atomic<bool> stopped{false};
    std::atomic<int> launched{0}, built{0}, completed{0};
    int next_id = 0;

    double now() override { return now_s(); }
    Status create_plan(const Key& k, PlanInfo* out, std::string*) override {
        std::lock_guard<std::mutex> lk(mu);
        Plan* p = new Plan{++next_id};
        plans[p] = p;
        out->handle = p;
        out->tensor_bytes = (size_t)k.N[0] * 1000;
        out->workspace_bytes = (size_t)k.N[1] * 1000;
        return ST_OK;
    }
    Status build_plan(const PlanInfo& pi, std::string*) override {
        std::lock_guard<std::mutex> lk(mu);
        Plan* p = (Plan*)pi.handle;
        CHECK(!p->destroyed && !p->built);
        p->built = true;
        ++built;
        return ST_OK;
    }
    void destroy_plan(const PlanInfo& pi) override {
        std::lock_guard<std::mutex> lk(mu);
        Plan* p = (Plan*)pi.handle;
        CHECK(!p->destroyed);
        p->destroyed = true;  // kept allocated, so use after destroy is caught above
    }
    Status launch(const Request& r, const PlanInfo& pi, int slot, std::string*) override {
        {
            std::lock_guard<std::mutex> lk(mu);
            Plan* p = (Plan*)pi.handle;
            CHECK(p->built && !p->destroyed);
        }
        Queue& q = queues[(size_t)slot % queues.size()];
        const double service = 20e-6 * (double)(1 + r.key.N[1] % 4);
        {
            std::lock_guard<std::mutex> lk(q.mu);
            q.busy_until = std::max(q.busy_until, now_s()) + service;
            q.fifo.push_back(Job{r.ticket, q.busy_until});
        }
        q.cv.notify_one();
        ++launched;
        return ST_OK;
    }
    int n_queues() const override { return (int)queues.size(); }
    bool wait_next(int qi, Completion* out) override {
        Queue& q = queues[(size_t)qi];
        Job j;
        {
            std::unique_lock<std::mutex> lk(q.mu);
            q.cv.wait(lk, [&] { return !q.fifo.empty() || stopped.load(); });
            if (q.fifo.empty()) return false;
            j = q.fifo.front();
            q.fifo.pop_front();
        }
        const double wait = j.t_done - now_s();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        out->ticket = j.ticket;
        out->status = ST_OK;
        out->t_done = now_s();
        ++completed;
        return true;
    }
    void stop() override {
        stopped.store(true);
        for (Queue& q : queues) {
            std::lock_guard<std::mutex> lk(q.mu);
            q.cv.notify_all();
        }
    }
    ~FakeDevice() override {
        for (auto& kv : plans) delete kv.second;
    }
};

static Key key_of(int i) {
    Key k;
    k.kind = 1 + i % 3;
    k.d = 2;
    k.N[0] = 1 + i % 5;  // tensor 1000 .. 5000 bytes
    k.N[1] = 1 + i % 4;  // workspace 1000 .. 4000 bytes
    k.L[0] = k.L[1] = 1.0 + (i % 7);
    return k;
}

int main() {
    const size_t budget = 30000;
    FakeDevice dev(3);
    Scheduler sched(&dev, budget, 4);
    std::atomic<size_t> peak_seen{0};
    std::vector<std::vector<uint64_t>> tickets(8);
    std::vector<std::vector<int>> cancelled(8);
    {
        Runner run(&sched, &dev);
        std::vector<std::thread> clients;
        for (int c = 0; c < 8; ++c) {
            clients.emplace_back([&, c] {
                std::mt19937 rng(1234 + c);
                for (int i = 0; i < 150; ++i) {
                    uint64_t t = 0;
                    std::string err;
                    const Status st = run.submit(key_of((int)(rng() % 40)), &dev, &dev, &t, &err,
                                                 (rng() % 2) ? now_s() - 1e-4 : -1.0);
                    CHECK(st == ST_OK);
                    tickets[c].push_back(t);
                    bool done = false;
                    Status res = ST_OK;
                    switch (rng() % 5) {
                    case 0:
                        CHECK(run.wait(t, -1.0, &done, &res) == ST_OK);
                        CHECK(done && res == ST_OK);
                        break;
                    case 1:
                        CHECK(run.wait(t, 1e-5, &done, &res) == ST_OK);
                        break;
                    case 2:
                        if (sched.cancel(t) == ST_OK) cancelled[c].push_back(1);
                        break;
                    default:
                        CHECK(sched.poll(t, &done, &res) == ST_OK);
                    }
                    const Stats s = sched.stats();
                    CHECK(s.hbm_in_use <= budget);
                    size_t p = peak_seen.load();
                    while (s.hbm_peak > p && !peak_seen.compare_exchange_weak(p, s.hbm_peak)) {}
                }
            });
        }
        for (auto& t : clients) t.join();
        // wait for everything that was not cancelled, then stop with nothing
        // in flight; a second phase stops with requests still running
        for (int c = 0; c < 8; ++c)
            for (uint64_t t : tickets[c]) {
                bool done = false;
                Status res = ST_OK;
                CHECK(run.wait(t, 10.0, &done, &res) == ST_OK);
                CHECK(done && (res == ST_OK || res == ST_ECANCELLED));
            }
        // a queue timeout shorter than the backlog: submitters on several
        // threads, every request ends OK or timed out, each exactly once
        sched.set_queue_timeout(2e-4);
        std::vector<std::vector<uint64_t>> late(4);
        std::vector<std::thread> bursts;
        for (int c = 0; c < 4; ++c)
            bursts.emplace_back([&, c] {
                for (int i = 0; i < 30; ++i) {
                    uint64_t t = 0;
                    std::string err;
                    CHECK(run.submit(key_of(i + c), &dev, &dev, &t, &err) == ST_OK);
                    late[c].push_back(t);
                }
                for (uint64_t t : late[c]) {
                    bool done = false;
                    Status res = ST_OK;
                    CHECK(run.wait(t, 10.0, &done, &res) == ST_OK);
                    CHECK(done && (res == ST_OK || res == ST_ETIMEDOUT));
                }
            });
        for (auto& t : bursts) t.join();
        sched.set_queue_timeout(0);
        for (int i = 0; i < 40; ++i) {
            uint64_t t = 0;
            std::string err;
            CHECK(run.submit(key_of(i), &dev, &dev, &t, &err) == ST_OK);
        }
        run.shutdown();  // cancels the queue, lets in-flight requests finish
    }
    const Stats s = sched.stats();
    size_t n_cancel = 0;
    for (auto& v : cancelled) n_cancel += v.size();
    CHECK(s.done == (uint64_t)dev.completed.load());
    CHECK(dev.launched.load() == dev.completed.load());
    CHECK(s.done + s.cancelled + s.timed_out >= 8 * 150 + 4 * 30);
    CHECK(s.cancelled >= n_cancel);
    CHECK(s.hbm_peak <= budget && peak_seen.load() <= budget);
    CHECK(s.cache_misses == (uint64_t)dev.built.load());
    CHECK(s.p50_ms > 0 && s.p99_ms >= s.p50_ms);
    CHECK(s.timed_out > 0);  // the burst outran its queue timeout
    std::printf("%s (%d failures): %llu done, %llu cancelled, %llu timed out, %d builds, "
                "peak %zu of %zu\n",
                g_fail.load() ? "FAILED" : "OK", g_fail.load(), (unsigned long long)s.done,
                (unsigned long long)s.cancelled, (unsigned long long)s.timed_out, dev.built.load(),
                s.hbm_peak, budget);
    return g_fail.load() ? 1 : 0;
}
