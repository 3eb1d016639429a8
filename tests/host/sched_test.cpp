// Host-only tests of the server's scheduling core (fsa_sched.hpp) with a
// scripted backend and a virtual clock: admission order and HBM budget,
// continuous admission as completions free resources, rejection of requests
// that can never fit, cancellation, queue timeouts, the tensor cache (hits,
// misses, LRU eviction), failure isolation, slot limits and latency
// percentiles.
// Exit status 0 = all checks passed.
#include <cmath>
#include <cstdio>
#include <set>
#include <vector>

#include "../../paper_2504_19410_amd/csrc/fsa_sched.hpp"

using namespace fsa::sched;

static int g_fail = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            ++g_fail;                                                  \
        }                                                              \
    } while (0)

struct Fake : Backend {
    double t = 0;
    int created = 0, built = 0, destroyed = 0;
    std::vector<uint64_t> launched;
    std::set<int> fail_kinds;
    double now() override { return t; }
    Status create_plan(const Key& k, PlanInfo* out, std::string* err) override {
        if (k.N[0] <= 0) {
            if (err) *err = "bad N";
            return ST_EINVAL;
        }
        ++created;
        out->handle = new int(created);
        out->tensor_bytes = (size_t)k.N[0] * 1000;  // scripted sizes
        out->workspace_bytes = (size_t)k.N[1] * 1000;
        return ST_OK;
    }
    Status build_plan(const PlanInfo&, std::string*) override {
        ++built;
        return ST_OK;
    }
    void destroy_plan(const PlanInfo& p) override {
        ++destroyed;
        delete (int*)p.handle;
    }
    Status launch(const Request& r, const PlanInfo&, int, std::string* err) override {
        if (fail_kinds.count(r.key.kind)) {
            if (err) *err = "injected device failure";
            return ST_EDEVICE;
        }
        launched.push_back(r.ticket);
        return ST_OK;
    }
};

static Key key(int kind, int64_t tensor_k, int64_t ws_k, double L = 1.0) {
    Key k;
    k.kind = kind;
    k.d = 2;
    k.N[0] = tensor_k;
    k.N[1] = ws_k;
    k.L[0] = L;
    k.L[1] = L;
    return k;
}

static void test_budget_fifo_continuous() {
    Fake be;
    Scheduler s(&be, 10000, 8);
    uint64_t t[5];
    // same key: tensor 1000, workspace 3000
    for (int i = 0; i < 5; ++i) CHECK(s.submit(key(1, 1, 3), nullptr, nullptr, &t[i], nullptr) == ST_OK);
    CHECK(s.pump() == 3);  // 1000 + 3*3000 = 10000
    CHECK(be.launched.size() == 3 && be.launched[0] == t[0] && be.launched[2] == t[2]);
    CHECK(s.stats().hbm_in_use == 10000);
    CHECK(s.pump() == 0);  // no room
    be.t = 0.004;
    s.complete(t[1], ST_OK, be.t);  // out of order completion frees 3000
    CHECK(s.pump() == 1 && be.launched.back() == t[3]);
    s.complete(t[0], ST_OK, 0.005);
    CHECK(s.pump() == 1 && be.launched.back() == t[4]);
    CHECK(s.stats().hbm_peak <= 10000);
    CHECK(be.built == 1 && s.stats().cache_misses == 1 && s.stats().cache_hits == 4);
}

static void test_head_of_line_order() {
    Fake be;
    Scheduler s(&be, 10000, 8);
    uint64_t a, b, c;
    CHECK(s.submit(key(1, 1, 6), nullptr, nullptr, &a, nullptr) == ST_OK);  // 7000
    CHECK(s.submit(key(2, 1, 5), nullptr, nullptr, &b, nullptr) == ST_OK);  // needs 6000
    CHECK(s.submit(key(3, 1, 1), nullptr, nullptr, &c, nullptr) == ST_OK);  // would fit, must wait
    CHECK(s.pump() == 1);
    CHECK(be.launched.size() == 1);
    s.complete(a, ST_OK, 0.001);
    CHECK(s.pump() == 2);  // b then c, in order
    CHECK(be.launched[1] == b && be.launched[2] == c);
}

static void test_bypass_of_a_blocked_head() {
    Fake be;
    Scheduler s(&be, 10000, 8);
    uint64_t a, warm, big, small1, small2;
    // a cached small key first
    CHECK(s.submit(key(3, 1, 1), nullptr, nullptr, &warm, nullptr) == ST_OK);
    CHECK(s.pump() == 1);
    s.complete(warm, ST_OK, 0.001);
    CHECK(s.submit(key(1, 1, 5), nullptr, nullptr, &a, nullptr) == ST_OK);    // 6000 (+1000 cached)
    CHECK(s.pump() == 1);                                                        // in use 7000
    CHECK(s.submit(key(2, 1, 5), nullptr, nullptr, &big, nullptr) == ST_OK);  // needs 6000: waits
    CHECK(s.submit(key(3, 1, 1), nullptr, nullptr, &small1, nullptr) == ST_OK);  // cached, 1000
    CHECK(s.submit(key(4, 1, 1), nullptr, nullptr, &small2, nullptr) == ST_OK);  // not cached
    CHECK(s.pump() == 1);  // small1 passes the blocked head; small2 (a miss) does not
    CHECK(be.launched.back() == small1);
    CHECK(be.destroyed == 0);  // nothing evicted while work is in flight
    s.complete(a, ST_OK, 0.002);
    s.complete(small1, ST_OK, 0.003);
    CHECK(s.pump() == 2);  // the head, then small2
    CHECK(be.launched[be.launched.size() - 2] == big && be.launched.back() == small2);
}

static void test_reject_and_cancel() {
    Fake be;
    Scheduler s(&be, 10000, 1);
    uint64_t big, a, b;
    std::string err;
    CHECK(s.submit(key(1, 6, 5), nullptr, nullptr, &big, &err) == ST_EBUDGET);
    CHECK(s.stats().rejected == 1);
    CHECK(s.submit(key(1, 0, 1), nullptr, nullptr, &a, &err) == ST_EINVAL);
    CHECK(s.submit(key(2, 1, 1), nullptr, nullptr, &a, nullptr) == ST_OK);
    CHECK(s.submit(key(2, 1, 1), nullptr, nullptr, &b, nullptr) == ST_OK);
    CHECK(s.pump() == 1);  // one slot
    CHECK(s.cancel(a) == ST_ESTATE);
    CHECK(s.cancel(b) == ST_OK);
    bool done = false;
    Status r = ST_OK;
    CHECK(s.poll(b, &done, &r) == ST_OK && done && r == ST_ECANCELLED);
    s.complete(a, ST_OK, 0.002);
    CHECK(s.pump() == 0);
    CHECK(s.idle());
    CHECK(s.stats().cancelled == 1 && s.stats().done == 1);
}

static void test_cache_eviction_lru() {
    Fake be;
    Scheduler s(&be, 10000, 4);
    uint64_t t;
    // A: tensor 4000, ws 1000; B: tensor 4000, ws 1000; C: tensor 5000, ws 1000
    CHECK(s.submit(key(1, 4, 1), nullptr, nullptr, &t, nullptr) == ST_OK);
    CHECK(s.pump() == 1);
    s.complete(t, ST_OK, 0.001);
    CHECK(s.submit(key(2, 4, 1), nullptr, nullptr, &t, nullptr) == ST_OK);
    CHECK(s.pump() == 1);
    s.complete(t, ST_OK, 0.002);
    CHECK(s.cached_plans() == 2);  // 8000 cached
    CHECK(s.submit(key(3, 5, 1), nullptr, nullptr, &t, nullptr) == ST_OK);
    CHECK(s.pump() == 1);           // evicts A (least recently used)
    CHECK(be.destroyed == 1);
    s.complete(t, ST_OK, 0.003);
    CHECK(s.stats().hbm_in_use == 9000);  // B 4000 + C 5000
    CHECK(s.submit(key(1, 4, 1), nullptr, nullptr, &t, nullptr) == ST_OK);  // A again: miss
    CHECK(s.pump() == 1);
    CHECK(s.stats().cache_misses == 4);
    CHECK(s.stats().hbm_peak <= 10000);
}

static void test_failure_isolation() {
    Fake be;
    be.fail_kinds.insert(7);
    Scheduler s(&be, 100000, 8);
    uint64_t ok1, bad, ok2;
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &ok1, nullptr) == ST_OK);
    CHECK(s.submit(key(7, 1, 1), nullptr, nullptr, &bad, nullptr) == ST_OK);
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &ok2, nullptr) == ST_OK);
    CHECK(s.pump() == 2);
    bool done = false;
    Status r = ST_OK;
    CHECK(s.poll(bad, &done, &r) == ST_OK && done && r == ST_EDEVICE);
    CHECK(s.inflight() == 2);
    s.complete(ok1, ST_OK, 0.001);
    s.complete(ok2, ST_OK, 0.001);
    CHECK(s.idle());
    // only the two cached tensors remain accounted
    CHECK(s.stats().hbm_in_use == 2000);
}

static void test_slots_and_latency() {
    Fake be;
    Scheduler s(&be, 1 << 30, 2);
    std::vector<uint64_t> t(10);
    for (int i = 0; i < 10; ++i) CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &t[i], nullptr) == ST_OK);
    int in_flight = 0;
    std::vector<double> lat;
    for (int i = 0; i < 10; ++i) {
        in_flight += s.pump();
        CHECK(s.inflight() <= 2);
        be.t = 0.001 * (i + 1);
        s.complete(t[i], ST_OK, be.t);
        lat.push_back(be.t * 1e3);
    }
    Stats st = s.stats();
    CHECK(st.done == 10);
    std::vector<double> v = lat;
    CHECK(std::fabs(st.p50_ms - Scheduler::quantile(v, 0.5)) < 1e-12);
    CHECK(std::fabs(st.p50_ms - 5.5) < 1e-9);   // latencies 1..10 ms
    CHECK(std::fabs(st.p99_ms - 9.91) < 1e-9);
    CHECK(std::fabs(st.throughput_rps - 1000.0) < 1e-6);
}

static void test_cancel_all() {
    Fake be;
    Scheduler s(&be, 1 << 30, 1);
    uint64_t a, b, c;
    s.submit(key(1, 1, 1), nullptr, nullptr, &a, nullptr);
    s.submit(key(1, 1, 1), nullptr, nullptr, &b, nullptr);
    s.submit(key(1, 1, 1), nullptr, nullptr, &c, nullptr);
    CHECK(s.pump() == 1);
    CHECK(s.cancel_all() == 2);
    s.complete(a, ST_OK, 0.001);
    CHECK(s.idle());
}

// Requests that wait in the queue past the timeout (from their arrival)
// finish ST_ETIMEDOUT without launching; a launched one is never timed out;
// the limit can be turned off again.
static void test_queue_timeout() {
    Fake be;
    Scheduler s(&be, 1 << 30, 1);  // one slot: everything after the first waits
    s.set_queue_timeout(0.010);
    uint64_t a, b, c, d;
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &a, nullptr) == ST_OK);
    CHECK(s.pump() == 1);
    be.t = 0.002;
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &b, nullptr) == ST_OK);  // arrives 0.002
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &c, nullptr, 0.008) == ST_OK);
    be.t = 0.013;  // b has waited 11 ms, c 5 ms; a (launched) is still running
    bool done = false;
    Status res = ST_OK;
    CHECK(s.poll(b, &done, &res) == ST_OK && done && res == ST_ETIMEDOUT);
    CHECK(s.poll(c, &done, &res) == ST_OK && !done);
    CHECK(s.poll(a, &done, &res) == ST_OK && !done);
    s.complete(a, ST_OK, 0.014);
    be.t = 0.014;
    CHECK(s.pump() == 1 && be.launched.back() == c);
    CHECK(s.stats().timed_out == 1 && s.stats().done == 1);
    // a queued request past the limit is dropped at the next pump as well
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &d, nullptr) == ST_OK);
    be.t = 0.030;
    CHECK(s.pump() == 0);
    CHECK(s.poll(d, &done, &res) == ST_OK && done && res == ST_ETIMEDOUT);
    CHECK(s.stats().timed_out == 2);
    s.complete(c, ST_OK, 0.031);
    s.set_queue_timeout(0);  // off: a long wait is fine
    CHECK(s.submit(key(1, 1, 1), nullptr, nullptr, &d, nullptr) == ST_OK);
    be.t = 10.0;
    CHECK(s.pump() == 1 && be.launched.back() == d);
    CHECK(be.launched.size() == 3);
}

int main() {
    test_queue_timeout();
    test_budget_fifo_continuous();
    test_head_of_line_order();
    test_reject_and_cancel();
    test_cache_eviction_lru();
    test_bypass_of_a_blocked_head();
    test_failure_isolation();
    test_slots_and_latency();
    test_cancel_all();
    std::printf("%s (%d failures)\n", g_fail ? "FAILED" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
