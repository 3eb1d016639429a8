// fsa_sched.hpp -- device-independent core of the convolution server.
//
// Continuous batching under an HBM budget: requests queue in arrival order;
// whenever a slot and enough budget are free, the request at the head is
// admitted -- its kernel tensor taken from the cache (built on a miss), its
// workspace reserved -- and launched; it then runs on the device alongside
// every other admitted request.  Completions release their workspace and
// slot, which admits the next requests.  Cached tensors that no in-flight
// request uses are evicted least-recently-used first when the budget is
// short.  The core knows nothing about HIP: a Backend builds plans, launches
// requests and reports completions, so the same logic runs on the GPU and,
// with a scripted backend and clock, in host-only tests.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace fsa {
namespace sched {

enum Status { ST_OK = 0, ST_EINVAL = 1, ST_EUNSUPPORTED = 2, ST_ENOMEM = 3, ST_EDEVICE = 4, ST_ESTATE = 5,
              ST_EBUDGET = 6, ST_ECANCELLED = 7, ST_ETIMEDOUT = 8 };

// Identity of a kernel tensor: everything that determines it.
struct Key {
    int kind = 0, d = 0, prec = 0;
    int general = 0;  // general construction requested
    double lam = 0, eps = 0;
    double L[3] = {0, 0, 0};
    int64_t N[3] = {0, 0, 0};
    bool operator<(const Key& o) const {
        if (kind != o.kind) return kind < o.kind;
        if (d != o.d) return d < o.d;
        if (prec != o.prec) return prec < o.prec;
        if (general != o.general) return general < o.general;
        if (lam != o.lam) return lam < o.lam;
        if (eps != o.eps) return eps < o.eps;
        for (int j = 0; j < 3; ++j) {
            if (L[j] != o.L[j]) return L[j] < o.L[j];
            if (N[j] != o.N[j]) return N[j] < o.N[j];
        }
        return false;
    }
    int64_t points() const {
        int64_t p = 1;
        for (int j = 0; j < d; ++j) p *= N[j];
        return p;
    }
};

// What a backend reports about a plan it created (host-side, no device work).
struct PlanInfo {
    void* handle = nullptr;
    size_t tensor_bytes = 0;     // device bytes the cached tensor occupies
    size_t workspace_bytes = 0;  // device bytes one evaluation needs
};

struct Request {
    uint64_t ticket = 0;
    Key key;
    const void* rho = nullptr;
    void* phi = nullptr;
    // t_arrival: when the request arose (the caller's, else the submission
    // time); latency = t_done - t_arrival, queueing before submission included
    double t_arrival = 0, t_submit = 0, t_admit = 0, t_done = 0;
    int slot = -1;
    bool done = false;
    Status result = ST_OK;
};

class Backend {
public:
    virtual ~Backend() = default;
    virtual double now() = 0;  // seconds, monotonic
    // host-side plan creation and sizing; no device work
    virtual Status create_plan(const Key& k, PlanInfo* out, std::string* err) = 0;
    // asynchronous tensor generation for a new cache entry
    virtual Status build_plan(const PlanInfo& p, std::string* err) = 0;
    virtual void destroy_plan(const PlanInfo& p) = 0;
    // asynchronous evaluation; the backend must later report its completion
    // through Scheduler::complete
    virtual Status launch(const Request& r, const PlanInfo& p, int slot, std::string* err) = 0;
};

struct Completion {
    uint64_t ticket;
    Status status;
    double t_done;
};

struct Stats {
    double p50_ms = 0, p99_ms = 0, throughput_rps = 0, gpts_per_s = 0;
    uint64_t done = 0, rejected = 0, cancelled = 0, cache_hits = 0, cache_misses = 0;
    size_t hbm_in_use = 0, hbm_peak = 0;
    uint64_t timed_out = 0;  // queued past the queue timeout (ST_ETIMEDOUT)
};

class Scheduler {
public:
    Scheduler(Backend* be, size_t budget, int max_inflight)
        : be_(be), budget_(budget), slots_(std::max(1, max_inflight)), t0_(be->now()) {
        free_slots_.resize(slots_);
        for (int i = 0; i < slots_; ++i) free_slots_[i] = slots_ - 1 - i;
    }

    ~Scheduler() {
        for (auto& kv : cache_) be_->destroy_plan(kv.second.info);
    }

    // Queues a request.  ST_EBUDGET if it could never fit: its workspace plus
    // its tensor exceed the whole budget.  t_arrival < 0: now.
    Status submit(const Key& k, const void* rho, void* phi, uint64_t* ticket, std::string* err,
                  double t_arrival = -1.0) {
        std::lock_guard<std::mutex> lk(mu_);
        PlanInfo probe;
        size_t tensor_bytes, ws_bytes;
        auto it = cache_.find(k);
        if (it != cache_.end()) {
            tensor_bytes = it->second.info.tensor_bytes;
            ws_bytes = it->second.info.workspace_bytes;
        } else {
            Status s = be_->create_plan(k, &probe, err);
            if (s != ST_OK) return s;
            tensor_bytes = probe.tensor_bytes;
            ws_bytes = probe.workspace_bytes;
            // keep the created (unbuilt) plan for admission
            Entry e;
            e.info = probe;
            e.built = false;
            cache_.emplace(k, e);
        }
        if (tensor_bytes + ws_bytes > budget_) {
            ++rejected_;
            if (err) *err = "request exceeds the HBM budget on its own";
            drop_if_unused_unbuilt(k);
            return ST_EBUDGET;
        }
        Request r;
        r.ticket = next_ticket_++;
        r.key = k;
        r.rho = rho;
        r.phi = phi;
        r.t_submit = be_->now();
        r.t_arrival = t_arrival >= 0 ? t_arrival : r.t_submit;
        reqs_[r.ticket] = r;
        queue_.push_back(r.ticket);
        *ticket = r.ticket;
        return ST_OK;
    }

    // Admits and launches as many queued requests as slots and budget allow,
    // in arrival order except for the bounded bypass of admit_locked, from
    // any thread; returns the number this call launched.  One pump runs at a
    // time: a caller that finds another pump running leaves a request for
    // it and returns, and the running pump goes round again, so a request
    // queued before a pump() call is always considered.  The state lock is
    // released while the backend builds a tensor or launches, so
    // submissions, completions and polls are not held up by device calls.
    int pump() {
        pending_.store(true);
        int total = 0;
        while (pending_.load()) {
            std::unique_lock<std::mutex> pl(pump_mu_, std::try_to_lock);
            if (!pl.owns_lock()) return total;  // the running pump sees pending_
            pending_.store(false);
            total += pump_locked();
        }
        return total;
    }

    // A launched request's work has finished at time t_done (backend clock).
    void complete(const Completion& c) { complete(c.ticket, c.status, c.t_done); }

    // A launched request's work has finished at time t_done (backend clock).
    void complete(uint64_t ticket, Status s, double t_done) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end() || it->second.done) return;
        release_locked(it->second);
        finish_locked(it->second, s, t_done);
    }

    Status poll(uint64_t ticket, bool* done, Status* result) {
        std::lock_guard<std::mutex> lk(mu_);
        expire_locked();
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return ST_EINVAL;
        *done = it->second.done;
        if (it->second.done && result) *result = it->second.result;
        return ST_OK;
    }

    // Requests still queued this long after their arrival finish with
    // ST_ETIMEDOUT instead of launching (seconds; <= 0: no limit).  A
    // launched request runs to completion.  Checked whenever the queue is
    // pumped or a request is polled.
    void set_queue_timeout(double seconds) {
        std::lock_guard<std::mutex> lk(mu_);
        queue_timeout_ = seconds;
        expire_locked();
    }

    // Cancels a request that is still queued (ST_ESTATE once it has launched).
    Status cancel(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return ST_EINVAL;
        auto q = std::find(queue_.begin(), queue_.end(), ticket);
        if (q == queue_.end()) return ST_ESTATE;
        queue_.erase(q);
        ++cancelled_;
        finish_locked(it->second, ST_ECANCELLED);
        return ST_OK;
    }

    // Cancels every queued request (used when the server shuts down).
    int cancel_all() {
        std::lock_guard<std::mutex> lk(mu_);
        int n = 0;
        while (!queue_.empty()) {
            Request& r = reqs_[queue_.front()];
            queue_.pop_front();
            ++cancelled_;
            finish_locked(r, ST_ECANCELLED);
            ++n;
        }
        return n;
    }

    // Starts a new statistics window (latencies, counters, peak); the cache
    // and any queued or in-flight work are kept.
    void reset_stats() {
        std::lock_guard<std::mutex> lk(mu_);
        lat_ms_.clear();
        done_ok_ = rejected_ = cancelled_ = hits_ = misses_ = timed_out_ = 0;
        points_ = 0;
        t0_ = be_->now();
        last_done_ = t0_;
        peak_ = in_use_;
    }

    // Forgets a finished request (frees its bookkeeping).
    void forget(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it != reqs_.end() && it->second.done) reqs_.erase(it);
    }

    Stats stats() {
        std::lock_guard<std::mutex> lk(mu_);
        Stats s;
        std::vector<double> v = lat_ms_;
        if (!v.empty()) {
            std::sort(v.begin(), v.end());
            s.p50_ms = quantile(v, 0.50);
            s.p99_ms = quantile(v, 0.99);
        }
        const double up = std::max(1e-9, last_done_ - t0_);
        s.done = done_ok_;
        s.throughput_rps = done_ok_ ? (double)done_ok_ / up : 0.0;
        s.gpts_per_s = done_ok_ ? (double)points_ / up / 1e9 : 0.0;
        s.rejected = rejected_;
        s.timed_out = timed_out_;
        s.cancelled = cancelled_;
        s.cache_hits = hits_;
        s.cache_misses = misses_;
        s.hbm_in_use = in_use_;
        s.hbm_peak = peak_;
        return s;
    }

    bool idle() {
        std::lock_guard<std::mutex> lk(mu_);
        return queue_.empty() && inflight_ == 0;
    }
    bool has_queued() {
        std::lock_guard<std::mutex> lk(mu_);
        return !queue_.empty();
    }
    int inflight() {
        std::lock_guard<std::mutex> lk(mu_);
        return inflight_;
    }
    size_t cached_plans() {
        std::lock_guard<std::mutex> lk(mu_);
        size_t n = 0;
        for (auto& kv : cache_) n += kv.second.built;
        return n;
    }
    // Latency percentile over completed requests: linear interpolation
    // between order statistics, q in [0, 1].
    static double quantile(const std::vector<double>& sorted, double q) {
        if (sorted.empty()) return 0.0;
        const double pos = q * (double)(sorted.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - (double)i;
        return i + 1 < sorted.size() ? sorted[i] * (1 - f) + sorted[i + 1] * f : sorted[i];
    }

private:
    struct Entry {
        PlanInfo info;
        bool built = false;
        int refs = 0;
        uint64_t lru = 0;
    };

    // An admission decided under the state lock and carried out without it.
    struct Admission {
        Request req;
        PlanInfo info;
        bool build = false;
    };

    // Admits the next request if a slot and budget allow: reserves the slot,
    // the workspace and (on a miss) the tensor, and marks the entry built and
    // referenced, so no other admission builds or evicts it.
    //   The head of the queue goes first.  When it does not fit, cached
    // tensors are evicted for it only if nothing is in flight (in-flight
    // requests will free their workspaces; evicting now would only make
    // later requests rebuild).  While it waits, a request among the next
    // kBypassWindow whose tensor is cached and which fits without eviction
    // may go ahead, at most kMaxBypass times per head, so that small requests
    // keep the device busy without starving a large one.
    static constexpr int kBypassWindow = 16, kMaxBypass = 64;
    bool admit_locked(Admission* a) {
        expire_locked();
        while (!queue_.empty() && !free_slots_.empty()) {
            size_t pos = 0;
            {
                Request& h = reqs_[queue_.front()];
                Entry& e = cache_[h.key];
                const size_t need = e.info.workspace_bytes + (e.built ? 0 : e.info.tensor_bytes);
                const bool fits = in_use_ + need <= budget_ ||
                                  (inflight_ == 0 && evict_for(need, h.key));
                if (!fits) {
                    if (bypassed_ >= kMaxBypass) return false;
                    pos = 0;
                    for (size_t i = 1; i < queue_.size() && i <= (size_t)kBypassWindow; ++i) {
                        const Request& c = reqs_[queue_[i]];
                        const Entry& ce = cache_[c.key];
                        if (ce.built && in_use_ + ce.info.workspace_bytes <= budget_) {
                            pos = i;
                            break;
                        }
                    }
                    if (pos == 0) return false;
                    ++bypassed_;
                } else {
                    bypassed_ = 0;
                }
            }
            Request& r = reqs_[queue_[pos]];
            Entry& e = cache_[r.key];
            queue_.erase(queue_.begin() + (long)pos);
            a->build = !e.built;
            if (a->build) {
                ++misses_;
                e.built = true;
                in_use_ += e.info.tensor_bytes;
            } else {
                ++hits_;
            }
            in_use_ += e.info.workspace_bytes;
            peak_ = std::max(peak_, in_use_);
            ++e.refs;
            touch(r.key);
            r.slot = free_slots_.back();
            free_slots_.pop_back();
            r.t_admit = be_->now();
            ++inflight_;
            a->req = r;
            a->info = e.info;
            return true;
        }
        return false;
    }

    int pump_locked() {
        int launched = 0;
        for (;;) {
            Admission a;
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (!admit_locked(&a)) break;
            }
            std::string err;
            Status s = a.build ? be_->build_plan(a.info, &err) : ST_OK;
            const bool built = s == ST_OK;
            if (s == ST_OK) s = be_->launch(a.req, a.info, a.req.slot, &err);
            std::lock_guard<std::mutex> lk(mu_);
            if (!built) {  // the tensor never came to be: undo its reservation
                Entry& e = cache_[a.req.key];
                e.built = false;
                in_use_ -= e.info.tensor_bytes;
            }
            if (s != ST_OK) {
                Request& r = reqs_[a.req.ticket];
                r.slot = a.req.slot;
                release_locked(r);
                finish_locked(r, s);
                continue;
            }
            ++launched;
        }
        return launched;
    }

    void touch(const Key& k) { cache_[k].lru = ++lru_clock_; }

    void drop_if_unused_unbuilt(const Key& k) {
        auto it = cache_.find(k);
        if (it != cache_.end() && !it->second.built && it->second.refs == 0 &&
            std::none_of(queue_.begin(), queue_.end(),
                         [&](uint64_t t) { return !(reqs_[t].key < k) && !(k < reqs_[t].key); })) {
            be_->destroy_plan(it->second.info);
            cache_.erase(it);
        }
    }

    // Evicts built, unreferenced tensors (least recently used first) until
    // `need` more bytes fit; never evicts the key about to be used.
    bool evict_for(size_t need, const Key& keep) {
        while (in_use_ + need > budget_) {
            auto victim = cache_.end();
            for (auto it = cache_.begin(); it != cache_.end(); ++it) {
                const bool same = !(it->first < keep) && !(keep < it->first);
                if (!it->second.built || it->second.refs > 0 || same) continue;
                if (victim == cache_.end() || it->second.lru < victim->second.lru) victim = it;
            }
            if (victim == cache_.end()) return false;
            in_use_ -= victim->second.info.tensor_bytes;
            be_->destroy_plan(victim->second.info);
            // an evicted key may be re-created later by submit()
            const bool queued = std::any_of(queue_.begin(), queue_.end(), [&](uint64_t t) {
                return !(reqs_[t].key < victim->first) && !(victim->first < reqs_[t].key);
            });
            if (queued) {
                PlanInfo fresh;
                std::string err;
                if (be_->create_plan(victim->first, &fresh, &err) == ST_OK) {
                    victim->second.info = fresh;
                    victim->second.built = false;
                    continue;
                }
            }
            cache_.erase(victim);
        }
        return true;
    }

    // Finishes the queued requests that have waited longer than the queue
    // timeout since their arrival.
    void expire_locked() {
        if (queue_timeout_ <= 0 || queue_.empty()) return;
        const double now = be_->now();
        for (size_t i = 0; i < queue_.size();) {
            Request& r = reqs_[queue_[i]];
            if (now - r.t_arrival > queue_timeout_) {
                queue_.erase(queue_.begin() + (long)i);
                ++timed_out_;
                finish_locked(r, ST_ETIMEDOUT);
                drop_if_unused_unbuilt(r.key);
            } else {
                ++i;
            }
        }
    }

    void release_locked(Request& r) {
        auto it = cache_.find(r.key);
        if (it != cache_.end()) {
            in_use_ -= it->second.info.workspace_bytes;
            --it->second.refs;
        }
        if (r.slot >= 0) {
            free_slots_.push_back(r.slot);
            r.slot = -1;
        }
        --inflight_;
    }

    void finish_locked(Request& r, Status s, double t_done = -1.0) {
        r.done = true;
        r.result = s;
        r.t_done = t_done >= 0 ? t_done : be_->now();
        if (s == ST_OK) {
            ++done_ok_;
            points_ += (double)r.key.points();
            lat_ms_.push_back((r.t_done - r.t_arrival) * 1e3);
            last_done_ = std::max(last_done_, r.t_done);
        }
    }

    Backend* be_;
    size_t budget_;
    int slots_;
    double t0_;
    std::mutex pump_mu_;  // taken before mu_, never while holding it
    std::atomic<bool> pending_{false};
    std::mutex mu_;
    std::map<Key, Entry> cache_;
    std::unordered_map<uint64_t, Request> reqs_;
    std::deque<uint64_t> queue_;
    std::vector<int> free_slots_;
    uint64_t next_ticket_ = 1, lru_clock_ = 0;
    int bypassed_ = 0;  // admissions ahead of the current head
    size_t in_use_ = 0, peak_ = 0;
    int inflight_ = 0;
    uint64_t done_ok_ = 0, rejected_ = 0, cancelled_ = 0, hits_ = 0, misses_ = 0, timed_out_ = 0;
    double queue_timeout_ = 0;  // seconds; <= 0: none
    double points_ = 0, last_done_ = 0;
    std::vector<double> lat_ms_;
};

// Where a served scheduler learns of completions: one in-order queue of
// launched requests per device stream.
class CompletionSource {
public:
    virtual ~CompletionSource() = default;
    virtual int n_queues() const = 0;
    // Blocks until the oldest request launched on queue q has finished and
    // returns it; false once stop() has been called and q is empty.
    virtual bool wait_next(int q, Completion* out) = 0;
    // Wakes every wait_next on an empty queue for good.
    virtual void stop() = 0;
    // Called first on every waiter thread (e.g. to select the device).
    virtual void thread_init() {}
};

// The threads of a served scheduler.  A submitting thread queues its request
// and pumps (admits and launches) itself, so an idle server starts a request
// without a thread hand-off; one waiter thread per device queue sleeps until
// that queue's oldest request finishes, records the completion and pumps the
// requests that the freed slot and budget admit.  No thread polls.
class Runner {
public:
    Runner(Scheduler* s, CompletionSource* src) : s_(s), src_(src) {
        for (int q = 0; q < src_->n_queues(); ++q)
            waiters_.emplace_back([this, q] { wait_loop(q); });
    }
    ~Runner() { shutdown(); }

    Status submit(const Key& k, const void* rho, void* phi, uint64_t* ticket, std::string* err,
                  double t_arrival = -1.0) {
        const Status st = s_->submit(k, rho, phi, ticket, err, t_arrival);
        if (st != ST_OK) return st;
        s_->pump();
        notify_done();  // a request may have failed at admission
        return ST_OK;
    }

    // Waits until the request has finished (true) or timeout_s has passed
    // (false; timeout_s < 0: no limit).  ST_EINVAL for an unknown ticket.
    Status wait(uint64_t ticket, double timeout_s, bool* done, Status* result) {
        const auto t_end = std::chrono::steady_clock::now() +
                           std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                               std::chrono::duration<double>(timeout_s < 0 ? 0.0 : timeout_s));
        std::unique_lock<std::mutex> lk(done_mu_);
        for (;;) {
            const Status st = s_->poll(ticket, done, result);
            if (st != ST_OK || *done) return st;
            if (timeout_s >= 0 && std::chrono::steady_clock::now() >= t_end) return ST_OK;
            // completions and admission failures notify; the timed wait is a
            // safety net only (system_clock: pthread_cond_timedwait, which
            // thread sanitizers intercept; the deadline above is steady)
            done_cv_.wait_until(lk,
                                std::chrono::system_clock::now() + std::chrono::milliseconds(2));
        }
    }

    // Cancels what is queued, lets what is in flight finish, joins the threads.
    void shutdown() {
        if (down_) return;
        down_ = true;
        s_->cancel_all();
        notify_done();
        src_->stop();
        for (auto& t : waiters_) t.join();
        waiters_.clear();
    }

    void notify_done() {
        std::lock_guard<std::mutex> lk(done_mu_);
        done_cv_.notify_all();
    }

private:
    void wait_loop(int q) {
        src_->thread_init();
        Completion c;
        while (src_->wait_next(q, &c)) {
            s_->complete(c);
            notify_done();
            s_->pump();
            notify_done();
        }
    }

    Scheduler* s_;
    CompletionSource* src_;
    std::vector<std::thread> waiters_;
    std::mutex done_mu_;
    std::condition_variable done_cv_;
    bool down_ = false;
};

}  // namespace sched
}  // namespace fsa
