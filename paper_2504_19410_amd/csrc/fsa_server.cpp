// fsa_server.cpp -- the served variant: continuous batching of convolution
// requests on one GPU under an HBM budget (scheduling logic and threads in
// fsa_sched.hpp).
//
// Device side of a request: on its slot's stream the request waits for its
// cached tensor's build event, runs the evaluation passes in the slot's
// resident workspace and records a completion event.  A slot's workspace is
// sized to the largest request it has run (grown, rarely, between requests,
// when the slot is idle), so the steady state allocates nothing.  Requests
// on different slots run concurrently on the device.  Completion events are
// created with hipEventBlockingSync: the waiter thread of each stream sleeps
// in hipEventSynchronize until its oldest request finishes (woken by the
// device's interrupt a few microseconds after the kernel ends), instead of
// a thread polling every event.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "fsa_internal.hpp"
#include "fsa_sched.hpp"

namespace fsa {
void set_last_error(const char* msg);
}

namespace {

using fsa::sched::Completion;
using fsa::sched::Key;
using fsa::sched::PlanInfo;
using fsa::sched::Request;
using fsa::sched::Runner;
using fsa::sched::Scheduler;
using Status = fsa::sched::Status;

double steady_now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

class HipBackend : public fsa::sched::Backend, public fsa::sched::CompletionSource {
public:
    HipBackend(int device, int n_streams) : device_(device) {
        for (int i = 0; i < n_streams; ++i) {
            hipStream_t s = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess)
                streams_.push_back(s);
        }
        queues_ = std::vector<Queue>(streams_.size());
        (void)hipStreamCreateWithFlags(&build_stream_, hipStreamNonBlocking);
    }
    ~HipBackend() override {
        for (auto w : slot_ws_)
            if (w) (void)hipFree(w);
        for (auto e : all_events_) (void)hipEventDestroy(e);
        for (auto s : streams_) (void)hipStreamDestroy(s);
        if (build_stream_) (void)hipStreamDestroy(build_stream_);
    }
    bool ok() const { return !streams_.empty() && build_stream_ != nullptr; }

    double now() override { return steady_now(); }

    Status create_plan(const Key& k, PlanInfo* out, std::string* err) override {
        fsa_kernel kk{};
        kk.kind = k.kind;
        kk.lambda = k.lam;
        kk.eps = k.eps;
        kk.general = k.general;
        fsa_plan pl = nullptr;
        fsa_status s = fsa_plan_create(&kk, k.d, k.L, k.N, (fsa_precision)k.prec, &pl);
        if (s != FSA_OK) {
            if (err) *err = fsa_last_error();
            return (Status)s;
        }
        size_t tb = 0, wb = 0;
        fsa_plan_query(pl, nullptr, nullptr, &tb, &wb);
        out->handle = pl;
        // tensor + twiddle tables + (3D, an upper bound) the tensor build's
        // line order, kept by plans whose box has equal sides
        const size_t order = k.d == 3 ? sizeof(int) * (size_t)(k.N[1] + 1) * (size_t)(k.N[2] + 1) : 0;
        out->tensor_bytes = tb + pl->tw_elems * pl->csize + order;
        out->workspace_bytes = wb + 256;                      // + alignment slack
        return fsa::sched::ST_OK;
    }

    Status build_plan(const PlanInfo& p, std::string* err) override {
    fsa::Range range("fsa_server tensor build");
        fsa_plan pl = (fsa_plan)p.handle;
        fsa_status s = fsa_build_tensor(pl, build_stream_);
        if (s != FSA_OK) {
            if (err) *err = fsa_last_error();
            return (Status)s;
        }
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev, build_stream_) != hipSuccess) {
            if (err) *err = "build event";
            return fsa::sched::ST_EDEVICE;
        }
        std::lock_guard<std::mutex> lk(ev_mu_);
        built_[pl] = ev;
        return fsa::sched::ST_OK;
    }

    void destroy_plan(const PlanInfo& p) override {
        fsa_plan pl = (fsa_plan)p.handle;
        {
            std::lock_guard<std::mutex> lk(ev_mu_);
            auto it = built_.find(pl);
            if (it != built_.end()) {
                (void)hipEventSynchronize(it->second);
                (void)hipEventDestroy(it->second);
                built_.erase(it);
            }
        }
        fsa_plan_destroy(pl);
    }

    // Large requests (at least kLargePoints grid points, e.g. 256^3) run one
    // after another on stream 0; the others rotate over the remaining
    // streams.  Two large requests sharing the device would each take about
    // twice as long, so running them in turn keeps the tail latency of the
    // large ones at their own run time, while small requests, which leave
    // most of the device idle, still overlap with them and each other.
    static constexpr int64_t kLargePoints = int64_t(1) << 23;
    size_t stream_of(const Request& r, int slot) const {
        const size_t n = streams_.size();
        if (n == 1) return 0;
        if (r.key.points() >= kLargePoints) return 0;
        return 1 + (size_t)slot % (n - 1);
    }

    // Called by the scheduler's pump, one at a time, with the slot reserved
    // for this request (its previous request has completed).
    Status launch(const Request& r, const PlanInfo& p, int slot, std::string* err) override {
    fsa::Range range("fsa_server launch");
        const size_t q = stream_of(r, slot);
        hipStream_t st = streams_[q];
        fsa_plan pl = (fsa_plan)p.handle;
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(ev_mu_);
            auto it = built_.find(pl);
            if (it != built_.end()) ev = it->second;
        }
        if (ev && hipStreamWaitEvent(st, ev, 0) != hipSuccess) {
            if (err) *err = "hipStreamWaitEvent failed";
            return fsa::sched::ST_EDEVICE;
        }
        if ((size_t)slot >= slot_ws_.size()) {
            slot_ws_.resize(slot + 1, nullptr);
            slot_bytes_.resize(slot + 1, 0);
        }
        if (slot_bytes_[slot] < p.workspace_bytes) {
            // the slot is idle (its previous request completed), so the old
            // buffer can go; this happens once per slot and size class
            if (slot_ws_[slot]) (void)hipFree(slot_ws_[slot]);
            slot_ws_[slot] = nullptr;
            slot_bytes_[slot] = 0;
            if (hipMalloc(&slot_ws_[slot], p.workspace_bytes) != hipSuccess) {
                slot_ws_[slot] = nullptr;
                if (err) *err = "workspace allocation failed";
                return fsa::sched::ST_ENOMEM;
            }
            slot_bytes_[slot] = p.workspace_bytes;
        }
        void* ws = (void*)(((uintptr_t)slot_ws_[slot] + 255) & ~(uintptr_t)255);
        fsa_status s = fsa_apply(pl, r.rho, r.phi, ws, st);
        if (s != FSA_OK) {
            if (err) *err = fsa_last_error();
            return (Status)s;
        }
        hipEvent_t done = take_event();
        if (!done || hipEventRecord(done, st) != hipSuccess) {
            if (err) *err = "completion event";
            return fsa::sched::ST_EDEVICE;
        }
        Queue& qu = queues_[q];
        {
            std::lock_guard<std::mutex> lk(qu.mu);
            qu.fifo.push_back(Inflight{r.ticket, done});
        }
        qu.cv.notify_one();
        return fsa::sched::ST_OK;
    }

    // CompletionSource: requests on one stream finish in launch order.
    int n_queues() const override { return (int)streams_.size(); }

    bool wait_next(int q, Completion* out) override {
        Queue& qu = queues_[(size_t)q];
        Inflight f;
        {
            std::unique_lock<std::mutex> lk(qu.mu);
            qu.cv.wait(lk, [&] { return !qu.fifo.empty() || stopped_.load(); });
            if (qu.fifo.empty()) return false;
            f = qu.fifo.front();
            qu.fifo.pop_front();
        }
        const hipError_t e = hipEventSynchronize(f.ev);  // sleeps; no polling
        out->ticket = f.ticket;
        out->status = e == hipSuccess ? fsa::sched::ST_OK : fsa::sched::ST_EDEVICE;
        out->t_done = steady_now();
        std::lock_guard<std::mutex> lk(ev_pool_mu_);
        free_events_.push_back(f.ev);
        return true;
    }

    void stop() override {
        stopped_.store(true);
        for (Queue& qu : queues_) {
            std::lock_guard<std::mutex> lk(qu.mu);
            qu.cv.notify_all();
        }
    }

    void thread_init() override { (void)hipSetDevice(device_); }

private:
    struct Inflight {
        uint64_t ticket = 0;
        hipEvent_t ev = nullptr;
    };
    struct Queue {
        std::mutex mu;
        std::condition_variable cv;
        std::deque<Inflight> fifo;
    };
    hipEvent_t take_event() {
        {
            std::lock_guard<std::mutex> lk(ev_pool_mu_);
            if (!free_events_.empty()) {
                hipEvent_t e = free_events_.back();
                free_events_.pop_back();
                return e;
            }
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventBlockingSync) !=
            hipSuccess)
            return nullptr;
        std::lock_guard<std::mutex> lk(ev_pool_mu_);
        all_events_.push_back(e);
        return e;
    }

    int device_;
    std::vector<hipStream_t> streams_;
    std::vector<Queue> queues_;
    std::atomic<bool> stopped_{false};
    hipStream_t build_stream_ = nullptr;
    std::vector<void*> slot_ws_;  // resident workspace per slot (pump thread only)
    std::vector<size_t> slot_bytes_;
    std::mutex ev_pool_mu_;
    std::vector<hipEvent_t> free_events_, all_events_;
    std::mutex ev_mu_;
    std::map<fsa_plan, hipEvent_t> built_;
};

}  // namespace

struct fsa_server_s {
    int device = 0;
    std::unique_ptr<HipBackend> be;
    std::unique_ptr<Scheduler> sched;
    std::unique_ptr<Runner> runner;
};

extern "C" {

fsa_status fsa_server_create(size_t hbm_budget_bytes, int max_inflight, int n_streams,
                             fsa_server* out) {
    if (!out || hbm_budget_bytes == 0 || max_inflight < 1 || n_streams < 1) {
        fsa::set_last_error("fsa_server_create: bad arguments");
        return FSA_EINVAL;
    }
    auto s = std::make_unique<fsa_server_s>();
    if (hipGetDevice(&s->device) != hipSuccess) {
        fsa::set_last_error("fsa_server_create: no device");
        return FSA_EDEVICE;
    }
    s->be = std::make_unique<HipBackend>(s->device, n_streams);
    if (!s->be->ok()) {
        fsa::set_last_error("fsa_server_create: stream creation failed");
        return FSA_EDEVICE;
    }
    s->sched = std::make_unique<Scheduler>(s->be.get(), hbm_budget_bytes, max_inflight);
    s->runner = std::make_unique<Runner>(s->sched.get(), s->be.get());
    *out = s.release();
    return FSA_OK;
}

fsa_status fsa_server_submit_at(fsa_server s, const fsa_kernel* k, int d, const double* L,
                                const int64_t* N, fsa_precision p, const void* rho, void* phi,
                                double t_arrival, uint64_t* ticket) {
    fsa::Range range("fsa_server_submit");
    if (!s || !k || !L || !N || !rho || !phi || !ticket || d < 2 || d > 3) {
        fsa::set_last_error("fsa_server_submit: bad arguments");
        return FSA_EINVAL;
    }
    if (p == FSA_DD) {
        fsa::set_last_error("fsa_server_submit: double-double requests are not served "
                            "(use a plan and fsa_apply)");
        return FSA_EUNSUPPORTED;
    }
    if (k->kind == FSA_DDI_3D || k->kind == FSA_QUASI2D_DDI) {
        fsa::set_last_error("fsa_server_submit: dipole-dipole requests are not served "
                            "(use a plan and fsa_apply)");
        return FSA_EUNSUPPORTED;
    }
    Key key;
    key.kind = k->kind;
    key.d = d;
    key.prec = (int)p;
    key.lam = (k->kind == FSA_YUKAWA_3D || k->kind == FSA_YUKAWA_2D) ? k->lambda : 0.0;
    key.eps = k->eps > 0 ? k->eps : 0.0;
    key.general = k->general != 0 ? 1 : 0;
    for (int j = 0; j < d; ++j) {
        key.L[j] = L[j];
        key.N[j] = N[j];
    }
    std::string err;
    const Status st = s->runner->submit(key, rho, phi, ticket, &err, t_arrival);
    if (st != fsa::sched::ST_OK) {
        fsa::set_last_error(err.c_str());
        return (fsa_status)st;
    }
    return FSA_OK;
}

fsa_status fsa_server_submit(fsa_server s, const fsa_kernel* k, int d, const double* L,
                             const int64_t* N, fsa_precision p, const void* rho, void* phi,
                             uint64_t* ticket) {
    return fsa_server_submit_at(s, k, d, L, N, p, rho, phi, -1.0, ticket);
}

fsa_status fsa_server_clock(double* t) {
    if (!t) {
        fsa::set_last_error("fsa_server_clock: null argument");
        return FSA_EINVAL;
    }
    *t = steady_now();
    return FSA_OK;
}

fsa_status fsa_server_poll(fsa_server s, uint64_t ticket, int* done, fsa_status* result) {
    if (!s || !done) {
        fsa::set_last_error("fsa_server_poll: bad arguments");
        return FSA_EINVAL;
    }
    bool d = false;
    Status r = fsa::sched::ST_OK;
    if (s->sched->poll(ticket, &d, &r) != fsa::sched::ST_OK) {
        fsa::set_last_error("fsa_server_poll: unknown ticket");
        return FSA_EINVAL;
    }
    *done = d ? 1 : 0;
    if (d && result) *result = (fsa_status)r;
    return FSA_OK;
}

fsa_status fsa_server_wait_for(fsa_server s, uint64_t ticket, double timeout_ms, int* done,
                               fsa_status* result) {
    if (!s || !done) {
        fsa::set_last_error("fsa_server_wait: bad arguments");
        return FSA_EINVAL;
    }
    bool d = false;
    Status r = fsa::sched::ST_OK;
    if (s->runner->wait(ticket, timeout_ms < 0 ? -1.0 : timeout_ms * 1e-3, &d, &r) !=
        fsa::sched::ST_OK) {
        fsa::set_last_error("fsa_server_wait: unknown ticket");
        return FSA_EINVAL;
    }
    *done = d ? 1 : 0;
    if (d && result) *result = (fsa_status)r;
    return FSA_OK;
}

fsa_status fsa_server_wait(fsa_server s, uint64_t ticket, fsa_status* result) {
    int done = 0;
    return fsa_server_wait_for(s, ticket, -1.0, &done, result);
}

fsa_status fsa_server_cancel(fsa_server s, uint64_t ticket) {
    if (!s) {
        fsa::set_last_error("fsa_server_cancel: bad arguments");
        return FSA_EINVAL;
    }
    Status st = s->sched->cancel(ticket);
    if (st == fsa::sched::ST_ESTATE) {
        fsa::set_last_error("fsa_server_cancel: request already launched or finished");
        return FSA_ESTATE;
    }
    if (st != fsa::sched::ST_OK) {
        fsa::set_last_error("fsa_server_cancel: unknown ticket");
        return FSA_EINVAL;
    }
    s->runner->notify_done();
    return FSA_OK;
}

fsa_status fsa_server_stats(fsa_server s, fsa_stats* out) {
    if (!s || !out) {
        fsa::set_last_error("fsa_server_stats: bad arguments");
        return FSA_EINVAL;
    }
    fsa::sched::Stats st = s->sched->stats();
    out->p50_ms = st.p50_ms;
    out->p99_ms = st.p99_ms;
    out->throughput_rps = st.throughput_rps;
    out->gpts_per_s = st.gpts_per_s;
    out->done = st.done;
    out->rejected = st.rejected;
    out->cancelled = st.cancelled;
    out->cache_hits = st.cache_hits;
    out->cache_misses = st.cache_misses;
    out->hbm_in_use = st.hbm_in_use;
    out->hbm_peak = st.hbm_peak;
    out->timed_out = st.timed_out;
    return FSA_OK;
}

fsa_status fsa_server_set_queue_timeout(fsa_server s, double timeout_ms) {
    if (!s || !(timeout_ms == timeout_ms)) {
        fsa::set_last_error("fsa_server_set_queue_timeout: bad arguments");
        return FSA_EINVAL;
    }
    s->sched->set_queue_timeout(timeout_ms > 0 ? timeout_ms * 1e-3 : 0.0);
    s->runner->notify_done();  // waiters of requests that just timed out
    return FSA_OK;
}

fsa_status fsa_server_reset_stats(fsa_server s) {
    if (!s) {
        fsa::set_last_error("fsa_server_reset_stats: bad arguments");
        return FSA_EINVAL;
    }
    s->sched->reset_stats();
    return FSA_OK;
}

fsa_status fsa_server_destroy(fsa_server s) {
    if (!s) return FSA_OK;
    s->runner->shutdown();     // cancels the queue, lets in-flight work finish
    (void)hipDeviceSynchronize();
    s->runner.reset();
    s->sched.reset();  // destroys cached plans through the backend
    s->be.reset();
    delete s;
    return FSA_OK;
}

}  // extern "C"
