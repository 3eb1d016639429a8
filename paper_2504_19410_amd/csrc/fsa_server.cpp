// fsa_server.cpp -- the served variant: continuous batching of convolution
// requests on one GPU under an HBM budget (scheduling logic in fsa_sched.hpp).
//
// Device side of a request: on its slot's stream the request waits for its
// cached tensor's build event, runs the evaluation passes in the slot's
// resident workspace and records a completion event.  A slot's workspace is
// sized to the largest request it has run (grown, rarely, between requests,
// when the slot is idle), so the steady state allocates nothing.  Requests on different slots run concurrently on the device.  A
// server thread polls the in-flight events (time-stamping completions as it
// sees them) and admits queued requests.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "fsa_internal.hpp"
#include "fsa_sched.hpp"

namespace fsa {
void set_last_error(const char* msg);
}

namespace {

using fsa::sched::Key;
using fsa::sched::PlanInfo;
using fsa::sched::Request;
using fsa::sched::Scheduler;
using Status = fsa::sched::Status;

double steady_now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Completion {
    uint64_t ticket;
    Status status;
    double t_done;
};

class HipBackend : public fsa::sched::Backend {
public:
    HipBackend(int device, int n_streams) : device_(device) {
        for (int i = 0; i < n_streams; ++i) {
            hipStream_t s = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess)
                streams_.push_back(s);
        }
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
        out->tensor_bytes = tb + pl->tw_elems * pl->csize;  // tensor + twiddle tables
        out->workspace_bytes = wb + 256;                      // + alignment slack
        return fsa::sched::ST_OK;
    }

    Status build_plan(const PlanInfo& p, std::string* err) override {
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

    Status launch(const Request& r, const PlanInfo& p, int slot, std::string* err) override {
        hipStream_t st = streams_[(size_t)slot % streams_.size()];
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
        std::lock_guard<std::mutex> lk(c_mu_);
        inflight_.push_back(Inflight{r.ticket, done});
        return fsa::sched::ST_OK;
    }

    // Completed requests, in the order the server thread observed them.
    std::vector<Completion> take_completions() {
        std::vector<Completion> out;
        std::lock_guard<std::mutex> lk(c_mu_);
        for (size_t i = 0; i < inflight_.size();) {
            const hipError_t q = hipEventQuery(inflight_[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            out.push_back(Completion{inflight_[i].ticket,
                                     q == hipSuccess ? fsa::sched::ST_OK : fsa::sched::ST_EDEVICE,
                                     steady_now()});
            free_events_.push_back(inflight_[i].ev);
            inflight_[i] = inflight_.back();
            inflight_.pop_back();
        }
        return out;
    }
    bool any_inflight() {
        std::lock_guard<std::mutex> lk(c_mu_);
        return !inflight_.empty();
    }
    std::mutex c_mu_;
    std::condition_variable* wake = nullptr;

private:
    struct Inflight {
        uint64_t ticket;
        hipEvent_t ev;
    };
    hipEvent_t take_event() {
        {
            std::lock_guard<std::mutex> lk(c_mu_);
            if (!free_events_.empty()) {
                hipEvent_t e = free_events_.back();
                free_events_.pop_back();
                return e;
            }
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(c_mu_);
        all_events_.push_back(e);
        return e;
    }

    std::vector<Inflight> inflight_;
    std::vector<void*> slot_ws_;  // resident workspace per slot
    std::vector<size_t> slot_bytes_;
    std::vector<hipEvent_t> free_events_, all_events_;
    int device_;
    std::vector<hipStream_t> streams_;
    hipStream_t build_stream_ = nullptr;
    std::mutex ev_mu_;
    std::map<fsa_plan, hipEvent_t> built_;
};

}  // namespace

struct fsa_server_s {
    int device = 0;
    std::unique_ptr<HipBackend> be;
    std::unique_ptr<Scheduler> sched;
    std::thread worker;
    std::atomic<bool> stop{false};
    std::condition_variable wake;       // new submissions / completions (with be->c_mu_)
    std::mutex done_mu;                 // for waiters
    std::condition_variable done_cv;

    void run() {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Completion> done = be->take_completions();
            for (const Completion& c : done) sched->complete(c.ticket, c.status, c.t_done);
            if (!done.empty()) {
                std::lock_guard<std::mutex> lk(done_mu);
                done_cv.notify_all();
            }
            sched->pump();
            {
                std::lock_guard<std::mutex> lk(done_mu);
                done_cv.notify_all();  // requests finished at admission (errors)
            }
            if (stop.load() && sched->idle()) break;
            if (be->any_inflight()) {
                // completions are observed by polling: spin (yielding) while
                // work is in flight; a timed sleep would add the kernel's
                // timer slack (tens of microseconds) to every latency
                std::this_thread::yield();
                continue;
            }
            std::unique_lock<std::mutex> lk(be->c_mu_);
            wake.wait_for(lk, std::chrono::microseconds(500));
        }
    }
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
    s->be->wake = &s->wake;
    s->sched = std::make_unique<Scheduler>(s->be.get(), hbm_budget_bytes, max_inflight);
    fsa_server_s* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    *out = s.release();
    return FSA_OK;
}

fsa_status fsa_server_submit(fsa_server s, const fsa_kernel* k, int d, const double* L,
                             const int64_t* N, fsa_precision p, const void* rho, void* phi,
                             uint64_t* ticket) {
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
    Status st = s->sched->submit(key, rho, phi, ticket, &err);
    if (st != fsa::sched::ST_OK) {
        fsa::set_last_error(err.c_str());
        return (fsa_status)st;
    }
    {
        std::lock_guard<std::mutex> lk(s->be->c_mu_);
        s->wake.notify_all();
    }
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

fsa_status fsa_server_wait(fsa_server s, uint64_t ticket, fsa_status* result) {
    if (!s) {
        fsa::set_last_error("fsa_server_wait: bad arguments");
        return FSA_EINVAL;
    }
    for (;;) {
        bool d = false;
        Status r = fsa::sched::ST_OK;
        if (s->sched->poll(ticket, &d, &r) != fsa::sched::ST_OK) {
            fsa::set_last_error("fsa_server_wait: unknown ticket");
            return FSA_EINVAL;
        }
        if (d) {
            if (result) *result = (fsa_status)r;
            return FSA_OK;
        }
        std::unique_lock<std::mutex> lk(s->done_mu);
        s->done_cv.wait_for(lk, std::chrono::microseconds(500));
    }
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
    std::lock_guard<std::mutex> lk(s->done_mu);
    s->done_cv.notify_all();
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
    s->sched->cancel_all();
    s->stop.store(true);
    {
        std::lock_guard<std::mutex> lk(s->be->c_mu_);
        s->wake.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipDeviceSynchronize();
    s->sched.reset();  // destroys cached plans through the backend
    s->be.reset();
    delete s;
    return FSA_OK;
}

}  // extern "C"
