// fsa_batch.cpp -- batched evaluation of independent problems.
//
// A batch of n problems (any mix of kernels, boxes, grid shapes and
// precisions) runs as a hipGraph of persistent launches: for every pass
// (A, B, C, D, E, in dependency order) and every transform length used by
// that pass, ONE launch walks the work items of all problems that share the
// length, through a device table of per-problem jobs.  Kernel boundaries
// order the passes, so no cross-workgroup synchronisation (and no multi-XCD
// L2 write-back/invalidate traffic) is needed inside a launch.  Each item
// runs exactly the code of the single-problem path, so a batched result is
// bitwise equal to fsa_apply on that problem alone.
//
// The graph (and the device job tables it reads) is built on the first call
// with a given signature -- plans, device pointers, workspace, and the
// generation of the tuning table whose launch choices it snapshots -- and
// replayed on later calls.
//
// A group's launch choice is the tuning table's batched entry for the
// group's total number of transforms (the single-evaluation entries where
// there is none): a launch over a job table of many problems is another
// kernel instantiation than the single-problem launch, and a large batch
// reaches size classes no single problem does.  fsa_autotune_batched times
// every candidate of every group launch of a batch and stores the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fsa_internal.hpp"

namespace fsa {
void set_last_error(const char* msg);
}  // namespace fsa

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Lengths the pass kernels are compiled for.
bool fft_length_ok(fsa::Pass pass, int len) {
    if (!fsa::fft_length_supported(len)) return false;
    if (pass == fsa::Pass::R2C || pass == fsa::Pass::C2R) return len >= 8 && len <= 2048;
    return len >= 16 && len <= 4096;
}

struct Group {
    fsa::Pass pass;
    int len;
    fsa_precision prec;
    const void* tw = nullptr;   // twiddles of length len (any member plan's table)
    const void* tw2 = nullptr;  // second table of the real transforms (length 2 len)
    fsa::Choice ch;             // launch choice, fixed when the groups are complete
    long lines = 0;             // transforms of all member jobs (the size class)
    std::vector<unsigned char> jobs;  // packed job structs
    std::vector<int> start{0};
    size_t job_size = 0;
    int n = 0;
};

struct Entry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* tables = nullptr;
    std::vector<uint64_t> plan_ids;
    int launches = 0;
    ~Entry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (tables) (void)hipFree(tables);
    }
};

std::mutex g_mu;
// most recently used last; deliberately never destroyed, so that no HIP call
// runs from static destructors after the runtime has shut down
std::vector<std::unique_ptr<Entry>>& g_cache = *new std::vector<std::unique_ptr<Entry>>();
constexpr size_t kCacheCap = 16;

// Adds one problem's job to its (pass, length, precision) group.  Returns
// false for an unsupported length.
template <class Job>
bool add_job(std::map<std::tuple<int, int, int>, Group>& groups, fsa::Pass pass, int len,
             fsa_precision prec, const void* tw, const void* tw2, const Job& job, long lines) {
    if (!fft_length_ok(pass, len)) return false;
    Group& g = groups[std::make_tuple((int)pass, len, (int)prec)];
    if (g.n == 0) {
        g.pass = pass;
        g.len = len;
        g.prec = prec;
        g.tw = tw;
        g.tw2 = tw2;
        g.job_size = sizeof(Job);
    }
    const unsigned char* p = (const unsigned char*)&job;
    g.jobs.insert(g.jobs.end(), p, p + sizeof(Job));
    g.lines += lines;
    ++g.n;
    return true;
}

// Fixes a group's launch choice and the item prefix its jobs follow under
// that choice.
template <class Job>
void finish_group_as(Group& g, fsa::Choice c) {
    g.ch = c;
    g.start.assign(1, 0);
    for (int i = 0; i < g.n; ++i) {
        Job job;
        std::memcpy(&job, g.jobs.data() + (size_t)i * sizeof(Job), sizeof(Job));
        const int items = g.prec == FSA_F32 ? fsa::Launch<float>::items(g.pass, g.len, &job, g.ch)
                                            : fsa::Launch<double>::items(g.pass, g.len, &job, g.ch);
        g.start.push_back(g.start.back() + items);
    }
}

void finish_group(Group& g, fsa::Choice c) {
    switch (g.pass) {
    case fsa::Pass::R2C: finish_group_as<fsa::JobR2c>(g, c); break;
    case fsa::Pass::C2R: finish_group_as<fsa::JobC2r>(g, c); break;
    case fsa::Pass::FWD_T:
    case fsa::Pass::INV_T: finish_group_as<fsa::JobT>(g, c); break;
    case fsa::Pass::CONV: finish_group_as<fsa::JobConv>(g, c); break;
    }
}

// Device bytes of a group's tables: [jobs | start], each 256-byte aligned.
size_t table_bytes(const Group& g) {
    return align256(g.jobs.size()) + align256(g.start.size() * sizeof(int));
}

hipError_t upload_tables(const Group& g, char* dst) {
    hipError_t e = hipMemcpy(dst, g.jobs.data(), g.jobs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(dst + align256(g.jobs.size()), g.start.data(),
                      g.start.size() * sizeof(int), hipMemcpyHostToDevice);
    return e;
}

// The group's persistent launch over tables at `tables` (laid out as
// upload_tables writes them).
hipError_t launch_group(const Group& g, const char* tables, hipStream_t st) {
    const int* start = (const int*)(tables + align256(g.jobs.size()));
    const int total = g.start.back();
    return g.prec == FSA_F32 ? fsa::Launch<float>::batch(g.pass, g.len, tables, start, g.n, total,
                                                         g.tw, g.tw2, g.ch, st)
                             : fsa::Launch<double>::batch(g.pass, g.len, tables, start, g.n,
                                                          total, g.tw, g.tw2, g.ch, st);
}

using Groups = std::map<std::tuple<int, int, int>, Group>;

// Sorts the problems' jobs into (pass, length, precision) groups; the
// launch choices are not fixed yet.
fsa_status make_groups(int n, const fsa_plan* plans, const void* const* rho, void* const* phi,
                       char* ws, Groups& groups) {
    for (int i = 0; i < n; ++i) {
        const fsa_plan_s* pl = plans[i];
        const size_t cs = pl->csize;
        const char* tw = (const char*)pl->twiddles;
        const void* tw_p0 = tw + pl->tw_off_p0 * cs;
        const void* tw_p1 = tw + pl->tw_off_p1 * cs;
        const void* tw_m = tw + pl->tw_off_m * cs;
        const void* tw_pl = tw + pl->tw_off_pl * cs;
        const int N0 = (int)pl->N[0], N1 = (int)pl->N[1], H = (int)pl->H;
        char* w1 = ws;
        char* w2 = w1 + align256(pl->ws1_elems * cs);
        ws += align256(pl->ws_bytes);
        const fsa_precision pr = pl->prec;
        auto add = [&](auto job, fsa::Pass pass, int len, const void* t1, const void* t2,
                       long lines) { return add_job(groups, pass, len, pr, t1, t2, job, lines); };
        const long n0 = N0, n1 = N1, h = H;
        bool ok;
        if (pl->d == 3) {
            const int N2 = (int)pl->N[2];
            ok = add(fsa::JobR2c{rho[i], w1, N0, N1}, fsa::Pass::R2C, N2, tw_m, tw_pl, n0 * n1) &&
                 add(fsa::JobT{w1, w2, N0, H, 0, H}, fsa::Pass::FWD_T, 2 * N1, tw_p1, nullptr,
                     n0 * h) &&
                 add(fsa::JobConv{w2, pl->tensor, H * 2 * N1, 2 * N1, N1, 0}, fsa::Pass::CONV,
                     2 * N0, tw_p0, nullptr, h * 2 * n1) &&
                 add(fsa::JobT{w2, w1, N0, H, 0, H}, fsa::Pass::INV_T, 2 * N1, tw_p1, nullptr,
                     n0 * h) &&
                 add(fsa::JobC2r{w1, phi[i], N0, N1}, fsa::Pass::C2R, N2, tw_m, tw_pl, n0 * n1);
        } else {
            ok = add(fsa::JobR2c{rho[i], w1, 1, N0}, fsa::Pass::R2C, N1, tw_m, tw_pl, n0) &&
                 add(fsa::JobConv{w1, pl->tensor, H, 1, 0, 0}, fsa::Pass::CONV, 2 * N0, tw_p0,
                     nullptr, h) &&
                 add(fsa::JobC2r{w1, phi[i], 1, N0}, fsa::Pass::C2R, N1, tw_m, tw_pl, n0);
        }
        if (!ok) {
            fsa::set_last_error("unsupported transform length in a batch");
            return FSA_EUNSUPPORTED;
        }
    }
    return FSA_OK;
}

fsa_status build_entry(int n, const fsa_plan* plans, const void* const* rho, void* const* phi,
                       char* ws, Entry& e) {
    Groups groups;
    fsa_status st = make_groups(n, plans, rho, phi, ws, groups);
    if (st != FSA_OK) return st;
    for (auto& kv : groups) {
        Group& g = kv.second;
        finish_group(g, fsa::tune::get(g.prec, g.pass, g.len, g.lines, true));
    }
    // one device buffer: per group [jobs | start], each part 256-byte aligned
    size_t bytes = 0;
    std::vector<size_t> offs;
    for (auto& kv : groups) {
        offs.push_back(bytes);
        bytes += table_bytes(kv.second);
    }
    std::vector<unsigned char> host(bytes, 0);
    size_t gi = 0;
    for (auto& kv : groups) {
        const Group& g = kv.second;
        std::memcpy(host.data() + offs[gi], g.jobs.data(), g.jobs.size());
        std::memcpy(host.data() + offs[gi] + align256(g.jobs.size()), g.start.data(),
                    g.start.size() * sizeof(int));
        ++gi;
    }
    hipError_t err = hipMalloc(&e.tables, bytes > 0 ? bytes : 256);
    if (err != hipSuccess) {
        e.tables = nullptr;
        fsa::set_last_error("fsa_apply_batched: job table allocation failed");
        return FSA_ENOMEM;
    }
    err = hipMemcpy(e.tables, host.data(), bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        fsa::set_last_error(hipGetErrorString(err));
        return FSA_EDEVICE;
    }
    // capture the stage-ordered launches on a private stream
    fsa::Range range("fsa_apply_batched capture");
    hipStream_t cap = nullptr;
    err = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (err != hipSuccess) {
        fsa::set_last_error(hipGetErrorString(err));
        return FSA_EDEVICE;
    }
    err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t lerr = hipSuccess;
    if (err == hipSuccess) {
        for (int stage = 0; stage <= (int)fsa::Pass::C2R; ++stage) {
            gi = 0;
            for (auto& kv : groups) {
                const Group& g = kv.second;
                const size_t off = offs[gi++];
                if ((int)g.pass != stage || lerr != hipSuccess) continue;
                lerr = launch_group(g, (const char*)e.tables + off, cap);
                ++e.launches;
            }
        }
        hipError_t cerr = hipStreamEndCapture(cap, &e.graph);
        if (err == hipSuccess) err = cerr;
    }
    if (err == hipSuccess) err = lerr;
    if (err == hipSuccess) err = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (err != hipSuccess) {
        fsa::set_last_error(hipGetErrorString(err));
        return FSA_EDEVICE;
    }
    return FSA_OK;
}

// Argument checks shared by the batched entry points (`fn` names the caller
// in the error message); on success *dev is the current device.
fsa_status check_batch(const char* fn, int n, const fsa_plan* plans, const void* const* rho,
                       void* const* phi, const void* workspace, size_t workspace_bytes,
                       int* dev) {
    size_t need = 0;
    fsa_status s = fsa_batch_workspace_bytes(n, plans, &need);
    if (s != FSA_OK) return s;
    if (n == 0) return FSA_OK;
    const std::string f(fn);
    if (!rho || !phi || !workspace) {
        fsa::set_last_error((f + ": null array").c_str());
        return FSA_EINVAL;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        fsa::set_last_error((f + ": workspace must be 256-byte aligned").c_str());
        return FSA_EINVAL;
    }
    if (workspace_bytes < need) {
        fsa::set_last_error((f + ": workspace too small").c_str());
        return FSA_EINVAL;
    }
    if (hipGetDevice(dev) != hipSuccess) {
        fsa::set_last_error((f + ": hipGetDevice failed").c_str());
        return FSA_EDEVICE;
    }
    for (int i = 0; i < n; ++i) {
        if (!rho[i] || !phi[i]) {
            fsa::set_last_error((f + ": null device pointer").c_str());
            return FSA_EINVAL;
        }
        if (!plans[i]->built || plans[i]->device != *dev) {
            fsa::set_last_error((f + ": a plan is not built on the current device").c_str());
            return FSA_ESTATE;
        }
        if (plans[i]->prec == FSA_DD) {
            fsa::set_last_error(
                (f + ": double-double plans are not batched (use fsa_apply)").c_str());
            return FSA_EUNSUPPORTED;
        }
        if (plans[i]->n_spectral) {
            fsa::set_last_error(
                (f + ": dipole-dipole plans are not batched (use fsa_apply)").c_str());
            return FSA_EUNSUPPORTED;
        }
    }
    return FSA_OK;
}

}  // namespace

namespace fsa {
// Drops cached batch graphs that reference a plan (called when it is destroyed).
void batch_forget_plan(uint64_t plan_id) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.erase(std::remove_if(g_cache.begin(), g_cache.end(),
                                 [&](const std::unique_ptr<Entry>& e) {
                                     return std::find(e->plan_ids.begin(), e->plan_ids.end(),
                                                      plan_id) != e->plan_ids.end();
                                 }),
                  g_cache.end());
}
}  // namespace fsa

extern "C" {

fsa_status fsa_batch_workspace_bytes(int n, const fsa_plan* plans, size_t* bytes) {
    if (n < 0 || (n > 0 && !plans) || !bytes) {
        fsa::set_last_error("fsa_batch_workspace_bytes: bad arguments");
        return FSA_EINVAL;
    }
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) {
            fsa::set_last_error("fsa_batch_workspace_bytes: null plan");
            return FSA_EINVAL;
        }
        total += align256(plans[i]->ws_bytes);
    }
    *bytes = total;
    return FSA_OK;
}

fsa_status fsa_apply_batched(int n, const fsa_plan* plans, const void* const* rho,
                             void* const* phi, void* workspace, size_t workspace_bytes,
                             void* stream) {
    fsa::Range range("fsa_apply_batched");
    int dev = 0;
    fsa_status s = check_batch("fsa_apply_batched", n, plans, rho, phi, workspace,
                               workspace_bytes, &dev);
    if (s != FSA_OK || n == 0) return s;
    std::vector<uint64_t> key;
    key.reserve(3 * (size_t)n + 3);
    key.push_back((uint64_t)dev);
    key.push_back((uint64_t)(uintptr_t)workspace);
    key.push_back((uint64_t)n);
    for (int i = 0; i < n; ++i) {
        key.push_back(plans[i]->id);
        key.push_back((uint64_t)(uintptr_t)rho[i]);
        key.push_back((uint64_t)(uintptr_t)phi[i]);
    }
    key.push_back(fsa::tune::generation());
    std::lock_guard<std::mutex> lk(g_mu);
    Entry* hit = nullptr;
    for (size_t i = 0; i < g_cache.size(); ++i) {
        if (g_cache[i]->key == key) {
            std::unique_ptr<Entry> e = std::move(g_cache[i]);
            g_cache.erase(g_cache.begin() + (long)i);
            g_cache.push_back(std::move(e));
            hit = g_cache.back().get();
            break;
        }
    }
    if (!hit) {
        auto e = std::make_unique<Entry>();
        e->key = key;
        for (int i = 0; i < n; ++i) e->plan_ids.push_back(plans[i]->id);
        s = build_entry(n, plans, rho, phi, (char*)workspace, *e);
        if (s != FSA_OK) return s;
        if (g_cache.size() >= kCacheCap) g_cache.erase(g_cache.begin());
        g_cache.push_back(std::move(e));
        hit = g_cache.back().get();
    }
    fsa::Range replay("fsa_apply_batched replay");
    hipError_t err = hipGraphLaunch(hit->exec, (hipStream_t)stream);
    if (err != hipSuccess) {
        fsa::set_last_error(hipGetErrorString(err));
        return FSA_EDEVICE;
    }
    return FSA_OK;
}

fsa_status fsa_batch_launches(int n, const fsa_plan* plans, const void* const* rho,
                              void* const* phi, void* workspace, int* launches) {
    if (!launches) return FSA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    // most recent first: an older entry may hold the same batch under an
    // earlier tuning generation
    for (auto it = g_cache.rbegin(); it != g_cache.rend(); ++it) {
        const auto& e = *it;
        if ((int)e->key[2] == n && e->key[1] == (uint64_t)(uintptr_t)workspace) {
            bool same = true;
            for (int i = 0; i < n && same; ++i)
                same = e->key[3 + 3 * i] == plans[i]->id &&
                       e->key[4 + 3 * i] == (uint64_t)(uintptr_t)rho[i] &&
                       e->key[5 + 3 * i] == (uint64_t)(uintptr_t)phi[i];
            if (same) {
                *launches = e->launches;
                return FSA_OK;
            }
        }
    }
    fsa::set_last_error("fsa_batch_launches: no captured graph for this batch");
    return FSA_ESTATE;
}

fsa_status fsa_autotune_batched(int n, const fsa_plan* plans, const void* const* rho,
                                void* const* phi, void* workspace, size_t workspace_bytes,
                                void* stream, int reps) {
    int dev = 0;
    fsa_status s = check_batch("fsa_autotune_batched", n, plans, rho, phi, workspace,
                               workspace_bytes, &dev);
    if (s != FSA_OK) return s;
    if (reps < 1 || reps > 1000) {
        fsa::set_last_error("fsa_autotune_batched: reps must be 1..1000");
        return FSA_EINVAL;
    }
    if (n == 0) return FSA_OK;
    Groups groups;
    s = make_groups(n, plans, rho, phi, (char*)workspace, groups);
    if (s != FSA_OK) return s;
    // every group's tables under its current choice (`fixed`), and room for
    // one group's tables under a candidate (`trial`); the start prefix is
    // the only part that depends on the choice, and it has n + 1 entries
    std::vector<Group*> order;
    for (int stage = 0; stage <= (int)fsa::Pass::C2R; ++stage)
        for (auto& kv : groups)
            if ((int)kv.second.pass == stage) order.push_back(&kv.second);
    size_t fixed_bytes = 0, trial_bytes = 0;
    std::vector<size_t> offs;
    for (Group* g : order) {
        finish_group(*g, fsa::tune::get(g->prec, g->pass, g->len, g->lines, true));
        offs.push_back(fixed_bytes);
        fixed_bytes += table_bytes(*g);
        trial_bytes = std::max(trial_bytes, table_bytes(*g));
    }
    char* dbuf = nullptr;
    // one trial slot per candidate of a group (at most two per variant)
    constexpr int kMaxCands = 2 * fsa::kNumVariants;
    if (hipMalloc((void**)&dbuf, fixed_bytes + kMaxCands * trial_bytes) != hipSuccess) {
        fsa::set_last_error("fsa_autotune_batched: table allocation failed");
        return FSA_ENOMEM;
    }
    char* trial = dbuf + fixed_bytes;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // timing events without the system-scope fence of a default event, whose
    // cache write-back and invalidation would give the timed launch a cold L2
    hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableSystemFence);
    for (size_t i = 0; i < order.size() && e == hipSuccess; ++i)
        e = upload_tables(*order[i], dbuf + offs[i]);
    // launches of every group of the passes before `stage`, with the fixed
    // choices: one evaluation up to that pass
    auto run_before = [&](int stage) {
        hipError_t r = hipSuccess;
        for (size_t i = 0; i < order.size() && r == hipSuccess; ++i)
            if ((int)order[i]->pass < stage) r = launch_group(*order[i], dbuf + offs[i], st);
        return r;
    };
    // fill every buffer with data once
    if (e == hipSuccess) e = run_before((int)fsa::Pass::C2R + 1);
    for (size_t gi = 0; gi < order.size() && e == hipSuccess; ++gi) {
        Group& g = *order[gi];
        const fsa::Choice current = g.ch;
        int mask = 0;
        if (fsa_tune_variants((int)g.prec, (int)g.pass, g.len, &mask) != FSA_OK) mask = 1;
        std::vector<fsa::Choice> cands;
        for (int v = 0; v < fsa::kNumVariants; ++v) {
            if (!(mask >> v & 1)) continue;
            const int mo = g.prec == FSA_F32 ? fsa::Launch<float>::max_occ(g.pass, g.len, v)
                                             : fsa::Launch<double>::max_occ(g.pass, g.len, v);
            cands.push_back(fsa::Choice{v, 0});
            if (mo >= 2) cands.push_back(fsa::Choice{v, mo / 2});
        }
        // every candidate's tables in its own trial slot, then `reps` rounds
        // that run each candidate once (after a warm-up round), so slow drifts
        // fall on all of them alike; median per candidate.  Each run is a
        // whole evaluation of the batch with this group's launch replaced by
        // the candidate and timed alone: the launches before it leave the
        // caches as a replay of the batch does (a group timed on its own,
        // over and over, found its input in the Infinity Cache and favoured
        // the variants that gain from that).
        const int nc = (int)cands.size();
        std::vector<Group> trials((size_t)nc, g);
        for (int c = 0; c < nc && e == hipSuccess; ++c) {
            finish_group(trials[(size_t)c], cands[(size_t)c]);
            e = upload_tables(trials[(size_t)c], trial + (size_t)c * trial_bytes);
        }
        std::vector<std::vector<float>> ms((size_t)nc);
        for (int i = -1; i < reps && e == hipSuccess; ++i) {
            for (int c = 0; c < nc && e == hipSuccess; ++c) {
                for (size_t oi = 0; oi < order.size() && e == hipSuccess; ++oi) {
                    if (oi != gi) {
                        e = launch_group(*order[oi], dbuf + offs[oi], st);
                        continue;
                    }
                    e = hipEventRecord(ev[0], st);
                    if (e == hipSuccess)
                        e = launch_group(trials[(size_t)c], trial + (size_t)c * trial_bytes, st);
                    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
                }
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float t = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
                if (e == hipSuccess && i >= 0) ms[(size_t)c].push_back(t);
            }
        }
        if (e != hipSuccess) break;
        double best = 1e300;
        fsa::Choice best_c = current;
        for (int c = 0; c < nc; ++c) {
            std::sort(ms[(size_t)c].begin(), ms[(size_t)c].end());
            const double us = 1e3 * ms[(size_t)c][ms[(size_t)c].size() / 2];
            if (us < best) {
                best = us;
                best_c = cands[(size_t)c];
            }
        }
        finish_group(g, best_c);
        e = upload_tables(g, dbuf + offs[gi]);
        fsa::tune::set(g.prec, g.pass, g.len, g.lines, best_c, best, true);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(dbuf);
    if (e != hipSuccess) {
        fsa::set_last_error((std::string("fsa_autotune_batched: ") + hipGetErrorString(e)).c_str());
        return FSA_EDEVICE;
    }
    // leave the outputs holding a valid evaluation under the tuned choices
    return fsa_apply_batched(n, plans, rho, phi, workspace, workspace_bytes, stream);
}

}  // extern "C"
