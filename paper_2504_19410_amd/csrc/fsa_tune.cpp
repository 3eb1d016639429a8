// fsa_tune.cpp -- the autotuner and its table of launch choices.
//
// Every pass kernel is compiled in up to five variants per transform length
// (default; alternate radix family, i.e. another radix split and number of
// threads per transform; half-size workgroups, i.e. fewer lines per tile or
// teams per group; exchanges across lanes; first stage on the matrix cores).
// At run time the persistent grid can also use fewer resident workgroups per
// CU than fit.  fsa_autotune times every distinct (variant, occupancy)
// candidate of every pass of a plan on the device with hipEvents, each inside
// a whole evaluation, and keeps the fastest per (precision, pass, length) in a
// process-wide table; for a 3D grid it then times the schedule, i.e. how many
// slabs of bins p2 the middle passes B, C, D are run in (B, C, D of one slab
// back to back, so the slab's spectrum can stay in the memory-side cache
// between them), and keeps the fastest per (precision, grid).  fsa_apply,
// fsa_apply_batched and the server read the tables at launch time.  They can
// be saved to and loaded from a JSON file, and are loaded on first use from
// the file named by the environment variable FSA_TUNE_CACHE when that is set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fsa_internal.hpp"

namespace fsa {
void set_last_error(const char* msg);
}

namespace {

struct TuneEntry {
    fsa::Choice ch;
    double us = 0.0;  // measured time of the chosen candidate (0: set by hand)
};

// precision, pass (| FSA_PASS_BATCHED for the batched launches), length,
// size class
using Key = std::tuple<int, int, int, int>;
using GridKey = std::tuple<int, int64_t, int64_t, int64_t>;  // precision, N0, N1, N2

struct SlabEntry {
    int slabs = 1;
    double us = 0.0;
};

std::mutex g_mu;
std::map<Key, TuneEntry>& g_table = *new std::map<Key, TuneEntry>();
std::map<GridKey, SlabEntry>& g_slabs = *new std::map<GridKey, SlabEntry>();
std::atomic<uint64_t> g_generation{1};
std::once_flag g_env_once;

const char* const kPassNames[5] = {"r2c", "fwd_t", "conv", "inv_t", "c2r"};
const char* const kBatchedPrefix = "batched_";

std::string pass_name(int pass) {
    return std::string((pass & FSA_PASS_BATCHED) ? kBatchedPrefix : "") +
           kPassNames[pass & ~FSA_PASS_BATCHED];
}

int pass_from_name(const std::string& name) {
    std::string base = name;
    int flag = 0;
    const std::string pre(kBatchedPrefix);
    if (base.compare(0, pre.size(), pre) == 0) {
        base = base.substr(pre.size());
        flag = FSA_PASS_BATCHED;
    }
    for (int k = 0; k < 5; ++k)
        if (base == kPassNames[k]) return k | flag;
    return -1;
}

fsa_status fail(fsa_status s, const std::string& msg) {
    fsa::set_last_error(msg.c_str());
    return s;
}

// A pass of fsa_pass, optionally with the FSA_PASS_BATCHED flag.
bool pass_ok(int pass) {
    const int base = pass & ~FSA_PASS_BATCHED;
    return base >= 0 && base <= (int)fsa::Pass::C2R;
}

// Transform lengths the passes support: the real passes take the half
// length M of the padded row, the complex passes the padded length P.
bool length_ok(int pass, int len) {
    pass &= ~FSA_PASS_BATCHED;
    if (!fsa::fft_length_supported(len)) return false;
    if (pass == (int)fsa::Pass::R2C || pass == (int)fsa::Pass::C2R) return len >= 8 && len <= 2048;
    return len >= 16 && len <= 4096;
}

bool variant_ok(fsa_precision prec, int pass, int len, int var) {
    pass &= ~FSA_PASS_BATCHED;
    if (var < 0 || var >= fsa::kNumVariants) return false;
    return prec == FSA_F32 ? fsa::Launch<float>::distinct((fsa::Pass)pass, len, var)
                           : fsa::Launch<double>::distinct((fsa::Pass)pass, len, var);
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    return std::string(prop.gcnArchName);
}

// --- a small reader for the flat JSON the saver writes ----------------------

struct Reader {
    const std::string& s;
    size_t i = 0;
    explicit Reader(const std::string& text) : s(text) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\') return false;  // the saver never escapes
            out.push_back(s[i++]);
        }
        if (i >= s.size()) return false;
        ++i;
        return true;
    }
    bool num(double& out) {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        out = std::strtod(b, &e);
        if (e == b) return false;
        i += (size_t)(e - b);
        return true;
    }
};

struct Parsed {
    std::string format, arch;
    struct Row {
        std::string prec, pass;
        double len = -1, var = -1, occ = -1, us = 0;
        double cls = -1;
        double slabs = -1;
        std::vector<double> grid;
    };
    std::vector<Row> rows;   // "entries"
    std::vector<Row> sched;  // "schedules"
};

bool parse_row(Reader& r, Parsed::Row& row) {
    if (!r.eat('{')) return false;
    if (r.eat('}')) return true;
    do {
        std::string k;
        if (!r.str(k) || !r.eat(':')) return false;
        if (k == "precision" || k == "pass") {
            std::string v;
            if (!r.str(v)) return false;
            (k == "precision" ? row.prec : row.pass) = v;
        } else if (k == "grid") {
            if (!r.eat('[')) return false;
            do {
                double v;
                if (!r.num(v)) return false;
                row.grid.push_back(v);
            } while (r.eat(','));
            if (!r.eat(']')) return false;
        } else {
            double v;
            if (!r.num(v)) return false;
            if (k == "length") row.len = v;
            else if (k == "variant") row.var = v;
            else if (k == "occupancy") row.occ = v;
            else if (k == "us") row.us = v;
            else if (k == "class") row.cls = v;
            else if (k == "slabs") row.slabs = v;
            else return false;
        }
    } while (r.eat(','));
    return r.eat('}');
}

bool parse(const std::string& text, Parsed& out) {
    Reader r(text);
    if (!r.eat('{')) return false;
    if (r.eat('}')) return true;
    do {
        std::string k;
        if (!r.str(k) || !r.eat(':')) return false;
        if (k == "format" || k == "arch") {
            std::string v;
            if (!r.str(v)) return false;
            (k == "format" ? out.format : out.arch) = v;
        } else if (k == "entries" || k == "schedules") {
            auto& dst = k == "entries" ? out.rows : out.sched;
            if (!r.eat('[')) return false;
            if (!r.eat(']')) {
                do {
                    Parsed::Row row;
                    if (!parse_row(r, row)) return false;
                    dst.push_back(row);
                } while (r.eat(','));
                if (!r.eat(']')) return false;
            }
        } else {
            return false;
        }
    } while (r.eat(','));
    if (!r.eat('}')) return false;
    r.ws();
    return r.i == text.size();
}

fsa_status load_file(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(FSA_EINVAL, std::string("fsa_tune_load: cannot open ") + path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    Parsed p;
    if (!parse(text, p)) return fail(FSA_EINVAL, std::string("fsa_tune_load: malformed ") + path);
    if (p.format != "fsa-tune-1")
        return fail(FSA_EINVAL, "fsa_tune_load: unknown format '" + p.format + "'");
    const std::string arch = device_arch();
    if (!arch.empty() && p.arch != arch)
        return fail(FSA_EINVAL, "fsa_tune_load: table was tuned on '" + p.arch +
                                    "', this device is '" + arch + "'");
    std::map<Key, TuneEntry> fresh;
    auto small_int = [](double v) { return v >= 0.0 && v <= 1e6 && v == (double)(int)v; };
    for (const auto& row : p.rows) {
        int prec = row.prec == "f32" ? FSA_F32 : row.prec == "f64" ? FSA_F64 : -1;
        const int pass = pass_from_name(row.pass);
        const bool ints = small_int(row.len) && small_int(row.var) && small_int(row.occ) &&
                          small_int(row.cls) && row.cls <= 62;
        const int len = ints ? (int)row.len : -1, var = ints ? (int)row.var : -1;
        const int occ = ints ? (int)row.occ : -1;
        if (prec < 0 || pass < 0 || !ints || !length_ok(pass, len) ||
            !variant_ok((fsa_precision)prec, pass, len, var))
            return fail(FSA_EINVAL, "fsa_tune_load: invalid entry (" + row.prec + ", " +
                                        row.pass + ", " + std::to_string(len) + ")");
        fresh[Key(prec, pass, len, (int)row.cls)] = TuneEntry{fsa::Choice{var, occ}, row.us};
    }
    std::map<GridKey, SlabEntry> fresh_slabs;
    for (const auto& row : p.sched) {
        const int prec = row.prec == "f32" ? FSA_F32 : row.prec == "f64" ? FSA_F64 : -1;
        bool ok = prec >= 0 && row.grid.size() == 3 && small_int(row.slabs) && row.slabs >= 1 &&
                  row.slabs <= fsa::kMaxSlabs;
        for (double g : row.grid) ok = ok && small_int(g) && fsa::grid_length_supported((int64_t)g);
        if (!ok)
            return fail(FSA_EINVAL, "fsa_tune_load: invalid schedule entry (" + row.prec + ")");
        fresh_slabs[GridKey(prec, (int64_t)row.grid[0], (int64_t)row.grid[1],
                            (int64_t)row.grid[2])] = SlabEntry{(int)row.slabs, row.us};
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto& kv : fresh) g_table[kv.first] = kv.second;
        for (const auto& kv : fresh_slabs) g_slabs[kv.first] = kv.second;
    }
    ++g_generation;
    return FSA_OK;
}

void load_env_once() {
    std::call_once(g_env_once, [] {
        const char* path = std::getenv("FSA_TUNE_CACHE");
        if (!path || !*path) return;
        FILE* f = std::fopen(path, "rb");
        if (!f) return;  // not written yet: defaults until someone saves one
        std::fclose(f);
        if (load_file(path) != FSA_OK)
            std::fprintf(stderr, "fsa: ignoring FSA_TUNE_CACHE=%s\n", path);
    });
}

}  // namespace

namespace fsa {
namespace tune {

int size_class(long lines) {
    int c = 0;
    while (c < 62 && (2L << c) <= lines) ++c;
    return c;
}

namespace {
// The entry of the nearest class among the entries of (prec, key_pass, len);
// false if there is none.  Caller holds g_mu.
bool nearest(int prec, int key_pass, int len, int cls, Choice* out) {
    // entries of (prec, pass, len) are adjacent in the map, ordered by class
    auto lo = g_table.lower_bound(Key(prec, key_pass, len, 0));
    int dist = 1 << 30;
    for (auto it = lo; it != g_table.end(); ++it) {
        if (std::get<0>(it->first) != prec || std::get<1>(it->first) != key_pass ||
            std::get<2>(it->first) != len)
            break;
        const int d = std::abs(std::get<3>(it->first) - cls);
        if (d < dist) {
            dist = d;
            *out = it->second.ch;
        }
    }
    return dist != (1 << 30);
}
}  // namespace

Choice get(fsa_precision prec, Pass pass, int len, long lines, bool batched) {
    load_env_once();
    const int cls = size_class(lines);
    std::lock_guard<std::mutex> lk(g_mu);
    Choice best;
    // a batched launch prefers the batched entries, then the single ones
    if (batched && nearest((int)prec, (int)pass | FSA_PASS_BATCHED, len, cls, &best)) return best;
    nearest((int)prec, (int)pass, len, cls, &best);
    return best;
}

void set(fsa_precision prec, Pass pass, int len, long lines, Choice c, double us, bool batched) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const int kp = (int)pass | (batched ? FSA_PASS_BATCHED : 0);
        g_table[Key((int)prec, kp, len, size_class(lines))] = TuneEntry{c, us};
    }
    ++g_generation;
}

uint64_t generation() { return g_generation.load(); }

int get_slabs(const fsa_plan_s* pl) {
    if (pl->d != 3) return 1;
    load_env_once();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_slabs.find(GridKey((int)pl->prec, pl->N[0], pl->N[1], pl->N[2]));
    return it == g_slabs.end() ? 1 : it->second.slabs;
}

void set_slabs(const fsa_plan_s* pl, int slabs, double us) {
    if (pl->d != 3) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_slabs[GridKey((int)pl->prec, pl->N[0], pl->N[1], pl->N[2])] = SlabEntry{slabs, us};
    }
    ++g_generation;
}

}  // namespace tune
}  // namespace fsa

extern "C" {

fsa_status fsa_tune_set(int precision, int pass, int length, int64_t lines, int variant,
                        int occupancy) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !pass_ok(pass) ||
        !length_ok(pass, length) || lines < 1)
        return fail(FSA_EINVAL, "fsa_tune_set: bad precision, pass, length or line count");
    if (occupancy < 0 || !variant_ok((fsa_precision)precision, pass, length, variant))
        return fail(FSA_EINVAL, "fsa_tune_set: variant " + std::to_string(variant) +
                                    " does not exist at this pass and length");
    load_env_once();
    fsa::tune::set((fsa_precision)precision, (fsa::Pass)(pass & ~FSA_PASS_BATCHED), length,
                   (long)lines, fsa::Choice{variant, occupancy}, 0.0,
                   (pass & FSA_PASS_BATCHED) != 0);
    return FSA_OK;
}

fsa_status fsa_tune_get(int precision, int pass, int length, int64_t lines, int* variant,
                        int* occupancy, double* us) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !pass_ok(pass) ||
        !length_ok(pass, length) || lines < 1 || !variant || !occupancy)
        return fail(FSA_EINVAL, "fsa_tune_get: bad arguments");
    load_env_once();
    const fsa::Choice c = fsa::tune::get((fsa_precision)precision,
                                         (fsa::Pass)(pass & ~FSA_PASS_BATCHED), length,
                                         (long)lines, (pass & FSA_PASS_BATCHED) != 0);
    double t = 0.0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(Key(precision, pass, length, fsa::tune::size_class((long)lines)));
        if (it != g_table.end()) t = it->second.us;
    }
    *variant = c.var;
    *occupancy = c.occ;
    if (us) *us = t;
    return FSA_OK;
}

fsa_status fsa_tune_variants(int precision, int pass, int length, int* mask) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !pass_ok(pass) ||
        !length_ok(pass, length) || !mask)
        return fail(FSA_EINVAL, "fsa_tune_variants: bad arguments");
    int m = 0;
    for (int v = 0; v < fsa::kNumVariants; ++v)
        if (variant_ok((fsa_precision)precision, pass, length, v)) m |= 1 << v;
    *mask = m;
    return FSA_OK;
}

fsa_status fsa_tune_reset(void) {
    load_env_once();  // an environment table loaded later must not undo the reset
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
        g_slabs.clear();
    }
    ++g_generation;
    return FSA_OK;
}

fsa_status fsa_tune_save(const char* path) {
    if (!path) return fail(FSA_EINVAL, "fsa_tune_save: null path");
    load_env_once();
    std::string out = "{\n  \"format\": \"fsa-tune-1\",\n  \"arch\": \"" + device_arch() +
                      "\",\n  \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        bool first = true;
        for (const auto& kv : g_table) {
            char line[256];
            std::snprintf(line, sizeof line,
                          "%s\n    {\"precision\": \"%s\", \"pass\": \"%s\", \"length\": %d, "
                          "\"class\": %d, \"variant\": %d, \"occupancy\": %d, \"us\": %.3f}",
                          first ? "" : ",", std::get<0>(kv.first) == FSA_F32 ? "f32" : "f64",
                          pass_name(std::get<1>(kv.first)).c_str(), std::get<2>(kv.first),
                          std::get<3>(kv.first), kv.second.ch.var, kv.second.ch.occ,
                          kv.second.us);
            out += line;
            first = false;
        }
    }
    out += "\n  ],\n  \"schedules\": [";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        bool first = true;
        for (const auto& kv : g_slabs) {
            char line[256];
            std::snprintf(line, sizeof line,
                          "%s\n    {\"precision\": \"%s\", \"grid\": [%lld, %lld, %lld], "
                          "\"slabs\": %d, \"us\": %.3f}",
                          first ? "" : ",", std::get<0>(kv.first) == FSA_F32 ? "f32" : "f64",
                          (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                          (long long)std::get<3>(kv.first), kv.second.slabs, kv.second.us);
            out += line;
            first = false;
        }
    }
    out += "\n  ]\n}\n";
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(FSA_EINVAL, std::string("fsa_tune_save: cannot write ") + tmp);
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(FSA_EINVAL, std::string("fsa_tune_save: cannot write ") + path);
    }
    return FSA_OK;
}

fsa_status fsa_tune_load(const char* path) {
    if (!path) return fail(FSA_EINVAL, "fsa_tune_load: null path");
    load_env_once();
    return load_file(path);
}

fsa_status fsa_tune_set_slabs(int precision, const int64_t* N, int slabs) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !N || slabs < 1 ||
        slabs > fsa::kMaxSlabs)
        return fail(FSA_EINVAL, "fsa_tune_set_slabs: bad precision, grid or slab count");
    for (int j = 0; j < 3; ++j)
        if (!fsa::grid_length_supported(N[j]))
            return fail(FSA_EINVAL, "fsa_tune_set_slabs: unsupported grid length");
    load_env_once();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_slabs[GridKey(precision, N[0], N[1], N[2])] = SlabEntry{slabs, 0.0};
    }
    ++g_generation;
    return FSA_OK;
}

fsa_status fsa_tune_get_slabs(int precision, const int64_t* N, int* slabs, double* us) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !N || !slabs)
        return fail(FSA_EINVAL, "fsa_tune_get_slabs: bad arguments");
    load_env_once();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_slabs.find(GridKey(precision, N[0], N[1], N[2]));
    const SlabEntry e = it == g_slabs.end() ? SlabEntry{} : it->second;
    *slabs = e.slabs;
    if (us) *us = e.us;
    return FSA_OK;
}

fsa_status fsa_autotune(fsa_plan pl, const void* rho, void* phi, void* workspace, void* stream,
                        int reps) {
    fsa::Range range("fsa_autotune");
    if (!pl || !rho || !phi || !workspace)
        return fail(FSA_EINVAL, "fsa_autotune: null argument");
    if (!pl->built) return fail(FSA_ESTATE, "fsa_autotune: tensor not built");
    if (pl->prec == FSA_DD)
        return fail(FSA_EUNSUPPORTED, "fsa_autotune: double-double plans have no launch choices");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(FSA_EINVAL, "fsa_autotune: workspace must be 256-byte aligned");
    if (reps < 1 || reps > 1000) return fail(FSA_EINVAL, "fsa_autotune: reps must be 1..1000");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
        return fail(FSA_ESTATE, "fsa_autotune: plan is not built on the current device");
    load_env_once();
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // timing events without the system-scope fence of a default event, whose
    // cache write-back and invalidation would give the timed launch a cold L2
    hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableSystemFence);
    const int np = fsa::n_passes(pl);
    const int H = (int)pl->H;
    auto whole = [&](int k) { return fsa::Step{k, 0, H}; };
    auto run_all = [&](int slabs) {
        fsa::Step steps[fsa::kMaxSteps];
        const int ns = fsa::schedule(pl, slabs, steps);
        hipError_t r = hipSuccess;
        for (int i = 0; i < ns && r == hipSuccess; ++i)
            r = fsa::launch_step(pl, steps[i], rho, phi, workspace,
                                 fsa::step_choice(pl, steps[i]), st);
        return r;
    };
    auto nothing = [] { return hipSuccess; };
    // median time (us) of every candidate over `reps` rounds after a warm-up
    // round; a round runs each candidate once, so slow drifts of the clock
    // or of the memory system fall on all of them alike
    // (prep and post run untimed before and after each timed body)
    auto time_rounds = [&](int n, auto&& prep, auto&& body, auto&& post,
                           std::vector<double>& us) {
        std::vector<std::vector<float>> ms((size_t)n);
        hipError_t r = hipSuccess;
        for (int i = -1; i < reps && r == hipSuccess; ++i) {
            for (int c = 0; c < n && r == hipSuccess; ++c) {
                r = prep();
                if (r == hipSuccess) r = hipEventRecord(ev[0], st);
                if (r == hipSuccess) r = body(c);
                if (r == hipSuccess) r = hipEventRecord(ev[1], st);
                if (r == hipSuccess) r = post();
                if (r == hipSuccess) r = hipEventSynchronize(ev[1]);
                float t = 0.0f;
                if (r == hipSuccess) r = hipEventElapsedTime(&t, ev[0], ev[1]);
                if (r == hipSuccess && i >= 0) ms[(size_t)c].push_back(t);
            }
        }
        us.assign((size_t)n, 0.0);
        if (r == hipSuccess)
            for (int c = 0; c < n; ++c) {
                std::sort(ms[(size_t)c].begin(), ms[(size_t)c].end());
                us[(size_t)c] = 1e3 * ms[(size_t)c][ms[(size_t)c].size() / 2];
            }
        return r;
    };
    // one evaluation with the current choices fills every buffer with data
    if (e == hipSuccess) e = run_all(1);
    for (int k = 0; k < np && e == hipSuccess; ++k) {
        fsa::Pass pass;
        int len;
        fsa::pass_of(pl, k, &pass, &len);
        std::vector<fsa::Choice> cands;
        for (int v = 0; v < fsa::kNumVariants; ++v) {
            if (!variant_ok(pl->prec, (int)pass, len, v)) continue;
            const int mo = pl->prec == FSA_F32 ? fsa::Launch<float>::max_occ(pass, len, v)
                                               : fsa::Launch<double>::max_occ(pass, len, v);
            cands.push_back(fsa::Choice{v, 0});
            if (mo >= 2) cands.push_back(fsa::Choice{v, mo / 2});
        }
        // Each candidate is timed inside a whole evaluation: the passes
        // before it run first (which also re-creates the input of the
        // in-place fused pass) and the passes after it once it is timed, so
        // the caches hold what they hold when evaluations follow each other.
        // (A pass timed on its own, over and over, finds its input in the
        // Infinity Cache and favours the variants that gain from that.)
        auto run_range = [&](int from, int to) {
            hipError_t r = hipSuccess;
            for (int j = from; j < to && r == hipSuccess; ++j)
                r = fsa::launch_step(pl, whole(j), rho, phi, workspace,
                                     fsa::step_choice(pl, whole(j)), st);
            return r;
        };
        std::vector<double> us;
        e = time_rounds(
            (int)cands.size(), [&] { return run_range(0, k); },
            [&](int c) {
                return fsa::launch_step(pl, whole(k), rho, phi, workspace, cands[(size_t)c], st);
            },
            [&] { return run_range(k + 1, np); }, us);
        if (e == hipSuccess) {
            size_t b = 0;
            for (size_t c = 1; c < cands.size(); ++c)
                if (us[c] < us[b]) b = c;
            fsa::tune::set(pl->prec, pass, len, fsa::step_lines(pl, whole(k)), cands[b], us[b]);
        }
    }
    // schedule: slabs of bins for the middle passes (3D)
    if (e == hipSuccess && pl->d == 3) {
        std::vector<int> counts;
        for (int slabs = 1; slabs <= fsa::kMaxSlabs && slabs <= H; slabs *= 2)
            counts.push_back(slabs);
        // evaluations back to back, as a caller streams them
        constexpr int kBack = 4;
        std::vector<double> us;
        e = time_rounds((int)counts.size(), nothing,
                        [&](int c) {
                            hipError_t r = hipSuccess;
                            for (int i = 0; i < kBack && r == hipSuccess; ++i)
                                r = run_all(counts[(size_t)c]);
                            return r;
                        },
                        nothing, us);
        if (e == hipSuccess) {
            size_t b = 0;
            for (size_t c = 1; c < counts.size(); ++c)
                if (us[c] < us[b]) b = c;
            fsa::tune::set_slabs(pl, counts[b], us[b] / kBack);
        }
    }
    // leave the caller's buffers holding a valid evaluation
    if (e == hipSuccess) e = run_all(fsa::tune::get_slabs(pl));
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess)
        return fail(FSA_EDEVICE, std::string("fsa_autotune: ") + hipGetErrorString(e));
    return FSA_OK;
}

}  // extern "C"
