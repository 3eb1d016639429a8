// fsa_tune.cpp -- the autotuner and its table of launch choices.
//
// Every pass kernel is compiled in up to three variants per transform length
// (default; alternate radix family, i.e. another radix split and number of
// threads per transform; half-size workgroups, i.e. fewer lines per tile or
// teams per group).  At run time the persistent grid can also use fewer
// resident workgroups per CU than fit.  fsa_autotune times every distinct
// (variant, occupancy) candidate of every pass of a plan on the device with
// hipEvents and keeps the fastest per (precision, pass, length) in a
// process-wide table; fsa_apply, fsa_apply_batched and the server read the
// table at launch time.  The table can be saved to and loaded from a JSON
// file, and is loaded on first use from the file named by the environment
// variable FSA_TUNE_CACHE when that is set.
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

using Key = std::tuple<int, int, int>;  // precision, pass, length

std::mutex g_mu;
std::map<Key, TuneEntry>& g_table = *new std::map<Key, TuneEntry>();
std::atomic<uint64_t> g_generation{1};
std::once_flag g_env_once;

const char* const kPassNames[5] = {"r2c", "fwd_t", "conv", "inv_t", "c2r"};

fsa_status fail(fsa_status s, const std::string& msg) {
    fsa::set_last_error(msg.c_str());
    return s;
}

bool pass_ok(int pass) { return pass >= 0 && pass <= (int)fsa::Pass::C2R; }

// Transform lengths the passes support: the real passes take the half
// length M of the padded row, the complex passes the padded length P.
bool length_ok(int pass, int len) {
    if (!fsa::fft_length_supported(len)) return false;
    if (pass == (int)fsa::Pass::R2C || pass == (int)fsa::Pass::C2R) return len >= 8 && len <= 2048;
    return len >= 16 && len <= 4096;
}

bool variant_ok(fsa_precision prec, int pass, int len, int var) {
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
    };
    std::vector<Row> rows;
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
        } else {
            double v;
            if (!r.num(v)) return false;
            if (k == "length") row.len = v;
            else if (k == "variant") row.var = v;
            else if (k == "occupancy") row.occ = v;
            else if (k == "us") row.us = v;
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
        } else if (k == "entries") {
            if (!r.eat('[')) return false;
            if (!r.eat(']')) {
                do {
                    Parsed::Row row;
                    if (!parse_row(r, row)) return false;
                    out.rows.push_back(row);
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
    for (const auto& row : p.rows) {
        int prec = row.prec == "f32" ? FSA_F32 : row.prec == "f64" ? FSA_F64 : -1;
        int pass = -1;
        for (int k = 0; k < 5; ++k)
            if (row.pass == kPassNames[k]) pass = k;
        auto small_int = [](double v) { return v >= 0.0 && v <= 1e6 && v == (double)(int)v; };
        const bool ints = small_int(row.len) && small_int(row.var) && small_int(row.occ);
        const int len = ints ? (int)row.len : -1, var = ints ? (int)row.var : -1;
        const int occ = ints ? (int)row.occ : -1;
        if (prec < 0 || pass < 0 || !ints || !length_ok(pass, len) ||
            !variant_ok((fsa_precision)prec, pass, len, var))
            return fail(FSA_EINVAL, "fsa_tune_load: invalid entry (" + row.prec + ", " +
                                        row.pass + ", " + std::to_string(len) + ")");
        fresh[Key(prec, pass, len)] = TuneEntry{fsa::Choice{var, occ}, row.us};
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto& kv : fresh) g_table[kv.first] = kv.second;
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

Choice get(fsa_precision prec, Pass pass, int len) {
    load_env_once();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(Key((int)prec, (int)pass, len));
    return it == g_table.end() ? Choice{} : it->second.ch;
}

void set(fsa_precision prec, Pass pass, int len, Choice c, double us) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[Key((int)prec, (int)pass, len)] = TuneEntry{c, us};
    }
    ++g_generation;
}

uint64_t generation() { return g_generation.load(); }

}  // namespace tune
}  // namespace fsa

extern "C" {

fsa_status fsa_tune_set(int precision, int pass, int length, int variant, int occupancy) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !pass_ok(pass) ||
        !length_ok(pass, length))
        return fail(FSA_EINVAL, "fsa_tune_set: bad precision, pass or length");
    if (occupancy < 0 || !variant_ok((fsa_precision)precision, pass, length, variant))
        return fail(FSA_EINVAL, "fsa_tune_set: variant " + std::to_string(variant) +
                                    " does not exist at this pass and length");
    load_env_once();
    fsa::tune::set((fsa_precision)precision, (fsa::Pass)pass, length,
                   fsa::Choice{variant, occupancy}, 0.0);
    return FSA_OK;
}

fsa_status fsa_tune_get(int precision, int pass, int length, int* variant, int* occupancy,
                        double* us) {
    if ((precision != FSA_F32 && precision != FSA_F64) || !pass_ok(pass) ||
        !length_ok(pass, length) || !variant || !occupancy)
        return fail(FSA_EINVAL, "fsa_tune_get: bad arguments");
    load_env_once();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(Key(precision, pass, length));
    const TuneEntry e = it == g_table.end() ? TuneEntry{} : it->second;
    *variant = e.ch.var;
    *occupancy = e.ch.occ;
    if (us) *us = e.us;
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
                          "\"variant\": %d, \"occupancy\": %d, \"us\": %.3f}",
                          first ? "" : ",", std::get<0>(kv.first) == FSA_F32 ? "f32" : "f64",
                          kPassNames[std::get<1>(kv.first)], std::get<2>(kv.first),
                          kv.second.ch.var, kv.second.ch.occ, kv.second.us);
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

fsa_status fsa_autotune(fsa_plan pl, const void* rho, void* phi, void* workspace, void* stream,
                        int reps) {
    if (!pl || !rho || !phi || !workspace)
        return fail(FSA_EINVAL, "fsa_autotune: null argument");
    if (!pl->built) return fail(FSA_ESTATE, "fsa_autotune: tensor not built");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(FSA_EINVAL, "fsa_autotune: workspace must be 256-byte aligned");
    if (reps < 1 || reps > 1000) return fail(FSA_EINVAL, "fsa_autotune: reps must be 1..1000");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
        return fail(FSA_ESTATE, "fsa_autotune: plan is not built on the current device");
    load_env_once();
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    const int np = fsa::n_passes(pl);
    auto tuned = [&](int k) {
        fsa::Pass pass;
        int len;
        fsa::pass_of(pl, k, &pass, &len);
        return fsa::tune::get(pl->prec, pass, len);
    };
    // one evaluation with the current choices fills every buffer with data
    for (int k = 0; k < np && e == hipSuccess; ++k)
        e = fsa::launch_pass(pl, k, rho, phi, workspace, tuned(k), st);
    for (int k = 0; k < np && e == hipSuccess; ++k) {
        fsa::Pass pass;
        int len;
        fsa::pass_of(pl, k, &pass, &len);
        // the fused pass works in place: re-create its input before each run
        const bool refill = pass == fsa::Pass::CONV;
        std::vector<fsa::Choice> cands;
        for (int v = 0; v < fsa::kNumVariants; ++v) {
            if (!variant_ok(pl->prec, (int)pass, len, v)) continue;
            const int mo = pl->prec == FSA_F32 ? fsa::Launch<float>::max_occ(pass, len, v)
                                               : fsa::Launch<double>::max_occ(pass, len, v);
            cands.push_back(fsa::Choice{v, 0});
            if (mo >= 2) cands.push_back(fsa::Choice{v, mo / 2});
        }
        double best = 1e300;
        fsa::Choice best_c;
        for (const fsa::Choice& c : cands) {
            std::vector<float> ms;
            for (int r = -1; r < reps && e == hipSuccess; ++r) {  // r = -1: warm-up
                if (refill) e = fsa::launch_pass(pl, k - 1, rho, phi, workspace, tuned(k - 1), st);
                if (e == hipSuccess) e = hipEventRecord(ev[0], st);
                if (e == hipSuccess) e = fsa::launch_pass(pl, k, rho, phi, workspace, c, st);
                if (e == hipSuccess) e = hipEventRecord(ev[1], st);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float t = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
                if (e == hipSuccess && r >= 0) ms.push_back(t);
            }
            if (e != hipSuccess) break;
            std::sort(ms.begin(), ms.end());
            const double med = 1e3 * ms[ms.size() / 2];
            if (med < best) {
                best = med;
                best_c = c;
            }
        }
        if (e == hipSuccess) fsa::tune::set(pl->prec, pass, len, best_c, best);
    }
    // leave the caller's buffers holding a valid evaluation
    for (int k = 0; k < np && e == hipSuccess; ++k)
        e = fsa::launch_pass(pl, k, rho, phi, workspace, tuned(k), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess)
        return fail(FSA_EDEVICE, std::string("fsa_autotune: ") + hipGetErrorString(e));
    return FSA_OK;
}

}  // extern "C"
