// fsa_api.cpp -- the C ABI of include/fsa.h: plans, tensor build, apply.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <string>

#include "fsa_internal.hpp"

namespace {

thread_local std::string g_last_error;

fsa_status fail(fsa_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fsa_status fail(fsa_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

fsa_status hip_fail(hipError_t e, const char* what) {
    return fail(FSA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int kernel_dim(int kind) {
    switch (kind) {
    case FSA_COULOMB_3D:
    case FSA_YUKAWA_3D:
    case FSA_BIHARMONIC_3D:
    case FSA_DDI_3D: return 3;
    case FSA_LOG_2D:
    case FSA_COULOMB_2D:
    case FSA_BIHARMONIC_2D:
    case FSA_YUKAWA_2D:
    case FSA_QUASI2D_DDI: return 2;
    }
    return 0;
}

bool finite_nonzero(const double* v) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) {
        if (!std::isfinite(v[j])) return false;
        s += v[j] * v[j];
    }
    return s > 0.0;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

namespace fsa {
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace fsa

extern "C" {

const char* fsa_last_error(void) { return g_last_error.c_str(); }

fsa_status fsa_plan_create(const fsa_kernel* k, int d, const double* L, const int64_t* N,
                           fsa_precision p, fsa_plan* out) {
    fsa::Range range("fsa_plan_create");
    if (!k || !L || !N || !out) return fail(FSA_EINVAL, "fsa_plan_create: null argument");
    const int kd = kernel_dim(k->kind);
    if (kd == 0) return fail(FSA_EINVAL, "fsa_plan_create: unknown kernel kind %d", k->kind);
    if (d != kd)
        return fail(FSA_EINVAL, "fsa_plan_create: kernel kind %d needs d = %d, got %d", k->kind,
                    kd, d);
    if (p != FSA_F32 && p != FSA_F64 && p != FSA_DD)
        return fail(FSA_EINVAL, "fsa_plan_create: unknown precision %d", (int)p);
    if (p == FSA_DD) {
        if ((k->kind != FSA_COULOMB_3D && k->kind != FSA_COULOMB_2D) || k->general)
            return fail(FSA_EUNSUPPORTED,
                        "fsa_plan_create: double-double precision supports the Coulomb "
                        "kernels (closed-form construction) only");
        for (int j = 0; j < d; ++j)
            if (N[j] < 8 || N[j] > 1024 || (N[j] & (N[j] - 1)) != 0)
                return fail(FSA_EUNSUPPORTED,
                            "fsa_plan_create: double-double precision needs N[%d] = 2^a in "
                            "[8, 1024], got %lld",
                            j, (long long)N[j]);
    }
    const bool yukawa = k->kind == FSA_YUKAWA_3D || k->kind == FSA_YUKAWA_2D;
    if (yukawa && !(k->lambda > 0.0 && std::isfinite(k->lambda)))
        return fail(FSA_EINVAL, "fsa_plan_create: Yukawa needs lambda > 0");
    if (k->kind == FSA_DDI_3D && !(finite_nonzero(k->n) && finite_nonzero(k->m)))
        return fail(FSA_EINVAL, "fsa_plan_create: DDI needs finite, nonzero n and m");
    if (k->kind == FSA_QUASI2D_DDI) {
        if (!finite_nonzero(k->n))
            return fail(FSA_EINVAL, "fsa_plan_create: quasi-2D DDI needs a finite, nonzero n");
        if (!(k->eta > 0.0 && std::isfinite(k->eta)))
            return fail(FSA_EINVAL, "fsa_plan_create: quasi-2D DDI needs eta > 0");
    }
    const bool general =
        k->general != 0 || k->kind == FSA_YUKAWA_2D || k->kind == FSA_QUASI2D_DDI;
    const bool windowed = general && fsa::kernel_windowed(k->kind);
    double minL = 1e300;
    for (int j = 0; j < d; ++j) {
        if (!(L[j] > 0.0 && std::isfinite(L[j])))
            return fail(FSA_EINVAL, "fsa_plan_create: L[%d] must be positive", j);
        if (N[j] < 8 || (N[j] % 2) != 0)
            return fail(FSA_EINVAL, "fsa_plan_create: N[%d] = %lld must be even and >= 8", j,
                        (long long)N[j]);
        if (!fsa::grid_length_supported(N[j]))
            return fail(FSA_EUNSUPPORTED,
                        "fsa_plan_create: N[%d] = %lld unsupported (need 2^a or 3*2^a, <= 2048)",
                        j, (long long)N[j]);
        minL = std::fmin(minL, L[j]);
    }
    const double R0 = 2.0 * minL;
    double eps = k->eps;
    if (!(eps > 0.0)) eps = windowed ? R0 / 16.0 : R0 / 8.0;
    if (!std::isfinite(eps) || eps > R0 / 4.0)
        return fail(FSA_EINVAL,
                    "fsa_plan_create: eps = %g violates the far-field condition (need eps <= "
                    "R0/4 = %g; 16 digits need eps <= R0/5.85)",
                    eps, R0 / 4.0);
    // the window erfc((r - 6 eps)/eps)/2 must have decayed at R0
    if (windowed && eps > R0 / 12.0)
        return fail(FSA_EINVAL,
                    "fsa_plan_create: eps = %g too large for the windowed general construction "
                    "(need eps <= R0/12 = %g)",
                    eps, R0 / 12.0);

    fsa_plan_s* pl = new (std::nothrow) fsa_plan_s();
    if (!pl) return fail(FSA_ENOMEM, "fsa_plan_create: out of host memory");
    static std::atomic<uint64_t> next_id{1};
    pl->id = next_id.fetch_add(1);
    // a 3D dipole-dipole plan convolves with the Coulomb tensor
    pl->ddi = k->kind == FSA_DDI_3D;
    pl->n_spectral = pl->ddi ? 5 : (k->kind == FSA_QUASI2D_DDI ? 3 : 0);
    pl->kp = fsa::KernelParams{pl->ddi ? FSA_COULOMB_3D : k->kind, yukawa ? k->lambda : 0.0, eps,
                               general ? 1 : 0,
                               k->kind == FSA_QUASI2D_DDI ? k->eta : 0.0};
    if (pl->n_spectral)
        for (int j = 0; j < 3; ++j) {
            pl->dn[j] = k->n[j];
            pl->dm[j] = pl->ddi ? k->m[j] : 0.0;
        }
    pl->d = d;
    pl->prec = p;
    for (int j = 0; j < d; ++j) {
        pl->L[j] = L[j];
        pl->N[j] = N[j];
        pl->h[j] = 2.0 * L[j] / (double)N[j];
    }
    const size_t rsize = p == FSA_F32 ? 4 : (p == FSA_F64 ? 8 : 16);
    pl->csize = 2 * rsize;
    const int64_t Nl = N[d - 1];
    pl->H = Nl + 1;
    if (d == 3) {
        pl->ws1_elems = (size_t)N[0] * pl->H * N[1];
        pl->ws2_elems = (size_t)pl->H * 2 * N[1] * N[0];
    } else {
        pl->ws1_elems = (size_t)pl->H * N[0];
        // quasi-2D DDI: the real source N_0 x N_1 (the complex N-grid array of
        // the derivative fits the first array, H > N_1)
        pl->ws2_elems = pl->n_spectral ? (size_t)N[0] * N[1] / 2 : 0;
    }
    if (p == FSA_DD) {  // the whole padded complex spectrum
        pl->ws1_elems = 1;
        for (int j = 0; j < d; ++j) pl->ws1_elems *= (size_t)(2 * N[j]);
        pl->ws2_elems = 0;
    }
    pl->ws_bytes = align256(pl->ws1_elems * pl->csize) + align256(pl->ws2_elems * pl->csize);
    pl->tensor_elems = 1;
    for (int j = 0; j < d; ++j) pl->tensor_elems *= (size_t)(N[j] + 1);
    if (p == FSA_DD) {  // complex DD twiddles of every axis
        pl->tw_elems = fsa::dd_twiddle_elems(pl);
        *out = pl;
        return FSA_OK;
    }
    // twiddle tables: P0 = 2 N0; P1 = 2 N1 (3D); M = N_last; P_last = 2 N_last
    size_t off = 0;
    pl->tw_off_p0 = off;
    off += 2 * N[0];
    pl->tw_off_p1 = off;
    if (d == 3) off += 2 * N[1];
    pl->tw_off_m = off;
    off += Nl;
    pl->tw_off_pl = off;
    off += 2 * Nl;
    if (pl->n_spectral) {  // unpadded transforms of the derivative on the N-grid
        pl->tw_off_n0 = off;
        off += N[0];
        pl->tw_off_n1 = off;
        off += N[1];
    }
    pl->tw_elems = off;
    *out = pl;
    return FSA_OK;
}

fsa_status fsa_plan_query(fsa_plan pl, double* eps_used, double* h, size_t* tensor_bytes,
                          size_t* workspace_bytes) {
    if (!pl) return fail(FSA_EINVAL, "fsa_plan_query: null plan");
    if (eps_used) *eps_used = pl->kp.eps;
    if (h)
        for (int j = 0; j < pl->d; ++j) h[j] = pl->h[j];
    if (tensor_bytes) *tensor_bytes = pl->tensor_elems * (pl->csize / 2);
    if (workspace_bytes) *workspace_bytes = pl->ws_bytes;
    return FSA_OK;
}

fsa_status fsa_build_tensor(fsa_plan pl, void* stream) {
    fsa::Range range("fsa_build_tensor");
    if (!pl) return fail(FSA_EINVAL, "fsa_build_tensor: null plan");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "fsa_build_tensor: hipGetDevice");
    if (pl->built && pl->device != dev)
        return fail(FSA_ESTATE, "fsa_build_tensor: plan was built on device %d, current is %d",
                    pl->device, dev);
    const size_t rsize = pl->csize / 2;
    if (!pl->tensor) {
        e = hipMalloc(&pl->tensor, pl->tensor_elems * rsize);
        if (e != hipSuccess) {
            pl->tensor = nullptr;
            return fail(FSA_ENOMEM, "fsa_build_tensor: tensor allocation (%zu bytes): %s",
                        pl->tensor_elems * rsize, hipGetErrorString(e));
        }
    }
    if (!pl->twiddles) {
        e = hipMalloc(&pl->twiddles, pl->tw_elems * pl->csize);
        if (e != hipSuccess) {
            pl->twiddles = nullptr;
            return fail(FSA_ENOMEM, "fsa_build_tensor: twiddle allocation: %s",
                        hipGetErrorString(e));
        }
    }
    if (pl->prec == FSA_DD) {
        e = fsa::build_tensor_dd(pl, st);
        if (e == hipErrorOutOfMemory)
            return fail(FSA_ENOMEM, "fsa_build_tensor: temporary DD octant: %s",
                        hipGetErrorString(e));
        if (e != hipSuccess) return hip_fail(e, "fsa_build_tensor: double-double kernels");
        pl->device = dev;
        pl->built = true;
        return FSA_OK;
    }
    char* tw = (char*)pl->twiddles;
    const int64_t Nl = pl->N[pl->d - 1];
    e = fsa::build_twiddles(pl->prec, (int)(2 * pl->N[0]), tw + pl->tw_off_p0 * pl->csize, st);
    if (e == hipSuccess && pl->d == 3)
        e = fsa::build_twiddles(pl->prec, (int)(2 * pl->N[1]), tw + pl->tw_off_p1 * pl->csize, st);
    if (e == hipSuccess)
        e = fsa::build_twiddles(pl->prec, (int)Nl, tw + pl->tw_off_m * pl->csize, st);
    if (e == hipSuccess)
        e = fsa::build_twiddles(pl->prec, (int)(2 * Nl), tw + pl->tw_off_pl * pl->csize, st);
    if (e == hipSuccess && pl->n_spectral)
        e = fsa::build_twiddles(pl->prec, (int)pl->N[0], tw + pl->tw_off_n0 * pl->csize, st);
    if (e == hipSuccess && pl->n_spectral)
        e = fsa::build_twiddles(pl->prec, (int)pl->N[1], tw + pl->tw_off_n1 * pl->csize, st);
    if (e != hipSuccess) return hip_fail(e, "fsa_build_tensor: twiddle kernels");
    e = fsa::build_tensor_device(pl->kp, pl->d, pl->L, pl->N, pl->h, pl->prec, pl->tensor,
                                 &pl->line_order, st);
    if (e == hipErrorOutOfMemory)
        return fail(FSA_ENOMEM, "fsa_build_tensor: temporary FP64 octant: %s",
                    hipGetErrorString(e));
    if (e != hipSuccess) return hip_fail(e, "fsa_build_tensor: tensor kernels");
    pl->device = dev;
    pl->built = true;
    return FSA_OK;
}

}  // extern "C"

namespace fsa {

int n_passes(const fsa_plan_s* pl) { return pl->d == 3 ? 5 : 3; }

void pass_of(const fsa_plan_s* pl, int k, Pass* pass, int* len) {
    const int N0 = (int)pl->N[0], N1 = (int)pl->N[1];
    if (pl->d == 3) {
        const int N2 = (int)pl->N[2];
        static const Pass kind[5] = {Pass::R2C, Pass::FWD_T, Pass::CONV, Pass::INV_T, Pass::C2R};
        const int lens[5] = {N2, 2 * N1, 2 * N0, 2 * N1, N2};
        *pass = kind[k];
        *len = lens[k];
    } else {
        static const Pass kind[3] = {Pass::R2C, Pass::CONV, Pass::C2R};
        const int lens[3] = {N1, 2 * N0, N1};
        *pass = kind[k];
        *len = lens[k];
    }
}

template <typename R>
static hipError_t launch_pass_t(const fsa_plan_s* pl, int k, int lo, int n, const void* rho,
                                void* phi, void* ws, Choice c, hipStream_t st) {
    const char* tw = (const char*)pl->twiddles;
    const size_t cs = pl->csize;
    const void* tw_p0 = tw + pl->tw_off_p0 * cs;
    const void* tw_p1 = tw + pl->tw_off_p1 * cs;
    const void* tw_m = tw + pl->tw_off_m * cs;
    const void* tw_pl = tw + pl->tw_off_pl * cs;
    const int N0 = (int)pl->N[0], N1 = (int)pl->N[1];
    const int H = (int)pl->H;
    const R* tensor = (const R*)pl->tensor;
    char* w1 = (char*)ws;
    if (pl->d == 3) {
        const int N2 = (int)pl->N[2];
        char* w2 = w1 + ((pl->ws1_elems * cs + 255) & ~size_t(255));
        // dipole-dipole: pass A convolves -3 d_nm rho (left in the second
        // workspace array by the derivative launches) and pass E adds
        // -(m.n) rho
        const void* src = pl->ddi ? (const void*)w2 : rho;
        const void* add = pl->ddi ? rho : nullptr;
        const double alpha =
            pl->ddi ? -(pl->dn[0] * pl->dm[0] + pl->dn[1] * pl->dm[1] + pl->dn[2] * pl->dm[2])
                    : 0.0;
        switch (k) {
        case 0: return Launch<R>::r2c(N2, (const R*)src, w1, N0, N1, tw_m, tw_pl, c, st);
        case 1: return Launch<R>::fwd_t(2 * N1, w1, w2, N0, H, lo, n, tw_p1, c, st);
        case 2:
            return Launch<R>::conv(2 * N0, w2, tensor, n * 2 * N1, 2 * N1, N1, lo, tw_p0, c, st);
        case 3: return Launch<R>::inv_t(2 * N1, w2, w1, N0, H, lo, n, tw_p1, c, st);
        case 4:
            return Launch<R>::c2r(N2, w1, (R*)phi, N0, N1, add, alpha, tw_m, tw_pl, c, st);
        }
    } else {
        // quasi-2D dipole-dipole: pass A convolves the source the derivative
        // launches left in the second workspace array
        const void* src =
            pl->n_spectral ? (const void*)(w1 + ((pl->ws1_elems * cs + 255) & ~size_t(255)))
                           : rho;
        switch (k) {
        case 0: return Launch<R>::r2c(N1, (const R*)src, w1, 1, N0, tw_m, tw_pl, c, st);
        case 1: return Launch<R>::conv(2 * N0, w1, tensor, H, 1, 0, 0, tw_p0, c, st);
        case 2:
            return Launch<R>::c2r(N1, w1, (R*)phi, 1, N0, nullptr, 0.0, tw_m, tw_pl, c, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(const fsa_plan_s* pl, const Step& s, const void* rho, void* phi, void* ws,
                       Choice c, hipStream_t st) {
    if (pl->prec == FSA_DD) return launch_dd_step(pl, s.k, rho, phi, ws, st);
    if (s.k >= kSpectralStep) {  // derivative of a dipole-dipole plan
        char* w1 = (char*)ws;
        char* w2 = w1 + ((pl->ws1_elems * pl->csize + 255) & ~size_t(255));
        return spectral_step(pl, s.k - kSpectralStep, rho, w1, w2, st);
    }
    return pl->prec == FSA_F32
               ? launch_pass_t<float>(pl, s.k, s.lo, s.n, rho, phi, ws, c, st)
               : launch_pass_t<double>(pl, s.k, s.lo, s.n, rho, phi, ws, c, st);
}

int schedule(const fsa_plan_s* pl, int slabs, Step* out) {
    int m = 0;
    const int H = (int)pl->H;
    if (pl->prec == FSA_DD) {  // one launch per pass, no slabs
        for (int k = 0; k < n_passes(pl); ++k) out[m++] = Step{k, 0, 0};
        return m;
    }
    for (int i = 0; i < pl->n_spectral; ++i) out[m++] = Step{kSpectralStep + i, 0, 0};
    if (pl->d != 3) {
        for (int k = 0; k < 3; ++k) out[m++] = Step{k, 0, H};
        return m;
    }
    if (slabs < 1) slabs = 1;
    if (slabs > kMaxSlabs) slabs = kMaxSlabs;
    if (slabs > H) slabs = H;
    out[m++] = Step{0, 0, H};
    for (int c = 0; c < slabs; ++c) {
        const int lo = (int)((long)H * c / slabs), hi = (int)((long)H * (c + 1) / slabs);
        for (int k = 1; k <= 3; ++k) out[m++] = Step{k, lo, hi - lo};
    }
    out[m++] = Step{4, 0, H};
    return m;
}

long step_lines(const fsa_plan_s* pl, const Step& s) {
    const long N0 = pl->N[0], N1 = pl->N[1];
    if (pl->d == 3) {
        switch (s.k) {
        case 0:
        case 4: return N0 * N1;             // rows of the last axis
        case 1:
        case 3: return N0 * (long)s.n;      // axis-1 lines of the slab
        case 2: return 2 * N1 * (long)s.n;  // axis-0 pencils of the slab
        }
    }
    return s.k == 1 ? (long)pl->H : N0;     // 2D: pencils, else rows
}

Choice step_choice(const fsa_plan_s* pl, const Step& s) {
    if (s.k >= kSpectralStep || pl->prec == FSA_DD) return Choice{};
    Pass pass;
    int len;
    pass_of(pl, s.k, &pass, &len);
    return tune::get(pl->prec, pass, len, step_lines(pl, s));
}

// Enqueues one evaluation: pass A, then passes B, C, D per slab of bins p2
// (3D; the slab count is the tuned schedule of the grid), then pass E, each
// with its tuned launch choice.  With events, records ev[2i] right before
// launch i and ev[2i + 1] right after it (a null pair: launch i untimed).
static hipError_t apply_impl(const fsa_plan_s* pl, const void* rho, void* phi, void* ws,
                             hipStream_t st, hipEvent_t const* ev) {
    static const char* const kPassRange[6] = {"fsa pass A r2c", "fsa pass B fwd_t",
                                              "fsa pass C conv", "fsa pass D inv_t",
                                              "fsa pass E c2r", "fsa spectral"};
    Range range("fsa_apply");
    Step steps[kMaxSteps];
    const int ns = schedule(pl, tune::get_slabs(pl), steps);
    hipError_t e = hipSuccess;
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        int kind = steps[i].k >= kSpectralStep ? 5 : steps[i].k;
        if (kind < 5 && pl->prec != FSA_DD && pl->d == 2) kind = kind == 0 ? 0 : kind == 1 ? 2 : 4;
        Range pass_range(kPassRange[kind]);
        const bool timed = ev && ev[2 * i];
        if (timed) e = hipEventRecord(ev[2 * i], st);
        if (e == hipSuccess)
            e = launch_step(pl, steps[i], rho, phi, ws, step_choice(pl, steps[i]), st);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[2 * i + 1], st);
    }
    return e;
}

hipError_t apply_plan(const fsa_plan_s* pl, const void* rho, void* phi, void* ws,
                      hipStream_t st, hipEvent_t const* events) {
    return apply_impl(pl, rho, phi, ws, st, events);
}

}  // namespace fsa

extern "C" {

static fsa_status apply_checked(fsa_plan pl, const void* rho, void* phi, void* workspace,
                                void* stream, hipEvent_t const* events) {
    if (!pl) return fail(FSA_EINVAL, "fsa_apply: null plan");
    if (!rho || !phi || !workspace) return fail(FSA_EINVAL, "fsa_apply: null device pointer");
    if (!pl->built) return fail(FSA_ESTATE, "fsa_apply: tensor not built (call fsa_build_tensor)");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(FSA_EINVAL, "fsa_apply: workspace must be 256-byte aligned");
    const size_t align = pl->csize / 2;
    if (((uintptr_t)rho % align) != 0 || ((uintptr_t)phi % align) != 0)
        return fail(FSA_EINVAL, "fsa_apply: rho/phi misaligned for the plan precision");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "fsa_apply: hipGetDevice");
    if (dev != pl->device)
        return fail(FSA_ESTATE, "fsa_apply: plan built on device %d, current device is %d",
                    pl->device, dev);
    e = fsa::apply_plan(pl, rho, phi, workspace, (hipStream_t)stream, events);
    if (e != hipSuccess) return hip_fail(e, "fsa_apply: kernel launch");
    return FSA_OK;
}

fsa_status fsa_apply(fsa_plan pl, const void* rho, void* phi, void* workspace, void* stream) {
    return apply_checked(pl, rho, phi, workspace, stream, nullptr);
}

}  // extern "C"

// Workspace of fsa_apply_noalloc: a device array of the library's module,
// one copy per device, alive until the process ends.  In host code `scratch`
// names a host-side shadow, not device memory: kernels only ever receive the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[FSA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of `scratch` on device `dev` (which must be current),
// resolved once per device.
fsa_status scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(FSA_EUNSUPPORTED, "fsa_apply_noalloc: device %d beyond the %d supported", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "fsa_apply_noalloc: hipGetSymbolAddress");
        if (!ptr || ((uintptr_t)ptr & 255) != 0)
            return fail(FSA_EDEVICE, "fsa_apply_noalloc: scratch address %p unusable", ptr);
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return FSA_OK;
}

}  // namespace

extern "C" {

fsa_status fsa_apply_noalloc(fsa_plan pl, const void* rho, void* phi, void* stream) {
    if (!pl) return fail(FSA_EINVAL, "fsa_apply_noalloc: null plan");
    if (pl->ws_bytes > (size_t)FSA_NOALLOC_SCRATCH_BYTES)
        return fail(FSA_EINVAL,
                    "fsa_apply_noalloc: the plan needs %zu bytes of workspace, the static scratch "
                    "holds %zu (use fsa_apply with a caller workspace)",
                    pl->ws_bytes, (size_t)FSA_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "fsa_apply_noalloc: hipGetDevice");
    void* ws = nullptr;
    const fsa_status st = scratch_address(dev, &ws);
    if (st != FSA_OK) return st;
    return apply_checked(pl, rho, phi, ws, stream, nullptr);
}

fsa_status fsa_plan_launches(fsa_plan pl, int* n, int* passes, int cap) {
    if (!pl || !n) return fail(FSA_EINVAL, "fsa_plan_launches: null argument");
    fsa::Step steps[fsa::kMaxSteps];
    const int ns = fsa::schedule(pl, fsa::tune::get_slabs(pl), steps);
    if (passes) {
        if (cap < ns) return fail(FSA_EINVAL, "fsa_plan_launches: need room for %d entries", ns);
        for (int i = 0; i < ns; ++i) {
            if (steps[i].k >= fsa::kSpectralStep) {
                passes[i] = FSA_PASS_SPECTRAL;
                continue;
            }
            fsa::Pass pass;
            int len;
            fsa::pass_of(pl, steps[i].k, &pass, &len);
            passes[i] = (int)pass;
        }
    }
    *n = ns;
    return FSA_OK;
}

fsa_status fsa_apply_events(fsa_plan pl, const void* rho, void* phi, void* workspace,
                            void* stream, void* const* events, int n_events) {
    if (!pl || !events) return fail(FSA_EINVAL, "fsa_apply_events: null argument");
    fsa::Step steps[fsa::kMaxSteps];
    const int need = 2 * fsa::schedule(pl, fsa::tune::get_slabs(pl), steps);
    if (n_events != need)
        return fail(FSA_EINVAL, "fsa_apply_events: need %d events (2 per launch), got %d", need,
                    n_events);
    for (int i = 0; i < need; i += 2)
        if (!events[i] != !events[i + 1])
            return fail(FSA_EINVAL, "fsa_apply_events: launch %d has one null event", i / 2);
    return apply_checked(pl, rho, phi, workspace, stream, (hipEvent_t const*)events);
}

fsa_status fsa_plan_tensor(fsa_plan pl, const void** tensor, int64_t* dims) {
    if (!pl || !tensor || !dims) return fail(FSA_EINVAL, "fsa_plan_tensor: null argument");
    if (!pl->built) return fail(FSA_ESTATE, "fsa_plan_tensor: tensor not built");
    *tensor = pl->tensor;
    for (int j = 0; j < pl->d; ++j) dims[j] = pl->N[pl->d - 1 - j] + 1;
    return FSA_OK;
}

fsa_status fsa_plan_destroy(fsa_plan pl) {
    if (!pl) return FSA_OK;
    fsa::batch_forget_plan(pl->id);
    hipError_t e = hipSuccess;
    if (pl->tensor || pl->twiddles || pl->line_order) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (pl->device >= 0 && pl->device != cur) (void)hipSetDevice(pl->device);
        if (pl->tensor) e = hipFree(pl->tensor);
        if (pl->twiddles) {
            hipError_t e2 = hipFree(pl->twiddles);
            if (e == hipSuccess) e = e2;
        }
        if (pl->line_order) {
            hipError_t e2 = hipFree(pl->line_order);
            if (e == hipSuccess) e = e2;
        }
        if (pl->device >= 0 && pl->device != cur) (void)hipSetDevice(cur);
    }
    delete pl;
    if (e != hipSuccess) return hip_fail(e, "fsa_plan_destroy: hipFree");
    return FSA_OK;
}

}  // extern "C"
