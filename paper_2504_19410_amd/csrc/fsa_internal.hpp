// fsa_internal.hpp -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstddef>
#include <cstdint>

#include "../../include/fsa.h"
#include "fsa_fft.hpp"
#include "fsa_jobs.hpp"

struct fsa_plan_s;

namespace fsa {

// A named host-side range for profilers (roctx: rocprofv3 --marker-trace
// shows it on the calling thread's timeline); costs a library call when no
// tool is attached.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// Launches a kernel and returns the launch status.
template <typename... Params, typename... Args>
inline hipError_t launch_kernel(void (*kernel)(Params...), dim3 grid, dim3 block,
                                unsigned shmem, hipStream_t st, Args... args) {
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, static_cast<Params>(args)...);
    return hipGetLastError();
}

struct KernelParams {
    int kind;
    double lam;
    double eps;
    int general = 0;   // general construction: U^eps = U erf(r/eps)(1 - xi), W by quadrature
    double eta = 0.0;  // quasi-2D DDI confinement width
};

// Whether U erf(r/eps) is not smooth at r = 0, so that the general
// construction multiplies it by the window 1 - xi(r).
inline bool kernel_windowed(int kind) {
    return !(kind == FSA_COULOMB_3D || kind == FSA_COULOMB_2D || kind == FSA_BIHARMONIC_3D ||
             kind == FSA_DDI_3D);
}

// Supported grid lengths N (8 <= N <= 2048, N = 2^a or 3 * 2^a): the padded
// transform 2N and, on the contiguous axis, the half-length N must both be
// supported transform lengths.
inline bool grid_length_supported(int64_t n) {
    return n >= 8 && n <= 2048 && (n % 2) == 0 && fft_length_supported(n) &&
           fft_length_supported(2 * n);
}

// Forget cached batch graphs that use a plan (fsa_batch.cpp).
void batch_forget_plan(uint64_t plan_id);

// The source launches of a dipole-dipole plan (fsa_spectral.hip): step s in
// [0, n_spectral) of the spectral derivative on the N-grid, reading rho and
// leaving the real source (plan precision) at dst: -3 d_nm rho (3D, five
// launches) or -(3/2)(d_{n_perp n_perp} - n_3^2 Lap) rho (quasi-2D, three).
hipError_t spectral_step(const fsa_plan_s* pl, int s, const void* rho, void* z, void* dst,
                         hipStream_t st);

// Double-double mode (fsa_dd.hip): twiddle elements (complex DD) of a plan,
// its tensor build, and step k of its 2d - 1 evaluation launches.
size_t dd_twiddle_elems(const fsa_plan_s* pl);
hipError_t build_tensor_dd(const fsa_plan_s* pl, hipStream_t st);
hipError_t launch_dd_step(const fsa_plan_s* pl, int k, const void* rho, void* phi, void* ws,
                          hipStream_t st);

// Tensor generation (fsa_tensor.hip).  line_order: the caller's cache of the
// order in which the last axis of a 3D build takes its lines (it depends on
// the grid sizes only): filled with a new device allocation by the first build
// that uses it, reused after that, freed by the caller.
hipError_t build_tensor_device(const KernelParams& kp, int d, const double* L, const int64_t* N,
                               const double* h, fsa_precision prec, void* tensor_out,
                               int** line_order, hipStream_t st);
// tw[m] = exp(-2 pi i m / n), m in [0, n), computed in FP64, stored in prec.
hipError_t build_twiddles(fsa_precision prec, int n, void* out, hipStream_t st);

// Launch configuration of one pass: compile-time variant (0 default, 1
// alternate radix family, 2 half-size workgroups, 3 exchanges across lanes,
// 4 first stage on the matrix cores)
// and the number of resident workgroups per CU the persistent grid uses (0:
// as many as fit).
struct Choice {
    int var = 0;
    int occ = 0;
};
constexpr int kNumVariants = 5;

// Pass launchers of one variant (fsa_launch_<prec>_v<var>.hip).  Complex
// arrays are interleaved (re, im) of R.  Each returns hipErrorInvalidValue
// for an unsupported length, or for a variant that is not distinct from
// variant 0 at that length.
template <typename R, int VAR>
struct LaunchV {
    static hipError_t r2c(int M, const R* rho, void* out, int n_outer, int n_inner,
                          const void* twM, const void* tw2M, int occ, hipStream_t st);
    static hipError_t c2r(int M, const void* in, R* phi, int n_outer, int n_inner,
                          const void* add, double alpha, const void* twM, const void* tw2M,
                          int occ, hipStream_t st);
    static hipError_t fwd_t(int P, const void* in, void* out, int N0, int H, int p2_lo, int p2_n,
                            const void* tw, int occ, hipStream_t st);
    static hipError_t inv_t(int P, const void* in, void* out, int N0, int H, int p2_lo, int p2_n,
                            const void* tw, int occ, hipStream_t st);
    static hipError_t conv(int P, void* data, const R* tensor, int n_pencils, int P1, int N1,
                           int p2_lo, const void* tw, int occ, hipStream_t st);
    // Work items of one job of `pass` at transform length `len` (-1: unsupported).
    static int items(Pass pass, int len, const void* job);
    // One persistent launch of `pass` over n jobs (device table `jobs` of the
    // pass's job type, device prefix `start` of n + 1 item offsets).
    static hipError_t batch(Pass pass, int len, const void* jobs, const int* start, int n,
                            int total, const void* tw, const void* tw2, int occ,
                            hipStream_t st);
    // Whether this variant exists (differs from variant 0) at (pass, len).
    static bool distinct(Pass pass, int len);
    // Resident workgroups per CU of the single-evaluation kernel (0: none).
    static int max_occ(Pass pass, int len);
};

// Dispatch on the run-time choice.
template <typename R>
struct Launch {
#define FSA_DISPATCH(call)                                      \
    switch (c.var) {                                            \
    case 0: return LaunchV<R, 0>::call;                         \
    case 1: return LaunchV<R, 1>::call;                         \
    case 2: return LaunchV<R, 2>::call;                         \
    case 3: return LaunchV<R, 3>::call;                         \
    case 4: return LaunchV<R, 4>::call;                         \
    }                                                           \
    return hipErrorInvalidValue;
    static hipError_t r2c(int M, const R* rho, void* out, int n_outer, int n_inner,
                          const void* twM, const void* tw2M, Choice c, hipStream_t st) {
        FSA_DISPATCH(r2c(M, rho, out, n_outer, n_inner, twM, tw2M, c.occ, st))
    }
    static hipError_t c2r(int M, const void* in, R* phi, int n_outer, int n_inner,
                          const void* add, double alpha, const void* twM, const void* tw2M,
                          Choice c, hipStream_t st) {
        FSA_DISPATCH(c2r(M, in, phi, n_outer, n_inner, add, alpha, twM, tw2M, c.occ, st))
    }
    static hipError_t fwd_t(int P, const void* in, void* out, int N0, int H, int p2_lo, int p2_n,
                            const void* tw, Choice c, hipStream_t st) {
        FSA_DISPATCH(fwd_t(P, in, out, N0, H, p2_lo, p2_n, tw, c.occ, st))
    }
    static hipError_t inv_t(int P, const void* in, void* out, int N0, int H, int p2_lo, int p2_n,
                            const void* tw, Choice c, hipStream_t st) {
        FSA_DISPATCH(inv_t(P, in, out, N0, H, p2_lo, p2_n, tw, c.occ, st))
    }
    static hipError_t conv(int P, void* data, const R* tensor, int n_pencils, int P1, int N1,
                           int p2_lo, const void* tw, Choice c, hipStream_t st) {
        FSA_DISPATCH(conv(P, data, tensor, n_pencils, P1, N1, p2_lo, tw, c.occ, st))
    }
    static hipError_t batch(Pass pass, int len, const void* jobs, const int* start, int n,
                            int total, const void* tw, const void* tw2, Choice c,
                            hipStream_t st) {
        FSA_DISPATCH(batch(pass, len, jobs, start, n, total, tw, tw2, c.occ, st))
    }
#undef FSA_DISPATCH
    static int items(Pass pass, int len, const void* job, Choice c) {
        switch (c.var) {
        case 0: return LaunchV<R, 0>::items(pass, len, job);
        case 1: return LaunchV<R, 1>::items(pass, len, job);
        case 2: return LaunchV<R, 2>::items(pass, len, job);
        case 3: return LaunchV<R, 3>::items(pass, len, job);
        case 4: return LaunchV<R, 4>::items(pass, len, job);
        }
        return -1;
    }
    static bool distinct(Pass pass, int len, int var) {
        switch (var) {
        case 0: return LaunchV<R, 0>::distinct(pass, len);
        case 1: return LaunchV<R, 1>::distinct(pass, len);
        case 2: return LaunchV<R, 2>::distinct(pass, len);
        case 3: return LaunchV<R, 3>::distinct(pass, len);
        case 4: return LaunchV<R, 4>::distinct(pass, len);
        }
        return false;
    }
    static int max_occ(Pass pass, int len, int var) {
        switch (var) {
        case 0: return LaunchV<R, 0>::max_occ(pass, len);
        case 1: return LaunchV<R, 1>::max_occ(pass, len);
        case 2: return LaunchV<R, 2>::max_occ(pass, len);
        case 3: return LaunchV<R, 3>::max_occ(pass, len);
        case 4: return LaunchV<R, 4>::max_occ(pass, len);
        }
        return 0;
    }
};

// Tuning table (fsa_tune.cpp): the launch choice for (precision, pass,
// transform length, size class), the size class being floor(log2(lines)) of
// the transforms one launch runs (rows, lines or pencils): the best variant
// of a length differs between a few hundred lines and a hundred thousand.
// A lookup takes the entry of the nearest tuned size class of that (precision,
// pass, length); variant 0 at full occupancy if there is none.
namespace tune {
int size_class(long lines);
// `batched`: the entries of the batched persistent launches (a batched get
// falls back to the single-evaluation entries where it has none).
Choice get(fsa_precision prec, Pass pass, int len, long lines, bool batched = false);
void set(fsa_precision prec, Pass pass, int len, long lines, Choice c, double us,
         bool batched = false);
// Bumped on every change; batch graphs captured under another generation
// are re-captured.
uint64_t generation();
}  // namespace tune

// One launch of an evaluation: pass k (0-based, in execution order) over
// the bins p2 in [lo, lo + n) (passes B, C, D of a 3D plan; the other passes
// cover everything).
struct Step {
    int k, lo, n;
};
constexpr int kMaxSlabs = 16;
// a dipole-dipole plan runs its n_spectral (at most kSpectralSteps)
// derivative launches first, as steps k = kSpectralStep + i
constexpr int kSpectralStep = 5, kSpectralSteps = 5;
constexpr int kMaxSteps = 2 + 3 * kMaxSlabs + kSpectralSteps;
// Launch order of one evaluation with `slabs` slabs of bins (clamped to
// [1, min(H, kMaxSlabs)]; 2D plans always have 3 launches).
int schedule(const fsa_plan_s* pl, int slabs, Step* out);
hipError_t launch_step(const fsa_plan_s* pl, const Step& s, const void* rho, void* phi, void* ws,
                       Choice c, hipStream_t st);
Choice step_choice(const fsa_plan_s* pl, const Step& s);
// (pass kind, transform length) of pass k of a plan.
void pass_of(const fsa_plan_s* pl, int k, Pass* pass, int* len);
// Transforms (rows, lines or pencils) one launch of a step runs.
long step_lines(const fsa_plan_s* pl, const Step& s);
int n_passes(const fsa_plan_s* pl);

namespace tune {
// Slabs of the schedule for the plan's (precision, grid); 1 unless tuned.
int get_slabs(const fsa_plan_s* pl);
void set_slabs(const fsa_plan_s* pl, int slabs, double us);
}  // namespace tune

}  // namespace fsa

// Plan object behind the opaque fsa_plan handle.
struct fsa_plan_s {
    uint64_t id = 0;  // unique per plan for the lifetime of the process
    fsa::KernelParams kp{};
    int d = 0;
    double L[3] = {1, 1, 1};
    int64_t N[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    fsa_precision prec = FSA_F32;
    // derived sizes
    int64_t H = 0;            // N_{d-1} + 1 bins of the real transform
    size_t csize = 0;         // bytes of one complex value
    size_t ws1_elems = 0;     // complex elements of the first workspace array
    size_t ws2_elems = 0;     // complex elements of the second (3D only)
    size_t ws_bytes = 0;
    size_t tensor_elems = 0;  // octant elements
    // twiddle tables (elements from the start of `twiddles`)
    size_t tw_off_p0 = 0, tw_off_p1 = 0, tw_off_m = 0, tw_off_pl = 0;
    size_t tw_off_n0 = 0, tw_off_n1 = 0;  // DDI: lengths N_0, N_1 (N_last is tw_off_m)
    size_t tw_elems = 0;
    // dipole-dipole plans: the source derivative runs before the passes
    // (n_spectral launches); the 3D one convolves with the Coulomb tensor
    // (kp.kind) and adds -(m.n) rho in its last pass
    bool ddi = false;
    int n_spectral = 0;
    double dn[3] = {0, 0, 0}, dm[3] = {0, 0, 0};
    // device state
    int device = -1;
    void* tensor = nullptr;
    void* twiddles = nullptr;
    int* line_order = nullptr;  // the tensor build's line order (3D cubic boxes), kept
    bool built = false;
};
