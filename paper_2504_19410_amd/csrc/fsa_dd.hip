// fsa_dd.hip -- the extended-precision (double-double) mode: tensor build and
// evaluation, Coulomb kernels (Table 1), grids N_j = 2^a <= 1024.
//
// The paper runs its method in quadruple precision to reach errors near
// 1e-34 once the tensor is generated in high precision (Sec. 5.1, Table 2).
// gfx950 has no FP128; double-double (hi + lo, 106 bits, fsa_dd.hpp) is the
// closest native format.  The method is the same as in FP32/FP64:
//   tensor  T^[p] = (DCT-I(T(1))[p] + W(|k_p|)) / prod P_j  on the octant
//           (the DCT-I as the real part of the DFT of the even extension),
//           T(1) = prod h_j U^eps(|n h|), U^eps = erf(r/eps)/(4 pi r) (3D) or
//           erf(r/eps)/(2 pi r) (2D), W = (1 - e^{-k^2 eps^2/4})/k^2 (3D) or
//           erf(k eps/2)/k (2D);
//   passes  the 2x zero-padded convolution, forward FFTs along the axes from
//           the last to axis 1, the fused forward FFT x T^ x inverse FFT
//           along axis 0, inverse FFTs back; input zero padding and output
//           crop folded into the loads and stores.
// Unlike the FP32/FP64 path it keeps the whole complex padded spectrum
// (prod P_j values of 32 bytes) and transforms one line per workgroup with a
// radix-4 FFT in LDS: this mode is about accuracy, not bandwidth.
// Arrays of reals are interleaved (hi, lo) pairs; complex values are
// (re.hi, re.lo, im.hi, im.lo).
#include <hip/hip_runtime.h>

#include "fsa_dd.hpp"
#include "fsa_internal.hpp"

namespace fsa {

namespace {

struct cdd {
    dd re, im;
};

__device__ __forceinline__ cdd cadd(cdd a, cdd b) { return cdd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cdd csub(cdd a, cdd b) { return cdd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cdd cmul(cdd a, cdd b) {
    return cdd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cdd cconj(cdd a) { return cdd{a.re, -a.im}; }

constexpr int kDDThreads = 256;
constexpr int kDDMaxP = 2048;
// threads per line: one per radix-4 butterfly, at most kDDThreads
constexpr int dd_threads(int P) { return P / 4 < 1 ? 1 : P / 4 < kDDThreads ? P / 4 : kDDThreads; }

// tw[m] = exp(-2 pi i m / P), m < P/2
__global__ void k_dd_twiddle(cdd* __restrict__ tw, int P) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= P / 2) return;
    dd s, c;
    dd_sincos_turn((double)m / (double)P, &s, &c);
    tw[m] = cdd{c, -s};
}

struct DDGeom {
    int d;
    int N[3], P[3];
    double L[3];
    double eps;
    int kind;
};

__device__ void octant_index(long i, const int* D, int d, int* a) {
    a[0] = (int)(i % D[0]);
    long r = i / D[0];
    a[1] = d > 1 ? (int)(r % D[1]) : 0;
    a[2] = d > 2 ? (int)(r / D[1]) : 0;
}

// T(1) on the octant (axis 0 innermost), FP64-free: every step in DD.
__global__ void k_dd_sample(dd* __restrict__ out, DDGeom g) {
    int D[3] = {g.N[0] + 1, g.d > 1 ? g.N[1] + 1 : 1, g.d > 2 ? g.N[2] + 1 : 1};
    const long n = (long)D[0] * D[1] * D[2];
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a[3];
    octant_index(i, D, g.d, a);
    dd r2 = dd_of(0.0), hprod = dd_of(1.0);
    for (int j = 0; j < g.d; ++j) {
        const dd h = dd_of(2.0 * g.L[j]) / dd_of((double)g.N[j]);
        hprod = hprod * h;
        const dd x = h * (double)a[j];
        r2 = r2 + x * x;
    }
    const dd eps = dd_of(g.eps);
    const dd sqpi = dd_sqrt(dd_pi());
    dd u;
    if (r2.hi == 0.0) {
        // limits of erf(r/eps)/(c r): 2/(sqrt(pi) eps c)
        u = g.kind == FSA_COULOMB_3D ? dd_of(1.0) / (dd_pi() * sqpi * eps * 2.0)
                                     : dd_of(1.0) / (dd_pi() * sqpi * eps);
    } else {
        const dd r = dd_sqrt(r2);
        const dd e = dd_erf(r / eps);
        u = g.kind == FSA_COULOMB_3D ? e / (dd_pi() * r * 4.0) : e / (dd_pi() * r * 2.0);
    }
    out[i] = hprod * u;
}

// T^ = (DCT(T1) + W(|k|)) / prod P_j
__global__ void k_dd_finalize(const dd* __restrict__ dct, dd* __restrict__ out, DDGeom g) {
    int D[3] = {g.N[0] + 1, g.d > 1 ? g.N[1] + 1 : 1, g.d > 2 ? g.N[2] + 1 : 1};
    const long n = (long)D[0] * D[1] * D[2];
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a[3];
    octant_index(i, D, g.d, a);
    dd k2 = dd_of(0.0);
    double prodP = 1.0;
    for (int j = 0; j < g.d; ++j) {
        const dd k = dd_pi() * (double)a[j] / (2.0 * g.L[j]);
        k2 = k2 + k * k;
        prodP *= (double)g.P[j];
    }
    const dd eps = dd_of(g.eps);
    dd w;
    if (g.kind == FSA_COULOMB_3D) {
        w = k2.hi == 0.0 ? eps * eps * 0.25 : -dd_expm1(-(k2 * eps * eps * 0.25)) / k2;
    } else {
        const dd sqpi = dd_sqrt(dd_pi());
        if (k2.hi == 0.0) {
            w = eps / sqpi;
        } else {
            const dd k = dd_sqrt(k2);
            w = dd_erf(k * eps * 0.5) / k;
        }
    }
    out[i] = (dct[i] + w) / prodP;  // prod P_j is a power of two: exact
}

// ---------------------------------------------------------------------------
// Evaluation: one line per workgroup, radix-4 steps in LDS.
// ---------------------------------------------------------------------------

// In-place decimation in time on x[0, P) (bit-reversed order in, natural
// order out); tw[m] = exp(-2 pi i m / P), m < P/2.  The radix-2 stages run in
// pairs (len/2, len) as one radix-4 step per group of four points, with one
// exchange through LDS per pair, after a leading radix-2 stage when log2 P is
// odd: points i0, i0 + q, i0 + 2q, i0 + 3q (q = len/4, j = i0 mod len < q)
// take the len/2 stage's twiddle w_len^(2j) on the odd points of each half,
// then the len stage's w_len^j on the second half, times -i (forward) or +i
// (inverse) for the upper pair.
template <bool INV>
__device__ void dd_fft_lds(cdd* x, int P, int logP, const cdd* __restrict__ tw) {
    int len = 4;
    if (logP & 1) {
        for (int b = threadIdx.x; b < P / 2; b += blockDim.x) {
            const cdd u = x[2 * b], v = x[2 * b + 1];
            x[2 * b] = cadd(u, v);
            x[2 * b + 1] = csub(u, v);
        }
        __syncthreads();
        len = 8;
    }
    for (; len <= P; len <<= 2) {
        const int q = len >> 2, step = P / len;
        for (int b = threadIdx.x; b < P / 4; b += blockDim.x) {
            const int g = b / q, j = b - g * q;
            const int i0 = g * len + j;
            const cdd w2 = INV ? cconj(tw[2 * j * step]) : tw[2 * j * step];
            const cdd wa = INV ? cconj(tw[j * step]) : tw[j * step];
            const cdd a0 = x[i0], a1 = cmul(x[i0 + q], w2);
            const cdd a2 = x[i0 + 2 * q], a3 = cmul(x[i0 + 3 * q], w2);
            const cdd b0 = cadd(a0, a1), b1 = csub(a0, a1);
            const cdd b2 = cadd(a2, a3), b3 = csub(a2, a3);
            const cdd t2 = cmul(b2, wa);
            const cdd u3 = cmul(b3, wa);
            const cdd t3 = INV ? cdd{-u3.im, u3.re} : cdd{u3.im, -u3.re};
            x[i0] = cadd(b0, t2);
            x[i0 + 2 * q] = csub(b0, t2);
            x[i0 + q] = cadd(b1, t3);
            x[i0 + 3 * q] = csub(b1, t3);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int t, int logP) {
    return (int)(__brev((unsigned)t) >> (32 - logP));
}

// DCT-I along axis ax of the octant (D_j = N_j + 1 points per axis), as the
// real part of the length-2N DFT of each line's even extension (x[m] for
// m <= N, x[2N - m] above): sum_m c_m x[m] cos(pi p m / N), c_0 = c_N = 1,
// else 2.  One line per workgroup; tw: the axis' twiddles of length 2N.
__global__ __launch_bounds__(kDDThreads) void k_dd_dct(const dd* __restrict__ in,
                                                     dd* __restrict__ out, DDGeom g, int ax,
                                                     const cdd* __restrict__ tw) {
    extern __shared__ cdd x[];
    const int D0 = g.N[0] + 1, D1 = g.d > 1 ? g.N[1] + 1 : 1;
    const int N = g.N[ax], P = 2 * N;
    int logP = 0;
    while ((1 << logP) < P) ++logP;
    const long l = blockIdx.x;
    long base, stride;
    if (ax == 0) {
        base = l * D0;  // l = a2 D1 + a1
        stride = 1;
    } else if (ax == 1) {
        base = (l / D0) * (long)D1 * D0 + l % D0;  // l = a2 D0 + a0
        stride = D0;
    } else {
        base = l;  // l = a1 D0 + a0
        stride = (long)D0 * D1;
    }
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const int m = t <= N ? t : P - t;
        x[bitrev(t, logP)] = cdd{in[base + m * stride], dd_of(0.0)};
    }
    __syncthreads();
    dd_fft_lds<false>(x, P, logP, tw);
    for (int p = threadIdx.x; p <= N; p += blockDim.x) out[base + p * stride] = x[p].re;
}

// Where a line lives: element t of line l is at base(l) + t * es, with
// base(l) = (l / nb) * sa + (l % nb) * sb (a two-level line index).
struct DDLines {
    long sa, sb, es;
    int nb;
    __device__ long base(long l) const { return (l / nb) * sa + (l % nb) * sb; }
};

enum DDMode { DD_FWD_REAL = 0, DD_FWD = 1, DD_CONV = 2, DD_INV = 3, DD_INV_REAL = 4 };

struct DDConv {  // octant lookup of T^ along axis-0 lines at (p1, p2)
    const dd* tensor;
    int N[3], P[3], D0, D1, d;
};

// One line: load n_in inputs (the rest zero), transform, store n_out outputs.
template <int MODE>
__global__ __launch_bounds__(kDDThreads) void k_dd_pass(const void* __restrict__ in,
                                                        void* __restrict__ out, DDLines li,
                                                        DDLines lo, int P, int logP, int n_in,
                                                        int n_out, const cdd* __restrict__ tw,
                                                        DDConv cv) {
    extern __shared__ cdd x[];
    const long line = blockIdx.x;
    const long bi = li.base(line), bo = lo.base(line);
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        cdd v = cdd{dd_of(0.0), dd_of(0.0)};
        if (t < n_in) {
            if constexpr (MODE == DD_FWD_REAL) v.re = ((const dd*)in)[bi + t * li.es];
            else v = ((const cdd*)in)[bi + t * li.es];
        }
        x[bitrev(t, logP)] = v;
    }
    __syncthreads();
    if constexpr (MODE == DD_CONV) {
        dd_fft_lds<false>(x, P, logP, tw);
        // line at (p1, p2) = (line / P2, line % P2) in 3D, p1 = line in 2D
        int a1, a2 = 0;
        if (cv.d == 3) {
            const int p1 = (int)(line / cv.P[2]), p2 = (int)(line % cv.P[2]);
            a1 = p1 <= cv.N[1] ? p1 : cv.P[1] - p1;
            a2 = p2 <= cv.N[2] ? p2 : cv.P[2] - p2;
        } else {
            const int p1 = (int)line;
            a1 = p1 <= cv.N[1] ? p1 : cv.P[1] - p1;
        }
        const dd* trow = cv.tensor + ((long)a2 * cv.D1 + a1) * cv.D0;
        // x (natural order) times T^, back into bit-reversed order for the
        // inverse: every product is formed before any is written back (at
        // most P / blockDim <= 8 per thread)
        // (fixed trip counts keep the array in registers)
        constexpr int kKeep = kDDMaxP / kDDThreads;  // P / blockDim (blockDim = min(P/4, 256))
        static_assert(kDDMaxP / kDDThreads <= kKeep, "keep array too small");
        cdd keep[kKeep];
#pragma unroll
        for (int r = 0; r < kKeep; ++r) {
            const int t = threadIdx.x + r * blockDim.x;
            if (t < P) {
                const int a0 = t <= cv.N[0] ? t : P - t;
                const dd s = trow[a0];
                cdd v = x[t];
                v.re = v.re * s;
                v.im = v.im * s;
                keep[r] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kKeep; ++r) {
            const int t = threadIdx.x + r * blockDim.x;
            if (t < P) x[bitrev(t, logP)] = keep[r];
        }
        __syncthreads();
    }
    if constexpr (MODE == DD_FWD || MODE == DD_FWD_REAL) dd_fft_lds<false>(x, P, logP, tw);
    else dd_fft_lds<true>(x, P, logP, tw);
    for (int t = threadIdx.x; t < n_out; t += blockDim.x) {
        if constexpr (MODE == DD_INV_REAL) ((dd*)out)[bo + t * lo.es] = x[t].re;
        else ((cdd*)out)[bo + t * lo.es] = x[t];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

size_t dd_twiddle_elems(const fsa_plan_s* pl) {
    size_t n = 0;
    for (int j = 0; j < pl->d; ++j) n += (size_t)pl->N[j];  // P_j / 2 each
    return n;
}

static const cdd* dd_tw(const fsa_plan_s* pl, int ax) {
    size_t off = 0;
    for (int j = 0; j < ax; ++j) off += (size_t)pl->N[j];
    return (const cdd*)pl->twiddles + off;
}

hipError_t build_tensor_dd(const fsa_plan_s* pl, hipStream_t st) {
    DDGeom g{};
    g.d = pl->d;
    g.eps = pl->kp.eps;
    g.kind = pl->kp.kind;
    for (int j = 0; j < 3; ++j) {
        g.N[j] = j < pl->d ? (int)pl->N[j] : 1;
        g.P[j] = 2 * g.N[j];
        g.L[j] = j < pl->d ? pl->L[j] : 1.0;
    }
    // twiddles of every axis
    size_t off = 0;
    for (int j = 0; j < pl->d; ++j) {
        const int half = (int)pl->N[j];
        hipLaunchKernelGGL(k_dd_twiddle, dim3((half + 255) / 256), dim3(256), 0, st,
                           (cdd*)pl->twiddles + off, 2 * half);
        off += half;
    }
    const long n = (long)pl->tensor_elems;
    dd *a = nullptr, *b = nullptr;
    hipError_t e = hipMallocAsync((void**)&a, sizeof(dd) * n, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&b, sizeof(dd) * n, st);
    if (e == hipSuccess) {
        const int grid = (int)((n + 255) / 256);
        hipLaunchKernelGGL(k_dd_sample, dim3(grid), dim3(256), 0, st, a, g);
        dd* src = a;
        dd* dst = b;
        for (int ax = 0; ax < pl->d; ++ax) {
            const int P = 2 * g.N[ax];
            const long lines = n / (g.N[ax] + 1);
            const int threads = dd_threads(P);
            hipLaunchKernelGGL(k_dd_dct, dim3((unsigned)lines), dim3(threads),
                               sizeof(cdd) * (size_t)P, st, (const dd*)src, dst, g, ax,
                               dd_tw(pl, ax));
            dd* t = src;
            src = dst;
            dst = t;
        }
        hipLaunchKernelGGL(k_dd_finalize, dim3(grid), dim3(256), 0, st, (const dd*)src,
                           (dd*)pl->tensor, g);
        e = hipGetLastError();
    }
    if (a) (void)hipFreeAsync(a, st);
    if (b) (void)hipFreeAsync(b, st);
    return e;
}

// Step k of a double-double evaluation (2d - 1 launches).  X is the full
// padded complex array, C order (P_0, ..., P_{d-1}).
hipError_t launch_dd_step(const fsa_plan_s* pl, int k, const void* rho, void* phi, void* ws,
                          hipStream_t st) {
    const int d = pl->d;
    long N[3], P[3];
    int logP[3];
    for (int j = 0; j < d; ++j) {
        N[j] = pl->N[j];
        P[j] = 2 * N[j];
        int lg = 0;
        while ((1L << lg) < P[j]) ++lg;
        logP[j] = lg;
    }
    cdd* X = (cdd*)ws;
    DDConv cv{};
    cv.tensor = (const dd*)pl->tensor;
    cv.d = d;
    for (int j = 0; j < 3; ++j) {
        cv.N[j] = j < d ? (int)N[j] : 0;
        cv.P[j] = j < d ? (int)P[j] : 1;
    }
    cv.D0 = (int)N[0] + 1;
    cv.D1 = (int)N[1] + 1;
    // pass kinds in order: fwd last (real in), [fwd axis 1], conv axis 0,
    // [inv axis 1], inv last (real out)
    int ax, mode;
    if (d == 3) {
        static const int axes[5] = {2, 1, 0, 1, 2};
        static const int modes[5] = {DD_FWD_REAL, DD_FWD, DD_CONV, DD_INV, DD_INV_REAL};
        ax = axes[k];
        mode = modes[k];
    } else {
        static const int axes[3] = {1, 0, 1};
        static const int modes[3] = {DD_FWD_REAL, DD_CONV, DD_INV_REAL};
        ax = axes[k];
        mode = modes[k];
    }
    const int Pa = (int)P[ax], lg = logP[ax];
    DDLines li{}, lo{};
    long lines = 0;
    int n_in = 0, n_out = 0;
    if (d == 3) {
        switch (mode) {
        case DD_FWD_REAL:  // rows (i0 < N0, i1 < N1) of rho -> X[i0][i1][p2]
            lines = N[0] * N[1];
            li = DDLines{N[1] * N[2], N[2], 1, (int)N[1]};
            lo = DDLines{P[1] * P[2], P[2], 1, (int)N[1]};
            n_in = (int)N[2];
            n_out = (int)P[2];
            break;
        case DD_FWD:  // axis 1 at (i0 < N0, p2): X[i0][t][p2]
            lines = N[0] * P[2];
            li = lo = DDLines{P[1] * P[2], 1, P[2], (int)P[2]};
            n_in = (int)N[1];
            n_out = (int)P[1];
            break;
        case DD_CONV:  // axis 0 at (p1, p2): X[t][p1][p2]
            lines = P[1] * P[2];
            li = lo = DDLines{P[2], 1, P[1] * P[2], (int)P[2]};
            n_in = n_out = (int)N[0];
            break;
        case DD_INV:
            lines = N[0] * P[2];
            li = lo = DDLines{P[1] * P[2], 1, P[2], (int)P[2]};
            n_in = (int)P[1];
            n_out = (int)N[1];
            break;
        default:  // DD_INV_REAL: X[i0][i1][t] -> phi rows
            lines = N[0] * N[1];
            li = DDLines{P[1] * P[2], P[2], 1, (int)N[1]};
            lo = DDLines{N[1] * N[2], N[2], 1, (int)N[1]};
            n_in = (int)P[2];
            n_out = (int)N[2];
            break;
        }
    } else {
        switch (mode) {
        case DD_FWD_REAL:  // rows i0 < N0 -> X[i0][p1]
            lines = N[0];
            li = DDLines{N[1], 0, 1, 1};
            lo = DDLines{P[1], 0, 1, 1};
            n_in = (int)N[1];
            n_out = (int)P[1];
            break;
        case DD_CONV:  // axis 0 at p1: X[t][p1]
            lines = P[1];
            li = lo = DDLines{1, 0, P[1], 1};
            n_in = n_out = (int)N[0];
            break;
        default:
            lines = N[0];
            li = DDLines{P[1], 0, 1, 1};
            lo = DDLines{N[1], 0, 1, 1};
            n_in = (int)P[1];
            n_out = (int)N[1];
            break;
        }
    }
    if (Pa > kDDMaxP || lines <= 0 || lines > 0x7fffffffL) return hipErrorInvalidValue;
    const int threads = dd_threads(Pa);
    const size_t lds = sizeof(cdd) * (size_t)Pa;
    const cdd* tw = dd_tw(pl, ax);
    const void* src = mode == DD_FWD_REAL ? rho : (const void*)X;
    void* dst = mode == DD_INV_REAL ? phi : (void*)X;
    switch (mode) {
    case DD_FWD_REAL:
        return launch_kernel(k_dd_pass<DD_FWD_REAL>, dim3((unsigned)lines), dim3(threads), lds, st,
                             src, dst, li, lo, Pa, lg, n_in, n_out, tw, cv);
    case DD_FWD:
        return launch_kernel(k_dd_pass<DD_FWD>, dim3((unsigned)lines), dim3(threads), lds, st,
                             src, dst, li, lo, Pa, lg, n_in, n_out, tw, cv);
    case DD_CONV:
        return launch_kernel(k_dd_pass<DD_CONV>, dim3((unsigned)lines), dim3(threads), lds, st,
                             src, dst, li, lo, Pa, lg, n_in, n_out, tw, cv);
    case DD_INV:
        return launch_kernel(k_dd_pass<DD_INV>, dim3((unsigned)lines), dim3(threads), lds, st,
                             src, dst, li, lo, Pa, lg, n_in, n_out, tw, cv);
    default:
        return launch_kernel(k_dd_pass<DD_INV_REAL>, dim3((unsigned)lines), dim3(threads), lds, st,
                             src, dst, li, lo, Pa, lg, n_in, n_out, tw, cv);
    }
}

}  // namespace fsa
