// fsa_tensor.hip -- once-per-plan generation of the spectral kernel tensor
// (Precomp), in FP64 on the GPU.
//
// The tensor of eq. DiscConv is T = T(1) + T(2) with
//   T(1)_n = prod_j h_j U^eps(|n h|)                     (eq. Tensor1 / TensorAnis)
//   T(2)   = IDFT over prod_j P_j points of W(|k_p|),     (eq. Tensor2, eq. FouTran)
//            k_j = pi p_j / (2 L_j),  P_j = 2 N_j.
// The evaluation only ever needs DFT(T), and DFT(IDFT(W)) = W exactly, so
//   T^[p] = ( DFT(T(1))[p] + W(|k_p|) ) / prod_j P_j
// is generated directly.  T(1) is real and even on every axis (Sec. 2.3), so
// its DFT is a DCT-I of the octant 0 <= n_j <= N_j along each axis:
//   DFT(T1)[p] = sum_{n=0}^{N} c_n T1[n] cos(pi p n / N),  c_0 = c_N = 1, else 2,
// computed as the length-2N FFT of the even extension of each line.
// Octant storage: axis 0 innermost, index ((a2 D1 + a1) D0 + a0), D_j = N_j + 1.
#include <hip/hip_runtime.h>

#include "fsa_internal.hpp"

namespace fsa {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;

// Ein(x) = sum_{m>=1} (-1)^{m+1} x^m / (m m!)   (Abramowitz & Stegun 5.1.11)
__device__ double d_ein(double x) {
    double t = x, s = x;
    for (int m = 2; m < 80; ++m) {
        t *= -x / (double)m;
        const double add = t / (double)m;
        s += add;
        if (fabs(add) < 1e-17 * fabs(s)) break;
    }
    return s;
}

// E1(x): x < 1 from Ein; otherwise the continued fraction of A&S 5.1.22 in
// its even contraction e^{-x} / (x + 1 - 1/(x + 3 - 4/(x + 5 - ...))),
// evaluated with the modified Lentz method.
__device__ double d_e1(double x) {
    if (x < 1.0) return -kEulerGamma - log(x) + d_ein(x);
    double b = x + 1.0, c = 1e300, d = 1.0 / b, h = d;
    for (int i = 1; i < 300; ++i) {
        const double a = -(double)i * (double)i;
        b += 2.0;
        d = 1.0 / (a * d + b);
        c = b + a / c;
        const double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return h * exp(-x);
}

// (e^{-x}(1 + x + c2 x^2) - 1) / x^2 for small x by its Taylor series,
// coefficients (-1)^n (1/n! - 1/(n-1)! + c2/(n-2)!) of x^n, n >= 2.
__device__ double d_bih_series(double x, double c2) {
    double acc = 0.0, xp = 1.0;
    double fn2 = 1.0;  // (n-2)!
    for (int n = 2; n < 30; ++n) {
        if (n > 2) fn2 *= (double)(n - 2);
        const double fn1 = fn2 * (double)(n - 1), fn = fn1 * (double)n;
        const double sg = (n & 1) ? -1.0 : 1.0;
        acc += sg * (1.0 / fn - 1.0 / fn1 + c2 / fn2) * xp;
        xp *= x;
    }
    return acc;
}

__device__ double d_ueps(const KernelParams& kp, double r) {
    const double eps = kp.eps;
    switch (kp.kind) {
    case FSA_COULOMB_3D:
        return r == 0.0 ? 1.0 / (2.0 * kPi * sqrt(kPi) * eps) : erf(r / eps) / (4.0 * kPi * r);
    case FSA_COULOMB_2D:
        return r == 0.0 ? 1.0 / (kPi * sqrt(kPi) * eps) : erf(r / eps) / (2.0 * kPi * r);
    case FSA_BIHARMONIC_3D:
        return r * erf(r / eps) / (8.0 * kPi);
    case FSA_YUKAWA_3D: {
        const double lam = kp.lam, a = 0.5 * lam * eps;
        if (r == 0.0)
            return (2.0 * exp(-a * a) / (sqrt(kPi) * eps) - lam * erfc(a)) / (4.0 * kPi);
        const double q = r / eps;
        // e^{lam r} erfc(q + a) = exp(lam r - (q + a)^2) erfcx(q + a)
        const double up = exp(lam * r - (q + a) * (q + a)) * erfcx(q + a);
        return (exp(-lam * r) * (1.0 + erf(q - a)) - up) / (8.0 * kPi * r);
    }
    case FSA_LOG_2D: {
        const double x = (r / eps) * (r / eps);
        if (x < 1.0) return -(log(eps) + 0.5 * (d_ein(x) - kEulerGamma)) / (2.0 * kPi);
        return -(log(r) + 0.5 * d_e1(x)) / (2.0 * kPi);
    }
    case FSA_BIHARMONIC_2D: {
        if (r == 0.0) return 0.0;
        const double x = (r / eps) * (r / eps);
        const double in = (x < 1.0) ? log(eps) + 0.5 * (d_ein(x) - kEulerGamma) - 1.0
                                    : log(r) + 0.5 * d_e1(x) - 1.0;
        return -r * r * in / (8.0 * kPi);
    }
    }
    return 0.0;
}

__device__ double d_what(const KernelParams& kp, double k) {
    const double eps = kp.eps, k2 = k * k;
    switch (kp.kind) {
    case FSA_COULOMB_3D:
    case FSA_LOG_2D:
        return k == 0.0 ? 0.25 * eps * eps : -expm1(-0.25 * k2 * eps * eps) / k2;
    case FSA_YUKAWA_3D: {
        const double q = k2 + kp.lam * kp.lam;
        return q == 0.0 ? 0.25 * eps * eps : -expm1(-0.25 * q * eps * eps) / q;
    }
    case FSA_COULOMB_2D:
        return k == 0.0 ? eps / sqrt(kPi) : erf(0.5 * k * eps) / k;
    case FSA_BIHARMONIC_3D:
    case FSA_BIHARMONIC_2D: {
        const double c2 = kp.kind == FSA_BIHARMONIC_3D ? 2.0 : 1.0;
        const double x = 0.25 * k2 * eps * eps, e4 = eps * eps * eps * eps;
        const double g = (x < 0.5) ? d_bih_series(x, c2)
                                   : (exp(-x) * (1.0 + x + c2 * x * x) - 1.0) / (x * x);
        return e4 * g / 16.0;
    }
    }
    return 0.0;
}

struct Oct {
    int D0, D1, D2;
    __device__ void split(long i, int& a0, int& a1, int& a2) const {
        a0 = (int)(i % D0);
        const long r = i / D0;
        a1 = (int)(r % D1);
        a2 = (int)(r / D1);
    }
    __device__ long size() const { return (long)D0 * D1 * D2; }
};

__global__ void k_sample(double* __restrict__ out, Oct o, double h0, double h1, double h2,
                         double hprod, KernelParams kp) {
    const long n = o.size();
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        int a0, a1, a2;
        o.split(i, a0, a1, a2);
        const double x = a0 * h0, y = a1 * h1, z = a2 * h2;
        out[i] = hprod * d_ueps(kp, sqrt(x * x + y * y + z * z));
    }
}

// DCT-I of every octant line along one axis, as the real part of the
// length-2N DFT of the line's even extension (x[n] for n <= N, x[2N - n]
// above), which is sum_n c_n x[n] cos(pi p n / N), c_0 = c_N = 1, else 2.
// A workgroup takes WT lines that are adjacent in the array, stages them
// through LDS (coalesced along the contiguous direction), and each of its
// teams runs the FP64 team FFT of length P = 2N on one line.
constexpr int dct_lines_per_group(int T, int scr, int D) {
    int wt = 8;
    while (wt > 1 && (wt * T > 1024 || wt * scr * 16 + D * (wt + 1) * 8 > 160 * 1024)) wt /= 2;
    return wt;
}

template <int P>
struct Dct {
    using F = Fft<double, P, false>;
    static constexpr int N = P / 2, D = N + 1;
    static constexpr int T = F::T;
    static constexpr int WT = dct_lines_per_group(T, F::SCR, D);
    static constexpr int TS = WT + 1;
    static constexpr int THREADS = WT * T;
};

// Lines of one axis: line (u, v) starts at u * u_stride + v * v_stride and
// its element t sits at + t * es; groups take WT consecutive u.
struct Lines {
    int n_u, n_v;
    long u_stride, v_stride, es;
};

template <int P>
__global__ __launch_bounds__(Dct<P>::THREADS) void k_dct(const double* __restrict__ in,
                                                        double* __restrict__ out, Lines ln,
                                                        const cpx<double>* __restrict__ tw) {
    using K = Dct<P>;
    using F = typename K::F;
    using C = cpx<double>;
    __shared__ C scr[K::WT * F::SCR];
    __shared__ double tile[K::D * K::TS];
    const int team = threadIdx.x / K::T, tid = threadIdx.x % K::T;
    const int ntu = (ln.n_u + K::WT - 1) / K::WT;
    const int tu = blockIdx.x % ntu, v = blockIdx.x / ntu;
    const long base = (long)tu * K::WT * ln.u_stride + (long)v * ln.v_stride;
    const int nw = ln.n_u - tu * K::WT < K::WT ? ln.n_u - tu * K::WT : K::WT;
    // element e of the tile -> (t, w), contiguous direction fastest
    auto at = [&](int e, int& t, int& w) {
        if (ln.es == 1) {
            w = e / K::D;
            t = e - w * K::D;
        } else {
            t = e / K::WT;
            w = e - t * K::WT;
        }
    };
    for (int e = threadIdx.x; e < K::D * K::WT; e += K::THREADS) {
        int t, w;
        at(e, t, w);
        tile[t * K::TS + w] = w < nw ? in[base + w * ln.u_stride + t * ln.es] : 0.0;
    }
    __syncthreads();
    C x[F::V];
    F::load_first(x, tid, P, [&](int i) {
        const int t = i <= K::N ? i : P - i;
        return mk(tile[t * K::TS + team], 0.0);
    });
    __syncthreads();
    F::run_g(x, scr + team * F::SCR, tid, tw);
    F::store_last(x, tid, K::D, [&](int p, C c) { tile[p * K::TS + team] = c.x; });
    __syncthreads();
    for (int e = threadIdx.x; e < K::D * K::WT; e += K::THREADS) {
        int t, w;
        at(e, t, w);
        if (w < nw) out[base + w * ln.u_stride + t * ln.es] = tile[t * K::TS + w];
    }
}

hipError_t dct_axis(const double* in, double* out, Lines ln, int N, const void* tw,
                    hipStream_t st) {
    switch (2 * N) {
#define FSA_DCT_CASE(p)                                                                         \
    case p: {                                                                                   \
        using K = Dct<p>;                                                                       \
        const int groups = (ln.n_u + K::WT - 1) / K::WT * ln.n_v;                               \
        hipLaunchKernelGGL(k_dct<p>, dim3(groups), dim3(K::THREADS), 0, st, in, out, ln,        \
                           (const cpx<double>*)tw);                                             \
        return hipGetLastError();                                                               \
    }
        FSA_DCT_CASE(16) FSA_DCT_CASE(24) FSA_DCT_CASE(32) FSA_DCT_CASE(48) FSA_DCT_CASE(64)
        FSA_DCT_CASE(96) FSA_DCT_CASE(128) FSA_DCT_CASE(192) FSA_DCT_CASE(256) FSA_DCT_CASE(384)
        FSA_DCT_CASE(512) FSA_DCT_CASE(768) FSA_DCT_CASE(1024) FSA_DCT_CASE(1536)
        FSA_DCT_CASE(2048) FSA_DCT_CASE(3072) FSA_DCT_CASE(4096)
#undef FSA_DCT_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R>
__global__ void k_finalize(const double* __restrict__ dct, R* __restrict__ out, Oct o, double c0,
                           double c1, double c2, double inv_prod_p, KernelParams kp) {
    const long n = o.size();
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        int a0, a1, a2;
        o.split(i, a0, a1, a2);
        const double kx = a0 * c0, ky = a1 * c1, kz = a2 * c2;
        const double k = sqrt(kx * kx + ky * ky + kz * kz);
        out[i] = (R)((dct[i] + d_what(kp, k)) * inv_prod_p);
    }
}

template <typename R>
__global__ void k_twiddle(cpx<R>* __restrict__ tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = mk<R>((R)c, (R)-s);
    }
}

int grid_for(long n, int block) {
    const long g = (n + block - 1) / block;
    return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

}  // namespace

hipError_t build_twiddles(fsa_precision prec, int n, void* out, hipStream_t st) {
    const int block = 256, grid = (n + block - 1) / block;
    if (prec == FSA_F32)
        hipLaunchKernelGGL(k_twiddle<float>, dim3(grid), dim3(block), 0, st, (cpx<float>*)out, n);
    else
        hipLaunchKernelGGL(k_twiddle<double>, dim3(grid), dim3(block), 0, st, (cpx<double>*)out, n);
    return hipGetLastError();
}

hipError_t build_tensor_device(const KernelParams& kp, int d, const double* L, const int64_t* N,
                               const double* h, fsa_precision prec, void* tensor_out,
                               hipStream_t st) {
    // octant extents, axis 0 innermost; a 2D plan has D2 = 1
    Oct o{(int)N[0] + 1, (int)N[1] + 1, d == 3 ? (int)N[2] + 1 : 1};
    const long n = (long)o.D0 * o.D1 * o.D2;
    int maxN = 0;
    for (int j = 0; j < d; ++j) maxN = (int)N[j] > maxN ? (int)N[j] : maxN;
    double *a = nullptr, *b = nullptr;
    void* tw = nullptr;
    hipError_t e = hipMallocAsync((void**)&a, sizeof(double) * n, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&b, sizeof(double) * n, st);
    if (e == hipSuccess) e = hipMallocAsync(&tw, 2 * sizeof(double) * 2 * maxN, st);
    if (e != hipSuccess) {
        if (a) (void)hipFreeAsync(a, st);
        if (b) (void)hipFreeAsync(b, st);
        return e;
    }
    const int block = 256, grid = grid_for(n, block);
    const double h2 = d == 3 ? h[2] : 1.0;
    const double hprod = h[0] * h[1] * h2;
    hipLaunchKernelGGL(k_sample, dim3(grid), dim3(block), 0, st, a, o, h[0], h[1],
                       d == 3 ? h[2] : 0.0, hprod, kp);
    double* src = a;
    double* dst = b;
    const long D0 = o.D0, D1 = o.D1, D2 = o.D2;
    for (int ax = 0; ax < d && e == hipSuccess; ++ax) {
        // lines along axis ax; groups take lines adjacent in memory
        Lines ln;
        if (ax == 0) ln = Lines{(int)D1, (int)D2, D0, D0 * D1, 1};
        else if (ax == 1) ln = Lines{(int)D0, (int)D2, 1, D0 * D1, D0};
        else ln = Lines{(int)D0, (int)D1, 1, D0, D0 * D1};
        e = build_twiddles(FSA_F64, (int)(2 * N[ax]), tw, st);
        if (e == hipSuccess) e = dct_axis(src, dst, ln, (int)N[ax], tw, st);
        double* t = src;
        src = dst;
        dst = t;
    }
    double prodP = 1.0;
    for (int j = 0; j < d; ++j) prodP *= 2.0 * (double)N[j];
    const double c0 = kPi / (2.0 * L[0]), c1 = kPi / (2.0 * L[1]);
    const double c2 = d == 3 ? kPi / (2.0 * L[2]) : 0.0;
    if (prec == FSA_F32)
        hipLaunchKernelGGL(k_finalize<float>, dim3(grid), dim3(block), 0, st, (const double*)src,
                           (float*)tensor_out, o, c0, c1, c2, 1.0 / prodP, kp);
    else
        hipLaunchKernelGGL(k_finalize<double>, dim3(grid), dim3(block), 0, st, (const double*)src,
                           (double*)tensor_out, o, c0, c1, c2, 1.0 / prodP, kp);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipFreeAsync(a, st);
    (void)hipFreeAsync(b, st);
    (void)hipFreeAsync(tw, st);
    return e;
}

}  // namespace fsa
