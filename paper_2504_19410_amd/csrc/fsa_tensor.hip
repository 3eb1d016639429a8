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
//
// General construction (Sec. 4, eq. GeneralApprox1): U^eps = U erf(r/eps)
// (1 - xi(r)) with the window xi(r) = erfc((r - 6 eps)/eps)/2 where
// U erf(r/eps) is not smooth at r = 0, and W(k) the radial transform of
// U - U^eps (eq. Fourier-Symmetric) by quadrature.  W depends on |k| only and
// is smooth (analytic) in it, so it is computed at Chebyshev points of short
// panels of |k| and the finalize kernel evaluates the panel's Chebyshev
// interpolant at each lattice |k|:
//   k_wq_nodes   quadrature weights g_i = c_d w_i r_i^{d-1} (U - U^eps)(r_i)
//                on composite 16-point Gauss-Legendre panels of [0, R_end]
//                (geometrically graded towards r = 0 for the 2D kernels with
//                a logarithm there);
//   k_wq_sum     W(kappa) = sum_i g_i J0(kappa r_i)  (2D)  or
//                           sum_i g_i sin(kappa r_i)/(kappa r_i)  (3D),
//                one workgroup per Chebyshev node kappa;
//   k_cheb       Chebyshev coefficients of each panel's interpolant.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

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

// ---------------------------------------------------------------------------
// General construction
// ---------------------------------------------------------------------------

// K0(x), 0 < x <= 1, by its ascending series (A&S 9.6.13 with 9.6.12):
// K0 = -(ln(x/2) + gamma) I0(x) + sum_{k>=1} H_k (x^2/4)^k / (k!)^2.
__device__ double d_k0_series(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, i0 = 1.0, tail = 0.0, hk = 0.0;
    for (int k = 1; k < 30; ++k) {
        term *= q / ((double)k * (double)k);
        hk += 1.0 / (double)k;
        i0 += term;
        tail += hk * term;
        if (term < 1e-18 * i0) break;
    }
    return -(log(0.5 * x) + kEulerGamma) * i0 + tail;
}

// e^x K0(x), x > 1: the trapezoidal rule on
// e^x K0(x) = int_0^inf e^{-2 x sinh^2(t/2)} dt  (A&S 9.6.24).  The integrand
// is analytic in a strip and decays double-exponentially, so the rule
// converges geometrically; the step min(0.2, 0.65/sqrt(x)) also resolves its
// width 1/sqrt(x) at large x (relative error below 1e-15 for all x > 1, at
// most ~25 terms).
__device__ double d_k0e_large(double x) {
    const double tau = fmin(0.2, 0.65 / sqrt(x));
    double s = 0.5;
    for (int j = 1; j < 64; ++j) {
        const double sh = sinh(0.5 * j * tau);
        const double v = exp(-2.0 * x * sh * sh);
        s += v;
        if (v < 1e-18) break;
    }
    return tau * s;
}

__device__ double d_k0(double x) { return x <= 1.0 ? d_k0_series(x) : exp(-x) * d_k0e_large(x); }
__device__ double d_k0e(double x) {
    return x <= 1.0 ? exp(x) * d_k0_series(x) : d_k0e_large(x);
}

// U(r), r > 0
__device__ double d_u(const KernelParams& kp, double r) {
    switch (kp.kind) {
    case FSA_COULOMB_3D: return 1.0 / (4.0 * kPi * r);
    case FSA_YUKAWA_3D: return exp(-kp.lam * r) / (4.0 * kPi * r);
    case FSA_LOG_2D: return -log(r) / (2.0 * kPi);
    case FSA_COULOMB_2D: return 1.0 / (2.0 * kPi * r);
    case FSA_BIHARMONIC_3D: return r / (8.0 * kPi);
    case FSA_BIHARMONIC_2D: return -r * r * (log(r) - 1.0) / (8.0 * kPi);
    case FSA_YUKAWA_2D: return d_k0(kp.lam * r) / (2.0 * kPi);
    case FSA_QUASI2D_DDI: {
        const double x = r * r / (4.0 * kp.eta * kp.eta);
        return d_k0e(x) / (2.0 * kPi * sqrt(2.0 * kPi) * kp.eta);
    }
    }
    return 0.0;
}

__device__ bool d_windowed(int kind) {
    return !(kind == FSA_COULOMB_3D || kind == FSA_COULOMB_2D || kind == FSA_BIHARMONIC_3D);
}

// U^eps of the general construction; r = 0 takes the limit of
// U erf(r/eps) (1 - xi(r)).
__device__ double d_ueps_general(const KernelParams& kp, double r) {
    const double eps = kp.eps;
    const bool win = d_windowed(kp.kind);
    const double keep0 = 0.5 * erfc(6.0);  // 1 - xi(0)
    if (r == 0.0) {
        double lim = 0.0;  // r ln r, r and r^3 ln r vanish
        if (kp.kind == FSA_COULOMB_3D || kp.kind == FSA_YUKAWA_3D)
            lim = 1.0 / (2.0 * kPi * sqrt(kPi) * eps);
        else if (kp.kind == FSA_COULOMB_2D)
            lim = 1.0 / (kPi * sqrt(kPi) * eps);
        return win ? lim * keep0 : lim;
    }
    const double v = d_u(kp, r) * erf(r / eps);
    return win ? v * 0.5 * erfc((6.0 * eps - r) / eps) : v;
}

// (U - U^eps)(r) = U(r) [erfc(r/eps) + erf(r/eps) xi(r)], r > 0
__device__ double d_remainder(const KernelParams& kp, double r) {
    const double eps = kp.eps;
    double g = erfc(r / eps);
    if (d_windowed(kp.kind)) g += erf(r / eps) * 0.5 * erfc((r - 6.0 * eps) / eps);
    return d_u(kp, r) * g;
}

constexpr int kGl = 16;  // Gauss-Legendre points per panel
constexpr int kCheb = 24;  // Chebyshev degree per |k| panel

struct Gl16 {
    double x[kGl], w[kGl];  // nodes and weights on [-1, 1]
};

// Panels of [0, R_end]: n_uni uniform panels of width wu; with `graded`
// levels the first of them is replaced by [0, wu s^G], [wu s^{m+1}, wu s^m]
// (m = G-1 .. 0).
struct QMesh {
    double wu, sigma;
    int n_uni, graded;
    __device__ int n_panels() const { return graded ? n_uni + graded : n_uni; }
    __device__ void panel(int p, double& a, double& b) const {
        if (graded) {
            if (p == 0) {
                a = 0.0;
                b = wu * pow(sigma, (double)graded);
                return;
            }
            if (p <= graded) {
                a = wu * pow(sigma, (double)(graded - p + 1));
                b = wu * pow(sigma, (double)(graded - p));
                return;
            }
            p -= graded;
        }
        a = wu * p;
        b = wu * (p + 1);
    }
};

__global__ void k_wq_nodes(double* __restrict__ g, double* __restrict__ rn, QMesh m, Gl16 gl,
                           int d, KernelParams kp) {
    const int n = m.n_panels() * kGl;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a, b;
    m.panel(i / kGl, a, b);
    const int j = i % kGl;
    const double hw = 0.5 * (b - a), r = 0.5 * (a + b) + hw * gl.x[j];
    const double cd = d == 2 ? 2.0 * kPi * r : 4.0 * kPi * r * r;
    rn[i] = r;
    g[i] = hw * gl.w[j] * cd * d_remainder(kp, r);
}

// Chebyshev point l of |k| panel q
__device__ double cheb_node(int q, int l, double dk) {
    return dk * (q + 0.5 * (1.0 + cospi((double)l / kCheb)));
}

// out[node] = sum_i g_i J0(kappa r_i) (2D) or sin(kappa r_i)/(kappa r_i) (3D)
// at the Chebyshev points node = node0 + blockIdx.x
__global__ __launch_bounds__(256) void k_wq_sum(const double* __restrict__ g,
                                                const double* __restrict__ rn, int n, int d,
                                                double dk, int node0, double* __restrict__ out) {
    __shared__ double red[256];
    const int node = node0 + (int)blockIdx.x;
    const double kap = cheb_node(node / (kCheb + 1), node % (kCheb + 1), dk);
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double x = kap * rn[i];
        const double f = d == 2 ? j0(x) : (x == 0.0 ? 1.0 : sin(x) / x);
        s += g[i] * f;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (unsigned w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[node] = red[0];
}

// c_j = a_j (halved for j = 0 and j = n), a_j = (2/n) sum''_l f_l cos(pi j l/n):
// the interpolant at the Chebyshev-Lobatto points is sum_j c_j T_j(s).
__global__ void k_cheb(const double* __restrict__ v, double* __restrict__ c, int nq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq * (kCheb + 1)) return;
    const int q = i / (kCheb + 1), j = i % (kCheb + 1);
    const double* f = v + (long)q * (kCheb + 1);
    double a = 0.0;
    for (int l = 0; l <= kCheb; ++l) {
        const double w = (l == 0 || l == kCheb) ? 0.5 : 1.0;
        a += w * f[l] * cospi((double)(j * l % (2 * kCheb)) / kCheb);
    }
    a *= 2.0 / kCheb;
    if (j == 0 || j == kCheb) a *= 0.5;
    c[i] = a;
}

// W(kappa) from the panel's Chebyshev coefficients (Clenshaw)
__device__ double d_what_cheb(const double* __restrict__ cf, double dk, int nq, double kap) {
    int q = (int)(kap / dk);
    if (q >= nq) q = nq - 1;
    const double s = 2.0 * (kap / dk - q) - 1.0;
    const double* c = cf + (long)q * (kCheb + 1);
    double b1 = 0.0, b2 = 0.0;
    for (int j = kCheb; j >= 1; --j) {
        const double b0 = c[j] + 2.0 * s * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + s * b1 - b2;
}

// W of the general construction: Chebyshev coefficients cf of nq panels of
// width dk (null for the closed forms).
struct WTable {
    const double* cf;
    double dk;
    int nq;
};

// DCT-I of every octant line along one axis, as the real part of the
// length-2N DFT of the line's even extension (x[n] for n <= N, x[2N - n]
// above), which is sum_n c_n x[n] cos(pi p n / N), c_0 = c_N = 1, else 2.
// The even extension of a real line has a real DFT, so two lines share one
// complex transform: line a in the real part, line b in the imaginary part,
// and DFT(a + i b) = DFT(a) + i DFT(b) returns both, exactly, in its real and
// imaginary parts.  A workgroup takes WT lines that are adjacent in the
// array, stages them through LDS (coalesced along the contiguous direction),
// and each of its WT/2 teams runs the FP64 team FFT of length P = 2N on one
// pair.  The first axis generates its input instead of reading it:
// T(1)_n = prod_j h_j U^eps(|n h|) (eq. Tensor1 / TensorAnis); the last axis
// adds W(|k|) (eq. FouTran, or the general construction's table), scales by
// 1 / prod_j P_j and writes the tensor in the plan precision.
enum class DctStage { FIRST, MID, LAST };

// The tile of lines and the teams' FFT scratch share one LDS array (the
// tile is dead while the transforms run), so its size is the larger of the
// two.  The teams exchange one component at a time (Fft::run_g_split), so a
// team's scratch holds SCR doubles.
constexpr int dct_lds_bytes(int wt, int scr, int D) {
    return (wt / 2) * scr * 8 > D * (wt + 1) * 8 ? (wt / 2) * scr * 8 : D * (wt + 1) * 8;
}

constexpr int dct_lines_per_group(int T, int scr, int D) {
    // up to 16 lines (128-byte rows on the strided axes); at most 1024
    // threads; LDS within a fifth of a CU's 160 KB where possible, so that
    // five workgroups can share a CU (at length 512: 8 lines, 18.5 KB; with
    // 16 lines and two workgroups per CU the finishing axis took 164 us
    // instead of 157 and the generation of an anisotropic T(1) 184 us
    // instead of 160)
    int wt = 16;
    while (wt > 2 && ((wt / 2) * T > 1024 || dct_lds_bytes(wt, scr, D) > 32 * 1024)) wt /= 2;
    return wt;
}

// The default radix family (at lengths 3 * 2^a from 192 the mid-3
// palindrome on the wider team: at 384, 66 instead of 162 VGPRs in the
// generating and middle axes)
template <int P>
struct Dct {
    using F = Fft<double, P, false>;
    static constexpr int N = P / 2, D = N + 1;
    static constexpr int T = F::T;
    static constexpr int WT = dct_lines_per_group(T, F::SCR, D);
    static constexpr int TEAMS = WT / 2;
    static constexpr int TS = WT + 1;
    static constexpr int THREADS = TEAMS * T;
    static constexpr int LDS_D = (dct_lds_bytes(WT, F::SCR, D) + 7) / 8;  // doubles
    static_assert(LDS_D * 8 <= 160 * 1024, "DCT workgroup exceeds the LDS");
};

// Lines of one axis: line (u, v) starts at u * u_stride + v * v_stride and
// its element t sits at + t * es; groups take WT consecutive u.  Octant
// coordinates: a[ax] = t, and (u, v) are the other two in increasing order.
struct Lines {
    int n_u, n_v;
    long u_stride, v_stride, es;
    int ax;
    const int* rows;  // optional: the order in which tiles take the lines (k_row_order)
};

// Generation of T(1) (first axis) and the finishing of T^ (last axis).
// When the mesh is the same on every axis, |n h|^2 = h^2 m and |k|^2 = c^2 m
// with the integer m = sum_j a_j^2, and T(1) and W take one value per m:
// t1_tab[m] = hprod U^eps(h sqrt m) and w_tab[m] = W(c sqrt m) are computed
// once (k_radial) and looked up, instead of evaluating the special functions
// at every octant point (a 256^3 octant has 1.7e7 points and 196 609 values
// of m).
struct DctEnds {
    KernelParams kp;
    double h[3], hprod;          // T(1) = hprod U^eps(|(a_j h_j)|)
    double c[3], inv_prod_p;     // k_j = a_j c_j; T^ = (DCT + W(|k|)) inv_prod_p
    WTable wt;
    const double* t1_tab;        // radial tables (null: evaluate directly)
    const double* w_tab;
    void* out;                   // the tensor, float or double
};

// T(1) or W at r = step sqrt(m), m = 0 .. n-1
template <bool T1>
__global__ void k_radial(double* __restrict__ tab, long n, double step, DctEnds ends) {
    const long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double r = step * sqrt((double)m);
    if constexpr (T1) {
        tab[m] = ends.hprod * (ends.kp.general ? d_ueps_general(ends.kp, r) : d_ueps(ends.kp, r));
    } else {
        tab[m] = ends.wt.cf ? d_what_cheb(ends.wt.cf, ends.wt.dk, ends.wt.nq, r)
                            : d_what(ends.kp, r);
    }
}

// Order of the lines of the contiguous axis 0 of a 3D octant by
// c = a1^2 + a2^2 (ties by a1), for the last axis when it reads W from the
// radial table.  Along a line W is read at m = a0^2 + c; lines with nearly
// equal c read nearly the same entries at each a0, so a tile of 8 such lines,
// walked with 8 values of a0 per 8 lines in one 64-lane gather, touches a few
// cache lines of the table per instruction instead of one per lane (with 8
// adjacent lines c spreads over 14 a1 and every lane reads its own line).
// The rank of a line is the count of lines before it, summed over the
// columns b1: the b2 with b2^2 < c - b1^2 are 0 .. ceil(sqrt(c - b1^2)) - 1,
// plus the tie b2^2 = c - b1^2 when b1 < a1.  So no sort is needed:
// rows[rank] = a1 + D1 a2, a permutation of 0 .. D1 D2 - 1.  Eight lanes
// share a line (lane q sums the columns q, q + 8, ...), so the grid holds
// enough waves to hide the loop's latency; c < 2^24 for every supported
// grid (D <= 2049), so x converts to float exactly and the FP32 square
// root is at most one off before the integer correction.
constexpr int kRankLanes = 8;
__global__ __launch_bounds__(256) void k_row_order(int* __restrict__ rows, int d1, int d2) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = d1 * d2, r = gid / kRankLanes, q = gid % kRankLanes;
    const bool live = r < n;
    const int a1 = live ? r % d1 : 0, a2 = live ? r / d1 : 0, c = a1 * a1 + a2 * a2;
    int rank = 0;
    for (int b1 = q; b1 < d1; b1 += kRankLanes) {
        const int x = c - b1 * b1;
        if (x < 0) break;
        int s = (int)sqrtf((float)x);  // floor(sqrt(x)) after the corrections
        while (s * s > x) --s;
        while ((s + 1) * (s + 1) <= x) ++s;
        const bool square = s * s == x;
        const int lt = square ? s : s + 1;  // b2 = 0 .. lt - 1 have b2^2 < x
        rank += lt < d2 ? lt : d2;
        rank += (square && b1 < a1 && s < d2) ? 1 : 0;
    }
#pragma unroll
    for (int m = 1; m < kRankLanes; m *= 2) rank += __shfl_xor(rank, m, kRankLanes);
    if (live && q == 0 && rank < n) rows[rank] = r;
}

__device__ __forceinline__ void octant_coords(const Lines& ln, int u, int v, int t, int (&a)[3]) {
    if (ln.ax == 0) { a[0] = t; a[1] = u; a[2] = v; }
    else if (ln.ax == 1) { a[0] = u; a[1] = t; a[2] = v; }
    else { a[0] = u; a[1] = v; a[2] = t; }
}

// TAB: the first / last axis looks T(1) / W up in the radial table.  ROWS:
// tiles take the lines in the order of ln.rows (the contiguous axis only,
// whose lines are whole rows), and the tile is walked with the line index
// fastest.
template <int P, DctStage STAGE, typename R, bool TAB, bool ROWS = false>
__global__ __launch_bounds__(Dct<P>::THREADS) void k_dct(const double* __restrict__ in,
                                                        double* __restrict__ out, Lines ln,
                                                        const cpx<double>* __restrict__ tw,
                                                        DctEnds ends) {
    using K = Dct<P>;
    using F = typename K::F;
    using C = cpx<double>;
    __shared__ double lds[K::LDS_D];
    double* scr = lds;   // teams' FFT scratch ...
    double* tile = lds;  // ... and the tile, in turn
    const int team = team_index<K::T>(), tid = threadIdx.x % K::T;
    static_assert(!ROWS || K::THREADS % K::WT == 0, "a thread keeps one line of the tile");
    const int ntu = (ln.n_u + K::WT - 1) / K::WT;
    // Tiles of the strided axes in XCD order: the dispatcher deals
    // workgroups to the 8 XCDs in turn, each with its own L2, and a tile's
    // rows of up to 16 doubles start anywhere in a cache line (the octant
    // extents are N + 1), so neighbouring tiles share lines.  XCD x takes
    // the x-th eighth of the tiles, in order, so that neighbours run side by
    // side under one L2 (tiles in launch order: axis 1 fetched 1.94 and
    // wrote 1.19 times its bytes; in XCD order 1.00 and 1.00).  The lines of
    // the contiguous axis are whole rows and keep the launch order.  The grid
    // is rounded up to a multiple of 8; the extra groups have no tile.
    const int per = (int)gridDim.x / 8;
    const int ti = ln.es != 1 ? ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8 : (int)blockIdx.x;
    int tu, v, nw;
    long base;
    if constexpr (ROWS) {
        // line w = threadIdx.x % WT of the tile is rows[ti WT + w], at (u, v)
        const int nrow = ln.n_u * ln.n_v;
        if (ti * K::WT >= nrow) return;
        nw = nrow - ti * K::WT < K::WT ? nrow - ti * K::WT : K::WT;
        const int w = (int)threadIdx.x % K::WT;
        int r = ln.rows[ti * K::WT + (w < nw ? w : 0)];
        if ((unsigned)r >= (unsigned)nrow) r = 0;  // a permutation of the lines; never taken
        tu = r % ln.n_u;
        v = r / ln.n_u;
        base = (long)tu * ln.u_stride + (long)v * ln.v_stride;
    } else {
        if (ti >= ntu * ln.n_v) return;
        tu = ti % ntu;
        v = ti / ntu;
        base = (long)tu * K::WT * ln.u_stride + (long)v * ln.v_stride;
        nw = ln.n_u - tu * K::WT < K::WT ? ln.n_u - tu * K::WT : K::WT;
    }
    // line w of the tile: u = tu WT + w at v, or (ROWS) this thread's (tu, v)
    auto line_off = [&](int w) { return ROWS ? base : base + w * ln.u_stride; };
    auto line_u = [&](int w) { return ROWS ? tu : tu * K::WT + w; };
    // element e of the tile -> (t, w), contiguous direction fastest
    auto at = [&](int e, int& t, int& w) {
        if (!ROWS && ln.es == 1) {
            w = e / K::D;
            t = e - w * K::D;
        } else {
            t = e / K::WT;
            w = e - t * K::WT;
        }
    };
    // Tile elements e = threadIdx.x + k THREADS, k < EPT: the load and the
    // store loops visit the same elements in the same order.  Direct
    // evaluation takes one element per iteration (the special functions need
    // many registers, and unrolled copies would cost the FFT its occupancy);
    // table lookups and plain copies are unrolled so that their loads are in
    // flight together.  The last axis looks its W values up in the store
    // loop, three elements at a time: gathered before the transforms, they
    // stayed live across the FFT (113 instead of 77 VGPRs at length 512, four
    // waves per SIMD instead of six).
    constexpr int EPT = (K::D * K::WT + K::THREADS - 1) / K::THREADS;
    constexpr bool DIRECT = !TAB && STAGE == DctStage::FIRST;
    auto load_one = [&](int e) {
        int t, w;
        at(e, t, w);
        double x = 0.0;
        if (w < nw) {
            if constexpr (STAGE == DctStage::FIRST) {
                int a[3];
                octant_coords(ln, line_u(w), v, t, a);
                if constexpr (TAB) {
                    x = ends.t1_tab[a[0] * a[0] + a[1] * a[1] + a[2] * a[2]];
                } else {
                    const double x0 = a[0] * ends.h[0], x1 = a[1] * ends.h[1],
                                 x2 = a[2] * ends.h[2];
                    const double r = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
                    x = ends.hprod * (ends.kp.general ? d_ueps_general(ends.kp, r)
                                                      : d_ueps(ends.kp, r));
                }
            } else {
                x = in[line_off(w) + t * ln.es];
            }
        }
        tile[t * K::TS + w] = x;
    };
    if constexpr (DIRECT) {
#pragma unroll 1
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * K::THREADS;
            if (e < K::D * K::WT) load_one(e);
        }
    } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * K::THREADS;
            if (e < K::D * K::WT) load_one(e);
        }
    }
    __syncthreads();
    C z[F::V];
    F::load_first(z, tid, P, [&](int i) {
        const int t = i <= K::N ? i : P - i;
        return mk(tile[t * K::TS + 2 * team], tile[t * K::TS + 2 * team + 1]);
    });
    __syncthreads();
    F::run_g_split(z, scr + team * F::SCR, tid, tw);
    __syncthreads();
    F::store_last(z, tid, K::D, [&](int p, C c) {
        tile[p * K::TS + 2 * team] = c.x;
        tile[p * K::TS + 2 * team + 1] = c.y;
    });
    __syncthreads();
    auto store_one = [&](int e) {
        int t, w;
        at(e, t, w);
        if (w >= nw) return;
        const long o = line_off(w) + t * ln.es;
        if constexpr (STAGE == DctStage::LAST) {
            double wk;
            int a[3];
            octant_coords(ln, line_u(w), v, t, a);
            if constexpr (TAB) {
                wk = ends.w_tab[a[0] * a[0] + a[1] * a[1] + a[2] * a[2]];
            } else {
                const double k0 = a[0] * ends.c[0], k1 = a[1] * ends.c[1], k2 = a[2] * ends.c[2];
                const double kk = sqrt(k0 * k0 + k1 * k1 + k2 * k2);
                wk = ends.wt.cf ? d_what_cheb(ends.wt.cf, ends.wt.dk, ends.wt.nq, kk)
                                : d_what(ends.kp, kk);
            }
            ((R*)ends.out)[o] = (R)((tile[t * K::TS + w] + wk) * ends.inv_prod_p);
        } else {
            out[o] = tile[t * K::TS + w];
        }
    };
    if constexpr (!TAB && STAGE == DctStage::LAST) {
#pragma unroll 1
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * K::THREADS;
            if (e < K::D * K::WT) store_one(e);
        }
    } else if constexpr (STAGE == DctStage::LAST) {
#pragma unroll 3
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * K::THREADS;
            if (e < K::D * K::WT) store_one(e);
        }
    } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * K::THREADS;
            if (e < K::D * K::WT) store_one(e);
        }
    }
}

// ROWS: take the lines in the order of ln.rows where the length's workgroup
// allows it (a whole number of tiles' lines per thread block), else in
// memory order.
template <DctStage STAGE, typename R, bool TAB, bool ROWS = false>
hipError_t dct_axis(const double* in, double* out, Lines ln, int N, const void* tw,
                    const DctEnds& ends, hipStream_t st) {
    switch (2 * N) {
#define FSA_DCT_CASE(p)                                                                         \
    case p: {                                                                                   \
        using K = Dct<p>;                                                                       \
        constexpr bool RW = ROWS && K::THREADS % K::WT == 0;                                    \
        const int tiles = RW ? (ln.n_u * ln.n_v + K::WT - 1) / K::WT                            \
                             : (ln.n_u + K::WT - 1) / K::WT * ln.n_v;                            \
        return launch_kernel(k_dct<p, STAGE, R, TAB, RW>, dim3((tiles + 7) / 8 * 8),            \
                             dim3(K::THREADS), 0, st, in, out, ln, (const cpx<double>*)tw, ends); \
    }
        FSA_DCT_CASE(16) FSA_DCT_CASE(24) FSA_DCT_CASE(32) FSA_DCT_CASE(48) FSA_DCT_CASE(64)
        FSA_DCT_CASE(96) FSA_DCT_CASE(128) FSA_DCT_CASE(192) FSA_DCT_CASE(256) FSA_DCT_CASE(384)
        FSA_DCT_CASE(512) FSA_DCT_CASE(768) FSA_DCT_CASE(1024) FSA_DCT_CASE(1536)
        FSA_DCT_CASE(2048) FSA_DCT_CASE(3072) FSA_DCT_CASE(4096)
#undef FSA_DCT_CASE
    }
    return hipErrorInvalidValue;
}

// Gauss-Legendre nodes and weights by Newton's method on the Legendre
// recurrence (host, FP64).
Gl16 gauss_legendre16() {
    Gl16 g{};
    const int n = kGl;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        g.x[i] = x;
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

// The general construction's W table, on the stream; device buffers are
// returned in bufs for the caller to free after the finalize launch.
hipError_t build_w_table(const KernelParams& kp, int d, const double* L, const int64_t* N,
                         hipStream_t st, WTable* wt, std::vector<void*>* bufs) {
    const double eps = kp.eps;
    const bool win = !(kp.kind == FSA_COULOMB_3D || kp.kind == FSA_COULOMB_2D ||
                       kp.kind == FSA_BIHARMONIC_3D);
    // largest lattice |k| of the octant: k_j = pi p_j / (2 L_j), p_j <= N_j
    double k2 = 0.0;
    for (int j = 0; j < d; ++j) {
        const double kj = kPi * (double)N[j] / (2.0 * L[j]);
        k2 += kj * kj;
    }
    const double kmax = std::sqrt(k2);
    // U - U^eps is below 1e-20 of its scale beyond R_end
    const double r_end = win ? 13.0 * eps : 7.0 * eps;
    // |k| panels of width 0.5/eps, kCheb + 1 Chebyshev-Lobatto points each
    wt->dk = 0.5 / eps;
    wt->nq = (int)std::ceil(kmax / wt->dk);
    if (wt->nq < 1) wt->nq = 1;
    const int n_k = wt->nq * (kCheb + 1);
    // In 2D (J0, whose evaluations dominate the build) the |k| panels fall
    // into 8 bands of equal width, and each band has quadrature nodes of its
    // own, spaced for the largest |k| of the band:
    // panel width w with k_top w <= 6 (16 Gauss-Legendre nodes per panel
    // then integrate J0(k r) or sin(k r)/(k r) to far below double rounding),
    // and at most eps/4 (the window and erfc), 4/lam (the Yukawa decay) and
    // eta/2 (the quasi-2D kernel's scale).  The sum costs nodes x points, and
    // a band of low |k| needs a fraction of the nodes the top band does (2D
    // Yukawa 2048^2: 1.63 -> 1.33 ms per build).  In 3D, sin(x)/x is cheap and
    // one band is faster (eight took the 256^3 Yukawa build 0.41 -> 0.46 ms).
    // 2D kernels with a logarithm at r = 0 grade their first panel.
    const bool log0 = kp.kind == FSA_LOG_2D || kp.kind == FSA_BIHARMONIC_2D ||
                      kp.kind == FSA_YUKAWA_2D || kp.kind == FSA_QUASI2D_DDI;
    constexpr int kBands = 8;
    const int bands = d == 2 ? kBands : 1;
    QMesh mesh[kBands];
    int q0[kBands + 1], off[kBands + 1];
    q0[0] = 0;
    off[0] = 0;
    for (int b = 0; b < bands; ++b) {
        q0[b + 1] = (int)(((long)wt->nq * (b + 1) + bands - 1) / bands);
        const double ktop = std::fmin(kmax, q0[b + 1] * wt->dk);
        double w = std::fmin(6.0 / ktop, 0.25 * eps);
        if (kp.kind == FSA_YUKAWA_3D || kp.kind == FSA_YUKAWA_2D) w = std::fmin(w, 4.0 / kp.lam);
        if (kp.kind == FSA_QUASI2D_DDI) w = std::fmin(w, 0.5 * kp.eta);
        QMesh& m = mesh[b];
        m.n_uni = (int)std::ceil(r_end / w);
        m.wu = r_end / m.n_uni;
        m.sigma = 0.15;
        m.graded = log0 ? 14 : 0;
        off[b + 1] = off[b] + (q0[b + 1] > q0[b] ? (m.graded ? m.n_uni + m.graded : m.n_uni) * kGl : 0);
    }
    const int n_nodes = off[bands];
    double *g = nullptr, *rn = nullptr, *v = nullptr, *cf = nullptr;
    hipError_t e = hipMallocAsync((void**)&g, sizeof(double) * n_nodes, st);
    if (e == hipSuccess) bufs->push_back(g), e = hipMallocAsync((void**)&rn, sizeof(double) * n_nodes, st);
    if (e == hipSuccess) bufs->push_back(rn), e = hipMallocAsync((void**)&v, sizeof(double) * n_k, st);
    if (e == hipSuccess) bufs->push_back(v), e = hipMallocAsync((void**)&cf, sizeof(double) * n_k, st);
    if (e != hipSuccess) return e;
    bufs->push_back(cf);
    const Gl16 gl = gauss_legendre16();
    for (int b = 0; b < bands; ++b) {
        const int nb = off[b + 1] - off[b], np = q0[b + 1] - q0[b];
        if (np <= 0) continue;
        hipLaunchKernelGGL(k_wq_nodes, dim3((nb + 255) / 256), dim3(256), 0, st, g + off[b],
                           rn + off[b], mesh[b], gl, d, kp);
        hipLaunchKernelGGL(k_wq_sum, dim3(np * (kCheb + 1)), dim3(256), 0, st,
                           (const double*)(g + off[b]), (const double*)(rn + off[b]), nb, d,
                           wt->dk, q0[b] * (kCheb + 1), v);
    }
    hipLaunchKernelGGL(k_cheb, dim3((n_k + 255) / 256), dim3(256), 0, st, (const double*)v, cf,
                       wt->nq);
    wt->cf = cf;
    return hipGetLastError();
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
                               int** line_order, hipStream_t st) {
    // octant extents D_j = N_j + 1, axis 0 innermost; a 2D plan has D2 = 1
    const long D0 = N[0] + 1, D1 = N[1] + 1, D2 = d == 3 ? N[2] + 1 : 1;
    const long n = D0 * D1 * D2;
    int maxN = 0;
    for (int j = 0; j < d; ++j) maxN = (int)N[j] > maxN ? (int)N[j] : maxN;
    // the general construction's W table first (the last axis reads it)
    WTable wt{nullptr, 0.0, 0};
    std::vector<void*> wbufs;
    hipError_t e = kp.general ? build_w_table(kp, d, L, N, st, &wt, &wbufs) : hipSuccess;
    // intermediate octants between the axes: one for 2D, two for 3D
    double *a = nullptr, *b = nullptr;
    void* tw = nullptr;
    if (e == hipSuccess) e = hipMallocAsync((void**)&a, sizeof(double) * n, st);
    if (e == hipSuccess && d == 3) e = hipMallocAsync((void**)&b, sizeof(double) * n, st);
    if (e == hipSuccess) e = hipMallocAsync(&tw, 2 * sizeof(double) * 2 * maxN, st);
    DctEnds ends{};
    ends.kp = kp;
    double prodP = 1.0;
    for (int j = 0; j < 3; ++j) {
        ends.h[j] = j < d ? h[j] : 0.0;
        ends.c[j] = j < d ? kPi / (2.0 * L[j]) : 0.0;
        if (j < d) prodP *= 2.0 * (double)N[j];
    }
    ends.hprod = h[0] * h[1] * (d == 3 ? h[2] : 1.0);
    ends.inv_prod_p = 1.0 / prodP;
    ends.wt = wt;
    ends.out = tensor_out;
    // radial tables where the mesh (for T(1)) or the frequency step (for W)
    // is the same on every axis and the table is much smaller than the octant
    long msum = 0;
    bool same_h = true, same_c = true;
    for (int j = 0; j < d; ++j) {
        msum += N[j] * N[j];
        same_h = same_h && h[j] == h[0];
        same_c = same_c && L[j] == L[0];
    }
    const long ntab = msum + 1;
    const bool small = ntab * 4 <= n;
    double *t1_tab = nullptr, *w_tab = nullptr;
    if (e == hipSuccess && small && same_h) {
        e = hipMallocAsync((void**)&t1_tab, sizeof(double) * ntab, st);
        if (e == hipSuccess)
            e = launch_kernel(k_radial<true>, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0,
                              st, t1_tab, ntab, h[0], ends);
    }
    if (e == hipSuccess && small && same_c) {
        e = hipMallocAsync((void**)&w_tab, sizeof(double) * ntab, st);
        if (e == hipSuccess)
            e = launch_kernel(k_radial<false>, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0,
                              st, w_tab, ntab, ends.c[0], ends);
    }
    ends.t1_tab = t1_tab;
    ends.w_tab = w_tab;
    // the order of the rows of axis 0, where the last axis (axis 0) of a 3D
    // build reads W from the radial table: computed once, kept by the caller
    if (e == hipSuccess && w_tab && d == 3 && !*line_order) {
        int* order = nullptr;
        e = hipMalloc((void**)&order, sizeof(int) * D1 * D2);
        if (e == hipSuccess) {
            e = launch_kernel(k_row_order, dim3((unsigned)((D1 * D2 * kRankLanes + 255) / 256)),
                              dim3(256), 0, st, order, (int)D1, (int)D2);
            if (e == hipSuccess) *line_order = order;
            else (void)hipFree(order);
        }
    }
    int* rows = w_tab && d == 3 ? *line_order : nullptr;
    // lines along axis ax; groups take lines adjacent in memory (or, on
    // axis 0, in the order of rows)
    auto lines = [&](int ax) {
        if (ax == 0) return Lines{(int)D1, (int)D2, D0, D0 * D1, 1, 0, rows};
        if (ax == 1) return Lines{(int)D0, (int)D2, 1, D0 * D1, D0, 1, nullptr};
        return Lines{(int)D0, (int)D1, 1, D0, D0 * D1, 2, nullptr};
    };
    // axes from the last (strided) to axis 0 (contiguous): the axis that
    // only writes takes the long strides, the last one reads and writes
    // contiguous rows
    for (int step = 0; step < d && e == hipSuccess; ++step) {
        const int ax = d - 1 - step;
        e = build_twiddles(FSA_F64, (int)(2 * N[ax]), tw, st);
        if (e != hipSuccess) break;
        const Lines ln = lines(ax);
        const int nn = (int)N[ax];
        const double* last_in = d == 3 ? b : a;
        if (step == 0)
            e = t1_tab ? dct_axis<DctStage::FIRST, double, true>(nullptr, a, ln, nn, tw, ends, st)
                       : dct_axis<DctStage::FIRST, double, false>(nullptr, a, ln, nn, tw, ends, st);
        else if (step < d - 1)
            e = dct_axis<DctStage::MID, double, false>(a, b, ln, nn, tw, ends, st);
        else if (prec == FSA_F32)
            e = rows    ? dct_axis<DctStage::LAST, float, true, true>(last_in, nullptr, ln, nn, tw, ends, st)
                : w_tab ? dct_axis<DctStage::LAST, float, true>(last_in, nullptr, ln, nn, tw, ends, st)
                        : dct_axis<DctStage::LAST, float, false>(last_in, nullptr, ln, nn, tw, ends, st);
        else
            e = rows    ? dct_axis<DctStage::LAST, double, true, true>(last_in, nullptr, ln, nn, tw, ends, st)
                : w_tab ? dct_axis<DctStage::LAST, double, true>(last_in, nullptr, ln, nn, tw, ends, st)
                        : dct_axis<DctStage::LAST, double, false>(last_in, nullptr, ln, nn, tw, ends, st);
    }
    if (t1_tab) (void)hipFreeAsync(t1_tab, st);
    if (w_tab) (void)hipFreeAsync(w_tab, st);
    for (void* p : wbufs) (void)hipFreeAsync(p, st);
    if (a) (void)hipFreeAsync(a, st);
    if (b) (void)hipFreeAsync(b, st);
    if (tw) (void)hipFreeAsync(tw, st);
    return e;
}

}  // namespace fsa
