/*
 * fsa_oracle.c -- plain FP64 CPU oracle of the far-field smooth approximation
 * (FSA) convolution solver of Liu & Zhang, "Fast convolution solver based on
 * far-field smooth approximation" (arXiv 2504.19410).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the GPU library: it has its own special
 * functions, its own naive mixed-radix FFT and builds the tensor straight from
 * the paper's formulas, in the paper's order:
 *
 *   T(1)_n = (prod_j h_j) U^eps(|n h|)                 Sec. 2.1, eq. Tensor1 / TensorAnis
 *   W_p    = FT[U - U^eps](|k_p|),  k_j = pi p_j/(2L_j) Sec. 2.2, eq. FouTran, Table 1
 *   T(2)_n = (prod P_j)^-1 sum_p W_p e^{+2 pi i p.n/P}  Sec. 2.2, eq. Tensor2
 *   T      = T(1) + T(2)                                Sec. 2.3, eq. DiscConv
 *   Phi_i  = sum_{i'} T_{i-i'} rho_{i'}                 Sec. 2.3, eq. DiscConv
 *
 * with P_j = 2 N_j, h_j = 2 L_j / N_j, the periodic index n_j in [-N_j, N_j-1]
 * stored at n_j mod P_j, and the grid value rho[i] sitting at
 * x_j = -L_j + i_j h_j (eq. UniformMesh).
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *  - U^eps(0) is the r -> 0 limit of U^eps; W(0) the k -> 0 limit.
 *  - 3D Yukawa: the paper gives no U^eps.  We use the Gaussian-screened split
 *    whose transform is e^{-(k^2+lam^2) eps^2/4}/(k^2+lam^2); it is smooth,
 *    radial, has a Gaussian tail, and reduces to the Coulomb row of Table 1
 *    as lam -> 0.
 *  - per-axis N_j: all formulas are separable per axis, (2N)^d -> prod P_j.
 *
 *  - 3D DDI (Sec. 5.3): the source d_nm rho is the spectral derivative of rho
 *    on its own grid, periodic on the box (see orc_solve_ddi).
 *
 * Parity pins (tests/): the printed error tables (Tables 2, 4, 5), closed-form
 * Gaussian potentials, a direct O(N^2d) sum, an O(n^2) DFT, Ein/E1 against a
 * library routine, W against quadrature of eq. Fourier-Symmetric.
 * The 2D/3D biharmonic and 2D Coulomb rows of Table 1 are pinned only by
 * quadrature of eq. Fourier-Symmetric and, for 3D biharmonic, Table 5.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum {
    ORC_COULOMB_3D = 1,
    ORC_YUKAWA_3D = 2,
    ORC_LOG_2D = 3,
    ORC_COULOMB_2D = 4,
    ORC_BIHARMONIC_3D = 5,
    ORC_BIHARMONIC_2D = 6,
    ORC_DDI_3D = 7, /* through the Coulomb kernel, see orc_solve_ddi */
};

static const double ORC_PI = 3.14159265358979323846264338327950288;
static const double ORC_EULER_GAMMA = 0.57721566490153286060651209008240243;

/* ------------------------------------------------------------------------- */
/* Threads                                                                    */
/* ------------------------------------------------------------------------- */

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Exponential integrals (Abramowitz & Stegun 5.1.11 and 5.1.22)              */
/* ------------------------------------------------------------------------- */

/* Ein(x) = sum_{m>=1} (-1)^{m+1} x^m / (m m!), an entire function
 * (A&S 5.1.11: E1(x) = -gamma - ln x + Ein(x)).  Summed term by term. */
double orc_ein(double x)
{
    double term = 1.0, sum = 0.0;
    for (int m = 1; m < 400; ++m) {
        term *= -x / (double)m;          /* (-x)^m / m!               */
        double add = -term / (double)m;  /* (-1)^{m+1} x^m / (m m!)   */
        sum += add;
        if (fabs(add) <= 1e-18 * fabs(sum) && m > 2) break;
    }
    return sum;
}

/* E1(x) = int_x^inf e^{-t}/t dt.  For x <= 1 from Ein (5.1.11); otherwise
 * the continued fraction 5.1.22, E1(x) = e^{-x} / (x + 1/(1 + 1/(x + 2/(1 +
 * 2/(x + ...))))), evaluated bottom-up with a fixed depth that is ample for
 * x > 1 at double precision. */
double orc_e1(double x)
{
    if (x <= 0.0) return INFINITY;
    if (x <= 1.0) return -ORC_EULER_GAMMA - log(x) + orc_ein(x);
    const int depth = 200;
    double f = x; /* tail approximation */
    for (int m = depth; m >= 1; --m) {
        /* x + m/(1 + m/f) */
        f = x + (double)m / (1.0 + (double)m / f);
    }
    return exp(-x) / f;
}

/* ------------------------------------------------------------------------- */
/* Kernels U, far-field smooth approximations U^eps and W = FT(U - U^eps)     */
/* (Table 1, eqs. KerAppr and lnrAppr; Yukawa split: see header)              */
/* ------------------------------------------------------------------------- */

double orc_u(int kind, double lam, double r)
{
    switch (kind) {
    case ORC_COULOMB_3D:
    case ORC_DDI_3D: return 1.0 / (4.0 * ORC_PI * r);
    case ORC_YUKAWA_3D: return exp(-lam * r) / (4.0 * ORC_PI * r);
    case ORC_LOG_2D: return -log(r) / (2.0 * ORC_PI);
    case ORC_COULOMB_2D: return 1.0 / (2.0 * ORC_PI * r);
    case ORC_BIHARMONIC_3D: return r / (8.0 * ORC_PI);
    case ORC_BIHARMONIC_2D: return -r * r * (log(r) - 1.0) / (8.0 * ORC_PI);
    }
    return NAN;
}

/* U^eps(r) for r >= 0; r = 0 is the limit value. */
double orc_ueps(int kind, double lam, double eps, double r)
{
    const double pi = ORC_PI;
    switch (kind) {
    case ORC_COULOMB_3D:
    case ORC_DDI_3D:
        if (r == 0.0) return 1.0 / (2.0 * pow(pi, 1.5) * eps);
        return erf(r / eps) / (4.0 * pi * r);
    case ORC_COULOMB_2D:
        if (r == 0.0) return 1.0 / (pow(pi, 1.5) * eps);
        return erf(r / eps) / (2.0 * pi * r);
    case ORC_BIHARMONIC_3D:
        return r * erf(r / eps) / (8.0 * pi);
    case ORC_YUKAWA_3D: {
        const double a = 0.5 * lam * eps;
        if (r == 0.0)
            return (2.0 * exp(-a * a) / (sqrt(pi) * eps) - lam * erfc(a)) / (4.0 * pi);
        /* [e^{-lam r}(1 + erf(r/eps - a)) - e^{lam r} erfc(r/eps + a)] / (8 pi r) */
        const double q = r / eps;
        return (exp(-lam * r) * (1.0 + erf(q - a)) - exp(lam * r) * erfc(q + a)) /
               (8.0 * pi * r);
    }
    case ORC_LOG_2D: {
        /* -(1/2pi)[ln r + E1(r^2/eps^2)/2]; near 0 use E1 = -gamma - ln x + Ein */
        const double x = (r / eps) * (r / eps);
        if (x <= 1.0) return -(log(eps) + 0.5 * (orc_ein(x) - ORC_EULER_GAMMA)) / (2.0 * pi);
        return -(log(r) + 0.5 * orc_e1(x)) / (2.0 * pi);
    }
    case ORC_BIHARMONIC_2D: {
        /* -(r^2/8pi)[ln r + E1(r^2/eps^2)/2 - 1] */
        if (r == 0.0) return 0.0;
        const double x = (r / eps) * (r / eps);
        double inner;
        if (x <= 1.0) inner = log(eps) + 0.5 * (orc_ein(x) - ORC_EULER_GAMMA) - 1.0;
        else inner = log(r) + 0.5 * orc_e1(x) - 1.0;
        return -r * r * inner / (8.0 * pi);
    }
    }
    return NAN;
}

/* W(k) = FT[U - U^eps](k), whole-space transform (eq. FouTran, Table 1). */
double orc_what(int kind, double lam, double eps, double k)
{
    const double k2 = k * k;
    switch (kind) {
    case ORC_COULOMB_3D:
    case ORC_DDI_3D:
    case ORC_LOG_2D: {
        /* (1 - e^{-k^2 eps^2/4}) / k^2 */
        const double x = 0.25 * k2 * eps * eps;
        if (k == 0.0) return 0.25 * eps * eps;
        return -expm1(-x) / k2;
    }
    case ORC_YUKAWA_3D: {
        const double q = k2 + lam * lam;
        if (q == 0.0) return 0.25 * eps * eps;
        return -expm1(-0.25 * q * eps * eps) / q;
    }
    case ORC_COULOMB_2D:
        if (k == 0.0) return eps / sqrt(ORC_PI);
        return erf(0.5 * k * eps) / k;
    case ORC_BIHARMONIC_3D: {
        /* (-8 + e^{-x}(8 + 8x + 16x^2)) / (8 k^4),  x = k^2 eps^2/4
         *  = eps^4 (e^{-x}(1 + x + 2x^2) - 1) / (16 x^2).  Small x: Taylor
         *  series of e^{-x}(1 + x + 2x^2) - 1 = sum_n c_n x^n. */
        const double x = 0.25 * k2 * eps * eps;
        const double e4 = eps * eps * eps * eps;
        if (x < 0.5) {
            /* c_n = (-1)^n/n! + (-1)^{n-1}/(n-1)! + 2(-1)^{n-2}/(n-2)!, n >= 2 */
            double s = 0.0, fact_n2 = 1.0; /* (n-2)! */
            double xp = 1.0;               /* x^{n-2} */
            for (int n = 2; n < 40; ++n) {
                if (n > 2) { fact_n2 *= (double)(n - 2); xp *= x; }
                const double f_n1 = fact_n2 * (double)(n - 1);
                const double f_n = f_n1 * (double)n;
                const double sg = (n % 2 == 0) ? 1.0 : -1.0;
                const double c = sg / f_n - sg / f_n1 + 2.0 * sg / fact_n2;
                s += c * xp;
            }
            return e4 * s / 16.0;
        }
        return e4 * (exp(-x) * (1.0 + x + 2.0 * x * x) - 1.0) / (16.0 * x * x);
    }
    case ORC_BIHARMONIC_2D: {
        /* (-16 + e^{-x}(16 + 16x + 16x^2)) / (16 k^4) = eps^4 (e^{-x}(1+x+x^2) - 1)/(16 x^2) */
        const double x = 0.25 * k2 * eps * eps;
        const double e4 = eps * eps * eps * eps;
        if (x < 0.5) {
            /* c_n = (-1)^n/n! + (-1)^{n-1}/(n-1)! + (-1)^{n-2}/(n-2)! */
            double s = 0.0, fact_n2 = 1.0, xp = 1.0;
            for (int n = 2; n < 40; ++n) {
                if (n > 2) { fact_n2 *= (double)(n - 2); xp *= x; }
                const double f_n1 = fact_n2 * (double)(n - 1);
                const double f_n = f_n1 * (double)n;
                const double sg = (n % 2 == 0) ? 1.0 : -1.0;
                const double c = sg / f_n - sg / f_n1 + sg / fact_n2;
                s += c * xp;
            }
            return e4 * s / 16.0;
        }
        return e4 * (exp(-x) * (1.0 + x + x * x) - 1.0) / (16.0 * x * x);
    }
    }
    return NAN;
}

int orc_kernel_dim(int kind)
{
    switch (kind) {
    case ORC_COULOMB_3D:
    case ORC_YUKAWA_3D:
    case ORC_BIHARMONIC_3D:
    case ORC_DDI_3D: return 3;
    case ORC_LOG_2D:
    case ORC_COULOMB_2D:
    case ORC_BIHARMONIC_2D: return 2;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Naive mixed-radix FFT: recursive decimation in time, splitting off the     */
/* smallest prime factor p of n and combining with a plain length-p DFT.      */
/* Unnormalised; sign = -1 forward, +1 inverse.                               */
/* ------------------------------------------------------------------------- */

static int smallest_prime_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* tab[j] = exp(sign 2 pi i j / n0) for j in [0, n0); a sub-transform of
 * length n uses the root exp(sign 2 pi i / n) = tab[n0/n]. */
static void fft_rec(int n, const cplx *in, int istride, cplx *out, const cplx *tab, int n0,
                    cplx *tmp)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int p = smallest_prime_factor(n);
    const int m = n / p;
    const int root = n0 / n; /* tab index step for exp(sign 2 pi i / n) */
    for (int q = 0; q < p; ++q)
        fft_rec(m, in + (size_t)q * istride, istride * p, out + (size_t)q * m, tab, n0, tmp);
    /* X[k + s m] = sum_q w_n^{q (k + s m)} Y_q[k]; the p outputs for one k
     * overwrite exactly the p inputs Y_q[k] = out[q m + k]. */
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) tmp[q] = out[(size_t)q * m + k];
        for (int s = 0; s < p; ++s) {
            cplx acc = 0.0;
            for (int q = 0; q < p; ++q) {
                const long e = ((long)q * (long)(k + s * m)) % n;
                acc += tmp[q] * tab[(size_t)e * root];
            }
            out[(size_t)s * m + k] = acc;
        }
    }
}

static cplx *make_table(int n, int sign)
{
    cplx *tab = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!tab) return NULL;
    for (int j = 0; j < n; ++j) {
        const double a = 2.0 * ORC_PI * (double)j / (double)n;
        tab[j] = cos(a) + (double)sign * sin(a) * I;
    }
    return tab;
}

static int max_prime_factor(int n)
{
    int mp = 1;
    while (n > 1) {
        const int p = smallest_prime_factor(n);
        if (p > mp) mp = p;
        n /= p;
    }
    return mp;
}

/* One 1-D transform of length n, out-of-place (in and out must differ). */
int orc_fft1d(int n, const double *in_ri, double *out_ri, int sign)
{
    if (n < 1) return -1;
    cplx *tab = make_table(n, sign < 0 ? -1 : 1);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)max_prime_factor(n));
    if (!tab || !tmp) { free(tab); free(tmp); return -2; }
    fft_rec(n, (const cplx *)in_ri, 1, (cplx *)out_ri, tab, n, tmp);
    free(tab);
    free(tmp);
    return 0;
}

/* In-place transform of a d-dimensional C-order complex array along every
 * axis, one axis after the other; pencils are gathered, transformed with
 * fft_rec and scattered back. */
static int fft_nd(int d, const int64_t *shape, cplx *a, int sign)
{
    size_t total = 1;
    for (int j = 0; j < d; ++j) total *= (size_t)shape[j];
    for (int ax = 0; ax < d; ++ax) {
        const int n = (int)shape[ax];
        size_t stride = 1;
        for (int j = ax + 1; j < d; ++j) stride *= (size_t)shape[j];
        const size_t npencil = total / (size_t)n;
        cplx *tab = make_table(n, sign < 0 ? -1 : 1);
        if (!tab) return -2;
        const int mp = max_prime_factor(n);
        int fail = 0;
#pragma omp parallel
        {
            cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n * 2);
            cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)mp);
            if (!buf || !tmp) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(static)
                for (long q = 0; q < (long)npencil; ++q) {
                    /* pencil q: outer index = q / stride, inner = q % stride */
                    const size_t outer = (size_t)q / stride, inner = (size_t)q % stride;
                    const size_t base = outer * stride * (size_t)n + inner;
                    for (int i = 0; i < n; ++i) buf[i] = a[base + (size_t)i * stride];
                    fft_rec(n, buf, 1, buf + n, tab, n, tmp);
                    for (int i = 0; i < n; ++i) a[base + (size_t)i * stride] = buf[n + i];
                }
            }
            free(buf);
            free(tmp);
        }
        free(tab);
        if (fail) return -2;
    }
    return 0;
}

/* d-dimensional transform of an interleaved (re, im) array, in place. */
int orc_fftnd(int d, const int64_t *shape, double *a_ri, int sign)
{
    return fft_nd(d, shape, (cplx *)a_ri, sign);
}

/* ------------------------------------------------------------------------- */
/* Tensor generation                                                          */
/* ------------------------------------------------------------------------- */

static int check_geometry(int kind, int d, const double *L, const int64_t *N)
{
    if (d < 1 || d > 3) return -1;
    if (kind != 0 && orc_kernel_dim(kind) != d) return -1;
    for (int j = 0; j < d; ++j) {
        if (!(L[j] > 0.0)) return -1;
        if (N[j] < 2 || (N[j] % 2) != 0) return -1;
    }
    return 0;
}

/* signed periodic index of storage position m on an axis of period P = 2N */
static inline long signed_index(long m, long N) { return m < N ? m : m - 2 * N; }

/*
 * Builds T = T(1) + T(2) on the full periodic grid prod_j P_j (C order,
 * signed index n_j stored at n_j mod P_j).  Optional outputs: T1 and T2
 * separately, and max |Im T(2)| (the imaginary part must be round-off).
 */
int orc_build_tensor(int kind, double lam, double eps, int d, const double *L, const int64_t *N,
                     double *T, double *T1_out, double *T2_out, double *t2_imag_max)
{
    if (check_geometry(kind, d, L, N)) return -1;
    if (!(eps > 0.0)) return -1;
    int64_t P[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    double hprod = 1.0;
    size_t total = 1;
    for (int j = 0; j < d; ++j) {
        P[j] = 2 * N[j];
        h[j] = 2.0 * L[j] / (double)N[j];
        hprod *= h[j];
        total *= (size_t)P[j];
    }
    cplx *w = (cplx *)malloc(sizeof(cplx) * total);
    if (!w) return -2;

    /* T(1)_n = prod h_j U^eps(|n h|)  and  W_p = W(|k_p|), k_j = pi p_j / (2 L_j) */
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)total; ++q) {
        size_t rem = (size_t)q;
        double r2 = 0.0, k2 = 0.0;
        for (int j = d - 1; j >= 0; --j) {
            const long m = (long)(rem % (size_t)P[j]);
            rem /= (size_t)P[j];
            const long n = signed_index(m, N[j]);
            const double x = (double)n * h[j];
            const double k = ORC_PI * (double)n / (2.0 * L[j]);
            r2 += x * x;
            k2 += k * k;
        }
        T[q] = hprod * orc_ueps(kind, lam, eps, sqrt(r2));
        w[q] = orc_what(kind, lam, eps, sqrt(k2));
    }
    if (T1_out) memcpy(T1_out, T, sizeof(double) * total);

    /* T(2) = inverse DFT of W with the 1/prod P_j normalisation */
    const int rc = fft_nd(d, P, w, +1);
    if (rc) { free(w); return rc; }
    const double inv = 1.0 / (double)total;
    double imax = 0.0;
#pragma omp parallel for reduction(max : imax) schedule(static)
    for (long q = 0; q < (long)total; ++q) {
        const double re = creal(w[q]) * inv, im = cimag(w[q]) * inv;
        if (fabs(im) > imax) imax = fabs(im);
        if (T2_out) T2_out[q] = re;
        T[q] += re;
    }
    if (t2_imag_max) *t2_imag_max = imax;
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Discrete convolution Phi_i = sum_{i'} T_{i - i'} rho_{i'}  (eq. DiscConv)   */
/* ------------------------------------------------------------------------- */

/* Compensated (Neumaier) accumulation.  eq. DiscConv fixes the sum, not its
 * rounding: a plain running sum of the ~10^7 same-signed terms of a 256^3
 * grid drifts by ~1e-11 relative, so the direct sums carry the rounding error
 * of each addition in a second accumulator. */
typedef struct { double s, c; } kahan;
static inline void kahan_add(kahan *k, double x)
{
    const double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}

/* Direct O(prod N_j^2) sum over all output points. */
int orc_conv_direct(int d, const int64_t *N, const double *T, const double *rho, double *phi)
{
    if (check_geometry(0, d, (const double[]){1, 1, 1}, N)) return -1;
    int64_t Nn[3] = {1, 1, 1}, P[3] = {1, 1, 1};
    for (int j = 0; j < d; ++j) { Nn[3 - d + j] = N[j]; P[3 - d + j] = 2 * N[j]; }
    const long M = (long)(Nn[0] * Nn[1] * Nn[2]);
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < M; ++i) {
        const long i0 = i / (Nn[1] * Nn[2]), i1 = (i / Nn[2]) % Nn[1], i2 = i % Nn[2];
        kahan acc = {0.0, 0.0};
        for (long a = 0; a < Nn[0]; ++a) {
            const long m0 = ((i0 - a) % P[0] + P[0]) % P[0];
            for (long b = 0; b < Nn[1]; ++b) {
                const long m1 = ((i1 - b) % P[1] + P[1]) % P[1];
                const double *trow = T + ((size_t)m0 * P[1] + (size_t)m1) * P[2];
                const double *rrow = rho + ((size_t)a * Nn[1] + (size_t)b) * Nn[2];
                for (long c = 0; c < Nn[2]; ++c) {
                    const long m2 = ((i2 - c) % P[2] + P[2]) % P[2];
                    kahan_add(&acc, trow[m2] * rrow[c]);
                }
            }
        }
        phi[i] = acc.s + acc.c;
    }
    return 0;
}

/* Direct sum at selected output points (flat C-order indices into phi). */
int orc_conv_direct_points(int d, const int64_t *N, const double *T, const double *rho,
                           long npts, const int64_t *flat_idx, double *out)
{
    if (check_geometry(0, d, (const double[]){1, 1, 1}, N)) return -1;
    int64_t Nn[3] = {1, 1, 1}, P[3] = {1, 1, 1};
    for (int j = 0; j < d; ++j) { Nn[3 - d + j] = N[j]; P[3 - d + j] = 2 * N[j]; }
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < npts; ++t) {
        const long i = (long)flat_idx[t];
        const long i0 = i / (Nn[1] * Nn[2]), i1 = (i / Nn[2]) % Nn[1], i2 = i % Nn[2];
        kahan acc = {0.0, 0.0};
        for (long a = 0; a < Nn[0]; ++a) {
            const long m0 = ((i0 - a) % P[0] + P[0]) % P[0];
            for (long b = 0; b < Nn[1]; ++b) {
                const long m1 = ((i1 - b) % P[1] + P[1]) % P[1];
                const double *trow = T + ((size_t)m0 * P[1] + (size_t)m1) * P[2];
                const double *rrow = rho + ((size_t)a * Nn[1] + (size_t)b) * Nn[2];
                for (long c = 0; c < Nn[2]; ++c) {
                    const long m2 = ((i2 - c) % P[2] + P[2]) % P[2];
                    kahan_add(&acc, trow[m2] * rrow[c]);
                }
            }
        }
        out[t] = acc.s + acc.c;
    }
    return 0;
}

/* The same convolution through the oracle's FFT on the 2N-padded grid:
 * Phi = crop( IDFT( DFT(T) . DFT(pad rho) ) ) / prod P_j. */
int orc_conv_fft(int d, const int64_t *N, const double *T, const double *rho, double *phi)
{
    if (check_geometry(0, d, (const double[]){1, 1, 1}, N)) return -1;
    int64_t P[3] = {1, 1, 1};
    size_t total = 1;
    for (int j = 0; j < d; ++j) { P[j] = 2 * N[j]; total *= (size_t)P[j]; }
    cplx *t = (cplx *)malloc(sizeof(cplx) * total);
    cplx *r = (cplx *)calloc(total, sizeof(cplx));
    if (!t || !r) { free(t); free(r); return -2; }
    int64_t Nn[3] = {1, 1, 1}, Pp[3] = {1, 1, 1};
    for (int j = 0; j < d; ++j) { Nn[3 - d + j] = N[j]; Pp[3 - d + j] = P[j]; }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)total; ++q) t[q] = T[q];
#pragma omp parallel for schedule(static)
    for (long a = 0; a < Nn[0]; ++a)
        for (long b = 0; b < Nn[1]; ++b)
            for (long c = 0; c < Nn[2]; ++c)
                r[((size_t)a * Pp[1] + (size_t)b) * Pp[2] + (size_t)c] =
                    rho[((size_t)a * Nn[1] + (size_t)b) * Nn[2] + (size_t)c];
    int rc = fft_nd(d, P, t, -1);
    if (!rc) rc = fft_nd(d, P, r, -1);
    if (rc) { free(t); free(r); return rc; }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)total; ++q) r[q] *= t[q];
    free(t);
    rc = fft_nd(d, P, r, +1);
    if (rc) { free(r); return rc; }
    const double inv = 1.0 / (double)total;
#pragma omp parallel for schedule(static)
    for (long a = 0; a < Nn[0]; ++a)
        for (long b = 0; b < Nn[1]; ++b)
            for (long c = 0; c < Nn[2]; ++c)
                phi[((size_t)a * Nn[1] + (size_t)b) * Nn[2] + (size_t)c] =
                    creal(r[((size_t)a * Pp[1] + (size_t)b) * Pp[2] + (size_t)c]) * inv;
    free(r);
    return 0;
}

/* Convenience: build T and evaluate Phi by the FFT route. */
int orc_solve(int kind, double lam, double eps, int d, const double *L, const int64_t *N,
              const double *rho, double *phi)
{
    if (check_geometry(kind, d, L, N)) return -1;
    size_t total = 1;
    for (int j = 0; j < d; ++j) total *= (size_t)(2 * N[j]);
    double *T = (double *)malloc(sizeof(double) * total);
    if (!T) return -2;
    int rc = orc_build_tensor(kind, lam, eps, d, L, N, T, NULL, NULL, NULL);
    if (!rc) rc = orc_conv_fft(d, N, T, rho, phi);
    free(T);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* 3D dipole-dipole interaction (Sec. 5.3, Example 4)                         */
/* ------------------------------------------------------------------------- */

/*
 * The 3D DDI is evaluated through the Coulomb kernel with the source
 * d_nm rho = (n.grad)(m.grad) rho (Sec. 5.3):
 *     Phi = -(m.n) rho - 3 (U_Coulomb conv d_nm rho).
 * d_nm rho is the spectral derivative of rho on its own grid, taken as
 * periodic on the box: DFT over the N_j points of each axis, product with
 * -(k.n)(k.m), k_j = pi q_j / L_j, where storage position i_j < N_j/2 is
 * q_j = i_j and the others q_j = i_j - N_j, inverse DFT, real part.  (The
 * paper does not spell this step out; this reading reproduces its printed
 * DDI errors of Table 5.)  The Coulomb convolution is the FSA discrete
 * convolution of orc_solve.
 */
int orc_solve_ddi(double eps, const double *L, const int64_t *N, const double *nv,
                  const double *mv, const double *rho, double *phi)
{
    if (check_geometry(ORC_COULOMB_3D, 3, L, N)) return -1;
    const size_t total = (size_t)N[0] * (size_t)N[1] * (size_t)N[2];
    cplx *a = (cplx *)malloc(sizeof(cplx) * total);
    double *src = (double *)malloc(sizeof(double) * total);
    double *conv = (double *)malloc(sizeof(double) * total);
    if (!a || !src || !conv) { free(a); free(src); free(conv); return -2; }
    for (size_t i = 0; i < total; ++i) a[i] = rho[i];
    int rc = fft_nd(3, N, a, -1);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long i0 = 0; i0 < N[0]; ++i0)
            for (long i1 = 0; i1 < N[1]; ++i1)
                for (long i2 = 0; i2 < N[2]; ++i2) {
                    const long iv[3] = {i0, i1, i2};
                    double kn = 0.0, km = 0.0;
                    for (int j = 0; j < 3; ++j) {
                        const long q = iv[j] < N[j] / 2 ? iv[j] : iv[j] - N[j];
                        const double k = ORC_PI * (double)q / L[j];
                        kn += k * nv[j];
                        km += k * mv[j];
                    }
                    a[((size_t)i0 * N[1] + (size_t)i1) * N[2] + (size_t)i2] *= -kn * km;
                }
        rc = fft_nd(3, N, a, +1);
    }
    if (!rc) {
        for (size_t i = 0; i < total; ++i) src[i] = creal(a[i]) / (double)total;
        rc = orc_solve(ORC_COULOMB_3D, 0.0, eps, 3, L, N, src, conv);
    }
    if (!rc) {
        const double nm = nv[0] * mv[0] + nv[1] * mv[1] + nv[2] * mv[2];
        for (size_t i = 0; i < total; ++i) phi[i] = -nm * rho[i] - 3.0 * conv[i];
    }
    free(a);
    free(src);
    free(conv);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Vectorised evaluation helpers for the tests                                */
/* ------------------------------------------------------------------------- */

void orc_ueps_vec(int kind, double lam, double eps, long n, const double *r, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_ueps(kind, lam, eps, r[i]);
}

void orc_what_vec(int kind, double lam, double eps, long n, const double *k, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_what(kind, lam, eps, k[i]);
}

void orc_u_vec(int kind, double lam, long n, const double *r, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_u(kind, lam, r[i]);
}

void orc_e1_vec(long n, const double *x, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_e1(x[i]);
}

void orc_ein_vec(long n, const double *x, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = orc_ein(x[i]);
}
