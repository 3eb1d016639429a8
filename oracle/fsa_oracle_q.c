/*
 * fsa_oracle_q.c -- the FSA oracle in quadruple precision (__float128, 113-bit
 * significand) for the extended-precision mode, Coulomb kernels only.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite may load or call this
 * library.  It shares no code with the GPU library (nor with the FP64
 * oracle): its own mixed-radix FFT in __complex128, the tensor in the
 * paper's order, quadmath's erfq/expm1q for the special functions.
 *
 *   T(1)_n = (prod_j h_j) U^eps(|n h|)                 Sec. 2.1, eq. Tensor1
 *   W_p    = FT[U - U^eps](|k_p|),  k_j = pi p_j/(2L_j) Sec. 2.2, eq. FouTran, Table 1
 *   T(2)   = IDFT over prod_j P_j points of W          Sec. 2.2, eq. Tensor2
 *   Phi_i  = sum_{i'} T_{i-i'} rho_{i'}                Sec. 2.3, eq. DiscConv (FFT route)
 *
 * Kernels (Table 1): 3D Coulomb U^eps = erf(r/eps)/(4 pi r),
 * W = (1 - e^{-k^2 eps^2/4})/k^2; 2D Coulomb U^eps = erf(r/eps)/(2 pi r),
 * W = erf(k eps/2)/k; r = 0 and k = 0 take the limits.  The paper's quad
 * rows (Table 2) come from this discretisation run in quad precision.
 *
 * Arrays cross the interface as double-double pairs (hi, lo) of doubles,
 * interleaved, the value being hi + lo.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 Q;
typedef __complex128 QC;

enum { ORCQ_COULOMB_3D = 1, ORCQ_COULOMB_2D = 4 };

static Q q_of_dd(const double *p) { return (Q)p[0] + (Q)p[1]; }
static void dd_of_q(Q v, double *p)
{
    const double hi = (double)v;
    p[0] = hi;
    p[1] = (double)(v - (Q)hi);
}

static Q orcq_ueps(int kind, Q eps, Q r)
{
    const Q pi = M_PIq;
    if (kind == ORCQ_COULOMB_3D) {
        if (r == 0) return 1 / (2 * pi * sqrtq(pi) * eps);
        return erfq(r / eps) / (4 * pi * r);
    }
    if (r == 0) return 1 / (pi * sqrtq(pi) * eps);
    return erfq(r / eps) / (2 * pi * r);
}

static Q orcq_what(int kind, Q eps, Q k)
{
    if (kind == ORCQ_COULOMB_3D) {
        if (k == 0) return eps * eps / 4;
        return -expm1q(-k * k * eps * eps / 4) / (k * k);
    }
    if (k == 0) return eps / sqrtq(M_PIq);
    return erfq(k * eps / 2) / k;
}

/* ---- FFT: recursive decimation in time over the smallest prime factor ---- */

static int spf(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* tab[j] = exp(sign 2 pi i j / n0) */
static void fft_rec(int n, const QC *in, int is, QC *out, const QC *tab, int n0, QC *tmp)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int p = spf(n), m = n / p, root = n0 / n;
    for (int q = 0; q < p; ++q) fft_rec(m, in + (size_t)q * is, is * p, out + (size_t)q * m, tab, n0, tmp);
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) tmp[q] = out[(size_t)q * m + k];
        for (int s = 0; s < p; ++s) {
            QC acc = 0;
            for (int q = 0; q < p; ++q) acc += tmp[q] * tab[(size_t)(((long)q * (k + s * m)) % n) * root];
            out[(size_t)s * m + k] = acc;
        }
    }
}

static QC *table(int n, int sign)
{
    QC *t = (QC *)malloc(sizeof(QC) * (size_t)n);
    if (!t) return NULL;
    for (int j = 0; j < n; ++j) {
        /* exact reduction of the angle: cos/sin of 2 pi j / n */
        const Q a = 2 * M_PIq * (Q)j / (Q)n;
        __real__ t[j] = cosq(a);
        __imag__ t[j] = (Q)sign * sinq(a);
    }
    return t;
}

static int fft_nd(int d, const int64_t *shape, QC *a, int sign)
{
    size_t total = 1;
    for (int j = 0; j < d; ++j) total *= (size_t)shape[j];
    for (int ax = 0; ax < d; ++ax) {
        const int n = (int)shape[ax];
        size_t stride = 1;
        for (int j = ax + 1; j < d; ++j) stride *= (size_t)shape[j];
        const size_t np = total / (size_t)n;
        QC *tab = table(n, sign);
        if (!tab) return -2;
        int fail = 0;
#pragma omp parallel
        {
            QC *buf = (QC *)malloc(sizeof(QC) * (size_t)n * 2);
            QC *tmp = (QC *)malloc(sizeof(QC) * (size_t)n);
            if (!buf || !tmp) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(static)
                for (long q = 0; q < (long)np; ++q) {
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

/* One length-n transform of DD-pair complex input (re_hi, re_lo, im_hi,
 * im_lo per element), for the tests of the FFT itself. */
int orcq_fft1d(int n, const double *in, double *out, int sign)
{
    QC *a = (QC *)malloc(sizeof(QC) * (size_t)n);
    if (!a) return -2;
    for (int i = 0; i < n; ++i) {
        __real__ a[i] = q_of_dd(in + 4 * i);
        __imag__ a[i] = q_of_dd(in + 4 * i + 2);
    }
    const int64_t sh[1] = {n};
    const int rc = fft_nd(1, sh, a, sign);
    for (int i = 0; i < n && !rc; ++i) {
        dd_of_q(__real__ a[i], out + 4 * i);
        dd_of_q(__imag__ a[i], out + 4 * i + 2);
    }
    free(a);
    return rc;
}

/* Phi for the Coulomb kernels (kind 1: 3D, 4: 2D): builds T = T(1) + T(2)
 * on the full periodic grid and convolves by the FFT route.  rho and phi are
 * DD pairs, C order, shape N. */
int orcq_solve(int kind, double eps_d, int d, const double *L, const int64_t *N,
               const double *rho, double *phi)
{
    if (!((kind == ORCQ_COULOMB_3D && d == 3) || (kind == ORCQ_COULOMB_2D && d == 2))) return -1;
    if (!(eps_d > 0)) return -1;
    const Q eps = eps_d;
    int64_t P[3] = {1, 1, 1}, Nn[3] = {1, 1, 1}, Pp[3] = {1, 1, 1};
    Q h[3] = {1, 1, 1}, hprod = 1;
    size_t total = 1;
    for (int j = 0; j < d; ++j) {
        if (!(L[j] > 0) || N[j] < 2 || (N[j] % 2)) return -1;
        P[j] = 2 * N[j];
        h[j] = 2 * (Q)L[j] / (Q)N[j];
        hprod *= h[j];
        total *= (size_t)P[j];
        Nn[3 - d + j] = N[j];
        Pp[3 - d + j] = P[j];
    }
    QC *t = (QC *)malloc(sizeof(QC) * total);
    QC *w = (QC *)malloc(sizeof(QC) * total);
    QC *r = (QC *)calloc(total, sizeof(QC));
    if (!t || !w || !r) { free(t); free(w); free(r); return -2; }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)total; ++q) {
        size_t rem = (size_t)q;
        Q r2 = 0, k2 = 0;
        for (int j = d - 1; j >= 0; --j) {
            const long m = (long)(rem % (size_t)P[j]);
            rem /= (size_t)P[j];
            const long n = m < N[j] ? m : m - P[j];
            const Q x = (Q)n * h[j], k = M_PIq * (Q)n / (2 * (Q)L[j]);
            r2 += x * x;
            k2 += k * k;
        }
        t[q] = hprod * orcq_ueps(kind, eps, sqrtq(r2));
        w[q] = orcq_what(kind, eps, sqrtq(k2));
    }
    /* T(2) = IDFT(W) / prod P; T = T(1) + T(2) */
    int rc = fft_nd(d, P, w, +1);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long q = 0; q < (long)total; ++q) t[q] += crealq(w[q]) / (Q)total;
    }
    free(w);
    /* Phi = crop(IDFT(DFT(T) DFT(pad rho))) / prod P */
    for (long a = 0; a < Nn[0] && !rc; ++a)
        for (long b = 0; b < Nn[1]; ++b)
            for (long c = 0; c < Nn[2]; ++c)
                r[((size_t)a * Pp[1] + (size_t)b) * Pp[2] + (size_t)c] =
                    q_of_dd(rho + 2 * (((size_t)a * Nn[1] + (size_t)b) * Nn[2] + (size_t)c));
    if (!rc) rc = fft_nd(d, P, t, -1);
    if (!rc) rc = fft_nd(d, P, r, -1);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long q = 0; q < (long)total; ++q) r[q] *= t[q];
        rc = fft_nd(d, P, r, +1);
    }
    for (long a = 0; a < Nn[0] && !rc; ++a)
        for (long b = 0; b < Nn[1]; ++b)
            for (long c = 0; c < Nn[2]; ++c)
                dd_of_q(crealq(r[((size_t)a * Pp[1] + (size_t)b) * Pp[2] + (size_t)c]) / (Q)total,
                        phi + 2 * (((size_t)a * Nn[1] + (size_t)b) * Nn[2] + (size_t)c));
    free(t);
    free(r);
    return rc;
}
