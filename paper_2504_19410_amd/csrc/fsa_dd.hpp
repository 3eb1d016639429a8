// fsa_dd.hpp -- double-double arithmetic for the extended-precision mode.
//
// A double-double value is the unevaluated sum hi + lo of two doubles with
// |lo| <= ulp(hi)/2: 106 significant bits, relative rounding ~1.2e-32.  The
// building blocks are the error-free transformations: two_sum (Knuth) gives
// s + e = a + b exactly, and two_prod with a fused multiply-add gives
// p + e = a * b exactly.  Sums, products and quotients then follow the
// standard double-double algorithms (Dekker 1971; Hida, Li and Bailey 2001).
// Everything here is written for both host and device and relies on IEEE
// round-to-nearest without reassociation (no fast-math).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FSA_DD_HD __host__ __device__ __forceinline__
#else
#define FSA_DD_HD inline
#endif

#include <cmath>

// The error-free transformations need every product and sum rounded as
// written: a product fused into a later addition (floating-point contraction,
// on by default for HIP device code) would break them.  Contraction is off
// from here to the end of this header.
#if defined(__clang__)
#pragma clang fp contract(off)
#endif

namespace fsa {

struct dd {
    double hi, lo;
};

FSA_DD_HD dd dd_make(double hi, double lo) {
    dd r;
    r.hi = hi;
    r.lo = lo;
    return r;
}
FSA_DD_HD dd dd_of(double a) { return dd_make(a, 0.0); }

// s + e = a + b exactly
FSA_DD_HD dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return dd_make(s, e);
}
// s + e = a + b exactly, given |a| >= |b|
FSA_DD_HD dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return dd_make(s, b - (s - a));
}
// p + e = a * b exactly
FSA_DD_HD dd two_prod(double a, double b) {
    const double p = a * b;
    return dd_make(p, std::fma(a, b, -p));
}

FSA_DD_HD dd operator+(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
FSA_DD_HD dd operator-(dd a) { return dd_make(-a.hi, -a.lo); }
FSA_DD_HD dd operator-(dd a, dd b) { return a + (-b); }
FSA_DD_HD dd operator*(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
FSA_DD_HD dd operator*(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
// a / b for a double b (exact integers in the series below): the quotient's
// remainder is formed exactly and corrected once
FSA_DD_HD dd operator/(dd a, double b) {
    const double q1 = a.hi / b;
    const dd p = two_prod(q1, b);
    dd s = two_sum(a.hi, -p.hi);
    s.lo -= p.lo;
    s.lo += a.lo;
    const double q2 = (s.hi + s.lo) / b;
    return quick_two_sum(q1, q2);
}
// a / b: three correction steps of the quotient
FSA_DD_HD dd operator/(dd a, dd b) {
    const double q1 = a.hi / b.hi;
    dd r = a - b * q1;
    const double q2 = r.hi / b.hi;
    r = r - b * q2;
    const double q3 = r.hi / b.hi;
    const dd q = quick_two_sum(q1, q2);
    return q + dd_of(q3);
}
FSA_DD_HD dd dd_sqrt(dd a) {
    if (a.hi <= 0.0) return dd_of(0.0);
    const double y = std::sqrt(a.hi);
    // one Newton step: y + (a - y^2) / (2y), the residual in double-double
    const dd r = a - two_prod(y, y);
    return quick_two_sum(y, 0.5 * (r.hi + r.lo) / y);
}
FSA_DD_HD bool dd_lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// Constants to double-double accuracy.
FSA_DD_HD dd dd_pi() { return dd_make(3.141592653589793116e+00, 1.224646799147353207e-16); }
FSA_DD_HD dd dd_ln2() { return dd_make(6.931471805599452862e-01, 2.319046813846299558e-17); }
// 2 / sqrt(pi)
FSA_DD_HD dd dd_two_over_sqrtpi() {
    return dd_make(1.128379167095512558e+00, 1.533545961316588336e-17);
}

// e^x: x = k ln2 + r, |r| <= ln2/2; e^r = (e^{r/256})^256 with the Taylor
// series of e^{r/256} (|r/256| < 1.4e-3, 14 terms reach 1e-34).
FSA_DD_HD dd dd_exp(dd x) {
    if (x.hi > 700.0) return dd_of(INFINITY);
    if (x.hi < -700.0) return dd_of(0.0);
    const double k = std::nearbyint(x.hi / dd_ln2().hi);
    // k ln2 with ln2 split into three doubles and each product formed
    // exactly (|k| <= 1010), so that r carries no reduction error
    dd r = x - two_prod(dd_ln2().hi, k);
    r = r - two_prod(dd_ln2().lo, k);
    r = r - dd_of(5.707708438416212066e-34 * k);
    r = r * (1.0 / 256.0);
    dd term = r, sum = r;
    for (int n = 2; n <= 14; ++n) {
        term = term * r / (double)n;
        sum = sum + term;
    }
    // sum = e^{r/256} - 1; square 8 times keeping the "- 1" form:
    // (1 + s)^2 - 1 = 2s + s^2
    for (int i = 0; i < 8; ++i) sum = sum * 2.0 + sum * sum;
    const dd e = sum + dd_of(1.0);
    return dd_make(std::ldexp(e.hi, (int)k), std::ldexp(e.lo, (int)k));
}

// e^x - 1 without cancellation for |x| < 1/2 (Taylor series), else e^x - 1.
FSA_DD_HD dd dd_expm1(dd x) {
    if (std::fabs(x.hi) >= 0.5) return dd_exp(x) - dd_of(1.0);
    dd term = x, sum = x;
    for (int n = 2; n <= 40; ++n) {
        term = term * x / (double)n;
        sum = sum + term;
        if (std::fabs(term.hi) < 1e-36 * std::fabs(sum.hi)) break;
    }
    return sum;
}

// erf(x), x >= 0: (2/sqrt(pi)) e^{-x^2} sum_{n>=0} 2^n x^{2n+1} / (1 3 5 ... (2n+1))
// (Abramowitz & Stegun 7.1.6), a series of positive terms; erf = 1 to
// double-double precision beyond x = 9.5 (erfc(9.5) < 1e-40).
FSA_DD_HD dd dd_erf(dd x) {
    if (x.hi <= 0.0) return dd_of(0.0);
    if (x.hi > 9.5) return dd_of(1.0);
    const dd x2 = x * x;
    dd term = x, sum = x;
    for (int n = 1; n < 400; ++n) {
        term = term * x2 * 2.0 / (2.0 * n + 1.0);
        sum = sum + term;
        if (term.hi < 1e-36 * sum.hi) break;
    }
    return dd_two_over_sqrtpi() * dd_exp(-x2) * sum;
}

// cos and sin of 2 pi f for f in [0, 1) given as an exact double: reduced to
// [0, 1/8] by symmetry, then Taylor series (|theta| <= pi/4: 24 terms).
FSA_DD_HD void dd_sincos_turn(double f, dd* s, dd* c) {
    // f in [0,1): octant o = floor(8 f), remainder g = f - o/8 exact
    int o = (int)(f * 8.0);
    if (o > 7) o = 7;
    double g = f - o * 0.125;  // [0, 1/8)
    bool flip = o & 1;         // use 1/8 - g
    if (flip) g = 0.125 - g;   // exact (g is a multiple of a power of two fraction)
    const dd th = dd_pi() * (2.0 * g);
    const dd t2 = th * th;
    dd ts = th, ss = th, tc = dd_of(1.0), cc = dd_of(1.0);
    for (int n = 1; n <= 16; ++n) {
        tc = -(tc * t2) / ((2.0 * n - 1.0) * (2.0 * n));
        cc = cc + tc;
        ts = -(ts * t2) / ((2.0 * n) * (2.0 * n + 1.0));
        ss = ss + ts;
    }
    // angle within the first octant: (sin, cos) = (ss, cc); flipped: (cc, ss)
    dd sn = flip ? cc : ss, cs = flip ? ss : cc;
    // rotate by o * 45 degrees using quadrant symmetries
    switch (o >> 1) {  // quadrant
    case 0: *s = sn; *c = cs; break;
    case 1: *s = cs; *c = -sn; break;
    case 2: *s = -sn; *c = -cs; break;
    default: *s = -cs; *c = sn; break;
    }
}

}  // namespace fsa

#if defined(__clang__)
#pragma clang fp contract(fast)
#endif
