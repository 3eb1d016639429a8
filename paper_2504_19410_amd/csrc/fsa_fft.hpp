// fsa_fft.hpp -- Stockham FFT building blocks for gfx950 (wave64, LDS-staged).
//
// A "team" of T threads computes one complex transform of length P.  Each
// thread keeps its butterflies' operands in registers; stages exchange data
// through a padded LDS scratch of the team.  Stage s (radix R_s) with
// NS = R_0 ... R_{s-1} and NB = P / R_s butterflies follows the Stockham
// autosort recursion:
//
//   butterfly j in [0, NB):  k = j mod NS
//     inputs   x[j + q NB]                        q = 0 .. R_s - 1
//     operands a_q = x[j + q NB] * w^{q k},      w = exp(-/+ 2 pi i / (NS R_s))
//     outputs  y[(j / NS) NS R_s + k + q NS] = DFT_{R_s}(a)_q
//
// Thread t owns butterflies j = t + b T (b = 0 .. ceil(NB/T) - 1) and holds
// their operands in v[b R_s + q].  The first stage has NS = 1 (no twiddles),
// so its inputs can come straight from global memory; the last stage has
// NS = P / R_last, so thread t's outputs are x[j + q P / R_last] and can go
// straight to global memory.  An inverse transform runs the radices in
// reverse order, so the forward's last-stage layout IS the inverse's
// first-stage layout: a pointwise product between them needs no exchange.
//
// Every per-thread phase is __host__ __device__ so that the index logic can
// be emulated thread by thread on the CPU (tests/host).  Twiddles come from
// a table tw[m] = exp(-2 pi i m / P) built in FP64 on the host.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#else
// plain C++ (the CPU emulation of the team transforms): no device qualifiers
#define __host__
#define __device__
#define __forceinline__ inline
#endif

#include <cstdint>

namespace fsa {

#define FSA_HD __host__ __device__ __forceinline__

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <typename R>
FSA_HD cpx<R> mk(R a, R b) { cpx<R> c; c.x = a; c.y = b; return c; }
template <typename R>
FSA_HD cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
FSA_HD cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
FSA_HD cpx<R> cmul(cpx<R> a, cpx<R> b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
template <typename R>
FSA_HD cpx<R> cmulc(cpx<R> a, cpx<R> b) { return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
template <typename R>
FSA_HD cpx<R> conj(cpx<R> a) { return mk(a.x, -a.y); }
template <typename R>
FSA_HD cpx<R> scale(cpx<R> a, R s) { return mk(a.x * s, a.y * s); }
// multiplication by -i (forward) or +i (inverse)
template <bool INV, typename R>
FSA_HD cpx<R> rot90(cpx<R> a) { return INV ? mk(-a.y, a.x) : mk(a.y, -a.x); }

// ---------------------------------------------------------------------------
// Small DFTs in registers (natural order in, natural order out).
// Forward: y_q = sum_p a_p exp(-2 pi i p q / R); inverse: exp(+...).
// ---------------------------------------------------------------------------

template <bool INV, typename R>
FSA_HD void dft2(cpx<R>* a) {
    const cpx<R> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
}

template <bool INV, typename R>
FSA_HD void dft3(cpx<R>* a) {
    const R c = R(-0.5), s = R(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    const cpx<R> t = a[1] + a[2];
    const cpx<R> m = a[0] + scale(t, c);
    // (a1 - a2) * (-/+ i sin(2pi/3))
    const cpx<R> d = scale(rot90<INV>(a[1] - a[2]), s);
    a[0] = a[0] + t;
    a[1] = m + d;
    a[2] = m - d;
}

template <bool INV, typename R>
FSA_HD void dft4(cpx<R>* a) {
    const cpx<R> t0 = a[0] + a[2], t1 = a[0] - a[2];
    const cpx<R> t2 = a[1] + a[3], t3 = rot90<INV>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
}

// multiply by exp(-/+ 2 pi i q / 8)
template <bool INV, int q, typename R>
FSA_HD cpx<R> w8(cpx<R> a) {
    const R h = R(0.70710678118654752440084436210485);
    if constexpr (q == 0) return a;
    else if constexpr (q == 1) return INV ? mk((a.x - a.y) * h, (a.x + a.y) * h)
                                          : mk((a.x + a.y) * h, (a.y - a.x) * h);
    else if constexpr (q == 2) return rot90<INV>(a);
    else return INV ? mk(-(a.x + a.y) * h, (a.x - a.y) * h)
                    : mk((a.y - a.x) * h, -(a.x + a.y) * h);
}

template <bool INV, typename R>
FSA_HD void dft8(cpx<R>* a) {
    cpx<R> e[4] = {a[0], a[2], a[4], a[6]};
    cpx<R> o[4] = {a[1], a[3], a[5], a[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    o[1] = w8<INV, 1>(o[1]);
    o[2] = w8<INV, 2>(o[2]);
    o[3] = w8<INV, 3>(o[3]);
    for (int q = 0; q < 4; ++q) {
        a[q] = e[q] + o[q];
        a[q + 4] = e[q] - o[q];
    }
}

template <bool INV, typename R>
FSA_HD void dft16(cpx<R>* a) {
    cpx<R> e[8], o[8];
    for (int q = 0; q < 8; ++q) {
        e[q] = a[2 * q];
        o[q] = a[2 * q + 1];
    }
    dft8<INV>(e);
    dft8<INV>(o);
    // o[q] *= exp(-/+ 2 pi i q / 16)
    const R c1 = R(0.92387953251128675612818318939679);  // cos(pi/8)
    const R s1 = R(0.38268343236508977172845998403040);  // sin(pi/8)
    const R h = R(0.70710678118654752440084436210485);
    const R sg = INV ? R(1) : R(-1);
    const cpx<R> tw[8] = {mk(R(1), R(0)), mk(c1, sg * s1), mk(h, sg * h), mk(s1, sg * c1),
                          mk(R(0), sg),   mk(-s1, sg * c1), mk(-h, sg * h), mk(-c1, sg * s1)};
    for (int q = 1; q < 8; ++q) o[q] = cmul(o[q], tw[q]);
    for (int q = 0; q < 8; ++q) {
        a[q] = e[q] + o[q];
        a[q + 8] = e[q] - o[q];
    }
}

// multiply by exp(-/+ 2 pi i k / 12) (forward / inverse)
template <bool INV, int K, typename R>
FSA_HD cpx<R> w12(cpx<R> a) {
    constexpr int k = K % 12;
    const R c = R(0.86602540378443864676372317075294);  // cos(pi/6)
    const R h = R(0.5);
    // (cos, sin) of 2 pi k / 12; the forward factor is cos - i sin
    const R cs = k == 0 ? R(1) : k == 1 ? c : k == 2 ? h : k == 3 ? R(0) : k == 4 ? -h
               : k == 5 ? -c : k == 6 ? R(-1) : k == 7 ? -c : k == 8 ? -h : k == 9 ? R(0)
               : k == 10 ? h : c;
    const R sn = k == 0 ? R(0) : k == 1 ? h : k == 2 ? c : k == 3 ? R(1) : k == 4 ? c
               : k == 5 ? h : k == 6 ? R(0) : k == 7 ? -h : k == 8 ? -c : k == 9 ? R(-1)
               : k == 10 ? -c : -h;
    if constexpr (k == 0) return a;
    else if constexpr (k == 3 || k == 9) return (k == 3) == !INV ? rot90<false>(a) : rot90<true>(a);
    else if constexpr (k == 6) return mk(-a.x, -a.y);
    else {
        const R s = INV ? sn : -sn;  // w = cs + i s
        return mk(a.x * cs - a.y * s, a.x * s + a.y * cs);
    }
}

// length 6 = 2 x 3: DFT3 of the even and the odd points, combined with w6^k
template <bool INV, typename R>
FSA_HD void dft6(cpx<R>* a) {
    cpx<R> e[3] = {a[0], a[2], a[4]};
    cpx<R> o[3] = {a[1], a[3], a[5]};
    dft3<INV>(e);
    dft3<INV>(o);
    o[1] = w12<INV, 2>(o[1]);
    o[2] = w12<INV, 4>(o[2]);
    for (int q = 0; q < 3; ++q) {
        a[q] = e[q] + o[q];
        a[q + 3] = e[q] - o[q];
    }
}

// length 12 = 3 x 4: DFT4 of the points r, r + 3, r + 6, r + 9 (r < 3), then
// for each k1 < 4 the DFT3 over r of w12^(r k1) D_r[k1] gives y[k1 + 4 k2]
template <bool INV, typename R>
FSA_HD void dft12(cpx<R>* a) {
    cpx<R> d[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int m = 0; m < 4; ++m) d[r][m] = a[r + 3 * m];
        dft4<INV>(d[r]);
    }
    cpx<R> u[4][3];
    for (int k1 = 0; k1 < 4; ++k1) u[k1][0] = d[0][k1];
    u[0][1] = d[1][0];
    u[1][1] = w12<INV, 1>(d[1][1]);
    u[2][1] = w12<INV, 2>(d[1][2]);
    u[3][1] = w12<INV, 3>(d[1][3]);
    u[0][2] = d[2][0];
    u[1][2] = w12<INV, 2>(d[2][1]);
    u[2][2] = w12<INV, 4>(d[2][2]);
    u[3][2] = w12<INV, 6>(d[2][3]);
    for (int k1 = 0; k1 < 4; ++k1) {
        dft3<INV>(u[k1]);
        for (int k2 = 0; k2 < 3; ++k2) a[k1 + 4 * k2] = u[k1][k2];
    }
}

// DFTs of R points whose upper half a[R/2 .. R-1] is zero (the first stage of
// a zero-padded transform): the butterflies of dft<R> without the additions of
// the zero operands (x + 0 is not x in IEEE arithmetic when x = -0, so the
// compiler keeps them otherwise).
template <bool INV, typename R>
FSA_HD void dft4_zh(cpx<R>* a) {
    const cpx<R> a0 = a[0], a1 = a[1], t3 = rot90<INV>(a[1]);
    a[0] = a0 + a1;
    a[2] = a0 - a1;
    a[1] = a0 + t3;
    a[3] = a0 - t3;
}

template <bool INV, typename R>
FSA_HD void dft8_zh(cpx<R>* a) {
    cpx<R> e[4] = {a[0], a[2]}, o[4] = {a[1], a[3]};
    dft4_zh<INV>(e);
    dft4_zh<INV>(o);
    o[1] = w8<INV, 1>(o[1]);
    o[2] = w8<INV, 2>(o[2]);
    o[3] = w8<INV, 3>(o[3]);
    for (int q = 0; q < 4; ++q) {
        a[q] = e[q] + o[q];
        a[q + 4] = e[q] - o[q];
    }
}

template <bool INV, typename R>
FSA_HD void dft16_zh(cpx<R>* a) {
    cpx<R> e[8], o[8];
    for (int q = 0; q < 4; ++q) {
        e[q] = a[2 * q];
        o[q] = a[2 * q + 1];
    }
    dft8_zh<INV>(e);
    dft8_zh<INV>(o);
    const R c1 = R(0.92387953251128675612818318939679);  // cos(pi/8)
    const R s1 = R(0.38268343236508977172845998403040);  // sin(pi/8)
    const R h = R(0.70710678118654752440084436210485);
    const R sg = INV ? R(1) : R(-1);
    const cpx<R> tw[8] = {mk(R(1), R(0)), mk(c1, sg * s1), mk(h, sg * h), mk(s1, sg * c1),
                          mk(R(0), sg),   mk(-s1, sg * c1), mk(-h, sg * h), mk(-c1, sg * s1)};
    for (int q = 1; q < 8; ++q) o[q] = cmul(o[q], tw[q]);
    for (int q = 0; q < 8; ++q) {
        a[q] = e[q] + o[q];
        a[q + 8] = e[q] - o[q];
    }
}

template <int RADIX, bool INV, typename R>
FSA_HD void dft_zh(cpx<R>* a) {
    if constexpr (RADIX == 2) a[1] = a[0];
    else if constexpr (RADIX == 4) dft4_zh<INV>(a);
    else if constexpr (RADIX == 8) dft8_zh<INV>(a);
    else if constexpr (RADIX == 16) dft16_zh<INV>(a);
    else static_assert(RADIX == 2, "zero-half first stage: radix 2, 4, 8 or 16");
}

template <int RADIX, bool INV, typename R>
FSA_HD void dft(cpx<R>* a) {
    if constexpr (RADIX == 2) dft2<INV>(a);
    else if constexpr (RADIX == 3) dft3<INV>(a);
    else if constexpr (RADIX == 4) dft4<INV>(a);
    else if constexpr (RADIX == 6) dft6<INV>(a);
    else if constexpr (RADIX == 8) dft8<INV>(a);
    else if constexpr (RADIX == 12) dft12<INV>(a);
    else if constexpr (RADIX == 16) dft16<INV>(a);
    else static_assert(RADIX == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Transform plans
// ---------------------------------------------------------------------------

struct FftPlan {
    int P;      // length
    int T;      // threads per transform (power of two)
    int n;      // number of stages
    int r[16];  // radices, execution order of the FORWARD transform
    int vmax;   // complex registers per thread
};

constexpr int ilog2_exact(int x) {
    int b = 0;
    while ((1 << b) < x) ++b;
    return ((1 << b) == x) ? b : -1;
}

// Lengths 2^a (a >= 2) and 3 * 2^a (a >= 2; see make_fft_plan for their
// families).  For powers of two, the default family (alt = 0)
// uses power-of-two radices of at most 8 (P < 1024) or 16 (P >= 1024), with
// the bits spread so that the radix sequence reads the same both ways
// whenever possible (the inverse runs the radices reversed, so a palindromic
// plan lets the forward and inverse transforms of the fused pass share one
// set of twiddles); a factor 3 runs last, or, with mid3, sits in the middle
// stage of 2^e . (3 2^mid) . 2^e (mid <= 2); T is the largest power of two
// with T * E <= P (or <= span, which lets threads idle in some stages) for
// E = 8 (P < 1024) or 16 operands per thread, capped at 256.  The alternate
// family (alt = 1) swaps both choices -- radices up to 16
// and E = 16 below 1024, radices up to 8 and E = 8 from 1024 -- which changes
// the radix split and the threads per transform; the autotuner times both.
// It falls back to the default where it would leave teams of fewer than 8
// threads or more than 16 operands per thread.
constexpr FftPlan make_fft_plan_rule(int P, int maxbits, int E, bool mid3 = false, int span = 0) {
    FftPlan p{};
    p.P = P;
    int m = P, threes = 0;
    while (m % 3 == 0) {
        m /= 3;
        ++threes;
    }
    const int a = ilog2_exact(m);
    if (mid3 && threes == 1 && a >= 2) {
        // 2^e . (3 2^mid) . 2^e, mid <= 2 (radix 3, 6 or 12 in the middle)
        int mid = a % 2, e = (a - mid) / 2;
        if (e > maxbits) {
            mid += 2 * (e - maxbits);
            e = maxbits;
        }
        if (mid <= 2 && e >= 1) {
            p.r[0] = 1 << e;
            p.r[1] = 3 << mid;
            p.r[2] = 1 << e;
            p.n = 3;
            int T = 1;
            while (T * 2 * E <= (span ? span : P) && T < 256) T *= 2;
            p.T = T;
            int vmax = 0;
            for (int s = 0; s < 3; ++s) {
                const int nb = P / p.r[s];
                const int b = (nb + T - 1) / T;
                if (b * p.r[s] > vmax) vmax = b * p.r[s];
            }
            p.vmax = vmax;
            return p;
        }
    }
    const int nst = (a + maxbits - 1) / maxbits;
    int bits[16] = {};
    if (nst == 3) {
        // ends e, middle m, 2e + m = a: palindromic by construction
        int e = a / 3, mid = a - 2 * e;
        while (mid > maxbits) {
            ++e;
            mid -= 2;
        }
        bits[0] = e;
        bits[1] = mid;
        bits[2] = e;
    } else {
        for (int s = 0; s < nst; ++s) bits[s] = a / nst + (s < a % nst ? 1 : 0);
    }
    int n = 0;
    for (int s = 0; s < nst; ++s) p.r[n++] = 1 << bits[s];
    for (int t = 0; t < threes; ++t) p.r[n++] = 3;
    p.n = n;
    int T = 1;
    while (T * 2 * E <= P && T < 256) T *= 2;
    p.T = T;
    int vmax = 0;
    for (int s = 0; s < n; ++s) {
        const int nb = P / p.r[s];
        const int b = (nb + T - 1) / T;
        if (b * p.r[s] > vmax) vmax = b * p.r[s];
    }
    p.vmax = vmax;
    return p;
}

constexpr FftPlan make_fft_plan(int P, int alt = 0) {
    const bool big = P >= 1024;
    if (P % 3 == 0) {
        // lengths 3 * 2^a: three stages with the factor 3 in the middle one
        // (a palindrome: one LDS exchange fewer, and a fused forward /
        // inverse pair shares its twiddles).  From 192 the default runs it on
        // a team of twice the threads (T E <= 4P/3): the outer radix-2^e
        // stages then leave a quarter of the threads idle, but each thread
        // holds half the operands (at 384: 64 threads of 8 instead of 32 of
        // 16, 184 -> 146 VGPRs in the FP64 fused pass, 240 -> 127 us at
        // 192^3), and the alternate family is the palindrome on the narrower
        // team; below 192 the default is that palindrome and the alternate
        // the power-of-two split with the radix 3 last
        const FftPlan pal = make_fft_plan_rule(P, big ? 4 : 3, big ? 16 : 8, true);
        const FftPlan last = make_fft_plan_rule(P, big ? 4 : 3, big ? 16 : 8, false);
        const FftPlan wide = make_fft_plan_rule(P, big ? 4 : 3, big ? 16 : 8, true, 4 * P / 3);
        if (P >= 192 && wide.T > pal.T && wide.vmax <= 16) return alt ? pal : wide;
        return alt ? last : pal;
    }
    const FftPlan def = make_fft_plan_rule(P, big ? 4 : 3, big ? 16 : 8);
    if (!alt) return def;
    const FftPlan p = make_fft_plan_rule(P, big ? 3 : 4, big ? 8 : 16);
    return (p.T >= 8 && p.vmax <= 16) ? p : def;
}

// Whether the alternate family gives a different transform at length P.
constexpr bool fft_alt_distinct(int P) {
    const FftPlan a = make_fft_plan(P, 0), b = make_fft_plan(P, 1);
    if (a.T != b.T || a.n != b.n) return true;
    for (int s = 0; s < a.n; ++s)
        if (a.r[s] != b.r[s]) return true;
    return false;
}

constexpr bool fft_length_supported(long P) {
    if (P < 8 || P > 4096) return false;
    long m = P;
    if (m % 3 == 0) m /= 3;
    if (m < 4) return false;
    return (m & (m - 1)) == 0;
}

#if defined(__HIPCC__)
// Team index of the calling thread for teams of T threads.  A team of
// T >= 64 threads spans whole waves (wave64), so its index is the same on
// every lane of a wave; reading it from the first lane lets the compiler know
// that, and the work-item, pencil and tensor-row arithmetic derived from it
// runs once per wave on the scalar unit instead of on every lane.
template <int T>
__device__ __forceinline__ int team_index() {
    const int t = (int)threadIdx.x / T;
    if constexpr (T % 64 == 0) return __builtin_amdgcn_readfirstlane(t);
    else return t;
}

#endif

// ---------------------------------------------------------------------------
// Team transform of length P, direction INV.
// ---------------------------------------------------------------------------

template <typename R, int P_, bool INV, int ALT = 0, int XCH = 0>
struct Fft {
    using C = cpx<R>;
    static constexpr int P = P_;
    static constexpr FftPlan plan = make_fft_plan(P_, ALT);
    static constexpr int T = plan.T;
    static constexpr int V = plan.vmax;
    static constexpr int S = plan.n;
    // padded scratch: one dummy slot every 8 entries breaks the stride-R bank pattern
    static constexpr int SCR = P_ + (P_ >> 3) + 1;

    FSA_HD static constexpr int pad(int i) { return i + (i >> 3); }

    // radix of execution stage s (inverse runs the forward radices reversed)
    static constexpr int radix(int s) { return INV ? plan.r[S - 1 - s] : plan.r[s]; }
    static constexpr int ns(int s) {
        int v = 1;
        for (int t = 0; t < s; ++t) v *= radix(t);
        return v;
    }
    static constexpr int nb(int s) { return P_ / radix(s); }
    static constexpr int nbt(int s) { return (nb(s) + T - 1) / T; }  // butterflies per thread
    static constexpr int first_stride() { return nb(0); }            // x[j + q * this]
    static constexpr int last_stride() { return ns(S - 1); }         // y[j + q * this]
    static constexpr int first_radix() { return radix(0); }
    static constexpr int last_radix() { return radix(S - 1); }
    static constexpr int first_nbt() { return nbt(0); }

    // Input index of first-stage operand q of thread tid's butterfly b, or -1
    // where that butterfly does not exist: when NB is not a multiple of T the
    // last butterfly slot of some threads lies beyond NB, and its operand
    // "indices" would run past the end of the line.  For q < R/2 every index
    // is below P/2, the non-zero half of a zero-padded input.
    FSA_HD static constexpr int first_index(int tid, int b, int q) {
        return ((nb(0) % T) != 0 && tid + b * T >= nb(0)) ? -1 : tid + b * T + q * nb(0);
    }
    static constexpr int last_nbt() { return nbt(S - 1); }

    // twiddle + butterfly of stage s on the registers (ZH: stage 0 with the
    // upper half of every butterfly's operands zero, see dft_zh)
    template <int s, bool ZH = false>
    FSA_HD static void compute(C (&v)[V], int tid, const C* __restrict__ tw) {
        constexpr int RAD = radix(s), NS = ns(s), NB = nb(s), NBT = nbt(s);
        constexpr int STEP = P_ / (NS * RAD);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int q = 1; q < RAD; ++q) {
                    const C w = tw[q * k * STEP];
                    v[b * RAD + q] = INV ? cmulc(v[b * RAD + q], w) : cmul(v[b * RAD + q], w);
                }
            }
            if constexpr (ZH && s == 0) dft_zh<RAD, INV>(&v[b * RAD]);
            else dft<RAD, INV>(&v[b * RAD]);
        }
    }

    // ---- twiddles held in registers ----------------------------------------
    // Thread t's twiddles depend only on t, so a thread that transforms many
    // pencils loads them once: stage s >= 1, butterfly b, q = 1..R_s-1.
    static constexpr int tw_count(int s) { return nbt(s) * (radix(s) - 1); }
    static constexpr int tw_off(int s) {
        int o = 0;
        for (int t = 1; t < s; ++t) o += tw_count(t);
        return o;
    }
    static constexpr int NTW_ = tw_off(S) > 0 ? tw_off(S) : 1;
    static constexpr int NTW = NTW_;

    // forward-direction twiddles (the inverse conjugates them on use)
    FSA_HD static void load_tw(C (&w)[NTW], int tid, const C* __restrict__ tw) {
        load_tw_from<1>(w, tid, tw);
    }
    template <int s>
    FSA_HD static void load_tw_from(C (&w)[NTW], int tid, const C* __restrict__ tw) {
        if constexpr (s < S) {
            constexpr int RAD = radix(s), NS = ns(s), NB = nb(s), NBT = nbt(s);
            constexpr int STEP = P_ / (NS * RAD), OFF = tw_off(s);
#pragma unroll
            for (int b = 0; b < NBT; ++b) {
                const int j = tid + b * T;
                const int k = ((NB % T) != 0 && j >= NB) ? 0 : j % NS;
#pragma unroll
                for (int q = 1; q < RAD; ++q) w[OFF + b * (RAD - 1) + q - 1] = tw[q * k * STEP];
            }
            load_tw_from<s + 1>(w, tid, tw);
        }
    }

    // stage s with twiddles from registers laid out like load_tw's
    template <int s, bool ZH = false>
    FSA_HD static void compute_r(C (&v)[V], int tid, const C (&w)[NTW]) {
        constexpr int RAD = radix(s), NS = ns(s), NB = nb(s), NBT = nbt(s), OFF = tw_off(s);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
            if constexpr (NS > 1) {
#pragma unroll
                for (int q = 1; q < RAD; ++q) {
                    const C t = w[OFF + b * (RAD - 1) + q - 1];
                    v[b * RAD + q] = INV ? cmulc(v[b * RAD + q], t) : cmul(v[b * RAD + q], t);
                }
            }
            if constexpr (ZH && s == 0) dft_zh<RAD, INV>(&v[b * RAD]);
            else dft<RAD, INV>(&v[b * RAD]);
        }
    }

    // ---- exchanges in registers (XCH = 1) ----------------------------------
    // The exchange before stage s only trades the register index with lane
    // bits where the team is one wave (T = 64) whose threads run one radix-8
    // butterfly at stages s-1 and s, with ns(s-1) = 8: thread j leaves its
    // output q at y[(j / 8) 64 + j % 8 + 8 q], and thread j' = 8 a + b reads
    // its input q' at y[j' + 64 q'], which is output a of thread 8 q' + b.
    // So register bit i trades places with lane bit 3 + i (i = 0, 1, 2), and
    // with XCH = 1 that exchange is done across lanes instead of through the
    // LDS: for each pair of registers that differ in bit i, the lanes whose
    // bit 3 + i is set take the partner lane's upper register and give it
    // their lower one (swap_bit).  Everywhere else the exchange stays in LDS.
    static constexpr bool reg_exchange(int s) {
        return XCH == 1 && T == 64 && s >= 1 && s < S && radix(s - 1) == 8 && radix(s) == 8 &&
               nbt(s - 1) == 1 && nbt(s) == 1 && ns(s - 1) == 8;
    }
    static constexpr bool has_reg_exchange() {
        for (int s = 1; s < S; ++s)
            if (reg_exchange(s)) return true;
        return false;
    }
    struct Words {
        unsigned w[sizeof(C) / 4];
    };
    static constexpr int NW = (int)(sizeof(C) / 4);

    // The same exchange on the registers of the whole team, v[lane][q]: the
    // pair swap of every register bit with its lane bit, one bit at a time
    // (the host emulation of swap_bit).
    static void reg_exchange_team(C (*v)[V]) {
        for (int rb = 0; rb < 3; ++rb) {
            const int lb = 3 + rb;
            for (int q = 0; q < 8; ++q) {
                if ((q >> rb) & 1) continue;
                const int q1 = q | (1 << rb);
                C na[64], nb[64];
                for (int l = 0; l < 64; ++l) {
                    const int p = l ^ (1 << lb);
                    const bool hi = (l >> lb) & 1;
                    na[l] = hi ? v[p][q1] : v[l][q];
                    nb[l] = hi ? v[l][q1] : v[p][q];
                }
                for (int l = 0; l < 64; ++l) {
                    v[l][q] = na[l];
                    v[l][q1] = nb[l];
                }
            }
        }
    }

    // ---- the first forward stage as a matrix product (FP32 16x16x4 MFMA) --
    // For a one-wave team of one radix-8 butterfly per thread (length 512)
    // whose operands q >= 4 are zero (the zero-padded input): butterfly j
    // takes x[j + 64 q], q < 4, and gives y[j][k] = sum_q x[j + 64 q]
    // e^{-2 pi i q k / 8}.  In real form, Y = A X with X (8 x 64: real and
    // imaginary part of each operand, row u = 2 q + part) and Y (16 x 64:
    // row m = 2 k + part).  The MFMA computes D (16 x 16) += A (16 x 4)
    // B (4 x 16); lane l gives A[l % 16][l / 16] and B[l / 16][l % 16] and
    // holds D[4 (l / 16) + r][l % 16], r = 0..3.  Butterflies 16 g .. 16 g +
    // 15 form column block g, rows u = 4 ks .. 4 ks + 3 K step ks.
    static constexpr bool mfma_first_ok() {
        return !INV && T == 64 && radix(0) == 8 && nbt(0) == 1 && P_ == 512;
    }
    // lane's A operand at K step ks
    FSA_HD static float mfma0_a(int lane, int ks) {
        const float h = 0.70710678118654752f;  // cos and sin of 2 pi n / 8
        const float cs[8] = {1.f, h, 0.f, -h, -1.f, -h, 0.f, h};
        const float sn[8] = {0.f, h, 1.f, h, 0.f, -h, -1.f, -h};
        const int m = lane % 16, u = 4 * ks + lane / 16;
        const int n = ((u / 2) * (m / 2)) % 8;
        // (a + i b) e^{-i t} = (a cos t + b sin t) + i (b cos t - a sin t)
        if (m % 2 == 0) return (u % 2 == 0) ? cs[n] : sn[n];
        return (u % 2 == 0) ? -sn[n] : cs[n];
    }
    // input index whose part mfma0_part(lane) is lane's B operand for column
    // block g, K step ks (always < P / 2)
    FSA_HD static int mfma0_b_index(int lane, int g, int ks) {
        return 16 * g + lane % 16 + 64 * (2 * ks + (lane / 16) / 2);
    }
    FSA_HD static int mfma0_part(int lane) { return (lane / 16) % 2; }
    // D registers 2 h, 2 h + 1 (real, imaginary) of lane, column block g:
    // output k = 2 (lane / 16) + h of butterfly j = 16 g + lane % 16, which
    // the stage-0 store puts at scratch slot pad(8 j + k)
    FSA_HD static int mfma0_slot(int lane, int g, int h) {
        return pad(8 * (16 * g + lane % 16) + 2 * (lane / 16) + h);
    }

    // the inverse of a palindromic plan has the forward's (radix, NS) per
    // stage, hence the same twiddles (conjugated on use)
    static constexpr bool palindromic() {
        for (int s = 0; s < S; ++s)
            if (plan.r[s] != plan.r[S - 1 - s]) return false;
        return true;
    }

    // write the outputs of stage s to the scratch
    template <int s>
    FSA_HD static void store(const C (&v)[V], C* scr, int tid) {
        constexpr int RAD = radix(s), NS = ns(s), NB = nb(s), NBT = nbt(s);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
            const int k = j % NS;
            const int base = (j / NS) * NS * RAD + k;
#pragma unroll
            for (int q = 0; q < RAD; ++q) scr[pad(base + q * NS)] = v[b * RAD + q];
        }
    }

    // read the inputs of stage s from the scratch
    template <int s>
    FSA_HD static void load(C (&v)[V], const C* scr, int tid) {
        constexpr int RAD = radix(s), NB = nb(s), NBT = nbt(s);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
#pragma unroll
            for (int q = 0; q < RAD; ++q) v[b * RAD + q] = scr[pad(j + q * NB)];
        }
    }

    // One component (PART 0: real, 1: imaginary) of store<s> / load<s>,
    // through a real scratch of SCR values: an exchange done one component
    // at a time needs half the LDS of one done with complex values.
    template <int s, int PART>
    FSA_HD static void store_part(const C (&v)[V], R* scr, int tid) {
        constexpr int RAD = radix(s), NS = ns(s), NB = nb(s), NBT = nbt(s);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
            const int k = j % NS;
            const int base = (j / NS) * NS * RAD + k;
#pragma unroll
            for (int q = 0; q < RAD; ++q)
                scr[pad(base + q * NS)] = PART ? v[b * RAD + q].y : v[b * RAD + q].x;
        }
    }
    template <int s, int PART>
    FSA_HD static void load_part(C (&v)[V], const R* scr, int tid) {
        constexpr int RAD = radix(s), NB = nb(s), NBT = nbt(s);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                if constexpr (PART) v[b * RAD + q].y = scr[pad(j + q * NB)];
                else v[b * RAD + q].x = scr[pad(j + q * NB)];
            }
        }
    }

    // first-stage operands from an arbitrary source: v = f(index) for
    // index < n_in, zero beyond (zero-padded inputs)
    template <class F>
    FSA_HD static void load_first(C (&v)[V], int tid, int n_in, F&& f) {
        constexpr int RAD = radix(0), NB = nb(0), NBT = nbt(0);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                const int idx = j + q * NB;
                const bool ok = ((NB % T) == 0 || j < NB) && idx < n_in;
                v[b * RAD + q] = ok ? f(idx) : mk(R(0), R(0));
            }
        }
    }

    // as load_first, with the operand's register position: v[pos] = f(index, pos)
    template <class F>
    FSA_HD static void load_first_at(C (&v)[V], int tid, int n_in, F&& f) {
        constexpr int RAD = radix(0), NB = nb(0), NBT = nbt(0);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                const int idx = j + q * NB;
                const bool ok = ((NB % T) == 0 || j < NB) && idx < n_in;
                v[b * RAD + q] = ok ? f(idx, b * RAD + q) : mk(R(0), R(0));
            }
        }
    }

    // last-stage outputs to an arbitrary sink: f(index, value) for index < n_out
    template <class F>
    FSA_HD static void store_last(const C (&v)[V], int tid, int n_out, F&& f) {
        constexpr int RAD = radix(S - 1), NS = ns(S - 1), NB = nb(S - 1), NBT = nbt(S - 1);
        static_assert(NB == NS, "last stage writes y[j + q NS]");
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                const int idx = j + q * NS;
                if (idx < n_out) f(idx, v[b * RAD + q]);
            }
        }
    }

    // apply g(index, value&) to every last-stage output held by this thread
    template <class G>
    FSA_HD static void for_each_last(C (&v)[V], int tid, G&& g) {
        constexpr int RAD = radix(S - 1), NS = ns(S - 1), NB = nb(S - 1), NBT = nbt(S - 1);
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int j = tid + b * T;
            if ((NB % T) != 0 && j >= NB) continue;
#pragma unroll
            for (int q = 0; q < RAD; ++q) g(j + q * NS, v[b * RAD + q]);
        }
    }

#if defined(__HIPCC__)
    static __device__ __forceinline__ void sync() {
        if constexpr (T <= 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }

    // Orders LDS only: waits for this wave's LDS operations, then a wave
    // (T <= 64) or workgroup barrier; global loads in flight keep flying.
    static __device__ __forceinline__ void sync_lds() {
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt/expcnt untouched
        if constexpr (T <= 64) __builtin_amdgcn_wave_barrier();
        else __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }

    // Register bit RB trades places with lane bit 3 + RB (see reg_exchange):
    // lane bit 5 by v_permlane32_swap, lane bit 4 by v_permlane16_swap (each
    // swaps the upper half-wave, or the odd rows of 16 lanes, of its first
    // register with the lower half, or even rows, of its second), lane bit 3
    // by a DPP rotation of each 16-lane row by 8 (lane l reads lane l ^ 8)
    // and two selects.  Per 32-bit word of each value.
    template <int RB>
    static __device__ __forceinline__ void swap_bit(C (&v)[V], int lane) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if ((q >> RB) & 1) continue;
            constexpr int D = 1 << RB;
            Words a = __builtin_bit_cast(Words, v[q]), b = __builtin_bit_cast(Words, v[q + D]);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if constexpr (RB == 2) {
                    const auto r = __builtin_amdgcn_permlane32_swap(a.w[w], b.w[w], false, false);
                    a.w[w] = r[0];
                    b.w[w] = r[1];
                } else if constexpr (RB == 1) {
                    const auto r = __builtin_amdgcn_permlane16_swap(a.w[w], b.w[w], false, false);
                    a.w[w] = r[0];
                    b.w[w] = r[1];
                } else {
                    const unsigned ta =
                        (unsigned)__builtin_amdgcn_update_dpp(0, (int)a.w[w], 0x128, 0xf, 0xf, false);
                    const unsigned tb =
                        (unsigned)__builtin_amdgcn_update_dpp(0, (int)b.w[w], 0x128, 0xf, 0xf, false);
                    const bool hi = (lane >> 3) & 1;
                    const unsigned na = hi ? tb : a.w[w], nb = hi ? b.w[w] : ta;
                    a.w[w] = na;
                    b.w[w] = nb;
                }
            }
            v[q] = __builtin_bit_cast(C, a);
            v[q + D] = __builtin_bit_cast(C, b);
        }
    }

    // the exchange before stage s: in registers where reg_exchange(s), else
    // through the scratch with LDS-only synchronisation
    template <int s>
    static __device__ __forceinline__ void exchange(C (&v)[V], C* scr, int tid) {
        if constexpr (reg_exchange(s)) {
            swap_bit<0>(v, tid);
            swap_bit<1>(v, tid);
            swap_bit<2>(v, tid);
        } else {
            store<s - 1>(v, scr, tid);
            sync_lds();
            load<s>(v, scr, tid);
            sync_lds();
        }
    }

    template <int s>
    static __device__ __forceinline__ void run_r_from(C (&v)[V], C* scr, int tid,
                                                      const C (&w)[NTW]) {
        if constexpr (s < S) {
            exchange<s>(v, scr, tid);
            compute_r<s>(v, tid, w);
            run_r_from<s + 1>(v, scr, tid, w);
        }
    }

    template <int s>
    static __device__ __forceinline__ void run_g_from(C (&v)[V], C* scr, int tid,
                                                      const C* __restrict__ tw) {
        if constexpr (s < S) {
            exchange<s>(v, scr, tid);
            compute<s>(v, tid, tw);
            run_g_from<s + 1>(v, scr, tid, tw);
        }
    }

    // The exchange before stage s through a real scratch, the real parts
    // first and then the imaginary parts (load_part<s, 0> leaves the
    // imaginary parts of the previous stage in place for store_part<s-1, 1>).
    template <int s>
    static __device__ __forceinline__ void exchange_split(C (&v)[V], R* scr, int tid) {
        store_part<s - 1, 0>(v, scr, tid);
        sync_lds();
        load_part<s, 0>(v, scr, tid);
        sync_lds();
        store_part<s - 1, 1>(v, scr, tid);
        sync_lds();
        load_part<s, 1>(v, scr, tid);
        sync_lds();
    }

    template <int s>
    static __device__ __forceinline__ void run_g_split_from(C (&v)[V], R* scr, int tid,
                                                            const C* __restrict__ tw) {
        if constexpr (s < S) {
            exchange_split<s>(v, scr, tid);
            compute<s>(v, tid, tw);
            run_g_split_from<s + 1>(v, scr, tid, tw);
        }
    }

    // run_g with every exchange through a real scratch of SCR values
    static __device__ __forceinline__ void run_g_split(C (&v)[V], R* scr, int tid,
                                                       const C* __restrict__ tw) {
        compute<0>(v, tid, tw);
        run_g_split_from<1>(v, scr, tid, tw);
    }

    // twiddles from the (cached) global table, LDS-only synchronisation
    // (ZH: the upper half of every first-stage operand set is zero)
    template <bool ZH = false>
    static __device__ __forceinline__ void run_g(C (&v)[V], C* scr, int tid,
                                                 const C* __restrict__ tw) {
        compute<0, ZH>(v, tid, tw);
        run_g_from<1>(v, scr, tid, tw);
    }

    // Whether this thread's twiddles fit a register budget of ~56 VGPRs; the
    // kernels keep them in registers then, and read the table otherwise.
    static constexpr bool reg_tw(int budget_vgprs) {
        return NTW * (int)(sizeof(C) / 4) <= budget_vgprs;
    }
    static constexpr bool REG_TW = reg_tw(56);

    // run() with register twiddles and LDS-only synchronisation
    template <bool ZH = false>
    static __device__ __forceinline__ void run_r(C (&v)[V], C* scr, int tid, const C (&w)[NTW]) {
        compute_r<0, ZH>(v, tid, w);
        run_r_from<1>(v, scr, tid, w);
    }

    template <int s>
    static __device__ __forceinline__ void run_from(C (&v)[V], C* scr, int tid,
                                                    const C* __restrict__ tw) {
        if constexpr (s < S) {
            if constexpr (reg_exchange(s)) {
                swap_bit<0>(v, tid);
                swap_bit<1>(v, tid);
                swap_bit<2>(v, tid);
            } else {
                store<s - 1>(v, scr, tid);
                sync();
                load<s>(v, scr, tid);
                sync();
            }
            compute<s>(v, tid, tw);
            run_from<s + 1>(v, scr, tid, tw);
        }
    }

    // v: first-stage operands on entry, last-stage outputs on exit.  Every
    // thread of the team must call it (it synchronises the team); on return
    // the scratch may still be read by other threads until the next sync.
    static __device__ __forceinline__ void run(C (&v)[V], C* scr, int tid,
                                               const C* __restrict__ tw) {
        compute<0>(v, tid, tw);
        run_from<1>(v, scr, tid, tw);
    }
#endif
};

}  // namespace fsa
