// CPU emulation of the team Stockham transforms of fsa_fft.hpp.
//
// Runs every thread of one team phase by phase (a barrier between phases is
// implied by finishing a phase for all threads before the next), for every
// supported length, forward and inverse, and compares with a long-double DFT
// written from its definition.  Also checks the forward -> inverse register
// hand-off that the fused convolution pass relies on.  Exit status 0 = pass.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2504_19410_amd/csrc/fsa_fft.hpp"

using namespace fsa;

template <typename R>
static std::vector<cpx<R>> twiddles(int P) {
    std::vector<cpx<R>> t(P);
    for (int m = 0; m < P; ++m) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * m / P;
        t[m] = mk<R>((R)std::cos(a), (R)-std::sin(a));
    }
    return t;
}

// roots e^{+2 pi i m / P} in long double, m in [0, P)
struct Roots {
    std::vector<long double> c, s;
    explicit Roots(int P) : c(P), s(P) {
        for (int m = 0; m < P; ++m) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * m / P;
            c[m] = std::cos(a);
            s[m] = std::sin(a);
        }
    }
};

template <typename F, int s>
static void emu_from(typename F::C (*v)[F::V], typename F::C* scr, const typename F::C* tw) {
    if constexpr (s < F::S) {
        for (int t = 0; t < F::T; ++t) F::template store<s - 1>(v[t], scr, t);
        for (int t = 0; t < F::T; ++t) F::template load<s>(v[t], scr, t);
        for (int t = 0; t < F::T; ++t) F::template compute<s>(v[t], t, tw);
        emu_from<F, s + 1>(v, scr, tw);
    }
}

// the register-twiddle path: twiddles loaded per thread once, stages take them from registers
template <typename F, int s>
static void emu_r_from(typename F::C (*v)[F::V], typename F::C* scr,
                       const std::vector<std::vector<typename F::C>>& w) {
    if constexpr (s < F::S) {
        for (int t = 0; t < F::T; ++t) F::template store<s - 1>(v[t], scr, t);
        for (int t = 0; t < F::T; ++t) F::template load<s>(v[t], scr, t);
        for (int t = 0; t < F::T; ++t)
            F::template compute_r<s>(v[t], t,
                                     *reinterpret_cast<const typename F::C(*)[F::NTW]>(w[t].data()));
        emu_r_from<F, s + 1>(v, scr, w);
    }
}

static bool g_register_twiddles = false;

template <typename F>
static void emu_run(typename F::C (*v)[F::V], const typename F::C* tw) {
    std::vector<typename F::C> scr(F::SCR);
    if (!g_register_twiddles) {
        for (int t = 0; t < F::T; ++t) F::template compute<0>(v[t], t, tw);
        emu_from<F, 1>(v, scr.data(), tw);
        return;
    }
    std::vector<std::vector<typename F::C>> w(F::T, std::vector<typename F::C>(F::NTW));
    for (int t = 0; t < F::T; ++t)
        F::load_tw(*reinterpret_cast<typename F::C(*)[F::NTW]>(w[t].data()), t, tw);
    for (int t = 0; t < F::T; ++t)
        F::template compute_r<0>(v[t], t, *reinterpret_cast<const typename F::C(*)[F::NTW]>(w[t].data()));
    emu_r_from<F, 1>(v, scr.data(), w);
}

template <typename R, int P, int ALT>
static int check() {
    using Ff = Fft<R, P, false, ALT>;
    using Fi = Fft<R, P, true, ALT>;
    static_assert(Ff::T == Fi::T && Ff::V == Fi::V, "same team shape");
    static_assert(Ff::last_radix() == Fi::first_radix(), "register hand-off");
    using C = cpx<R>;
    const auto tw = twiddles<R>(P);
    const Roots rt(P);
    std::vector<C> x(P);
    for (int i = 0; i < P; ++i)
        x[i] = mk<R>((R)std::sin(1.3 * i + 0.2), (R)std::cos(0.7 * i * i + 0.1));
    int fails = 0;
    for (int pass = 0; pass < 3; ++pass) {
        // pass 0: full forward; 1: forward with the upper half zero; 2: inverse
        const bool inv = pass == 2;
        const int n_in = pass == 1 ? P / 2 : P;
        static C v[Ff::T][Ff::V];
        std::vector<C> y(P);
        if (!inv) {
            for (int t = 0; t < Ff::T; ++t)
                Ff::load_first(v[t], t, n_in, [&](int i) { return x[i]; });
            emu_run<Ff>(v, tw.data());
            for (int t = 0; t < Ff::T; ++t)
                Ff::store_last(v[t], t, P, [&](int i, C c) { y[i] = c; });
        } else {
            for (int t = 0; t < Fi::T; ++t)
                Fi::load_first(v[t], t, n_in, [&](int i) { return x[i]; });
            emu_run<Fi>(v, tw.data());
            for (int t = 0; t < Fi::T; ++t)
                Fi::store_last(v[t], t, P, [&](int i, C c) { y[i] = c; });
        }
        long double err = 0, mag = 0;
        for (int k = 0; k < P; ++k) {
            long double re = 0, im = 0;
            for (int n = 0; n < n_in; ++n) {
                const long m = (long)n * k % P;
                const long double ca = rt.c[m], sa = inv ? rt.s[m] : -rt.s[m];
                re += x[n].x * ca - x[n].y * sa;
                im += x[n].x * sa + x[n].y * ca;
            }
            err = std::fmax(err, std::hypot(re - y[k].x, im - y[k].y));
            mag = std::fmax(mag, std::hypot(re, im));
        }
        const long double tol = (sizeof(R) == 4 ? 2e-6L : 1e-14L) * mag;
        if (!(err <= tol)) {
            std::printf("FAIL P=%d alt=%d %s pass=%d err=%Lg mag=%Lg\n", P, ALT,
                        sizeof(R) == 4 ? "f32" : "f64", pass, err, mag);
            ++fails;
        }
    }
    // the pass kernels prefetch the non-zero half of a padded line straight
    // from global memory at first_index: every index must lie in [0, P/2)
    // (an index beyond it reads past the line, and past the buffer on its last
    // line) and each must be read exactly once
    {
        std::vector<int> hits(P / 2, 0);
        int bad = 0;
        for (int t = 0; t < Ff::T; ++t)
            for (int b = 0; b < Ff::first_nbt(); ++b)
                for (int q = 0; q < Ff::first_radix() / 2; ++q) {
                    const int i = Ff::first_index(t, b, q);
                    if (i < 0) continue;
                    if (i >= P / 2) ++bad;
                    else ++hits[i];
                }
        for (int h : hits) bad += h != 1;
        if (bad) {
            std::printf("FAIL P=%d alt=%d %s prefetch indices (%d bad)\n", P, ALT,
                        sizeof(R) == 4 ? "f32" : "f64", bad);
            ++fails;
        }
    }
    // forward (half-zero input) -> in-register product -> inverse, keep P/2 outputs
    {
        static C v[Ff::T][Ff::V];
        for (int t = 0; t < Ff::T; ++t) Ff::load_first(v[t], t, P / 2, [&](int i) { return x[i]; });
        emu_run<Ff>(v, tw.data());
        for (int t = 0; t < Ff::T; ++t)
            Ff::for_each_last(v[t], t, [&](int k, C& c) { c = scale(c, (R)(1.0 + 0.25 * std::cos(0.3 * k))); });
        emu_run<Fi>(v, tw.data());
        std::vector<C> y(P, mk<R>(0, 0));
        for (int t = 0; t < Fi::T; ++t)
            Fi::store_last(v[t], t, P / 2, [&](int i, C c) { y[i] = c; });
        // reference: circular convolution theorem done with long-double DFTs
        std::vector<long double> Xr(P), Xi(P);
        for (int k = 0; k < P; ++k) {
            long double re = 0, im = 0;
            for (int n = 0; n < P / 2; ++n) {
                const long m = (long)n * k % P;
                const long double ca = rt.c[m], sa = -rt.s[m];
                re += x[n].x * ca - x[n].y * sa;
                im += x[n].x * sa + x[n].y * ca;
            }
            const long double g = 1.0L + 0.25L * std::cos(0.3L * k);
            Xr[k] = re * g;
            Xi[k] = im * g;
        }
        long double err = 0, mag = 0;
        for (int n = 0; n < P / 2; ++n) {
            long double re = 0, im = 0;
            for (int k = 0; k < P; ++k) {
                const long m = (long)n * k % P;
                re += Xr[k] * rt.c[m] - Xi[k] * rt.s[m];
                im += Xr[k] * rt.s[m] + Xi[k] * rt.c[m];
            }
            err = std::fmax(err, std::hypot(re - y[n].x, im - y[n].y));
            mag = std::fmax(mag, std::hypot(re, im));
        }
        const long double tol = (sizeof(R) == 4 ? 4e-6L : 2e-14L) * mag;
        if (!(err <= tol)) {
            std::printf("FAIL P=%d alt=%d %s fused err=%Lg mag=%Lg\n", P, ALT,
                        sizeof(R) == 4 ? "f32" : "f64", err, mag);
            ++fails;
        }
    }
    return fails;
}

// every length with the default radix family, and with the alternate family
// where that gives a different transform
template <typename R, int P>
static int check_both() {
    int f = check<R, P, 0>();
    if constexpr (fft_alt_distinct(P)) f += check<R, P, 1>();
    return f;
}

template <typename R, int... Ps>
static int check_all() {
    return (check_both<R, Ps>() + ...);
}

int main() {
    int f = 0;
    for (int mode = 0; mode < 2; ++mode) {
    g_register_twiddles = mode == 1;
    f += check_all<double, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536,
                   2048, 3072, 4096>();
    f += check_all<float, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536,
                   2048, 3072, 4096>();
    }
    std::printf("%s (%d failures)\n", f ? "FAILED" : "OK", f);
    return f ? 1 : 0;
}
