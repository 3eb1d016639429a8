// CPU emulation of the team Stockham transforms of fsa_fft.hpp.
//
// Runs every thread of one team phase by phase (a barrier between phases is
// implied by finishing a phase for all threads before the next), for every
// supported length, forward and inverse, and compares with a long-double DFT
// written from its definition.  Also checks the forward -> inverse register
// hand-off that the fused convolution pass relies on, and the plans whose
// exchanges trade register and lane bits across lanes (XCH = 1), with the
// lane swaps emulated on the whole team.  Every length runs three ways:
// twiddles from the table, twiddles from registers, and the exchanges one
// component at a time through a real scratch (exchange_split, used by the
// tensor build).  Exit status 0 = pass.
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

static bool g_split_exchange = false;

// the exchange before stage s: across lanes where the plan does it there;
// with g_split_exchange one component at a time through a real scratch (the
// tensor build's exchange_split), the real parts first
template <typename F, int s>
static void emu_exchange(typename F::C (*v)[F::V], typename F::C* scr) {
    if constexpr (F::reg_exchange(s)) {
        F::reg_exchange_team(v);
    } else if (g_split_exchange) {
        using R = decltype(scr->x);
        R* rs = reinterpret_cast<R*>(scr);
        for (int t = 0; t < F::T; ++t) F::template store_part<s - 1, 0>(v[t], rs, t);
        for (int t = 0; t < F::T; ++t) F::template load_part<s, 0>(v[t], rs, t);
        for (int t = 0; t < F::T; ++t) F::template store_part<s - 1, 1>(v[t], rs, t);
        for (int t = 0; t < F::T; ++t) F::template load_part<s, 1>(v[t], rs, t);
    } else {
        for (int t = 0; t < F::T; ++t) F::template store<s - 1>(v[t], scr, t);
        for (int t = 0; t < F::T; ++t) F::template load<s>(v[t], scr, t);
    }
}

template <typename F, int s>
static void emu_from(typename F::C (*v)[F::V], typename F::C* scr, const typename F::C* tw) {
    if constexpr (s < F::S) {
        emu_exchange<F, s>(v, scr);
        for (int t = 0; t < F::T; ++t) F::template compute<s>(v[t], t, tw);
        emu_from<F, s + 1>(v, scr, tw);
    }
}

// the register-twiddle path: twiddles loaded per thread once, stages take them from registers
template <typename F, int s>
static void emu_r_from(typename F::C (*v)[F::V], typename F::C* scr,
                       const std::vector<std::vector<typename F::C>>& w) {
    if constexpr (s < F::S) {
        emu_exchange<F, s>(v, scr);
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

template <typename R, int P, int ALT, int XCH = 0>
static int check() {
    using Ff = Fft<R, P, false, ALT, XCH>;
    using Fi = Fft<R, P, true, ALT, XCH>;
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

// the plans with exchanges across lanes: exactly the one-wave 8 * 8 * 8 plan
template <typename R>
static int check_lane_exchange() {
    int f = 0;
    static_assert(Fft<R, 512, false, 0, 1>::has_reg_exchange() &&
                      Fft<R, 512, true, 0, 1>::has_reg_exchange(),
                  "length 512 exchanges across lanes");
    static_assert(!Fft<R, 256, false, 0, 1>::has_reg_exchange() &&
                      !Fft<R, 1024, false, 0, 1>::has_reg_exchange() &&
                      !Fft<R, 384, false, 0, 1>::has_reg_exchange(),
                  "no other length does");
    f += check<R, 512, 0, 1>();
    return f;
}

// The first forward stage as the matrix product of the fused pass's variant
// 4 (Fft::mfma0_*): every lane's A and B operands from the helpers, the
// 16x16x4 products with the MFMA's lane layouts (A[l % 16][l / 16] and
// B[l / 16][l % 16] from lane l, D[4 (l / 16) + r][l % 16] in its register
// r), the outputs stored to the scratch slots the helpers name; compared
// with the radix-8 stage 0 (zero upper half) and its store.
static int check_mfma_first_stage() {
    using F = Fft<float, 512, false, 0>;
    static_assert(F::mfma_first_ok(), "512-point one-wave plan");
    static_assert(!Fft<float, 256, false, 0>::mfma_first_ok() &&
                      !Fft<float, 1024, false, 0>::mfma_first_ok() &&
                      !Fft<float, 512, true, 0>::mfma_first_ok(),
                  "only the forward 512-point plan");
    using C = cpx<float>;
    std::vector<C> x(512, mk<float>(0, 0));
    for (int i = 0; i < 256; ++i)
        x[i] = mk<float>((float)std::sin(0.37 * i + 0.1), (float)std::cos(1.1 * i * i + 0.3));
    // reference: stage 0 on the VALU path, then its store
    static C v[F::T][F::V];
    std::vector<C> ref(F::SCR, mk<float>(0, 0)), got(F::SCR, mk<float>(0, 0));
    const auto tw = twiddles<float>(512);
    for (int t = 0; t < F::T; ++t) {
        F::load_first(v[t], t, 256, [&](int i) { return x[i]; });
        F::compute<0, true>(v[t], t, tw.data());
        F::store<0>(v[t], ref.data(), t);
    }
    std::vector<int> hits(F::SCR, 0);
    int bad = 0;
    for (int g = 0; g < 4; ++g) {
        float A[16][8] = {}, B[8][16] = {};
        for (int l = 0; l < 64; ++l)
            for (int ks = 0; ks < 2; ++ks) {
                A[l % 16][4 * ks + l / 16] = F::mfma0_a(l, ks);
                const int i = F::mfma0_b_index(l, g, ks);
                if (i < 0 || i >= 256) ++bad;
                const C c = x[i < 0 || i >= 256 ? 0 : i];
                B[4 * ks + l / 16][l % 16] = F::mfma0_part(l) ? c.y : c.x;
            }
        for (int l = 0; l < 64; ++l) {
            float d[4];
            for (int r = 0; r < 4; ++r) {
                double acc = 0;
                for (int u = 0; u < 8; ++u) acc += (double)A[4 * (l / 16) + r][u] * B[u][l % 16];
                d[r] = (float)acc;
            }
            for (int h = 0; h < 2; ++h) {
                const int slot = F::mfma0_slot(l, g, h);
                if (slot < 0 || slot >= F::SCR) { ++bad; continue; }
                got[slot] = mk<float>(d[2 * h], d[2 * h + 1]);
                ++hits[slot];
            }
        }
    }
    double err = 0, mag = 0;
    int slots = 0;
    for (int i = 0; i < F::SCR; ++i) {
        if (hits[i] > 1) ++bad;
        if (!hits[i]) continue;
        ++slots;
        err = std::fmax(err, std::hypot(got[i].x - ref[i].x, got[i].y - ref[i].y));
        mag = std::fmax(mag, std::hypot(ref[i].x, ref[i].y));
    }
    if (bad || slots != 512 || !(err <= 4e-6 * mag)) {
        std::printf("FAIL mfma first stage: bad %d slots %d err %g mag %g\n", bad, slots, err, mag);
        return 1;
    }
    return 0;
}

int main() {
    int f = 0;
    f += check_mfma_first_stage();
    for (int mode = 0; mode < 3; ++mode) {
    g_register_twiddles = mode == 1;
    g_split_exchange = mode == 2;
    f += check_lane_exchange<float>() + check_lane_exchange<double>();
    f += check_all<double, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536,
                   2048, 3072, 4096>();
    f += check_all<float, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536,
                   2048, 3072, 4096>();
    }
    std::printf("%s (%d failures)\n", f ? "FAILED" : "OK", f);
    return f ? 1 : 0;
}
