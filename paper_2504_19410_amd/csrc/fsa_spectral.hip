// fsa_spectral.hip -- the source terms of the dipole-dipole potentials.
//
// The 3D DDI is evaluated through the Coulomb kernel with the source
// d_nm rho = (n.grad)(m.grad) rho (Sec. 5.3):
//   Phi = -(m.n) rho - 3 Coulomb(d_nm rho).
// d_nm rho is the spectral derivative of rho on its own N-point grid,
// periodic on the box: a 3D DFT, the product with -(k.n)(k.m),
// k_j = pi q_j / L_j (q_j = i_j for i_j < N_j/2, else i_j - N_j), an inverse
// DFT and the real part.  Five launches on a complex N0 x N1 x (N2/2 + 1)
// array Z (the half spectrum, below) in the first workspace array, leaving
// -3 d_nm rho (real, plan precision) in the second one, where pass A of the
// Coulomb convolution reads it:
//   0  rows of rho (last axis, real) -> forward FFT -> Z
//   1  Z along axis 1, forward
//   2  Z along axis 0: forward, x 3 (k.n)(k.m) / (N0 N1 N2), inverse
//   3  Z along axis 1, inverse
//   4  Z rows, inverse, real part -> -3 d_nm rho
// (3 (k.n)(k.m) / prod N folds the -3, the sign of the derivative and the
// normalisation of the inverse DFT into one factor.)  The quasi-2D DDI
// (Sec. 5.3) convolves S = -(3/2)(d_{n_perp n_perp} - n_3^2 Lap) rho, whose
// transform is (3/2)((k.n_perp)^2 - n_3^2 |k|^2) rho^, in three launches:
// rows forward, axis 0 forward x factor x inverse, rows inverse.  Both
// factors are a scale times a quadratic form f(k) = k^T A k.
//
// rho is real, so Z keeps only the bins 0 <= i_last <= N_last/2 of the row
// transforms (a half spectrum: the other half is the conjugate), and the row
// inverse rebuilds each row from it.  Taking the real part of the full
// inverse DFT of f Z equals the inverse of g Z with g(k) = (f(k) + f(k~))/2,
// k~ the frequency of the bin that pairs with k under conjugation (-q_j,
// except that the Nyquist index N_j/2 pairs with itself); g is even under
// that pairing, so the half spectrum times g is consistent, and the axis-0
// launch multiplies by g.  Each team of a
// workgroup transforms one line with the team FFT.  Launches along the
// strided axes stage a tile of WT lines adjacent in memory through LDS, so
// they read and write rows of WT consecutive elements; the row launches read
// and write their contiguous rows directly.  Launches 1-3 work in
// place (each workgroup reads its whole tile before it writes it back).
#include <hip/hip_runtime.h>

#include "fsa_internal.hpp"

namespace fsa {

namespace {

enum SpecKind { ROW_FWD_REAL = 0, COL_FWD = 1, COL_MUL = 2, COL_INV = 3, ROW_INV_REAL = 4 };

// The team scratch and the tile share one LDS array (the tile is idle while
// the teams transform, the lines being in registers), so a group needs
// max(WT * SCR, P * (WT + 1)) complex values.
constexpr int spec_lines_per_group(int T, int scr, int P, int csize) {
    int wt = 128 / csize;
    while (wt > 1 && (wt * T > 1024 || (wt * scr > P * (wt + 1) ? wt * scr : P * (wt + 1)) *
                                               csize > 160 * 1024))
        wt /= 2;
    return wt;
}

template <typename R, int P>
struct Spec {
    using Ff = Fft<R, P, false>;
    using Fi = Fft<R, P, true>;
    static constexpr int T = Ff::T;
    static constexpr int WT = spec_lines_per_group(T, Ff::SCR, P, (int)sizeof(cpx<R>));
    static constexpr int TS = WT + 1;
    static constexpr int THREADS = WT * T;
    static constexpr int LDS = WT * Ff::SCR > P * TS ? WT * Ff::SCR : P * TS;
    static_assert(Ff::last_radix() == Fi::first_radix(), "register hand-off");
};

// Lines of one launch: line (u, v) starts at u * u_stride + v * v_stride
// (elements), its element t at + t * es; groups take WT consecutive u.  The
// row launches write (or read, for the inverse) rows of another length:
// their other array's row (u, v) starts at u * ou_stride + v * ov_stride.
struct SLines {
    int n_u, n_v;
    long u_stride, v_stride, es;
    long ou_stride, ov_stride;
};

// The derivative factor scale * k^T A k of the axis-0 launch, k = (k0, k1,
// k2) with k0 along the launch's lines, k2 from the line index u and k1 from
// v (a 2D plan maps its axis 1 to slot 2 and leaves slot 1 empty: c[1] = 0).
struct SMul {
    double c[3];  // pi / L_j
    double A[3][3];
    double scale;
    int N[3];
};

template <typename R, int P, int KIND>
__global__ __launch_bounds__((Spec<R, P>::THREADS)) void k_spec(const void* in,
                                                             void* out, SLines ln,
                                                             const cpx<R>* __restrict__ tw,
                                                             SMul mul) {
    using K = Spec<R, P>;
    using Ff = typename K::Ff;
    using Fi = typename K::Fi;
    using C = cpx<R>;
    __shared__ C lds[K::LDS];
    C* const tile = lds;  // [t][w], also the teams' scratch while they transform
    const int team = team_index<K::T>(), tid = threadIdx.x % K::T;
    const int ntu = (ln.n_u + K::WT - 1) / K::WT;
    const int tu = blockIdx.x % ntu, v = blockIdx.x / ntu;
    const long base = (long)tu * K::WT * ln.u_stride + (long)v * ln.v_stride;
    const int nw = ln.n_u - tu * K::WT < K::WT ? ln.n_u - tu * K::WT : K::WT;
    if constexpr (KIND == ROW_FWD_REAL || KIND == ROW_INV_REAL) {
        // rows are contiguous: each team reads and writes its own row straight
        // from and to global memory (the team's accesses are consecutive);
        // Z rows hold the half spectrum, H = P/2 + 1 bins
        constexpr int H = P / 2 + 1;
        const bool act = team < nw;
        const long u = (long)tu * K::WT + team;
        const long rb = base + team * ln.u_stride;
        const long ro = u * ln.ou_stride + (long)v * ln.ov_stride;
        C* sc = lds + team * Ff::SCR;
        C x[Ff::V];
        if constexpr (KIND == ROW_FWD_REAL) {
            Ff::load_first(x, tid, P, [&](int t) {
                return act ? mk(((const R*)in)[rb + t], R(0)) : mk(R(0), R(0));
            });
            Ff::run_g(x, sc, tid, tw);
            if (act)
                Ff::store_last(x, tid, P, [&](int t, C c) {
                    if (t < H) ((C*)out)[ro + t] = c;
                });
        } else {
            // Z[P - t] = conj Z[t] rebuilds the bins above P/2
            Fi::load_first(x, tid, P, [&](int t) {
                if (!act) return mk(R(0), R(0));
                return t < H ? ((const C*)in)[rb + t] : conj(((const C*)in)[rb + P - t]);
            });
            Fi::run_g(x, sc, tid, tw);
            if (act) Fi::store_last(x, tid, P, [&](int t, C c) { ((R*)out)[ro + t] = c.x; });
        }
        return;
    }
    // tile element e -> (t, w), the contiguous direction fastest
    auto at = [&](int e, int& t, int& w) {
        if (ln.es == 1) {
            w = e / P;
            t = e - w * P;
        } else {
            t = e / K::WT;
            w = e - t * K::WT;
        }
    };
    for (int e = threadIdx.x; e < P * K::WT; e += K::THREADS) {
        int t, w;
        at(e, t, w);
        C x = mk(R(0), R(0));
        if (w < nw) {
            const long i = base + w * ln.u_stride + t * ln.es;
            x = ((const C*)in)[i];
        }
        tile[t * K::TS + w] = x;
    }
    __syncthreads();
    C x[Ff::V];
    // the inverse runs the radices in reverse: its first stage has its own layout
    if constexpr (KIND == COL_INV)
        Fi::load_first(x, tid, P, [&](int t) { return tile[t * K::TS + team]; });
    else
        Ff::load_first(x, tid, P, [&](int t) { return tile[t * K::TS + team]; });
    __syncthreads();
    C* sc = lds + team * Ff::SCR;
    // every team has finished with its scratch before the tile is rewritten
    if constexpr (KIND == COL_FWD) {
        Ff::run_g(x, sc, tid, tw);
        __syncthreads();
        Ff::store_last(x, tid, P, [&](int t, C c) { tile[t * K::TS + team] = c; });
    } else if constexpr (KIND == COL_MUL) {
        Ff::run_g(x, sc, tid, tw);
        // line (u = i2, v = i1) along axis 0; the register holds output i0.
        // g = (f(k) + f(k~)) / 2 with f = a k0^2 + b k0 + c along the line
        const int i2 = tu * K::WT + team, i1 = v;
        auto qv = [](int i, int n) { return i < n / 2 ? i : i - n; };
        auto qp = [&](int i, int n) { return qv(i == 0 ? 0 : n - i, n); };  // the paired bin
        const double k1 = mul.c[1] * qv(i1, mul.N[1]), k2 = mul.c[2] * qv(i2, mul.N[2]);
        const double p1 = mul.c[1] * qp(i1, mul.N[1]), p2 = mul.c[2] * qp(i2, mul.N[2]);
        const double ha = 0.5 * mul.scale * mul.A[0][0];
        const double hb = mul.scale * (mul.A[0][1] * k1 + mul.A[0][2] * k2);
        const double hbp = mul.scale * (mul.A[0][1] * p1 + mul.A[0][2] * p2);
        const double hc = 0.5 * mul.scale *
                          (mul.A[1][1] * (k1 * k1 + p1 * p1) +
                           2.0 * mul.A[1][2] * (k1 * k2 + p1 * p2) +
                           mul.A[2][2] * (k2 * k2 + p2 * p2));
        Ff::for_each_last(x, tid, [&](int i0, C& c) {
            const double k0 = mul.c[0] * qv(i0, mul.N[0]), p0 = mul.c[0] * qp(i0, mul.N[0]);
            c = scale(c, (R)(ha * (k0 * k0 + p0 * p0) + hb * k0 + hbp * p0 + hc));
        });
        Fi::run_g(x, sc, tid, tw);
        __syncthreads();
        Fi::store_last(x, tid, P, [&](int t, C c) { tile[t * K::TS + team] = c; });
    } else {
        Fi::run_g(x, sc, tid, tw);
        __syncthreads();
        Fi::store_last(x, tid, P, [&](int t, C c) { tile[t * K::TS + team] = c; });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P * K::WT; e += K::THREADS) {
        int t, w;
        at(e, t, w);
        if (w < nw) {
            const long i = base + w * ln.u_stride + t * ln.es;
            ((C*)out)[i] = tile[t * K::TS + w];
        }
    }
}


template <typename R, int KIND>
hipError_t go(int P, const void* in, void* out, SLines ln, const void* tw, const SMul& mul,
              hipStream_t st) {
    switch (P) {
#define FSA_SPEC_CASE(p)                                                                        \
    case p: {                                                                                   \
        using K = Spec<R, p>;                                                                   \
        const int groups = (ln.n_u + K::WT - 1) / K::WT * ln.n_v;                               \
        return launch_kernel(k_spec<R, p, KIND>, dim3(groups), dim3(K::THREADS), 0, st, in, out, \
                             ln, (const cpx<R>*)tw, mul);                                       \
    }
        FSA_SPEC_CASE(8) FSA_SPEC_CASE(12) FSA_SPEC_CASE(16) FSA_SPEC_CASE(24) FSA_SPEC_CASE(32)
        FSA_SPEC_CASE(48) FSA_SPEC_CASE(64) FSA_SPEC_CASE(96) FSA_SPEC_CASE(128)
        FSA_SPEC_CASE(192) FSA_SPEC_CASE(256) FSA_SPEC_CASE(384) FSA_SPEC_CASE(512)
        FSA_SPEC_CASE(768) FSA_SPEC_CASE(1024) FSA_SPEC_CASE(1536) FSA_SPEC_CASE(2048)
#undef FSA_SPEC_CASE
    }
    return hipErrorInvalidValue;
}

constexpr double kPi = 3.14159265358979323846264338327950288;

// quasi-2D DDI: rows, axis 0 with the factor, rows inverse
template <typename R>
hipError_t step_2d(const fsa_plan_s* pl, int s, const void* rho, void* z, void* dst,
                   hipStream_t st) {
    const long N0 = pl->N[0], N1 = pl->N[1];
    const char* tw = (const char*)pl->twiddles;
    const void* tw0 = tw + pl->tw_off_n0 * pl->csize;
    const void* tw1 = tw + pl->tw_off_m * pl->csize;  // length N1
    SMul mul{};
    // 2D axes 0, 1 in slots 0, 2; (3/2)((k.n_perp)^2 - n_3^2 |k|^2) / (N0 N1)
    const double n0 = pl->dn[0], n1 = pl->dn[1], n3sq = pl->dn[2] * pl->dn[2];
    mul.c[0] = kPi / pl->L[0];
    mul.c[2] = kPi / pl->L[1];
    mul.N[0] = (int)N0;
    mul.N[1] = 1;
    mul.N[2] = (int)N1;
    mul.A[0][0] = n0 * n0 - n3sq;
    mul.A[2][2] = n1 * n1 - n3sq;
    mul.A[0][2] = mul.A[2][0] = n0 * n1;
    mul.scale = 1.5 / ((double)N0 * (double)N1);
    const long H1 = N1 / 2 + 1;  // half spectrum of the rows
    const SLines fwd{(int)N0, 1, N1, 0, 1, H1, 0};  // rho rows -> Z rows
    const SLines inv{(int)N0, 1, H1, 0, 1, N1, 0};  // Z rows -> source rows
    const SLines ax0{(int)H1, 1, 1, 0, H1, 0, 0};
    switch (s) {
    case 0: return go<R, ROW_FWD_REAL>((int)N1, rho, z, fwd, tw1, mul, st);
    case 1: return go<R, COL_MUL>((int)N0, z, z, ax0, tw0, mul, st);
    case 2: return go<R, ROW_INV_REAL>((int)N1, z, dst, inv, tw1, mul, st);
    }
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t step_t(const fsa_plan_s* pl, int s, const void* rho, void* z, void* dst,
                  hipStream_t st) {
    if (pl->d == 2) return step_2d<R>(pl, s, rho, z, dst, st);
    const long N0 = pl->N[0], N1 = pl->N[1], N2 = pl->N[2];
    const char* tw = (const char*)pl->twiddles;
    const void* tw0 = tw + pl->tw_off_n0 * pl->csize;
    const void* tw1 = tw + pl->tw_off_n1 * pl->csize;
    const void* tw2 = tw + pl->tw_off_m * pl->csize;  // length N2
    SMul mul{};
    double prodN = 1.0;
    for (int j = 0; j < 3; ++j) {
        mul.c[j] = kPi / pl->L[j];
        mul.N[j] = (int)pl->N[j];
        prodN *= (double)pl->N[j];
    }
    // (k.n)(k.m) = k^T A k with A the symmetric part of n m^T
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            mul.A[a][b] = 0.5 * (pl->dn[a] * pl->dm[b] + pl->dm[a] * pl->dn[b]);
    mul.scale = 3.0 / prodN;
    // Z is N0 x N1 x H2, the half spectrum of the rows
    const long H2 = N2 / 2 + 1;
    // rows: lines along axis 2, groups of consecutive rows
    const SLines fwd{(int)N1, (int)N0, N2, N1 * N2, 1, H2, N1 * H2};  // rho -> Z
    const SLines inv{(int)N1, (int)N0, H2, N1 * H2, 1, N2, N1 * N2};  // Z -> source
    // axis 1: lines at fixed (i0, i2), groups of consecutive i2
    const SLines ax1{(int)H2, (int)N0, 1, N1 * H2, H2, 0, 0};
    // axis 0: lines at fixed (i1, i2), groups of consecutive i2
    const SLines ax0{(int)H2, (int)N1, 1, H2, N1 * H2, 0, 0};
    switch (s) {
    case 0: return go<R, ROW_FWD_REAL>((int)N2, rho, z, fwd, tw2, mul, st);
    case 1: return go<R, COL_FWD>((int)N1, z, z, ax1, tw1, mul, st);
    case 2: return go<R, COL_MUL>((int)N0, z, z, ax0, tw0, mul, st);
    case 3: return go<R, COL_INV>((int)N1, z, z, ax1, tw1, mul, st);
    case 4: return go<R, ROW_INV_REAL>((int)N2, z, dst, inv, tw2, mul, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t spectral_step(const fsa_plan_s* pl, int s, const void* rho, void* z, void* dst,
                         hipStream_t st) {
    return pl->prec == FSA_F32 ? step_t<float>(pl, s, rho, z, dst, st)
                               : step_t<double>(pl, s, rho, z, dst, st);
}

}  // namespace fsa
