// fsa_passes.hpp -- the per-evaluation FFT-convolution passes (gfx950).
//
// One evaluation computes phi = crop(IDFT(T^ . DFT(pad(rho)))) on the 2N
// zero-padded grid (eq. DiscConv evaluated with FFTs, Sec. 2.2-2.3).  The
// transform of each axis is split so that every pass reads and writes HBM
// exactly once, with the zero-pad, the tensor product and the crop fused in:
//
//   3D (grid axes 0,1,2; axis 2 contiguous; H = N2 + 1; P_j = 2 N_j)
//     A  r2c      rho[i0][i1][i2] (real)   -> X1[i0][p2][i1]     pad+R2C on axis 2
//     B  fwd_t    X1[i0][p2][i1]           -> X2[p2][p1][i0]     pad+C2C on axis 1
//     C  conv     X2[p2][p1][i0]  in place: pad+C2C, x T^, C2C^-1, crop on axis 0
//     D  inv_t    X2[p2][p1][i0]           -> X1[i0][p2][i1]     C2C^-1+crop on axis 1
//     E  c2r      X1[i0][p2][i1]           -> phi[i0][i1][i2]    C2R+crop on axis 2
//   2D (axis 1 contiguous; H = N1 + 1)
//     A  r2c      rho[i0][i1] -> X[p1][i0];  C conv on X[p1][i0];  E c2r -> phi
//
// Every axis transform reads its pencils from contiguous memory or from
// 128-byte row segments of WT consecutive pencils, and writes the other way
// round through an LDS tile, so all HBM traffic is coalesced and the pencils
// of the fused pass C are contiguous.  The 1/prod P_j scale is folded into T^.
//
// Real transforms use the half-length complex transform of
// z[m] = x[2m] + i x[2m+1] (the standard two-for-one packing):
//   X[k] = (Z[k] + conj Z[M-k])/2 - i w^k (Z[k] - conj Z[M-k])/2,  w = e^{-pi i/M}
// and its inverse Z[k] = (X[k] + conj X[M-k]) + i w^{-k} (X[k] - conj X[M-k]),
// which returns 2M x[n] like every other unnormalised inverse here.
#pragma once

#include "fsa_fft.hpp"
#include "fsa_jobs.hpp"
#include "fsa_walk.hpp"

namespace fsa {

constexpr int kMaxLds = 160 * 1024;

// Width (pencils) of a transposing tile: 128 bytes of complex values, fewer
// if the LDS or the thread budget says so.  The thread budget keeps the
// per-thread register file large enough for the operands, the register
// twiddles and the prefetch buffers: a 1024-thread workgroup leaves 128
// VGPRs per thread, a 512-thread one 256.
constexpr int tile_width(int csize, int T, int scr, int rows, int max_threads = 1024) {
    int wt = 128 / csize;
    while (wt > 1 && (wt * T > max_threads ||
                      (wt * scr > rows * (wt + 1) ? wt * scr : rows * (wt + 1)) * csize > kMaxLds))
        wt /= 2;
    return wt;
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Compile-time variants of every pass; the autotuner picks one per (pass,
// transform length, precision) at run time.  0: default.  1: the alternate
// radix family of make_fft_plan (another radix split and number of threads
// per transform).  2: half-size workgroups (half the lines per tile, or half
// the teams per workgroup): less LDS and fewer threads per group, more
// resident groups per CU.  3: the default plan with the stage exchanges
// that only trade register and lane bits done across lanes instead of
// through the LDS (Fft::reg_exchange; the fused pass at length 512).  4:
// the default plan with the first forward stage of the fused pass as a
// matrix product on the matrix cores (FP32, length 512; Conv::MFMA0).  A
// variant that comes out identical to variant 0 at some length is marked
// not DISTINCT and never instantiated there.
constexpr int kVariants = 5;
constexpr int var_alt(int var) { return var == 1 ? 1 : 0; }
constexpr int var_cap(int var, int cap) { return var == 2 ? cap / 2 : cap; }
constexpr int var_xch(int var) { return var == 3 ? 1 : 0; }

// Workgroup barrier that orders LDS only: global loads in flight (prefetch)
// and global stores keep flying.
__device__ __forceinline__ void sync_wg_lds() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The lane index, made opaque to the optimiser.  The transforms' LDS and
// twiddle addresses depend only on it, so the compiler hoists all of them out
// of a kernel's work loop and keeps them live for the whole loop.  Where their
// strides do not fold into immediate offsets (lengths 3 * 2^a) and there are
// many of them (FP64 operands, or FP32 from length 768), that overflows the
// register file (one wave per SIMD, AGPR spills); there each work item takes
// a fresh copy of the lane index and recomputes its addresses, at a few VALU
// instructions per item.  Measured per evaluation: 192^3 FP64 654 -> 526 us,
// 384^3 FP64 6.1 -> 4.2 ms, 384^3 FP32 3.46 -> 2.77 ms.  Elsewhere the
// addresses fit and the recomputation only costs (power-of-two lengths, and
// FP32 below 768: 192^3 FP32 263 -> 289 us, 256^3 FP32 +6%).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
template <typename R, int P>
constexpr bool fresh_lane() {
    return (P & (P - 1)) != 0 && (sizeof(R) == 8 || P >= 768);
}

// Whether a transposing tile of WT lines of complex values of `csize` bytes
// reads and writes rows narrower than a cache line.  Pass A takes the XCD walk
// then (2D batch, rows of 1024: 300 -> 280 us, HBM fetches 1.075 -> 1.013 x
// the algorithmic bytes).  Pass E of the same rows ran slower under the XCD
// walk (292 -> 354 us, every workgroup of an XCD reading the same lines at
// once) and takes the pair walk instead: fetches 2.3 -> 1.09 x the
// algorithmic bytes at the same time (the Infinity Cache had served the
// re-reads).  The other transposing passes keep their chunks.
constexpr bool narrow_rows(int wt, int csize) { return wt * csize < 128; }

// This workgroup's walk over `items` items of the launch.
template <int MODE>
__device__ __forceinline__ Walk walk_of(int items) {
    return Walk::make<MODE>(items, (int)gridDim.x, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Work sources.  A pass kernel walks global work items; a source maps an
// item to its job (one problem's arrays and extents) and the item's index
// within that job.  JobOne serves a single evaluation (the job travels in
// the kernel arguments); JobList serves a batch of problems that share the
// transform length (device table of jobs plus the prefix of their item
// counts), so one persistent launch covers the pass for every problem.
// ---------------------------------------------------------------------------
// A caller walks its items in increasing order and keeps a cursor per walk
// (the job of its previous item, -1 before the first): the lookup then
// advances from the cursor over the job starts it passes, instead of a
// binary search of dependent loads for every item.
template <class Job>
struct JobOne {
    Job job;
    int total;
    __device__ __forceinline__ Job get(int item, int& local, int& /*cursor*/) const {
        local = item;
        return job;
    }
};

template <class Job>
struct JobList {
    const Job* jobs;
    const int* start;  // start[i] = first item of job i; start[n] = total
    int n, total;
    __device__ __forceinline__ Job get(int item, int& local, int& cursor) const {
        int lo;
        if (cursor >= 0 && start[cursor] <= item) {
            lo = cursor;
            while (lo + 1 < n && start[lo + 1] <= item) ++lo;
        } else {
            lo = 0;
            int hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (start[mid] <= item) lo = mid;
                else hi = mid - 1;
            }
        }
        cursor = lo;
        local = item - start[lo];
        return jobs[lo];
    }
};

// ---------------------------------------------------------------------------
// Pass A: zero-pad + real-to-complex along the contiguous axis, transposed out
//   rho rows r = outer * n_inner + inner of M reals (M = N_last), padded to
//   2M; out[(outer * (M+1) + k) * n_inner + inner] = X[k], k in [0, M].
// Work item = (outer, tile of WT rows); team w of the workgroup owns row
// tile * WT + w.  Persistent, with the next item's rows prefetched.
// ---------------------------------------------------------------------------
template <typename R, int M, int VAR = 0>
struct R2c {
    using F = Fft<R, M, false, var_alt(VAR)>;
    using C = cpx<R>;
    static constexpr int T = F::T;
    static constexpr int H = M + 1;
    static constexpr int WT = tile_width(sizeof(C), T, F::SCR, H, var_cap(VAR, 512));
    static constexpr int TS = WT + 1;
    static constexpr int LDS = cmax(WT * F::SCR, H * TS);
    static constexpr int THREADS = WT * T;
    static constexpr int NX = (H + T - 1) / T;
    static constexpr int R0 = F::first_radix(), NB0 = F::first_stride(), NBT0 = F::first_nbt();
    static constexpr int HALF = R0 / 2;
    static_assert(R0 % 2 == 0, "zero half = whole first-stage operands");
    static constexpr bool DISTINCT =
        VAR == 0 || (VAR == 1 ? fft_alt_distinct(M) : WT != R2c<R, M, 0>::WT);
};

template <typename R, int M, int VAR, class Src>
__global__ __launch_bounds__((R2c<R, M, VAR>::THREADS)) void k_r2c(
    Src src, const cpx<R>* __restrict__ twM, const cpx<R>* __restrict__ tw2M) {
    using K = R2c<R, M, VAR>;
    using F = typename K::F;
    using C = cpx<R>;
    __shared__ C lds[K::LDS];
    const int team = team_index<K::T>(), tid0 = threadIdx.x % K::T;
    const int tid = tid0;
    C* scr = lds + team * F::SCR;
    C w[F::REG_TW ? F::NTW : 1];
    if constexpr (F::REG_TW) F::load_tw(w, tid, twM);
    C w2[F::REG_TW ? K::NX : 1];  // post-processing twiddles e^{-i pi k / M}, k = tid + i T
    if constexpr (F::REG_TW) {
#pragma unroll
        for (int i = 0; i < K::NX; ++i) {
            const int k = tid + i * K::T;
            w2[i] = tw2M[k < K::H ? k : 0];
        }
    }
    const Walk ch =
        walk_of<narrow_rows(K::WT, (int)sizeof(C)) ? kWalkXcd : kWalkChunk>(src.total);
    C pf[K::NBT0 * K::HALF];
    int cur_pf = -1, cur_it = -1;  // job cursors of the prefetch and the item walks
    auto prefetch = [&](int item) {
        int loc;
        const JobR2c jb = src.get(item, loc, cur_pf);
        const int ntile = cdiv(jb.n_inner, K::WT);
        const int outer = loc / ntile, inner = (loc - outer * ntile) * K::WT + team;
        if (inner < jb.n_inner) {
            const R* row = (const R*)jb.rho + ((size_t)outer * jb.n_inner + inner) * M;
#pragma unroll
            for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
                for (int q = 0; q < K::HALF; ++q) {
                    const int i = F::first_index(tid, b, q);
                    if (i >= 0) pf[b * K::HALF + q] = *reinterpret_cast<const C*>(row + 2 * i);
                    else pf[b * K::HALF + q] = mk(R(0), R(0));
                }
        }
    };
    if (ch.first < ch.last) prefetch(ch.first);
    for (int item = ch.first; item < ch.last; item += ch.stride) {
        const int tid = fresh_lane<R, M>() ? opaque(tid0) : tid0;  // per item: fresh_lane
        int loc;
        const JobR2c jb = src.get(item, loc, cur_it);
        const int n_inner = jb.n_inner;
        const int ntile = cdiv(n_inner, K::WT);
        const int outer = loc / ntile, col0 = (loc - outer * ntile) * K::WT;
        const bool active = col0 + team < n_inner;
        C v[F::V];
#pragma unroll
        for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
            for (int q = 0; q < K::R0; ++q)
                v[b * K::R0 + q] = (q < K::HALF && active) ? pf[b * K::HALF + q] : mk(R(0), R(0));
        if (item + ch.stride < ch.last) prefetch(item + ch.stride);
        if constexpr (F::REG_TW) F::template run_r<true>(v, scr, tid, w);
        else F::template run_g<true>(v, scr, tid, twM);
        F::store_last(v, tid, M, [&](int k, C z) { scr[F::pad(k)] = z; });
        F::sync_lds();
        C x[K::NX];
#pragma unroll
        for (int i = 0; i < K::NX; ++i) {
            const int k = tid + i * K::T;
            if (k < K::H) {
                const C zk = scr[F::pad(k == M ? 0 : k)];
                const C zm = scr[F::pad(k == 0 ? 0 : M - k)];
                const C a = zk + conj(zm);
                const C b = rot90<false>(zk - conj(zm));
                C t;
                if constexpr (F::REG_TW) t = w2[i];
                else t = tw2M[k];
                x[i] = scale(a + cmul(t, b), R(0.5));
            }
        }
        sync_wg_lds();
#pragma unroll
        for (int i = 0; i < K::NX; ++i) {
            const int k = tid + i * K::T;
            if (k < K::H) lds[k * K::TS + team] = x[i];
        }
        sync_wg_lds();
        C* out = (C*)jb.out;
        for (int e = threadIdx.x; e < K::H * K::WT; e += K::THREADS) {
            const int k = e / K::WT, ww = e - k * K::WT;
            if (col0 + ww < n_inner)
                out[((size_t)outer * K::H + k) * n_inner + col0 + ww] = lds[k * K::TS + ww];
        }
        sync_wg_lds();
    }
}

// ---------------------------------------------------------------------------
// Pass E: complex-to-real along the contiguous axis with crop, transposed in
//   in[(outer * (M+1) + k) * n_inner + inner] -> phi row r, first M reals of 2M
// (plus alpha times the same row of `add` when the job carries one).
// Persistent; the next item's tile is prefetched into registers.
// ---------------------------------------------------------------------------
template <typename R, int M, int VAR = 0>
struct C2r {
    using F = Fft<R, M, true, var_alt(VAR)>;
    using C = cpx<R>;
    static constexpr int T = F::T;
    static constexpr int H = M + 1;
    static constexpr int WT = tile_width(sizeof(C), T, F::SCR, H, var_cap(VAR, 512));
    static constexpr int TS = WT + 1;
    static constexpr int LDS = cmax(WT * F::SCR, H * TS);
    static constexpr int THREADS = WT * T;
    static constexpr int NT = (H * WT + THREADS - 1) / THREADS;  // tile elements per thread
    // prefetch the next tile into registers only if it fits ~48 VGPRs, and
    // not beside the 16 operands per thread of an FP32 plan at M = 2048 (the
    // prefetch pushed that kernel past 256 VGPRs into scratch)
    static constexpr bool PREFETCH =
        NT * (int)(sizeof(C) / 4) <= 48 && !(sizeof(R) == 4 && F::V >= 16 && M >= 2048);
    static constexpr int R0 = F::first_radix(), NB0 = F::first_stride(), NBT0 = F::first_nbt();
    static constexpr bool DISTINCT =
        VAR == 0 || (VAR == 1 ? fft_alt_distinct(M) : WT != C2r<R, M, 0>::WT);
};

template <typename R, int M, int VAR, class Src>
__global__ __launch_bounds__((C2r<R, M, VAR>::THREADS)) void k_c2r(
    Src src, const cpx<R>* __restrict__ twM, const cpx<R>* __restrict__ tw2M) {
    using K = C2r<R, M, VAR>;
    using F = typename K::F;
    using C = cpx<R>;
    __shared__ C lds[K::LDS];
    const int team = team_index<K::T>(), tid0 = threadIdx.x % K::T;
    const int tid = tid0;
    C* scr = lds + team * F::SCR;
    C w[F::REG_TW ? F::NTW : 1];
    if constexpr (F::REG_TW) F::load_tw(w, tid, twM);
    C w2[F::REG_TW ? F::V : 1];  // e^{-i pi k / M} at this thread's first-stage indices k
    if constexpr (F::REG_TW) F::load_first(w2, tid, M, [&](int k) { return tw2M[k]; });
    const Walk ch =
        walk_of<narrow_rows(K::WT, (int)sizeof(C)) ? kWalkPair : kWalkChunk>(src.total);
    C tp[K::PREFETCH ? K::NT : 1];
    auto tile_elem = [&](const JobC2r& jb, int outer, int col0, int e) {
        const int k = e / K::WT, ww = e - k * K::WT;
        return (e < K::H * K::WT && col0 + ww < jb.n_inner)
                   ? ((const C*)jb.in)[((size_t)outer * K::H + k) * jb.n_inner + col0 + ww]
                   : mk(R(0), R(0));
    };
    int cur_pf = -1, cur_it = -1;  // job cursors of the prefetch and the item walks
    auto prefetch = [&](int item) {
        int loc;
        const JobC2r jb = src.get(item, loc, cur_pf);
        const int ntile = cdiv(jb.n_inner, K::WT);
        const int outer = loc / ntile, col0 = (loc - outer * ntile) * K::WT;
#pragma unroll
        for (int i = 0; i < K::NT; ++i) tp[i] = tile_elem(jb, outer, col0, threadIdx.x + i * K::THREADS);
    };
    if constexpr (K::PREFETCH) {
        if (ch.first < ch.last) prefetch(ch.first);
    }
    for (int item = ch.first; item < ch.last; item += ch.stride) {
        const int tid = fresh_lane<R, M>() ? opaque(tid0) : tid0;  // per item: fresh_lane
        int loc;
        const JobC2r jb = src.get(item, loc, cur_it);
        const int n_inner = jb.n_inner;
        const int ntile = cdiv(n_inner, K::WT);
        const int outer = loc / ntile, col0 = (loc - outer * ntile) * K::WT;
        if constexpr (K::PREFETCH) {
#pragma unroll
            for (int i = 0; i < K::NT; ++i) {
                const int e = threadIdx.x + i * K::THREADS;
                const int k = e / K::WT, ww = e - k * K::WT;
                if (e < K::H * K::WT) lds[k * K::TS + ww] = tp[i];
            }
        } else {
            for (int e = threadIdx.x; e < K::H * K::WT; e += K::THREADS) {
                const int k = e / K::WT, ww = e - k * K::WT;
                lds[k * K::TS + ww] = tile_elem(jb, outer, col0, e);
            }
        }
        sync_wg_lds();
        if constexpr (K::PREFETCH) {
            if (item + ch.stride < ch.last) prefetch(item + ch.stride);
        }
        C v[F::V];
        F::load_first_at(v, tid, M, [&](int k, int pos) {
            const C xk = lds[k * K::TS + team];
            const C xm = lds[(M - k) * K::TS + team];
            const C a = xk + conj(xm);
            C t;
            if constexpr (F::REG_TW) t = w2[pos];
            else t = tw2M[k];
            const C b = cmulc(xk - conj(xm), t);
            return a + rot90<true>(b);
        });
        sync_wg_lds();
        if constexpr (F::REG_TW) F::run_r(v, scr, tid, w);
        else F::run_g(v, scr, tid, twM);
        const int inner = col0 + team;
        if (inner < n_inner) {
            const size_t r0 = ((size_t)outer * n_inner + inner) * M;
            R* row = (R*)jb.phi + r0;
            if (jb.add) {  // phi += alpha * add, element by element (add may be phi)
                const R* arow = (const R*)jb.add + r0;
                const R al = (R)jb.alpha;
                F::store_last(v, tid, M / 2, [&](int m, C z) {
                    const C a = *reinterpret_cast<const C*>(arow + 2 * m);
                    *reinterpret_cast<C*>(row + 2 * m) = mk(z.x + al * a.x, z.y + al * a.y);
                });
            } else {
                F::store_last(v, tid, M / 2,
                              [&](int m, C z) { *reinterpret_cast<C*>(row + 2 * m) = z; });
            }
        }
        sync_wg_lds();
    }
}

// ---------------------------------------------------------------------------
// Pass B (3D): zero-pad + forward C2C along axis 1, contiguous in, transposed out
//   in[(i0 * H + p2) * N1 + i1] -> out[(p2 * P + p1) * N0 + i0],  P = 2 N1
// for the bins p2 in [p2_lo, p2_lo + p2_n) of the job.  Work item = (p2,
// tile of WT consecutive i0); persistent with prefetch.
// ---------------------------------------------------------------------------
template <typename R, int P, int VAR = 0>
struct FwdT {
    using F = Fft<R, P, false, var_alt(VAR)>;
    using C = cpx<R>;
    static constexpr int T = F::T;
    static constexpr int WT =
        tile_width(sizeof(C), T, F::SCR, P, var_cap(VAR, F::V <= 8 ? 1024 : 512));
    static constexpr int TS = WT + 1;
    static constexpr int LDS = cmax(WT * F::SCR, P * TS);
    static constexpr int THREADS = WT * T;
    static constexpr int R0 = F::first_radix(), NB0 = F::first_stride(), NBT0 = F::first_nbt();
    static constexpr int HALF = R0 / 2;
    static_assert(R0 % 2 == 0, "zero half = whole first-stage operands");
    static constexpr bool DISTINCT =
        VAR == 0 || (VAR == 1 ? fft_alt_distinct(P) : WT != FwdT<R, P, 0>::WT);
};

template <typename R, int P, int VAR, class Src>
__global__ __launch_bounds__((FwdT<R, P, VAR>::THREADS)) void k_fwd_t(
    Src src, const cpx<R>* __restrict__ tw) {
    using K = FwdT<R, P, VAR>;
    using F = typename K::F;
    using C = cpx<R>;
    constexpr int N1 = P / 2;
    __shared__ C lds[K::LDS];
    const int team = team_index<K::T>(), tid0 = threadIdx.x % K::T;
    const int tid = tid0;
    C* scr = lds + team * F::SCR;
    C w[F::REG_TW ? F::NTW : 1];
    if constexpr (F::REG_TW) F::load_tw(w, tid, tw);
    const Walk ch = walk_of<kWalkChunk>(src.total);
    C pf[K::NBT0 * K::HALF];
    int cur_pf = -1, cur_it = -1;  // job cursors of the prefetch and the item walks
    auto prefetch = [&](int item) {
        int loc;
        const JobT jb = src.get(item, loc, cur_pf);
        const int ntile = cdiv(jb.N0, K::WT);
        const int t2 = loc / ntile, i0 = (loc - t2 * ntile) * K::WT + team;
        const int p2 = jb.p2_lo + t2;
        if (i0 < jb.N0) {
            const C* in = (const C*)jb.in + ((size_t)i0 * jb.H + p2) * N1;
#pragma unroll
            for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
                for (int q = 0; q < K::HALF; ++q) {
                    const int i = F::first_index(tid, b, q);
                    pf[b * K::HALF + q] = i >= 0 ? in[i] : mk(R(0), R(0));
                }
        }
    };
    if (ch.first < ch.last) prefetch(ch.first);
    for (int item = ch.first; item < ch.last; item += ch.stride) {
        const int tid = fresh_lane<R, P>() ? opaque(tid0) : tid0;  // per item: fresh_lane
        int loc;
        const JobT jb = src.get(item, loc, cur_it);
        const int N0 = jb.N0;
        const int ntile = cdiv(N0, K::WT);
        const int t2 = loc / ntile, col0 = (loc - t2 * ntile) * K::WT;
        const int p2 = jb.p2_lo + t2;
        const bool active = col0 + team < N0;
        C v[F::V];
#pragma unroll
        for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
            for (int q = 0; q < K::R0; ++q)
                v[b * K::R0 + q] = (q < K::HALF && active) ? pf[b * K::HALF + q] : mk(R(0), R(0));
        if (item + ch.stride < ch.last) prefetch(item + ch.stride);
        if constexpr (F::REG_TW) F::template run_r<true>(v, scr, tid, w);
        else F::template run_g<true>(v, scr, tid, tw);
        sync_wg_lds();
        F::store_last(v, tid, P, [&](int p1, C c) { lds[p1 * K::TS + team] = c; });
        sync_wg_lds();
        C* out = (C*)jb.out;
        for (int e = threadIdx.x; e < P * K::WT; e += K::THREADS) {
            const int p1 = e / K::WT, ww = e - p1 * K::WT;
            if (col0 + ww < N0) out[((size_t)p2 * P + p1) * N0 + col0 + ww] = lds[p1 * K::TS + ww];
        }
        sync_wg_lds();
    }
}

// ---------------------------------------------------------------------------
// Pass D (3D): inverse C2C along axis 1 with crop, transposed in, contiguous out
//   in[(p2 * P + p1) * N0 + i0] -> out[(i0 * H + p2) * N1 + i1], i1 < N1
// Persistent; the next item's tile is prefetched into registers.
// ---------------------------------------------------------------------------
template <typename R, int P, int VAR = 0>
struct InvT {
    using F = Fft<R, P, true, var_alt(VAR)>;
    using C = cpx<R>;
    static constexpr int T = F::T;
    static constexpr int WT =
        tile_width(sizeof(C), T, F::SCR, P, var_cap(VAR, F::V <= 8 ? 1024 : 512));
    static constexpr int TS = WT + 1;
    static constexpr int LDS = cmax(WT * F::SCR, P * TS);
    static constexpr int THREADS = WT * T;
    static constexpr int NT = (P * WT + THREADS - 1) / THREADS;
    static constexpr bool PREFETCH = NT * (int)(sizeof(C) / 4) <= 48;
    static constexpr bool DISTINCT =
        VAR == 0 || (VAR == 1 ? fft_alt_distinct(P) : WT != InvT<R, P, 0>::WT);
};

template <typename R, int P, int VAR, class Src>
__global__ __launch_bounds__((InvT<R, P, VAR>::THREADS)) void k_inv_t(
    Src src, const cpx<R>* __restrict__ tw) {
    using K = InvT<R, P, VAR>;
    using F = typename K::F;
    using C = cpx<R>;
    constexpr int N1 = P / 2;
    __shared__ C lds[K::LDS];
    const int team = team_index<K::T>(), tid0 = threadIdx.x % K::T;
    const int tid = tid0;
    C* scr = lds + team * F::SCR;
    C w[F::REG_TW ? F::NTW : 1];
    if constexpr (F::REG_TW) F::load_tw(w, tid, tw);
    const Walk ch = walk_of<kWalkChunk>(src.total);
    C tp[K::PREFETCH ? K::NT : 1];
    auto tile_elem = [&](const JobT& jb, int p2, int col0, int e) {
        const int p1 = e / K::WT, ww = e - p1 * K::WT;
        return (e < P * K::WT && col0 + ww < jb.N0)
                   ? ((const C*)jb.in)[((size_t)p2 * P + p1) * jb.N0 + col0 + ww]
                   : mk(R(0), R(0));
    };
    int cur_pf = -1, cur_it = -1;  // job cursors of the prefetch and the item walks
    auto prefetch = [&](int item) {
        int loc;
        const JobT jb = src.get(item, loc, cur_pf);
        const int ntile = cdiv(jb.N0, K::WT);
        const int t2 = loc / ntile, col0 = (loc - t2 * ntile) * K::WT;
#pragma unroll
        for (int i = 0; i < K::NT; ++i)
            tp[i] = tile_elem(jb, jb.p2_lo + t2, col0, threadIdx.x + i * K::THREADS);
    };
    if constexpr (K::PREFETCH) {
        if (ch.first < ch.last) prefetch(ch.first);
    }
    for (int item = ch.first; item < ch.last; item += ch.stride) {
        const int tid = fresh_lane<R, P>() ? opaque(tid0) : tid0;  // per item: fresh_lane
        int loc;
        const JobT jb = src.get(item, loc, cur_it);
        const int N0 = jb.N0;
        const int ntile = cdiv(N0, K::WT);
        const int t2 = loc / ntile, col0 = (loc - t2 * ntile) * K::WT;
        const int p2 = jb.p2_lo + t2;
        if constexpr (K::PREFETCH) {
#pragma unroll
            for (int i = 0; i < K::NT; ++i) {
                const int e = threadIdx.x + i * K::THREADS;
                const int p1 = e / K::WT, ww = e - p1 * K::WT;
                if (e < P * K::WT) lds[p1 * K::TS + ww] = tp[i];
            }
        } else {
            for (int e = threadIdx.x; e < P * K::WT; e += K::THREADS) {
                const int p1 = e / K::WT, ww = e - p1 * K::WT;
                lds[p1 * K::TS + ww] = tile_elem(jb, p2, col0, e);
            }
        }
        sync_wg_lds();
        if constexpr (K::PREFETCH) {
            if (item + ch.stride < ch.last) prefetch(item + ch.stride);
        }
        C v[F::V];
        F::load_first(v, tid, P, [&](int p1) { return lds[p1 * K::TS + team]; });
        sync_wg_lds();
        if constexpr (F::REG_TW) F::run_r(v, scr, tid, w);
        else F::run_g(v, scr, tid, tw);
        const int i0 = col0 + team;
        if (i0 < N0) {
            C* dst = (C*)jb.out + ((size_t)i0 * jb.H + p2) * N1;
            F::store_last(v, tid, N1, [&](int i1, C c) { dst[i1] = c; });
        }
        sync_wg_lds();
    }
}

// ---------------------------------------------------------------------------
// Pass C: along the outermost axis, pencils contiguous: zero-pad, forward
// C2C, product with the real octant tensor, inverse C2C, crop -- in place.
//   pencil q = p2 * P1 + p1 (3D) or q = p1 (2D: P1 = 1, N1 = 0),
//   data[q * N0 + i0];  tensor[((p2 (N1+1) + |p1|) (N0+1)) + |p0|]
//
// Persistent: the grid fills the GPU once; every team walks a contiguous
// chunk of work items.  Its twiddles are loaded into registers once, the next
// pencil's non-zero half is prefetched while the current one is transformed,
// and items are ordered so that the mirror pencils p1 and P1 - p1, which read
// the same tensor row, follow each other.
// ---------------------------------------------------------------------------
template <typename R, int P, int VAR = 0>
struct Conv {
    using Ff = Fft<R, P, false, var_alt(VAR), var_xch(VAR)>;
    using Fi = Fft<R, P, true, var_alt(VAR), var_xch(VAR)>;
    using C = cpx<R>;
    static constexpr int T = Ff::T;
    static constexpr int TPW = cmax(1, var_cap(VAR, 256) / T);  // teams per workgroup
    static constexpr int THREADS = TPW * T;
    static constexpr int LDS = TPW * Ff::SCR;
    static constexpr bool SHARED_TW = Ff::palindromic();
    static constexpr int R0 = Ff::first_radix();
    static constexpr int NB0 = Ff::first_stride();
    static constexpr int NBT0 = Ff::first_nbt();
    static constexpr int HALF = R0 / 2;  // first-stage operands with index < P/2
    static constexpr int NPF = NBT0 * HALF;
    // The next pencil's operands are prefetched into registers, except for
    // FP32 plans of 16 operands per thread up to length 2048: there the
    // operands, twiddles and tensor values already take ~165 VGPRs, and the
    // prefetch held the kernel at two waves per SIMD instead of three (the
    // 2D batch's fused pass at 2048: 490 -> 428 us; at 4096 the kernel stays
    // at two waves either way and keeps the prefetch)
    static constexpr bool PREFETCH = !(sizeof(R) == 4 && Ff::V >= 16 && P <= 2048);
    static_assert(R0 % 2 == 0, "the zero half must be whole first-stage operands");
    static_assert(Ff::last_radix() == Fi::first_radix(), "register hand-off");
    // Variant 4: the first forward stage as a matrix product on the matrix
    // cores (Fft::mfma_first_ok: FP32, length 512): four pairs of FP32
    // 16x16x4 MFMAs over the 64 butterflies, operands loaded from HBM
    // straight into the B layout, outputs stored to the LDS where the
    // stage-0 store puts them; the transform goes on from stage 1.
    static constexpr bool MFMA0 = VAR == 4 && sizeof(R) == 4 && Ff::mfma_first_ok();
    static constexpr bool DISTINCT =
        VAR == 0 || (VAR == 1   ? fft_alt_distinct(P)
                     : VAR == 2 ? TPW != Conv<R, P, 0>::TPW
                     : VAR == 3 ? Ff::has_reg_exchange()
                                : MFMA0);
};

// work item t -> pencil, ordered (p2; p1 = 0, N1, 1, P1-1, 2, P1-2, ...)
__device__ __forceinline__ int conv_item_to_pencil(int t, int P1, int N1) {
    const int p2 = t / P1, u = t - p2 * P1;
    int p1;
    if (P1 == 1) p1 = 0;
    else if (u < 2) p1 = u ? N1 : 0;
    else p1 = (u & 1) ? P1 - (u >> 1) : (u >> 1);
    return p2 * P1 + p1;
}

template <typename R, int P, int VAR, class Src>
__global__ __launch_bounds__((Conv<R, P, VAR>::THREADS)) void k_conv(
    Src src, const cpx<R>* __restrict__ tw) {
    using K = Conv<R, P, VAR>;
    using Ff = typename K::Ff;
    using Fi = typename K::Fi;
    using C = cpx<R>;
    constexpr int N0 = P / 2;
    __shared__ C lds[K::LDS];
    const int team = team_index<K::T>(), tid0 = threadIdx.x % K::T;
    const int tid = tid0;
    C* scr = lds + team * Ff::SCR;

    // register twiddles when they fit (shared by both directions if palindromic)
    // (the 256-thread conv workgroups can spend up to ~64 VGPRs on them)
    constexpr bool REG = K::SHARED_TW ? Ff::reg_tw(64)
                                      : (Ff::NTW + Fi::NTW) * (int)(sizeof(C) / 4) <= 64;
    C wf[REG ? Ff::NTW : 1];
    if constexpr (REG) Ff::load_tw(wf, tid, tw);
    C wi[(REG && !K::SHARED_TW) ? Fi::NTW : 1];
    if constexpr (REG && !K::SHARED_TW) Fi::load_tw(wi, tid, tw);

    const int total = src.total;
    const int slots = gridDim.x * K::TPW;
    const int chunk = (total + slots - 1) / slots;
    const int first = (blockIdx.x * K::TPW + team) * chunk;

    C pf[(K::MFMA0 || !K::PREFETCH) ? 1 : K::NPF];
    // variant 4: this lane's B operands (butterfly group g, K step ks at
    // pb[2 g + ks]) and A operands (K step ks), see Conv::MFMA0.  Lane l
    // gives B row l / 16 (operand q = 2 ks + (l / 16) / 2, its real part for
    // even l / 16, imaginary for odd) of column l % 16 (butterfly 16 g +
    // l % 16), and A entry (l % 16, 4 ks + l / 16).
    float pb[K::MFMA0 ? 8 : 1];
    float am[2] = {0.f, 0.f};
    if constexpr (K::MFMA0) {
        am[0] = Ff::mfma0_a(tid, 0);
        am[1] = Ff::mfma0_a(tid, 1);
    }
    int cur_pf = -1, cur_it = -1;  // job cursors of the prefetch and the item walks
    auto prefetch = [&](int item) {
        if (item < total) {
            int loc;
            const JobConv jb = src.get(item, loc, cur_pf);
            const int qp = conv_item_to_pencil(loc, jb.P1, jb.N1) + jb.p2_lo * jb.P1;
            const C* pen = (const C*)jb.data + (size_t)qp * N0;
            if constexpr (K::MFMA0) {
                const R* pr = (const R*)pen;
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks)
                        pb[2 * g + ks] = pr[2 * Ff::mfma0_b_index(tid, g, ks) + Ff::mfma0_part(tid)];
            } else {
#pragma unroll
                for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
                    for (int q = 0; q < K::HALF; ++q) {
                        const int i = Ff::first_index(tid, b, q);
                        pf[b * K::HALF + q] = i >= 0 ? pen[i] : mk(R(0), R(0));
                    }
            }
        }
    };
    if constexpr (K::PREFETCH) prefetch(first);
    for (int it = 0; it < chunk; ++it) {
        const int tid = fresh_lane<R, P>() ? opaque(tid0) : tid0;  // per item: fresh_lane
        const int item = first + it;
        const bool active = item < total;
        int loc;
        const JobConv jb = src.get(active ? item : 0, loc, cur_it);
        C v[Ff::V];
        typedef float v4f __attribute__((ext_vector_type(4)));
        v4f d[K::MFMA0 ? 4 : 1];
        if constexpr (K::MFMA0) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                d[g] = v4f{0.f, 0.f, 0.f, 0.f};
                d[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[0], pb[2 * g], d[g], 0, 0, 0);
                d[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[1], pb[2 * g + 1], d[g], 0, 0, 0);
            }
        } else if constexpr (K::PREFETCH) {
#pragma unroll
            for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
                for (int q = 0; q < K::R0; ++q)
                    v[b * K::R0 + q] = q < K::HALF ? pf[b * K::HALF + q] : mk(R(0), R(0));
        } else {  // this pencil's non-zero half, loaded now
            const int qp0 = conv_item_to_pencil(loc, jb.P1, jb.N1) + jb.p2_lo * jb.P1;
            const C* pen = (const C*)jb.data + (size_t)qp0 * N0;
#pragma unroll
            for (int b = 0; b < K::NBT0; ++b)
#pragma unroll
                for (int q = 0; q < K::R0; ++q) {
                    const int i = q < K::HALF ? Ff::first_index(tid, b, q) : -1;
                    v[b * K::R0 + q] = (active && i >= 0) ? pen[i] : mk(R(0), R(0));
                }
        }
        if constexpr (K::PREFETCH) {
            if (it + 1 < chunk) prefetch(item + 1);
        }
        const int qp = conv_item_to_pencil(loc, jb.P1, jb.N1) + jb.p2_lo * jb.P1;
        const int p2 = qp / jb.P1, p1 = qp - p2 * jb.P1;
        const int a1 = p1 <= jb.N1 ? p1 : jb.P1 - p1;
        const R* trow = (const R*)jb.tensor + ((size_t)p2 * (jb.N1 + 1) + a1) * (N0 + 1);
        R tv[Ff::V];
        {
            int i = 0;
            Ff::for_each_last(v, tid, [&](int p0, C&) { tv[i++] = trow[p0 <= N0 ? p0 : P - p0]; });
        }
        if constexpr (K::MFMA0) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                scr[Ff::mfma0_slot(tid, g, 0)] = mk(d[g][0], d[g][1]);
                scr[Ff::mfma0_slot(tid, g, 1)] = mk(d[g][2], d[g][3]);
            }
            Ff::sync_lds();
            Ff::template load<1>(v, scr, tid);
            Ff::sync_lds();
            if constexpr (REG) {
                Ff::template compute_r<1>(v, tid, wf);
                Ff::template run_r_from<2>(v, scr, tid, wf);
            } else {
                Ff::template compute<1>(v, tid, tw);
                Ff::template run_g_from<2>(v, scr, tid, tw);
            }
        } else if constexpr (REG) {
            Ff::template run_r<true>(v, scr, tid, wf);
        } else {
            Ff::template run_g<true>(v, scr, tid, tw);
        }
        {
            int i = 0;
            Ff::for_each_last(v, tid, [&](int, C& c) { c = scale(c, tv[i++]); });
        }
        if constexpr (REG && K::SHARED_TW) Fi::run_r(v, scr, tid, wf);
        else if constexpr (REG) Fi::run_r(v, scr, tid, wi);
        else Fi::run_g(v, scr, tid, tw);
        if (active) {
            C* pen = (C*)jb.data + (size_t)qp * N0;
            Fi::store_last(v, tid, N0, [&](int i, C c) { pen[i] = c; });
        }
    }
}

}  // namespace fsa
