// fsa_launch.hpp -- compile-time length dispatch of the pass kernels.
// Included by one translation unit per precision.
#pragma once

#include "fsa_internal.hpp"
#include "fsa_passes.hpp"

// half-lengths M of the real transforms / padded lengths P of the complex ones
#define FSA_M_LIST(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) \
    X(1024) X(1536) X(2048)
#define FSA_P_LIST(X) \
    X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) \
    X(1536) X(2048) X(3072) X(4096)

namespace fsa {

// Compute units of the current device (the library drives one device).
inline int device_cus() {
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        return n;
    }();
    return cus;
}

// Resident workgroups per CU of a kernel at a block size.
template <typename Kern>
int blocks_per_cu(Kern kernel, int threads) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    return per_cu;
}

// Workgroups that fill every CU once, but no more than the work needs.
inline int persistent_grid(int per_cu, int work_groups_needed) {
    const int g = device_cus() * per_cu;
    return g < work_groups_needed ? g : (work_groups_needed > 0 ? work_groups_needed : 1);
}

template <typename R>
hipError_t Launch<R>::r2c(int M, const R* rho, void* out, int n_outer, int n_inner,
                          const void* twM, const void* tw2M, hipStream_t st) {
    switch (M) {
#define FSA_CASE(m)                                                                              \
    case m: {                                                                                    \
        using K = R2c<R, m>;                                                                     \
        using S = JobOne<JobR2c>;                                                                \
        static const int per_cu = blocks_per_cu(k_r2c<R, m, S>, K::THREADS);                    \
        const S src{JobR2c{rho, out, n_outer, n_inner}, cdiv(n_inner, K::WT) * n_outer};         \
        hipLaunchKernelGGL((k_r2c<R, m, S>), dim3(persistent_grid(per_cu, src.total)),          \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)twM,                     \
                           (const cpx<R>*)tw2M);                                                 \
        break;                                                                                   \
    }
        FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::c2r(int M, const void* in, R* phi, int n_outer, int n_inner,
                          const void* twM, const void* tw2M, hipStream_t st) {
    switch (M) {
#define FSA_CASE(m)                                                                              \
    case m: {                                                                                    \
        using K = C2r<R, m>;                                                                     \
        using S = JobOne<JobC2r>;                                                                \
        static const int per_cu = blocks_per_cu(k_c2r<R, m, S>, K::THREADS);                    \
        const S src{JobC2r{in, phi, n_outer, n_inner}, cdiv(n_inner, K::WT) * n_outer};          \
        hipLaunchKernelGGL((k_c2r<R, m, S>), dim3(persistent_grid(per_cu, src.total)),          \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)twM,                     \
                           (const cpx<R>*)tw2M);                                                 \
        break;                                                                                   \
    }
        FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::fwd_t(int P, const void* in, void* out, int N0, int H, const void* tw,
                            hipStream_t st) {
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = FwdT<R, p>;                                                                    \
        using S = JobOne<JobT>;                                                                  \
        static const int per_cu = blocks_per_cu(k_fwd_t<R, p, S>, K::THREADS);                  \
        const S src{JobT{in, out, N0, H}, cdiv(N0, K::WT) * H};                                  \
        hipLaunchKernelGGL((k_fwd_t<R, p, S>), dim3(persistent_grid(per_cu, src.total)),        \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        break;                                                                                   \
    }
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::inv_t(int P, const void* in, void* out, int N0, int H, const void* tw,
                            hipStream_t st) {
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = InvT<R, p>;                                                                    \
        using S = JobOne<JobT>;                                                                  \
        static const int per_cu = blocks_per_cu(k_inv_t<R, p, S>, K::THREADS);                  \
        const S src{JobT{in, out, N0, H}, cdiv(N0, K::WT) * H};                                  \
        hipLaunchKernelGGL((k_inv_t<R, p, S>), dim3(persistent_grid(per_cu, src.total)),        \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        break;                                                                                   \
    }
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::conv(int P, void* data, const R* tensor, int n_pencils, int P1, int N1,
                           const void* tw, hipStream_t st) {
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = Conv<R, p>;                                                                    \
        using S = JobOne<JobConv>;                                                               \
        static const int per_cu = blocks_per_cu(k_conv<R, p, S>, K::THREADS);                   \
        const S src{JobConv{data, tensor, n_pencils, P1, N1}, n_pencils};                        \
        hipLaunchKernelGGL((k_conv<R, p, S>),                                                    \
                           dim3(persistent_grid(per_cu, cdiv(n_pencils, K::TPW))),               \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        break;                                                                                   \
    }
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
int Launch<R>::items(Pass pass, int len, const void* job) {
    switch (pass) {
    case Pass::R2C: {
        const JobR2c& j = *(const JobR2c*)job;
        switch (len) {
#define FSA_CASE(m) case m: return cdiv(j.n_inner, R2c<R, m>::WT) * j.n_outer;
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return -1;
    }
    case Pass::C2R: {
        const JobC2r& j = *(const JobC2r*)job;
        switch (len) {
#define FSA_CASE(m) case m: return cdiv(j.n_inner, C2r<R, m>::WT) * j.n_outer;
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return -1;
    }
    case Pass::FWD_T:
    case Pass::INV_T: {
        const JobT& j = *(const JobT*)job;
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return cdiv(j.N0, pass == Pass::FWD_T ? FwdT<R, p>::WT : InvT<R, p>::WT) * j.H;
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return -1;
    }
    case Pass::CONV:
        return fft_length_supported(len) ? ((const JobConv*)job)->n_pencils : -1;
    }
    return -1;
}

template <typename R>
hipError_t Launch<R>::batch(Pass pass, int len, const void* jobs, const int* start, int n,
                            int total, const void* tw, const void* tw2, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    switch (pass) {
    case Pass::R2C:
        switch (len) {
#define FSA_CASE(m)                                                                              \
    case m: {                                                                                    \
        using K = R2c<R, m>;                                                                     \
        using S = JobList<JobR2c>;                                                               \
        static const int per_cu = blocks_per_cu(k_r2c<R, m, S>, K::THREADS);                    \
        const S src{(const JobR2c*)jobs, start, n, total};                                       \
        hipLaunchKernelGGL((k_r2c<R, m, S>), dim3(persistent_grid(per_cu, total)),              \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw, (const cpx<R>*)tw2); \
        return hipGetLastError();                                                                \
    }
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    case Pass::C2R:
        switch (len) {
#define FSA_CASE(m)                                                                              \
    case m: {                                                                                    \
        using K = C2r<R, m>;                                                                     \
        using S = JobList<JobC2r>;                                                               \
        static const int per_cu = blocks_per_cu(k_c2r<R, m, S>, K::THREADS);                    \
        const S src{(const JobC2r*)jobs, start, n, total};                                       \
        hipLaunchKernelGGL((k_c2r<R, m, S>), dim3(persistent_grid(per_cu, total)),              \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw, (const cpx<R>*)tw2); \
        return hipGetLastError();                                                                \
    }
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    case Pass::FWD_T:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = FwdT<R, p>;                                                                    \
        using S = JobList<JobT>;                                                                 \
        static const int per_cu = blocks_per_cu(k_fwd_t<R, p, S>, K::THREADS);                  \
        const S src{(const JobT*)jobs, start, n, total};                                         \
        hipLaunchKernelGGL((k_fwd_t<R, p, S>), dim3(persistent_grid(per_cu, total)),            \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        return hipGetLastError();                                                                \
    }
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    case Pass::INV_T:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = InvT<R, p>;                                                                    \
        using S = JobList<JobT>;                                                                 \
        static const int per_cu = blocks_per_cu(k_inv_t<R, p, S>, K::THREADS);                  \
        const S src{(const JobT*)jobs, start, n, total};                                         \
        hipLaunchKernelGGL((k_inv_t<R, p, S>), dim3(persistent_grid(per_cu, total)),            \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        return hipGetLastError();                                                                \
    }
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    case Pass::CONV:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p: {                                                                                    \
        using K = Conv<R, p>;                                                                    \
        using S = JobList<JobConv>;                                                              \
        static const int per_cu = blocks_per_cu(k_conv<R, p, S>, K::THREADS);                   \
        const S src{(const JobConv*)jobs, start, n, total};                                      \
        hipLaunchKernelGGL((k_conv<R, p, S>), dim3(persistent_grid(per_cu, cdiv(total, K::TPW))), \
                           dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);                     \
        return hipGetLastError();                                                                \
    }
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace fsa
