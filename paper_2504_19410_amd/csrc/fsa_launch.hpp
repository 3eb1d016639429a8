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
        static const int per_cu = blocks_per_cu(k_r2c<R, m>, K::THREADS);                       \
        const int grid = persistent_grid(per_cu, ((n_inner + K::WT - 1) / K::WT) * n_outer);    \
        hipLaunchKernelGGL((k_r2c<R, m>), dim3(grid), dim3(K::THREADS), 0, st, rho, (cpx<R>*)out,     \
                           n_outer, n_inner, (const cpx<R>*)twM, (const cpx<R>*)tw2M);           \
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
        static const int per_cu = blocks_per_cu(k_c2r<R, m>, K::THREADS);                       \
        const int grid = persistent_grid(per_cu, ((n_inner + K::WT - 1) / K::WT) * n_outer);    \
        hipLaunchKernelGGL((k_c2r<R, m>), dim3(grid), dim3(K::THREADS), 0, st, (const cpx<R>*)in, phi, \
                           n_outer, n_inner, (const cpx<R>*)twM, (const cpx<R>*)tw2M);           \
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
        static const int per_cu = blocks_per_cu(k_fwd_t<R, p>, K::THREADS);                     \
        const int grid = persistent_grid(per_cu, ((N0 + K::WT - 1) / K::WT) * H);               \
        hipLaunchKernelGGL((k_fwd_t<R, p>), dim3(grid), dim3(K::THREADS), 0, st, (const cpx<R>*)in,    \
                           (cpx<R>*)out, N0, H, (const cpx<R>*)tw);                              \
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
        static const int per_cu = blocks_per_cu(k_inv_t<R, p>, K::THREADS);                     \
        const int grid = persistent_grid(per_cu, ((N0 + K::WT - 1) / K::WT) * H);               \
        hipLaunchKernelGGL((k_inv_t<R, p>), dim3(grid), dim3(K::THREADS), 0, st, (const cpx<R>*)in,    \
                           (cpx<R>*)out, N0, H, (const cpx<R>*)tw);                              \
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
        static const int per_cu = blocks_per_cu(k_conv<R, p>, K::THREADS);                      \
        const int grid = persistent_grid(per_cu, (n_pencils + K::TPW - 1) / K::TPW);            \
        hipLaunchKernelGGL((k_conv<R, p>), dim3(grid), dim3(K::THREADS), 0, st, (cpx<R>*)data,   \
                           tensor, n_pencils, P1, N1, (const cpx<R>*)tw);                        \
        break;                                                                                   \
    }
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fsa
