// fsa_launch.hpp -- compile-time length dispatch of the pass kernels of one
// variant.  Included by one translation unit per (precision, variant).
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

// Workgroups that fill every CU `occ` times (occ <= 0 or above what fits:
// as many as fit), but no more than the work needs.
inline int persistent_grid(int per_cu, int occ, int work_groups_needed) {
    const int k = (occ > 0 && occ < per_cu) ? occ : per_cu;
    const int g = device_cus() * k;
    return g < work_groups_needed ? g : (work_groups_needed > 0 ? work_groups_needed : 1);
}

namespace detail {

template <typename R, int VAR, int M, class S>
hipError_t go_r2c(const S& src, const void* tw, const void* tw2, int occ, hipStream_t st) {
    using K = R2c<R, M, VAR>;
    if constexpr (!K::DISTINCT) {
        return hipErrorInvalidValue;
    } else {
        static const int per_cu = blocks_per_cu(k_r2c<R, M, VAR, S>, K::THREADS);
        return launch_kernel(k_r2c<R, M, VAR, S>, dim3(persistent_grid(per_cu, occ, src.total)),
                             dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw, (const cpx<R>*)tw2);
    }
}

template <typename R, int VAR, int M, class S>
hipError_t go_c2r(const S& src, const void* tw, const void* tw2, int occ, hipStream_t st) {
    using K = C2r<R, M, VAR>;
    if constexpr (!K::DISTINCT) {
        return hipErrorInvalidValue;
    } else {
        static const int per_cu = blocks_per_cu(k_c2r<R, M, VAR, S>, K::THREADS);
        return launch_kernel(k_c2r<R, M, VAR, S>, dim3(persistent_grid(per_cu, occ, src.total)),
                             dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw, (const cpx<R>*)tw2);
    }
}

template <typename R, int VAR, int P, class S>
hipError_t go_fwd_t(const S& src, const void* tw, int occ, hipStream_t st) {
    using K = FwdT<R, P, VAR>;
    if constexpr (!K::DISTINCT) {
        return hipErrorInvalidValue;
    } else {
        static const int per_cu = blocks_per_cu(k_fwd_t<R, P, VAR, S>, K::THREADS);
        return launch_kernel(k_fwd_t<R, P, VAR, S>,
                             dim3(persistent_grid(per_cu, occ, src.total)), dim3(K::THREADS), 0, st,
                             src, (const cpx<R>*)tw);
    }
}

template <typename R, int VAR, int P, class S>
hipError_t go_inv_t(const S& src, const void* tw, int occ, hipStream_t st) {
    using K = InvT<R, P, VAR>;
    if constexpr (!K::DISTINCT) {
        return hipErrorInvalidValue;
    } else {
        static const int per_cu = blocks_per_cu(k_inv_t<R, P, VAR, S>, K::THREADS);
        return launch_kernel(k_inv_t<R, P, VAR, S>,
                             dim3(persistent_grid(per_cu, occ, src.total)), dim3(K::THREADS), 0, st,
                             src, (const cpx<R>*)tw);
    }
}

template <typename R, int VAR, int P, class S>
hipError_t go_conv(const S& src, const void* tw, int occ, hipStream_t st) {
    using K = Conv<R, P, VAR>;
    if constexpr (!K::DISTINCT) {
        return hipErrorInvalidValue;
    } else {
        static const int per_cu = blocks_per_cu(k_conv<R, P, VAR, S>, K::THREADS);
        return launch_kernel(k_conv<R, P, VAR, S>,
                             dim3(persistent_grid(per_cu, occ, cdiv(src.total, K::TPW))),
                             dim3(K::THREADS), 0, st, src, (const cpx<R>*)tw);
    }
}

// Resident workgroups per CU of a variant's single-evaluation kernel (the
// kernel is named only where the variant exists).
#define FSA_OCC_HELPER(name, Cfg, kern, Job)                                                    \
    template <typename R, int VAR, int LEN>                                                      \
    int name() {                                                                                 \
        using K = Cfg<R, LEN, VAR>;                                                              \
        if constexpr (!K::DISTINCT) return 0;                                                    \
        else return blocks_per_cu(kern<R, LEN, VAR, JobOne<Job>>, K::THREADS);                   \
    }
FSA_OCC_HELPER(occ_r2c, R2c, k_r2c, JobR2c)
FSA_OCC_HELPER(occ_c2r, C2r, k_c2r, JobC2r)
FSA_OCC_HELPER(occ_fwd_t, FwdT, k_fwd_t, JobT)
FSA_OCC_HELPER(occ_inv_t, InvT, k_inv_t, JobT)
FSA_OCC_HELPER(occ_conv, Conv, k_conv, JobConv)
#undef FSA_OCC_HELPER

}  // namespace detail

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::r2c(int M, const R* rho, void* out, int n_outer, int n_inner,
                                const void* twM, const void* tw2M, int occ, hipStream_t st) {
    using S = JobOne<JobR2c>;
    switch (M) {
#define FSA_CASE(m)                                                                              \
    case m:                                                                                      \
        return detail::go_r2c<R, VAR, m>(                                                        \
            S{JobR2c{rho, out, n_outer, n_inner}, cdiv(n_inner, R2c<R, m, VAR>::WT) * n_outer},  \
            twM, tw2M, occ, st);
        FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::c2r(int M, const void* in, R* phi, int n_outer, int n_inner,
                                const void* add, double alpha, const void* twM,
                                const void* tw2M, int occ, hipStream_t st) {
    using S = JobOne<JobC2r>;
    switch (M) {
#define FSA_CASE(m)                                                                              \
    case m:                                                                                      \
        return detail::go_c2r<R, VAR, m>(S{JobC2r{in, phi, n_outer, n_inner, add, alpha},        \
                                           cdiv(n_inner, C2r<R, m, VAR>::WT) * n_outer},         \
                                         twM, tw2M, occ, st);
        FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::fwd_t(int P, const void* in, void* out, int N0, int H, int p2_lo,
                                  int p2_n, const void* tw, int occ, hipStream_t st) {
    using S = JobOne<JobT>;
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::go_fwd_t<R, VAR, p>(                                                      \
            S{JobT{in, out, N0, H, p2_lo, p2_n}, cdiv(N0, FwdT<R, p, VAR>::WT) * p2_n}, tw, occ,  \
            st);
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::inv_t(int P, const void* in, void* out, int N0, int H, int p2_lo,
                                  int p2_n, const void* tw, int occ, hipStream_t st) {
    using S = JobOne<JobT>;
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::go_inv_t<R, VAR, p>(                                                      \
            S{JobT{in, out, N0, H, p2_lo, p2_n}, cdiv(N0, InvT<R, p, VAR>::WT) * p2_n}, tw, occ,  \
            st);
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::conv(int P, void* data, const R* tensor, int n_pencils, int P1,
                                 int N1, int p2_lo, const void* tw, int occ, hipStream_t st) {
    using S = JobOne<JobConv>;
    switch (P) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::go_conv<R, VAR, p>(                                                       \
            S{JobConv{data, tensor, n_pencils, P1, N1, p2_lo}, n_pencils}, tw, occ, st);
        FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
int LaunchV<R, VAR>::items(Pass pass, int len, const void* job) {
    switch (pass) {
    case Pass::R2C: {
        const JobR2c& j = *(const JobR2c*)job;
        switch (len) {
#define FSA_CASE(m) case m: return cdiv(j.n_inner, R2c<R, m, VAR>::WT) * j.n_outer;
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return -1;
    }
    case Pass::C2R: {
        const JobC2r& j = *(const JobC2r*)job;
        switch (len) {
#define FSA_CASE(m) case m: return cdiv(j.n_inner, C2r<R, m, VAR>::WT) * j.n_outer;
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
        return cdiv(j.N0, pass == Pass::FWD_T ? FwdT<R, p, VAR>::WT : InvT<R, p, VAR>::WT) *     \
               j.p2_n;
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

template <typename R, int VAR>
hipError_t LaunchV<R, VAR>::batch(Pass pass, int len, const void* jobs, const int* start, int n,
                                  int total, const void* tw, const void* tw2, int occ,
                                  hipStream_t st) {
    if (total <= 0) return hipSuccess;
    switch (pass) {
    case Pass::R2C: {
        using S = JobList<JobR2c>;
        const S src{(const JobR2c*)jobs, start, n, total};
        switch (len) {
#define FSA_CASE(m) case m: return detail::go_r2c<R, VAR, m>(src, tw, tw2, occ, st);
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    case Pass::C2R: {
        using S = JobList<JobC2r>;
        const S src{(const JobC2r*)jobs, start, n, total};
        switch (len) {
#define FSA_CASE(m) case m: return detail::go_c2r<R, VAR, m>(src, tw, tw2, occ, st);
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    case Pass::FWD_T: {
        using S = JobList<JobT>;
        const S src{(const JobT*)jobs, start, n, total};
        switch (len) {
#define FSA_CASE(p) case p: return detail::go_fwd_t<R, VAR, p>(src, tw, occ, st);
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    case Pass::INV_T: {
        using S = JobList<JobT>;
        const S src{(const JobT*)jobs, start, n, total};
        switch (len) {
#define FSA_CASE(p) case p: return detail::go_inv_t<R, VAR, p>(src, tw, occ, st);
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    case Pass::CONV: {
        using S = JobList<JobConv>;
        const S src{(const JobConv*)jobs, start, n, total};
        switch (len) {
#define FSA_CASE(p) case p: return detail::go_conv<R, VAR, p>(src, tw, occ, st);
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        break;
    }
    }
    return hipErrorInvalidValue;
}

template <typename R, int VAR>
bool LaunchV<R, VAR>::distinct(Pass pass, int len) {
    switch (pass) {
    case Pass::R2C:
        switch (len) {
#define FSA_CASE(m) case m: return R2c<R, m, VAR>::DISTINCT;
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return false;
    case Pass::C2R:
        switch (len) {
#define FSA_CASE(m) case m: return C2r<R, m, VAR>::DISTINCT;
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return false;
    case Pass::FWD_T:
        switch (len) {
#define FSA_CASE(p) case p: return FwdT<R, p, VAR>::DISTINCT;
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return false;
    case Pass::INV_T:
        switch (len) {
#define FSA_CASE(p) case p: return InvT<R, p, VAR>::DISTINCT;
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return false;
    case Pass::CONV:
        switch (len) {
#define FSA_CASE(p) case p: return Conv<R, p, VAR>::DISTINCT;
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return false;
    }
    return false;
}

template <typename R, int VAR>
int LaunchV<R, VAR>::max_occ(Pass pass, int len) {
    switch (pass) {
    case Pass::R2C:
        switch (len) {
#define FSA_CASE(m)                                                                              \
    case m:                                                                                      \
        return detail::occ_r2c<R, VAR, m>();
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return 0;
    case Pass::C2R:
        switch (len) {
#define FSA_CASE(m)                                                                              \
    case m:                                                                                      \
        return detail::occ_c2r<R, VAR, m>();
            FSA_M_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return 0;
    case Pass::FWD_T:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::occ_fwd_t<R, VAR, p>();
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return 0;
    case Pass::INV_T:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::occ_inv_t<R, VAR, p>();
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return 0;
    case Pass::CONV:
        switch (len) {
#define FSA_CASE(p)                                                                              \
    case p:                                                                                      \
        return detail::occ_conv<R, VAR, p>();
            FSA_P_LIST(FSA_CASE)
#undef FSA_CASE
        }
        return 0;
    }
    return 0;
}

}  // namespace fsa
