// Dispatch of y = H x to the kernel instantiations (rank width by dim, value
// type by dtype); the kernels themselves are in sigma_impl.h.
#include "pd_internal.h"
#include "sigma_impl.h"

namespace pd {

hipError_t sigma_r32_f32(int, int, int64_t, const float *, const float *, float, const float *, float *, unsigned *,
                         hipStream_t);
hipError_t sigma_r32_f64(int, int, int64_t, const double *, const double *, double, const double *, double *,
                         unsigned *, hipStream_t);
hipError_t sigma_r64_f32(int, int, int64_t, const float *, const float *, float, const float *, float *, unsigned *,
                         hipStream_t);
hipError_t sigma_r64_f64(int, int, int64_t, const double *, const double *, double, const double *, double *,
                         unsigned *, hipStream_t);

hipError_t sigma_trunc_r32_f32(int, int, const TruncSpace &, const float *, const float *, float, const float *, float *,
                               hipStream_t);
hipError_t sigma_trunc_r32_f64(int, int, const TruncSpace &, const double *, const double *, double, const double *,
                               double *, hipStream_t);
hipError_t sigma_trunc_r64_f32(int, int, const TruncSpace &, const float *, const float *, float, const float *, float *,
                               hipStream_t);
hipError_t sigma_trunc_r64_f64(int, int, const TruncSpace &, const double *, const double *, double, const double *,
                               double *, hipStream_t);

hipError_t launch_sigma(int omega, int n, int64_t dim, const CoefBlock *coef, pd_dtype dt, const void *x, void *y,
                        hipStream_t s, double dsum64, float dsum32, const TruncSpace *tr) {
    if (dim <= 0) return hipSuccess;
    const unsigned char *base = reinterpret_cast<const unsigned char *>(coef);  // device address
    if (tr) {
        const bool small = trunc_ranks32(tr->full_dim);
        if (dt == PD_F64) {
            const double *d = reinterpret_cast<const double *>(base + offsetof(CoefBlock, d64));
            const double *V = reinterpret_cast<const double *>(base + offsetof(CoefBlock, V64));
            return (small ? sigma_trunc_r32_f64 : sigma_trunc_r64_f64)(omega, n, *tr, d, V, dsum64, (const double *)x,
                                                                     (double *)y, s);
        }
        const float *d = reinterpret_cast<const float *>(base + offsetof(CoefBlock, d32));
        const float *V = reinterpret_cast<const float *>(base + offsetof(CoefBlock, V32));
        return (small ? sigma_trunc_r32_f32 : sigma_trunc_r64_f32)(omega, n, *tr, d, V, dsum32, (const float *)x,
                                                                 (float *)y, s);
    }
    if (sigma_space_refused(omega, n)) return hipErrorNotSupported;
    const bool small = dim < (int64_t(1) << 32);
    unsigned *sched = reinterpret_cast<unsigned *>(const_cast<unsigned char *>(base) + offsetof(CoefBlock, sched));
    if (dt == PD_F64) {
        const double *d = reinterpret_cast<const double *>(base + offsetof(CoefBlock, d64));
        const double *V = reinterpret_cast<const double *>(base + offsetof(CoefBlock, V64));
        return (small ? sigma_r32_f64 : sigma_r64_f64)(omega, n, dim, d, V, dsum64, (const double *)x, (double *)y, sched,
                                                     s);
    }
    const float *d = reinterpret_cast<const float *>(base + offsetof(CoefBlock, d32));
    const float *V = reinterpret_cast<const float *>(base + offsetof(CoefBlock, V32));
    return (small ? sigma_r32_f32 : sigma_r64_f32)(omega, n, dim, d, V, dsum32, (const float *)x, (float *)y, sched, s);
}

bool sigma_launch_shape(int omega, int n, pd_dtype dt, int *threads, int64_t *lds, int64_t *limit) {
    const int nn = n > omega - n ? omega - n : n;
    const bool small = binom_host(omega, n) < (uint64_t(1) << 32);
    sigma_detail::LaunchShape sh{};
    bool ok;
    if (dt == PD_F64)
        ok = small ? sigma_detail::shape_for<uint32_t, double>(omega, nn, &sh)
                   : sigma_detail::shape_for<uint64_t, double>(omega, nn, &sh);
    else
        ok = small ? sigma_detail::shape_for<uint32_t, float>(omega, nn, &sh)
                   : sigma_detail::shape_for<uint64_t, float>(omega, nn, &sh);
    if (!ok) return false;
    *threads = sh.threads;
    *lds = (int64_t)sh.lds;
    *limit = (int64_t)sh.limit;
    return true;
}

}  // namespace pd
