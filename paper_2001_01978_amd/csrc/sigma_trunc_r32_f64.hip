// Instantiation of the truncated-space sigma kernels for 32-bit ranks and double values.
#include "sigma_impl.h"

namespace pd {
hipError_t sigma_trunc_r32_f64(int omega, int n, const TruncSpace &tr, const double *d, const double *V, double dsum,
                               const double *x, double *y, hipStream_t s) {
    return sigma_detail::launch_trunc_typed<uint32_t, double>(omega, n, tr, d, V, dsum, x, y, s);
}
}  // namespace pd
