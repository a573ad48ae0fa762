// Instantiation of the truncated-space sigma kernels for 64-bit ranks and double values.
#include "sigma_impl.h"

namespace pd {
hipError_t sigma_trunc_r64_f64(int omega, int n, const TruncSpace &tr, const double *d, const double *V, double dsum,
                               const double *x, double *y, hipStream_t s) {
    return sigma_detail::launch_trunc_typed<uint64_t, double>(omega, n, tr, d, V, dsum, x, y, s);
}
}  // namespace pd
