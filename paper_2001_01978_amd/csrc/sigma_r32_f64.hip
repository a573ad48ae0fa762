// Instantiation of the sigma kernels for 32-bit ranks and double values.
#include "sigma_impl.h"

namespace pd {
hipError_t sigma_r32_f64(int omega, int n, int64_t dim, const double *d, const double *V, double dsum, const double *x,
                        double *y, unsigned *sched, hipStream_t s) {
    return sigma_detail::launch_typed<uint32_t, double>(omega, n, dim, d, V, dsum, x, y, sched, s);
}
}  // namespace pd
