// Instantiation of the sigma kernels for 32-bit ranks and float values.
#include "sigma_impl.h"

namespace pd {
hipError_t sigma_r32_f32(int omega, int n, int64_t dim, const float *d, const float *V, float dsum, const float *x,
                        float *y, unsigned *sched, hipStream_t s) {
    return sigma_detail::launch_typed<uint32_t, float>(omega, n, dim, d, V, dsum, x, y, sched, s);
}
}  // namespace pd
