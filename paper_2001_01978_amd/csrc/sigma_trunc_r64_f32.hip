// Instantiation of the truncated-space sigma kernels for 64-bit ranks and float values.
#include "sigma_impl.h"

namespace pd {
hipError_t sigma_trunc_r64_f32(int omega, int n, const TruncSpace &tr, const float *d, const float *V, float dsum,
                               const float *x, float *y, hipStream_t s) {
    return sigma_detail::launch_trunc_typed<uint64_t, float>(omega, n, tr, d, V, dsum, x, y, s);
}
}  // namespace pd
