// Lanczos vector kernels (Sec. 3.4): projections onto the stored Krylov
// vectors, the Gram-Schmidt updates, norms, the Ritz combination and the
// occupation numbers of Sec. 4.3.  All FP64.  Every kernel streams its
// vectors once with a grid-stride loop; per-block partial sums go to a
// scratch array and a second small kernel adds them in a fixed order, so the
// results are deterministic.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kGrid = 2048;          // blocks of the streaming kernels
constexpr int kMaxCols = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Reduce acc[0..ncols) over the block; thread j < ncols writes partials[j*gridDim + block].
template <int KMAX>
__device__ __forceinline__ void block_partials(const double (&acc)[KMAX], int ncols, double *sh,
                                               double *__restrict__ partials) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < ncols) {
            double v = wave_sum(acc[j]);
            if (lane == 0) sh[wid * KMAX + j] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < ncols) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += sh[w * KMAX + threadIdx.x];
        partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

// out[j] = scale * sum_b partials[j*nb + b]; one block per column.
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double *__restrict__ partials, int nb,
                                                            double scale, double *__restrict__ out) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += partials[(size_t)j * nb + b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += sh[w];
        out[j] = scale * t;
    }
}

template <int KMAX>
__global__ __launch_bounds__(kThreads) void gemvt_kernel(const double *__restrict__ Q, int64_t ld, int ncols,
                                                         int64_t dim, const double *__restrict__ p,
                                                         double *__restrict__ partials) {
    __shared__ double sh[kWaves * KMAX];
    double acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        const double pi = p[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < ncols) acc[j] += Q[(size_t)j * ld + i] * pi;
    }
    block_partials<KMAX>(acc, ncols, sh, partials);
}

template <int KMAX>
__global__ __launch_bounds__(kThreads) void update_gemvt_kernel(const double *__restrict__ Q, int64_t ld,
                                                                int ncols, int64_t dim,
                                                                const double *__restrict__ c,
                                                                const double *pin, double *pout,
                                                                double *__restrict__ partials) {
    __shared__ double sh[kWaves * KMAX];
    double cj[KMAX], acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        cj[j] = (j < ncols) ? c[j] : 0.0;
        acc[j] = 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double q[KMAX];
        double v = pin[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            q[j] = (j < ncols) ? Q[(size_t)j * ld + i] : 0.0;
            v -= q[j] * cj[j];
        }
        pout[i] = v;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) acc[j] += q[j] * v;
    }
    block_partials<KMAX>(acc, ncols, sh, partials);
}

template <int KMAX>
__global__ __launch_bounds__(kThreads) void update_norm_kernel(const double *__restrict__ Q, int64_t ld,
                                                               int ncols, int64_t dim,
                                                               const double *__restrict__ c, const double *pin,
                                                               double *pout, double *__restrict__ partials) {
    __shared__ double sh[kWaves * 1];
    double cj[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) cj[j] = (j < ncols) ? c[j] : 0.0;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double v = pin[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < ncols) v -= Q[(size_t)j * ld + i] * cj[j];
        pout[i] = v;
        acc[0] += v * v;
    }
    block_partials<1>(acc, 1, sh, partials);
}

template <int KMAX>
__global__ __launch_bounds__(kThreads) void combine_kernel(const double *__restrict__ Q, int64_t ld, int ncols,
                                                           int64_t dim, SmallVec y, double *__restrict__ out,
                                                           double *__restrict__ partials) {
    __shared__ double sh[kWaves * 2];
    double yj[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) yj[j] = (j < ncols) ? y.v[j] : 0.0;
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < ncols) v += Q[(size_t)j * ld + i] * yj[j];
        out[i] = v;
        acc[0] += v * v;
        acc[1] += v;
    }
    block_partials<2>(acc, 2, sh, partials);
}

__global__ __launch_bounds__(kThreads) void norm_sum_kernel(const double *__restrict__ x, int64_t dim,
                                                            double *__restrict__ partials) {
    __shared__ double sh[kWaves * 2];
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double v = x[i];
        acc[0] += v * v;
        acc[1] += v;
    }
    block_partials<2>(acc, 2, sh, partials);
}

__global__ __launch_bounds__(kThreads) void scale_kernel(const double *x, int64_t dim, double a,
                                                         double *out, float *out32) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double v = x[i] * a;
        out[i] = v;
        if (out32) out32[i] = (float)v;
    }
}

__global__ __launch_bounds__(kThreads) void f32_to_f64_kernel(const float *__restrict__ x, int64_t dim,
                                                              double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) out[i] = (double)x[i];
}

__global__ __launch_bounds__(kThreads) void copy_kernel(const double *__restrict__ x, int64_t dim,
                                                        double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) out[i] = x[i];
}

// SplitMix64 (Steele, Lea, Flood 2014) at counter k of stream `seed`,
// mapped to [-1, 1) as 2 * (z >> 11) * 2^-53 - 1.
__global__ __launch_bounds__(kThreads) void fill_random_kernel(uint64_t seed, int64_t dim,
                                                               double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        out[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    }
}

__global__ __launch_bounds__(kThreads) void fill_unit_kernel(int64_t dim, int64_t index, double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride)
        out[i] = (i == index) ? 1.0 : 0.0;
}

// Occupations: per-lane accumulators for every orbit, state from the rank.
template <int MAXW>
__global__ __launch_bounds__(kThreads) void occupations_kernel(int omega, int n, int64_t dim,
                                                               const double *__restrict__ psi,
                                                               double *__restrict__ partials) {
    __shared__ double sh[kWaves * MAXW];
    double acc[MAXW];
#pragma unroll
    for (int i = 0; i < MAXW; ++i) acc[i] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < dim; k += stride) {
        uint64_t s = 0, r = (uint64_t)k;
        int m = n;
        for (int p = omega - 1; p >= 0; --p) {
            uint64_t c = g_binom.v[p][m];
            if (m > 0 && c <= r) {
                s |= 1ull << p;
                r -= c;
                --m;
            }
        }
        const double w = psi[k] * psi[k];
#pragma unroll
        for (int i = 0; i < MAXW; ++i) acc[i] += ((s >> i) & 1ull) ? w : 0.0;
    }
    block_partials<MAXW>(acc, omega, sh, partials);
}

inline unsigned grid_for(int64_t dim) {
    int64_t g = (dim + kThreads - 1) / kThreads;
    if (g > kGrid) g = kGrid;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t finalize(const double *partials, unsigned nb, int ncols, double scale, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(ncols), dim3(kThreads), 0, s, partials, (int)nb, scale, out);
    return hipGetLastError();
}

#define PD_DISPATCH_COLS(ncols, KERNEL, ...)                                                      \
    do {                                                                                         \
        if ((ncols) <= 4) hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                            \
        else if ((ncols) <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                       \
        else if ((ncols) <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                     \
        else if ((ncols) <= 32) hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                     \
        else hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__);                                        \
    } while (0)

}  // namespace

int vec_grid() { return kGrid; }
size_t partial_doubles() { return (size_t)kGrid * kMaxCols; }

hipError_t launch_gemvt(const double *Q, int64_t ld, int ncols, int64_t dim, const double *p, double *partials,
                        double *c_dev, hipStream_t s) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    PD_DISPATCH_COLS(ncols, gemvt_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, p, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, ncols, 1.0, c_dev, s);
}

hipError_t launch_update_gemvt(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c,
                               const double *pin, double *pout, double *partials, double *c2_dev, hipStream_t s) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    PD_DISPATCH_COLS(ncols, update_gemvt_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, c, pin, pout,
                     partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, ncols, 1.0, c2_dev, s);
}

hipError_t launch_update_norm(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c,
                              const double *pin, double *pout, double *partials, double *nrm2_dev,
                              hipStream_t s) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    PD_DISPATCH_COLS(ncols, update_norm_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, c, pin, pout,
                     partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, 1, 1.0, nrm2_dev, s);
}

hipError_t launch_combine(const double *Q, int64_t ld, int ncols, int64_t dim, const double *y_host, double *out,
                          double *partials, double *nrm2_dev, double *sum_dev, hipStream_t s) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    SmallVec y;
    for (int j = 0; j < kMaxCols; ++j) y.v[j] = j < ncols ? y_host[j] : 0.0;
    unsigned nb = grid_for(dim);
    PD_DISPATCH_COLS(ncols, combine_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, y, out, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = finalize(partials, nb, 1, 1.0, nrm2_dev, s);
    if (e != hipSuccess) return e;
    return finalize(partials + nb, nb, 1, 1.0, sum_dev, s);
}

hipError_t launch_norm_sum(const double *x, int64_t dim, double *partials, double *nrm2_dev, double *sum_dev,
                           hipStream_t s) {
    unsigned nb = grid_for(dim);
    hipLaunchKernelGGL(norm_sum_kernel, dim3(nb), dim3(kThreads), 0, s, x, dim, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = finalize(partials, nb, 1, 1.0, nrm2_dev, s);
    if (e != hipSuccess) return e;
    return finalize(partials + nb, nb, 1, 1.0, sum_dev, s);
}

hipError_t launch_scale(const double *x, int64_t dim, double scale, double *out, float *out32, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(dim)), dim3(kThreads), 0, s, x, dim, scale, out, out32);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *x, int64_t dim, double *out, hipStream_t s) {
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(grid_for(dim)), dim3(kThreads), 0, s, x, dim, out);
    return hipGetLastError();
}

hipError_t launch_copy(const double *x, int64_t dim, double *out, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(dim)), dim3(kThreads), 0, s, x, dim, out);
    return hipGetLastError();
}

hipError_t launch_fill_random(uint64_t seed, int64_t dim, double *out, hipStream_t s) {
    hipLaunchKernelGGL(fill_random_kernel, dim3(grid_for(dim)), dim3(kThreads), 0, s, seed, dim, out);
    return hipGetLastError();
}

hipError_t launch_fill_unit(int64_t dim, int64_t index, double *out, hipStream_t s) {
    hipLaunchKernelGGL(fill_unit_kernel, dim3(grid_for(dim)), dim3(kThreads), 0, s, dim, index, out);
    return hipGetLastError();
}

hipError_t launch_occupations(int omega, int n, int64_t dim, const double *psi, double *partials, double *occ_dev,
                              hipStream_t s) {
    unsigned nb = grid_for(dim);
    if (omega <= 32)
        hipLaunchKernelGGL(occupations_kernel<32>, dim3(nb), dim3(kThreads), 0, s, omega, n, dim, psi, partials);
    else
        hipLaunchKernelGGL(occupations_kernel<64>, dim3(nb), dim3(kThreads), 0, s, omega, n, dim, psi, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, omega, 2.0, occ_dev, s);
}

}  // namespace pd
