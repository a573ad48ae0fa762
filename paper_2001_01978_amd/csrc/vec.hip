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

// As block_partials for acc[0..ncols), plus extra[0..NX) reduced to partials
// rows ncols .. ncols + NX - 1.
template <int KMAX, int NX>
__device__ __forceinline__ void block_partials_extra(const double (&acc)[KMAX], const double (&extra)[NX],
                                                     int ncols, double *sh, double *__restrict__ partials) {
    constexpr int W = KMAX + NX;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < ncols) {
            double v = wave_sum(acc[j]);
            if (lane == 0) sh[wid * W + j] = v;
        }
    }
#pragma unroll
    for (int x = 0; x < NX; ++x) {
        double v = wave_sum(extra[x]);
        if (lane == 0) sh[wid * W + KMAX + x] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < ncols + NX) {
        const int j = (int)threadIdx.x < ncols ? (int)threadIdx.x : KMAX + ((int)threadIdx.x - ncols);
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += sh[w * W + j];
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

// The Krylov columns are stored unnormalised: q_j = sc_j * Qt_j (sc on the
// host, passed by value).  Columns j >= ncols are never read: every thread
// loads KMAX columns at index min(j, ncols - 1), so all loads of an element
// are issued together, and the duplicates get coefficient 0 (their dot
// products are discarded).

// Krylov column j of row i: column 0 is FP64 (Q); columns j >= 1 are FP64
// (Q + j ld) or, when Q32 is given (mixed precision), FP32 (Q32 + (j - 1) ld).
// SPLIT is a template parameter so that every column load is unconditional.
// Slots j >= ncols repeat column ncols - 1 (weight zero); with ncols == 1 they
// read the first FP32 column, which the caller keeps finite.
template <int KMAX, bool SPLIT>
__device__ __forceinline__ void load_cols(const double *__restrict__ Q, const float *__restrict__ Q32, int64_t ld,
                                          int ncols, int64_t i, double (&q)[KMAX]) {
    q[0] = Q[i];
#pragma unroll
    for (int j = 1; j < KMAX; ++j) {
        const int jj = j < ncols ? j : ncols - 1;
        if constexpr (SPLIT)
            q[j] = (double)Q32[(size_t)(jj > 0 ? jj - 1 : 0) * ld + i];
        else
            q[j] = Q[(size_t)jj * ld + i];
    }
}

// With pf = sp * p and ps = pf - sum_j d_j Qt_j (d: the part of the
// three-term recurrence known in advance), partials: raw_j = sum_i Qt_j[i]
// ps[i] (j < ncols), sum_i ps[i]^2 (row ncols), sum_i pf[i]^2 (row ncols + 1).
template <int KMAX, typename TIn, bool SPLIT>
__global__ __launch_bounds__(kThreads) void project_kernel(const double *__restrict__ Q, int64_t ld, int ncols,
                                                           int64_t dim, const TIn *__restrict__ p, double sp,
                                                           SmallVec d, double *__restrict__ partials,
                                                           const float *__restrict__ Q32) {
    __shared__ double sh[kWaves * (KMAX + 2)];
    double acc[KMAX], dj[KMAX], nrm[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        acc[j] = 0.0;
        dj[j] = (j < ncols) ? d.v[j] : 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        const double pf = sp * (double)p[i];
        double q[KMAX];
        load_cols<KMAX, SPLIT>(Q, Q32, ld, ncols, i, q);
        double ps = pf;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) ps -= q[j] * dj[j];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) acc[j] += q[j] * ps;
        nrm[0] += ps * ps;
        nrm[1] += pf * pf;
    }
    block_partials_extra<KMAX, 2>(acc, nrm, ncols, sh, partials);
}

// v = sp * p - sum_j (d_j + c_j sc_j) Qt_j  ->  out (and out32); partials:
// raw sum_i Qt_j[i] v[i] (j < ncols) and sum_i v[i]^2 (row ncols).  c: device.
template <int KMAX, typename TIn, bool SPLIT>
__global__ __launch_bounds__(kThreads) void update_project_kernel(const double *__restrict__ Q, int64_t ld,
                                                                  int ncols, int64_t dim,
                                                                  const double *__restrict__ c, SmallVec sc,
                                                                  SmallVec d, const TIn *__restrict__ p,
                                                                  double sp, double *__restrict__ out,
                                                                  float *__restrict__ out32,
                                                                  double *__restrict__ partials,
                                                                  const float *__restrict__ Q32) {
    __shared__ double sh[kWaves * (KMAX + 1)];
    double cj[KMAX], acc[KMAX], nrm[1] = {0.0};
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        cj[j] = (j < ncols) ? d.v[j] + c[j] * sc.v[j] : 0.0;
        acc[j] = 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double q[KMAX];
        load_cols<KMAX, SPLIT>(Q, Q32, ld, ncols, i, q);
        double v = sp * (double)p[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) v -= q[j] * cj[j];
        if (out) out[i] = v;
        if (out32) out32[i] = (float)v;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) acc[j] += q[j] * v;
        nrm[0] += v * v;
    }
    block_partials_extra<KMAX, 1>(acc, nrm, ncols, sh, partials);
}

// v -= sum_j (c_j sc_j) Qt_j in place (and out32); partials: sum_i v[i]^2.
template <int KMAX, bool SPLIT>
__global__ __launch_bounds__(kThreads) void update_norm_kernel(const double *__restrict__ Q, int64_t ld,
                                                               int ncols, int64_t dim,
                                                               const double *__restrict__ c, SmallVec sc,
                                                               double *v_io, float *out32,
                                                               double *__restrict__ partials,
                                                               const float *__restrict__ Q32) {
    __shared__ double sh[kWaves * 1];
    double cj[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) cj[j] = (j < ncols) ? c[j] * sc.v[j] : 0.0;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double q[KMAX];
        load_cols<KMAX, SPLIT>(Q, Q32, ld, ncols, i, q);
        // v_io null: the vector is FP32 only and is updated in place in out32
        double v = v_io ? v_io[i] : (double)out32[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) v -= q[j] * cj[j];
        if (v_io) v_io[i] = v;
        if (out32) out32[i] = (float)v;
        acc[0] += v * v;
    }
    block_partials<1>(acc, 1, sh, partials);
}

template <int KMAX, bool SPLIT>
__global__ __launch_bounds__(kThreads) void combine_kernel(const double *__restrict__ Q, int64_t ld, int ncols,
                                                           int64_t dim, SmallVec y, double *__restrict__ out,
                                                           double *__restrict__ partials,
                                                           const float *__restrict__ Q32) {
    __shared__ double sh[kWaves * 2];
    double yj[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) yj[j] = (j < ncols) ? y.v[j] : 0.0;
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double q[KMAX];
        load_cols<KMAX, SPLIT>(Q, Q32, ld, ncols, i, q);
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) v += q[j] * yj[j];
        out[i] = v;
        acc[0] += v * v;
        acc[1] += v;
    }
    block_partials<2>(acc, 2, sh, partials);
}

// Thick restart, in place and row by row: Q[o] = sum_{j < ncols} Y[j * k + o] Q[j]
// for o < k, and Q[k] = zs * Q[zcol] when zcol >= 0.  Each thread reads all
// ncols (+1) entries of its row before writing any, so no other row is read.
template <int KMAX>
__global__ __launch_bounds__(kThreads) void combine_many_kernel(double *__restrict__ Q, int64_t ld, int ncols,
                                                                int k, int64_t dim, const double *__restrict__ Y,
                                                                int zcol, double zs) {
    __shared__ double Ys[kMaxCols * kMaxCols];
    for (int t = threadIdx.x; t < KMAX * k; t += kThreads) Ys[t] = t < ncols * k ? Y[t] : 0.0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < dim; i += stride) {
        double q[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) q[j] = j < ncols ? Q[(size_t)j * ld + i] : 0.0;
        const double z = zcol >= 0 ? Q[(size_t)zcol * ld + i] : 0.0;
        for (int o = 0; o < k; ++o) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) v += Ys[j * k + o] * q[j];
            Q[(size_t)o * ld + i] = v;
        }
        if (zcol >= 0) Q[(size_t)k * ld + i] = zs * z;
    }
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
// kr32 / kr64 (at most one non-null): row k is the state of full rank kr[k]
// (truncated space); otherwise rank k.
__global__ __launch_bounds__(kThreads) void occupations_kernel(int omega, int n, int64_t dim,
                                                               const double *__restrict__ psi,
                                                               double *__restrict__ partials,
                                                               const uint32_t *__restrict__ kr32,
                                                               const uint64_t *__restrict__ kr64) {
    __shared__ double sh[kWaves * MAXW];
    double acc[MAXW];
#pragma unroll
    for (int i = 0; i < MAXW; ++i) acc[i] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < dim; k += stride) {
        uint64_t s = 0, r = kr32 ? (uint64_t)kr32[k] : kr64 ? kr64[k] : (uint64_t)k;
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

// out[j] = sc_j * sum_b partials[j*nb + b], j < nout.
struct ScaleVec {
    double v[kMaxCols + 2];
};

__global__ __launch_bounds__(kThreads) void finalize_scaled_kernel(const double *__restrict__ partials, int nb,
                                                                   ScaleVec sc, double *__restrict__ out) {
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
        out[j] = sc.v[j] * t;
    }
}

hipError_t finalize(const double *partials, unsigned nb, int ncols, double scale, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(ncols), dim3(kThreads), 0, s, partials, (int)nb, scale, out);
    return hipGetLastError();
}

#define PD_DISPATCH_COLS(ncols, KERNEL, ...)                                                      \
    do {                                                                                         \
        if ((ncols) <= 4) hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                            \
        else if ((ncols) <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                       \
        else if ((ncols) <= 12) hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__);                     \
        else if ((ncols) <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                     \
        else if ((ncols) <= 24) hipLaunchKernelGGL(KERNEL<24>, __VA_ARGS__);                     \
        else if ((ncols) <= 32) hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                     \
        else if ((ncols) <= 48) hipLaunchKernelGGL(KERNEL<48>, __VA_ARGS__);                     \
        else hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__);                                        \
    } while (0)
// Same, for kernels templated on the column bound and the input type.
#define PD_DISPATCH_COLS_T(ncols, T, KERNEL, ...)                                                 \
    do {                                                                                         \
        if ((ncols) <= 4) hipLaunchKernelGGL((KERNEL<4, T>), __VA_ARGS__);                       \
        else if ((ncols) <= 8) hipLaunchKernelGGL((KERNEL<8, T>), __VA_ARGS__);                  \
        else if ((ncols) <= 12) hipLaunchKernelGGL((KERNEL<12, T>), __VA_ARGS__);                \
        else if ((ncols) <= 16) hipLaunchKernelGGL((KERNEL<16, T>), __VA_ARGS__);                \
        else if ((ncols) <= 24) hipLaunchKernelGGL((KERNEL<24, T>), __VA_ARGS__);                \
        else if ((ncols) <= 32) hipLaunchKernelGGL((KERNEL<32, T>), __VA_ARGS__);                \
        else if ((ncols) <= 48) hipLaunchKernelGGL((KERNEL<48, T>), __VA_ARGS__);                \
        else hipLaunchKernelGGL((KERNEL<64, T>), __VA_ARGS__);                                   \
    } while (0)

// Kernels templated on the column bound and a flag (FP32 columns j >= 1).
#define PD_DISPATCH_COLS_B(ncols, B, KERNEL, ...)                                                 \
    do {                                                                                         \
        if ((ncols) <= 4) hipLaunchKernelGGL((KERNEL<4, B>), __VA_ARGS__);                       \
        else if ((ncols) <= 8) hipLaunchKernelGGL((KERNEL<8, B>), __VA_ARGS__);                  \
        else if ((ncols) <= 12) hipLaunchKernelGGL((KERNEL<12, B>), __VA_ARGS__);                \
        else if ((ncols) <= 16) hipLaunchKernelGGL((KERNEL<16, B>), __VA_ARGS__);                \
        else if ((ncols) <= 24) hipLaunchKernelGGL((KERNEL<24, B>), __VA_ARGS__);                \
        else if ((ncols) <= 32) hipLaunchKernelGGL((KERNEL<32, B>), __VA_ARGS__);                \
        else if ((ncols) <= 48) hipLaunchKernelGGL((KERNEL<48, B>), __VA_ARGS__);                \
        else hipLaunchKernelGGL((KERNEL<64, B>), __VA_ARGS__);                                   \
    } while (0)
#define PD_COMMA ,

hipError_t finalize_scaled(const double *partials, unsigned nb, int nout, const ScaleVec &sc, double *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(finalize_scaled_kernel, dim3(nout), dim3(kThreads), 0, s, partials, (int)nb, sc, out);
    return hipGetLastError();
}

}  // namespace

int vec_grid() { return kGrid; }
size_t partial_doubles() { return (size_t)kGrid * (kMaxCols + 2); }

hipError_t launch_project(const double *Q, int64_t ld, int ncols, int64_t dim, const void *p, bool p_f32, double sp,
                          const double *sc_host, const double *d_host, double *partials, double *out_dev,
                          hipStream_t s, const float *Q32) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    SmallVec d;
    for (int j = 0; j < 64; ++j) d.v[j] = j < ncols ? d_host[j] : 0.0;
    if (p_f32 && Q32)
        PD_DISPATCH_COLS_T(ncols, float PD_COMMA true, project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols,
                           dim, static_cast<const float *>(p), sp, d, partials, Q32);
    else if (p_f32)
        PD_DISPATCH_COLS_T(ncols, float PD_COMMA false, project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols,
                           dim, static_cast<const float *>(p), sp, d, partials, Q32);
    else if (Q32)
        PD_DISPATCH_COLS_T(ncols, double PD_COMMA true, project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols,
                           dim, static_cast<const double *>(p), sp, d, partials, Q32);
    else
        PD_DISPATCH_COLS_T(ncols, double PD_COMMA false, project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld,
                           ncols, dim, static_cast<const double *>(p), sp, d, partials, Q32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ScaleVec f;
    for (int j = 0; j < kMaxCols + 2; ++j) f.v[j] = j < ncols ? sc_host[j] : 1.0;
    return finalize_scaled(partials, nb, ncols + 2, f, out_dev, s);
}

hipError_t launch_update_project(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c_dev,
                                 const double *sc_host, const double *d_host, const void *p, bool p_f32, double sp,
                                 double *out, float *out32, double *partials, double *out_dev, hipStream_t s,
                                 const float *Q32) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    SmallVec sc, d;
    for (int j = 0; j < 64; ++j) {
        sc.v[j] = j < ncols ? sc_host[j] : 0.0;
        d.v[j] = j < ncols ? d_host[j] : 0.0;
    }
    if (p_f32 && Q32)
        PD_DISPATCH_COLS_T(ncols, float PD_COMMA true, update_project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld,
                           ncols, dim, c_dev, sc, d, static_cast<const float *>(p), sp, out, out32, partials, Q32);
    else if (p_f32)
        PD_DISPATCH_COLS_T(ncols, float PD_COMMA false, update_project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld,
                           ncols, dim, c_dev, sc, d, static_cast<const float *>(p), sp, out, out32, partials, Q32);
    else if (Q32)
        PD_DISPATCH_COLS_T(ncols, double PD_COMMA true, update_project_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld,
                           ncols, dim, c_dev, sc, d, static_cast<const double *>(p), sp, out, out32, partials, Q32);
    else
        PD_DISPATCH_COLS_T(ncols, double PD_COMMA false, update_project_kernel, dim3(nb), dim3(kThreads), 0, s, Q,
                           ld, ncols, dim, c_dev, sc, d, static_cast<const double *>(p), sp, out, out32, partials,
                           Q32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ScaleVec f;
    for (int j = 0; j < kMaxCols + 2; ++j) f.v[j] = j < ncols ? sc_host[j] : 1.0;
    return finalize_scaled(partials, nb, ncols + 1, f, out_dev, s);
}

hipError_t launch_update_norm(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c_dev,
                              const double *sc_host, double *v, float *out32, double *partials, double *nrm2_dev,
                              hipStream_t s, const float *Q32) {
    if (!v && !out32) return hipErrorInvalidValue;
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    unsigned nb = grid_for(dim);
    SmallVec sc;
    for (int j = 0; j < 64; ++j) sc.v[j] = j < ncols ? sc_host[j] : 0.0;
    if (Q32)
        PD_DISPATCH_COLS_B(ncols, true, update_norm_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, c_dev,
                           sc, v, out32, partials, Q32);
    else
        PD_DISPATCH_COLS_B(ncols, false, update_norm_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim,
                           c_dev, sc, v, out32, partials, Q32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, 1, 1.0, nrm2_dev, s);
}

hipError_t launch_combine_many(double *Q, int64_t ld, int ncols, int k, int64_t dim, const double *Y_dev, int zcol,
                               double zs, hipStream_t s) {
    if (ncols < 1 || ncols > kMaxCols || k < 1 || k > kMaxCols || zcol > kMaxCols || (zcol >= 0 && zcol < k))
        return hipErrorInvalidValue;
    const unsigned nb = grid_for(dim);
    PD_DISPATCH_COLS(ncols, combine_many_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, k, dim, Y_dev, zcol,
                     zs);
    return hipGetLastError();
}

hipError_t launch_combine(const double *Q, int64_t ld, int ncols, int64_t dim, const double *y_host, double *out,
                          double *partials, double *nrm2_dev, double *sum_dev, hipStream_t s, const float *Q32) {
    if (ncols < 1 || ncols > kMaxCols) return hipErrorInvalidValue;
    SmallVec y;
    for (int j = 0; j < kMaxCols; ++j) y.v[j] = j < ncols ? y_host[j] : 0.0;
    unsigned nb = grid_for(dim);
    if (Q32)
        PD_DISPATCH_COLS_B(ncols, true, combine_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, y, out,
                           partials, Q32);
    else
        PD_DISPATCH_COLS_B(ncols, false, combine_kernel, dim3(nb), dim3(kThreads), 0, s, Q, ld, ncols, dim, y, out,
                           partials, Q32);
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
                              hipStream_t s, const TruncSpace *tr) {
    unsigned nb = grid_for(dim);
    const uint32_t *kr32 = tr && trunc_ranks32(tr->full_dim) ? static_cast<const uint32_t *>(tr->kranks) : nullptr;
    const uint64_t *kr64 = tr && !trunc_ranks32(tr->full_dim) ? static_cast<const uint64_t *>(tr->kranks) : nullptr;
    if (omega <= 32)
        hipLaunchKernelGGL(occupations_kernel<32>, dim3(nb), dim3(kThreads), 0, s, omega, n, dim, psi, partials, kr32,
                           kr64);
    else
        hipLaunchKernelGGL(occupations_kernel<64>, dim3(nb), dim3(kThreads), 0, s, omega, n, dim, psi, partials, kr32,
                           kr64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(partials, nb, omega, 2.0, occ_dev, s);
}

}  // namespace pd
