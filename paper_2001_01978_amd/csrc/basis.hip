// Seniority-zero basis on the device (Sec. 3.1-3.2).
//
// The paper generates the ascending list of n-pair bitstrings serially with
// the '01' inversion (Alg. conversion) and notes it does not parallelise.
// Here every 8-state tile is independent: its first state comes from the
// rank by the inverse of the hash of Sec. 3.2 (greedy combinadic), and the
// other seven from the successor rule that Alg. conversion computes (lowest
// '01' pair flipped to '10', the ones below it moved to the bottom), written
// with bit operations.  Tiles are staged in LDS so the HBM writes coalesce.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int kBasisThreads = 256;
constexpr int kBasisPerThread = 8;

__device__ __forceinline__ uint64_t unrank64(uint64_t r, int omega, int n) {
    uint64_t s = 0;
    int k = n;
    for (int p = omega - 1; p >= 0; --p) {
        uint64_t c = g_binom.v[p][k];  // C(p, k); k <= p+1 always holds, C = 0 when p < k
        if (k > 0 && c <= r) {
            s |= 1ull << p;
            r -= c;
            --k;
        }
    }
    return s;
}

// Next larger integer with the same number of set bits: the lowest '01' pair
// becomes '10' (ripple) and the ones that were below it drop to the bottom.
__device__ __forceinline__ uint64_t successor(uint64_t s) {
    uint64_t low = s & (~s + 1ull);  // lowest set bit, 2^(ffs(s)-1)
    uint64_t ripple = s + low;
    uint64_t ones = ((ripple ^ s) >> 2) >> (__ffsll((unsigned long long)s) - 1);
    return ripple | ones;
}

__global__ __launch_bounds__(kBasisThreads) void basis_build_kernel(int omega, int n, int64_t dim,
                                                                    uint64_t *__restrict__ states) {
    __shared__ uint64_t tile[kBasisThreads * kBasisPerThread];
    const int64_t base = (int64_t)blockIdx.x * (kBasisThreads * kBasisPerThread);
    const int64_t r0 = base + (int64_t)threadIdx.x * kBasisPerThread;
    if (r0 < dim) {
        uint64_t s = unrank64((uint64_t)r0, omega, n);
        tile[threadIdx.x * kBasisPerThread] = s;
#pragma unroll
        for (int i = 1; i < kBasisPerThread; ++i) {
            if (r0 + i < dim) {
                s = successor(s);
                tile[threadIdx.x * kBasisPerThread + i] = s;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kBasisPerThread; ++i) {
        int64_t idx = base + (int64_t)i * kBasisThreads + threadIdx.x;
        if (idx < dim) states[idx] = tile[i * kBasisThreads + threadIdx.x];
    }
}

__global__ void basis_rank_kernel(int omega, int n, const uint64_t *__restrict__ states, int64_t count,
                                  int64_t *__restrict__ ranks) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    uint64_t s = states[q];
    bool ok = (__popcll(s) == n) && (omega == 64 || (s >> omega) == 0);
    uint64_t r = 0;
    int j = 0;
    for (int p = 0; p < omega; ++p) {
        if ((s >> p) & 1ull) {
            ++j;
            r += g_binom.v[p][j];
        }
    }
    ranks[q] = ok ? (int64_t)r : -1;
}

__global__ void basis_unrank_kernel(int omega, int n, int64_t dim, const int64_t *__restrict__ ranks,
                                    int64_t count, uint64_t *__restrict__ states) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    int64_t r = ranks[q];
    states[q] = (r >= 0 && r < dim) ? unrank64((uint64_t)r, omega, n) : ~0ull;
}

}  // namespace

hipError_t launch_basis_build(int omega, int n, int64_t dim, uint64_t *states, hipStream_t s) {
    if (dim <= 0) return hipSuccess;
    const int64_t per_block = kBasisThreads * kBasisPerThread;
    int64_t blocks = (dim + per_block - 1) / per_block;
    hipLaunchKernelGGL(basis_build_kernel, dim3((unsigned)blocks), dim3(kBasisThreads), 0, s, omega, n,
                       dim, states);
    return hipGetLastError();
}

hipError_t launch_basis_rank(int omega, int n, const uint64_t *states, int64_t count, int64_t *ranks,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(basis_rank_kernel, dim3((unsigned)blocks), dim3(256), 0, s, omega, n, states, count,
                       ranks);
    return hipGetLastError();
}

hipError_t launch_basis_unrank(int omega, int n, const int64_t *ranks, int64_t count, uint64_t *states,
                               hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t dim = (int64_t)binom_host(omega, n);
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(basis_unrank_kernel, dim3((unsigned)blocks), dim3(256), 0, s, omega, n, dim, ranks,
                       count, states);
    return hipGetLastError();
}

}  // namespace pd
