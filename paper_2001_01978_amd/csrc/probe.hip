// Streaming kernels of known byte count: the achievable HBM bandwidth that
// the product and the Lanczos vector passes are measured against.  Each
// kernel moves every element once with 16-byte vector accesses in a
// grid-stride loop (four vectors in flight per lane), so its bytes are exact:
//   read   sum of a               4 n bytes read
//   copy   c = a                  4 n read + 4 n written
//   triad  c = a + s b            8 n read + 4 n written
//   write  c = s                  4 n written
// The nontemporal variants mark the accesses as streaming (no reuse), which
// keeps them from displacing cache lines they will never touch again.
#include <algorithm>

#include "pd_internal.h"

namespace pd {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kProbeUnroll = 4;

template <bool NT>
__device__ __forceinline__ f4 ld4(const f4 *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void st4(f4 *p, f4 v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// n4 = number of 4-float vectors (the entry point takes n as a multiple of 1024 floats).
template <int KIND, bool NT, int kProbeThreads>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(const f4 *__restrict__ a,
                                                              const f4 *__restrict__ b, f4 *__restrict__ c,
                                                              int64_t n4, float s, float *__restrict__ partial) {
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    float acc = 0.0f;
    for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
        f4 va[kProbeUnroll], vb[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            if constexpr (KIND != PD_PROBE_WRITE) va[u] = ld4<NT>(a + i + u * stride);
            if constexpr (KIND == PD_PROBE_TRIAD) vb[u] = ld4<NT>(b + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            if constexpr (KIND == PD_PROBE_READ) acc += (va[u].x + va[u].y) + (va[u].z + va[u].w);
            if constexpr (KIND == PD_PROBE_COPY) st4<NT>(c + i + u * stride, va[u]);
            if constexpr (KIND == PD_PROBE_TRIAD)
                st4<NT>(c + i + u * stride, va[u] + s * vb[u]);
            if constexpr (KIND == PD_PROBE_WRITE) st4<NT>(c + i + u * stride, f4{s, s, s, s});
        }
    }
    for (; i < n4; i += stride) {
        f4 va = f4{0.f, 0.f, 0.f, 0.f}, vb = va;
        if constexpr (KIND != PD_PROBE_WRITE) va = ld4<NT>(a + i);
        if constexpr (KIND == PD_PROBE_TRIAD) vb = ld4<NT>(b + i);
        if constexpr (KIND == PD_PROBE_READ) acc += (va.x + va.y) + (va.z + va.w);
        if constexpr (KIND == PD_PROBE_COPY) st4<NT>(c + i, va);
        if constexpr (KIND == PD_PROBE_TRIAD)
            st4<NT>(c + i, va + s * vb);
        if constexpr (KIND == PD_PROBE_WRITE) st4<NT>(c + i, f4{s, s, s, s});
    }
    if constexpr (KIND == PD_PROBE_READ) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        __shared__ float sh[kProbeThreads / 64];
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int w = 0; w < kProbeThreads / 64; ++w) t += sh[w];
            partial[blockIdx.x] = t;
        }
    }
}

// Launch shapes from a sweep on MI355X (block 256..1024, grid 1K..64K, 1..8
// vectors in flight): reads stream best from 512-thread workgroups on a
// 16K grid, writes and copies from 1024-thread workgroups on a 64K grid.
constexpr int probe_block(int kind) { return kind == PD_PROBE_READ ? 512 : 1024; }
constexpr int64_t probe_max_grid(int kind) { return kind == PD_PROBE_READ ? 16384 : kProbeMaxGrid; }

template <int KIND, bool NT>
hipError_t launch_probe(const float *a, const float *b, float *c, int64_t n, float s, int grid, hipStream_t st) {
    constexpr int B = probe_block(KIND);
    hipLaunchKernelGGL((probe_kernel<KIND, NT, B>), dim3(grid), dim3(B), 0, st, reinterpret_cast<const f4 *>(a),
                       reinterpret_cast<const f4 *>(b), reinterpret_cast<f4 *>(c), n / 4, s, c);
    return hipGetLastError();
}

}  // namespace

int probe_grid(int kind, int64_t n) {
    const int64_t per = (int64_t)probe_block(kind) * kProbeUnroll;
    int64_t g = (n / 4 + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, probe_max_grid(kind)));
}

hipError_t launch_stream_probe(int kind, bool nt, const float *a, const float *b, float *c, int64_t n,
                               hipStream_t st) {
    const int grid = probe_grid(kind, n);
    const float s = 0.5f;
    switch (kind) {
        case PD_PROBE_READ:
            return nt ? launch_probe<PD_PROBE_READ, true>(a, b, c, n, s, grid, st)
                      : launch_probe<PD_PROBE_READ, false>(a, b, c, n, s, grid, st);
        case PD_PROBE_COPY:
            return nt ? launch_probe<PD_PROBE_COPY, true>(a, b, c, n, s, grid, st)
                      : launch_probe<PD_PROBE_COPY, false>(a, b, c, n, s, grid, st);
        case PD_PROBE_TRIAD:
            return nt ? launch_probe<PD_PROBE_TRIAD, true>(a, b, c, n, s, grid, st)
                      : launch_probe<PD_PROBE_TRIAD, false>(a, b, c, n, s, grid, st);
        case PD_PROBE_WRITE:
            return nt ? launch_probe<PD_PROBE_WRITE, true>(a, b, c, n, s, grid, st)
                      : launch_probe<PD_PROBE_WRITE, false>(a, b, c, n, s, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pd
