// Warm-start network and start-vector expansion.
//
// The network maps an instance (pair energies, couplings) to one logit l_i
// per orbit; sigmoid(l_i) is trained against the half occupation <N_i>/2 of
// the exact ground state.  Reading sigmoid(l) as the BCS occupation v^2 gives
// the pair amplitude v/u = exp(l/2), and projecting that product state onto n
// pairs gives the start vector psi_k ~ prod_{i occupied in k} exp(l_i/2).
//
// Dense layers run on the matrix cores: operands are rounded from FP32 to
// BF16 while tiles are staged in LDS, products accumulate in FP32
// (gfx950's v_mfma_f32_16x16x32_bf16: 32 products per output per
// instruction), and bias / GELU are fused into the store.
#include <cmath>

#include "pd_internal.h"

namespace pd {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
    // round to nearest even on the upper 16 bits (inputs are finite)
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float gelu_tanh(float x) {
    const float c = 0.7978845608028654f;  // sqrt(2/pi)
    return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float gelu_tanh_grad(float x) {
    const float c = 0.7978845608028654f;
    const float t = tanhf(c * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

constexpr int kTile = 64;
constexpr int kK = 32;            // k per MFMA (16x16x32)
constexpr int kRow = kK + 8;      // LDS row of a staged tile: 32 BF16 + 16 bytes of padding

// C = op(A) op(B) (M x N, K inner).  op(A)(m, k) = TA ? A[k*lda + m] : A[m*lda + k];
// op(B)(k, n) = TB ? B[n*ldb + k] : B[k*ldb + n].
// epilogue 0: C = acc; 1: C = acc + bias[n]; 2: Z = acc + bias[n] stored in C, H = gelu(Z).
// A 64 x 64 tile per workgroup, four waves of 32 x 32 (2 x 2 MFMA tiles).  Both
// operands are staged k-contiguous (op(A) as rows m, op(B) transposed as rows
// n), each thread converting 8 consecutive k of one row and storing them as
// one 16-byte LDS write, so every MFMA operand is one 16-byte LDS read: lane l
// takes row (l % 16) of its 16-row slice at k = 8 (l / 16) .. 8 (l / 16) + 7.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                        int ldc, const float *__restrict__ bias, int epilogue,
                                                        float *__restrict__ H) {
    __shared__ __align__(16) short As[kTile][kRow];
    __shared__ __align__(16) short Bs[kTile][kRow];   // Bs[n][k] = op(B)(k, n)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int srow = tid >> 2, sk = (tid & 3) * 8;     // this thread's staging row and k offset
    for (int k0 = 0; k0 < K; k0 += kK) {
        shortx8 av, bv;
        const int gm = m0 + srow, gn = n0 + srow;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int gk = k0 + sk + i;
            float a = 0.f, b = 0.f;
            if (gm < M && gk < K) a = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            if (gn < N && gk < K) b = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
            av[i] = to_bf16(a);
            bv[i] = to_bf16(b);
        }
        *reinterpret_cast<shortx8 *>(&As[srow][sk]) = av;
        *reinterpret_cast<shortx8 *>(&Bs[srow][sk]) = bv;
        __syncthreads();
        const int r = lane & 15, kq = (lane >> 4) * 8;
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const shortx8 *>(&As[wm + i * 16 + r][kq]));
            b[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const shortx8 *>(&Bs[wn + i * 16 + r][kq]));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result: lane holds C[4*(lane/16) + v][lane % 16] of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wm + i * 16 + (lane >> 4) * 4 + v;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    float z = acc[i][j][v];
                    if (epilogue >= 1) z += bias[gn];
                    C[(int64_t)gm * ldc + gn] = z;
                    if (epilogue == 2) H[(int64_t)gm * ldc + gn] = gelu_tanh(z);
                }
            }
}

// loss = mean (sigmoid(l) - t)^2 over B x F; dl = d loss / d l.
__global__ void loss_kernel(int count, const float *__restrict__ logits, const float *__restrict__ target,
                            float *__restrict__ dl, float *__restrict__ partial) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float sg = 1.0f / (1.0f + expf(-logits[i]));
        const float r = sg - target[i];
        s += r * r;
        dl[i] = 2.0f * r * sg * (1.0f - sg) / (float)count;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void sum_partials_kernel(int nb, const float *__restrict__ partial, float scale, float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int b = 0; b < nb; ++b) s += partial[b];
        *out = s * scale;
    }
}

// g *= gelu'(z), elementwise
__global__ void gelu_back_kernel(int count, const float *__restrict__ z, float *__restrict__ g) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        g[i] *= gelu_tanh_grad(z[i]);
}

// db[n] = sum_m G[m*ld + n]
__global__ void colsum_kernel(int M, int N, const float *__restrict__ G, float *__restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += G[(int64_t)m * N + n];
    db[n] = s;
}

// Adam (Kingma & Ba 2015) with bias correction.
__global__ void adam_kernel(int count, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// psi_k = exp(0.5 * (sum_{i occupied in k} l_i - lmax)); lmax = sum of the n largest l.
__global__ void warm_expand_kernel(int omega, int n, int64_t dim, const float *__restrict__ logits, double lmax,
                                   double *__restrict__ psi) {
    __shared__ double l[64];
    if ((int)threadIdx.x < omega) l[threadIdx.x] = (double)logits[threadIdx.x];
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < dim; k += (int64_t)gridDim.x * blockDim.x) {
        uint64_t r = (uint64_t)k;
        int m = n;
        double s = 0.0;
        for (int p = omega - 1; p >= 0; --p) {
            uint64_t c = g_binom.v[p][m];
            if (m > 0 && c <= r) {
                r -= c;
                --m;
                s += l[p];
            }
        }
        psi[k] = exp(0.5 * (s - lmax));
    }
}

}  // namespace mlp

hipError_t launch_gemm_bf16(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                            float *C, int ldc, const float *bias, int epilogue, float *H, hipStream_t s) {
    using namespace mlp;
    dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    if (ta && tb) hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, epilogue, H);
    else if (ta) hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, epilogue, H);
    else if (tb) hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, epilogue, H);
    else hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, epilogue, H);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(int count, const float *logits, const float *target, float *dl, float *partial,
                           float *loss, hipStream_t s) {
    const int nb = 64;
    hipLaunchKernelGGL(mlp::loss_kernel, dim3(nb), dim3(256), 0, s, count, logits, target, dl, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp::sum_partials_kernel, dim3(1), dim3(64), 0, s, nb, partial, 1.0f / (float)count, loss);
    return hipGetLastError();
}

hipError_t launch_gelu_back(int count, const float *z, float *g, hipStream_t s) {
    hipLaunchKernelGGL(mlp::gelu_back_kernel, dim3((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024), dim3(256),
                       0, s, count, z, g);
    return hipGetLastError();
}

hipError_t launch_colsum(int M, int N, const float *G, float *db, hipStream_t s) {
    hipLaunchKernelGGL(mlp::colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, M, N, G, db);
    return hipGetLastError();
}

hipError_t launch_adam(int count, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(mlp::adam_kernel, dim3((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024), dim3(256), 0,
                       s, count, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_warm_expand(int omega, int n, int64_t dim, const float *logits, double lmax, double *psi,
                              hipStream_t s) {
    int64_t g = (dim + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(mlp::warm_expand_kernel, dim3((unsigned)g), dim3(256), 0, s, omega, n, dim, logits, lmax, psi);
    return hipGetLastError();
}

}  // namespace pd
