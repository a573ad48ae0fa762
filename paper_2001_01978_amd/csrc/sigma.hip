// Matrix-free y = H x over the seniority-zero basis (Sec. 3.3).
//
// Row k of H has the diagonal of Eq. diagonal and one element V_EO for every
// pair hop |j> = S+_E S-_O |k> (occupied O, empty E), n(omega-n) of them.  The
// paper regenerates these elements on the fly and finds j with the hash of
// Sec. 3.2; here one lane owns one row and finds j without any search:
//
//   * the lane recovers its state from the rank k (greedy inverse of the
//     hash) so no basis array is read;
//   * with occupied positions p_1 < ... < p_n, rank = sum_j C(p_j, j).  A hop
//     a = p_r -> b shifts the indices of the occupied orbits between a and b
//     by one, so the target rank is rank + A(a) + B(b), where A depends only
//     on the removed orbit and B only on the added one (the "up" pair of terms
//     when b > a, the "down" pair when b < a).  Both are differences of suffix
//     sums of binomials over the occupied orbits above a (resp. b):
//         up:   A = S_m(a) - S_0(a) - C(a, r),      B = S_0(b) - S_m(b) + C(b, t)
//         down: A = S_0(a) - S_p(a) - C(a, r+1),    B = S_p(b) - S_0(b) + C(b, t+1)
//     with S_c(q) = sum over occupied p_j > q of C(p_j, j + c) (c = 0, -1, +1)
//     and t = number of occupied orbits below b;
//   * A for every occupied orbit sits in registers (fully unrolled loop); the
//     lane then walks the orbits from the top, updating the suffix sums, and
//     at every empty orbit b issues the n gathers x[rank + A + B] at once.
//
// Lanes of a wave hold consecutive ranks, which share their high orbits.
// Walking and numbering orbits from the top makes every lane do the same
// physical hop at the same time on those shared orbits, so those gathers hit
// consecutive addresses.
//
// When n > omega - n the kernel works in the complementary space (holes as
// particles): the state s^ = ~s of rank dim-1-k has omega-n pairs, a hop O->E
// of s is the hop E->O of s^, and V is symmetric, so the same code applies
// with ranks mirrored.  This keeps the register side at most min(n, omega-n)
// wide; more than 20 would mean dim >= C(42, 21) ~ 5e11, beyond any GPU memory.
//
// Rank arithmetic is modular in R (uint32 whenever dim < 2^32): every target
// lies in [0, dim), so wrap-around in intermediate sums cancels.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int kSigmaThreads = 256;

template <typename R, typename T>
struct SigmaParams {
    int omega;
    int nn;        // pairs in the working space (n, or omega - n when mirrored)
    int comp;      // 1: working space is the complement
    int ks;        // binomial table row stride (nn + 2)
    int64_t dim;
    int64_t ntiles;
    const T *__restrict__ x;
    T *__restrict__ y;
    const T *__restrict__ d;   // omega pair energies
    const T *__restrict__ V;   // omega x omega
    T dsum;                    // sum of d (for the mirrored diagonal)
};

template <typename R, typename T, int MAXO>
__global__ __launch_bounds__(kSigmaThreads) void sigma_kernel(SigmaParams<R, T> P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int omega = P.omega, nn = P.nn, ks = P.ks;
    R *Ct = reinterpret_cast<R *>(smem);
    const int ct_elems = omega * ks;
    T *Vs = reinterpret_cast<T *>(smem + ((ct_elems * (int)sizeof(R) + 15) & ~15));
    T *ds = Vs + omega * omega;

    for (int i = threadIdx.x; i < ct_elems; i += kSigmaThreads) {
        int p = i / ks, k = i - p * ks;
        Ct[i] = (R)g_binom.v[p][k];
    }
    for (int i = threadIdx.x; i < omega * omega; i += kSigmaThreads) Vs[i] = P.V[i];
    for (int i = threadIdx.x; i < omega; i += kSigmaThreads) ds[i] = P.d[i];
    __syncthreads();

    const int64_t dim = P.dim;
    const bool comp = P.comp != 0;
    for (int64_t tile = blockIdx.x; tile < P.ntiles; tile += gridDim.x) {
        const int64_t row = tile * kSigmaThreads + threadIdx.x;
        if (row >= dim) continue;
        const R rk = comp ? (R)(dim - 1 - row) : (R)row;

        // state of rank rk: greedy, orbits from the top
        uint64_t s = 0;
        R rem = rk;
        int k = nn;
        T dacc = T(0);
        for (int p = omega - 1; p >= 0; --p) {
            R c = Ct[p * ks + k];
            if (k > 0 && c <= rem) {
                s |= 1ull << p;
                rem -= c;
                --k;
                dacc += ds[p];
            }
        }

        // removed-orbit terms, occupied orbits numbered from the top
        R Aup[MAXO], Adn[MAXO];
        int apos[MAXO];
        {
            uint64_t occ = s;
            R s0 = 0, sm = 0, sp = 0;
#pragma unroll
            for (int r = 0; r < MAXO; ++r) {
                if (r < nn) {
                    int a = 63 - __clzll((long long)occ);
                    occ &= ~(1ull << a);
                    int j = nn - r;
                    R c0 = Ct[a * ks + j], cm = Ct[a * ks + j - 1], cp = Ct[a * ks + j + 1];
                    Aup[r] = sm - s0 - c0;
                    Adn[r] = s0 - sp - cp;
                    apos[r] = a;
                    s0 += c0;
                    sm += cm;
                    sp += cp;
                } else {
                    Aup[r] = 0;
                    Adn[r] = 0;
                    apos[r] = 0;
                }
            }
        }

        T acc = (comp ? (P.dsum - dacc) : dacc) * P.x[row];
        R s0 = 0, sm = 0, sp = 0;
        int above = 0;
        for (int p = omega - 1; p >= 0; --p) {
            if ((s >> p) & 1ull) {
                int j = nn - above;
                s0 += Ct[p * ks + j];
                sm += Ct[p * ks + j - 1];
                sp += Ct[p * ks + j + 1];
                ++above;
            } else {
                const int t = nn - above;
                const R bup = s0 - sm + Ct[p * ks + t];
                const R bdn = sp - s0 + Ct[p * ks + t + 1];
                const T *Vrow = Vs + p * omega;
#pragma unroll
                for (int r = 0; r < MAXO; ++r) {
                    if (r < nn) {
                        const int a = apos[r];
                        const R jt = rk + ((p > a) ? (R)(Aup[r] + bup) : (R)(Adn[r] + bdn));
                        const int64_t jx = comp ? (dim - 1 - (int64_t)jt) : (int64_t)jt;
                        acc += Vrow[a] * P.x[jx];
                    }
                }
            }
        }
        P.y[row] = acc;
    }
}

template <typename R, typename T, int MAXO>
hipError_t launch_one(const SigmaParams<R, T> &P, hipStream_t stream) {
    size_t ct_bytes = ((size_t)P.omega * P.ks * sizeof(R) + 15) & ~size_t(15);
    size_t smem = ct_bytes + ((size_t)P.omega * P.omega + P.omega) * sizeof(T);
    int64_t grid = P.ntiles;
    const int64_t max_grid = 256 * 16;
    if (grid > max_grid) grid = max_grid;
    hipLaunchKernelGGL((sigma_kernel<R, T, MAXO>), dim3((unsigned)grid), dim3(kSigmaThreads), smem, stream, P);
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t dispatch(const SigmaParams<R, T> &P, hipStream_t stream) {
    const int nn = P.nn;
    if (nn <= 4) return launch_one<R, T, 4>(P, stream);
    if (nn <= 8) return launch_one<R, T, 8>(P, stream);
    if (nn <= 12) return launch_one<R, T, 12>(P, stream);
    if (nn <= 16) return launch_one<R, T, 16>(P, stream);
    if (nn <= 20) return launch_one<R, T, 20>(P, stream);
    return hipErrorInvalidValue;  // rejected by the caller: dim >= C(42, 21)
}

template <typename R, typename T>
hipError_t launch_typed(int omega, int n, int64_t dim, const T *d, const T *V, T dsum, const T *x, T *y,
                        hipStream_t stream) {
    SigmaParams<R, T> P;
    P.omega = omega;
    P.comp = (n > omega - n) ? 1 : 0;
    P.nn = P.comp ? omega - n : n;
    P.ks = P.nn + 2;
    P.dim = dim;
    P.ntiles = (dim + kSigmaThreads - 1) / kSigmaThreads;
    P.x = x;
    P.y = y;
    P.d = d;
    P.V = V;
    P.dsum = dsum;
    return dispatch<R, T>(P, stream);
}

}  // namespace

hipError_t launch_sigma(int omega, int n, int64_t dim, const CoefBlock *coef, pd_dtype dt, const void *x,
                        void *y, hipStream_t s, double dsum64, float dsum32) {
    if (dim <= 0) return hipSuccess;
    const bool small = dim < (int64_t(1) << 32);
    const unsigned char *base = reinterpret_cast<const unsigned char *>(coef);  // device address
    if (dt == PD_F64) {
        const double *d = reinterpret_cast<const double *>(base + offsetof(CoefBlock, d64));
        const double *V = reinterpret_cast<const double *>(base + offsetof(CoefBlock, V64));
        if (small)
            return launch_typed<uint32_t, double>(omega, n, dim, d, V, dsum64, (const double *)x, (double *)y, s);
        return launch_typed<uint64_t, double>(omega, n, dim, d, V, dsum64, (const double *)x, (double *)y, s);
    }
    const float *d = reinterpret_cast<const float *>(base + offsetof(CoefBlock, d32));
    const float *V = reinterpret_cast<const float *>(base + offsetof(CoefBlock, V32));
    if (small) return launch_typed<uint32_t, float>(omega, n, dim, d, V, dsum32, (const float *)x, (float *)y, s);
    return launch_typed<uint64_t, float>(omega, n, dim, d, V, dsum32, (const float *)x, (float *)y, s);
}

}  // namespace pd
