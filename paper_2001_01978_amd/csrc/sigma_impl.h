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
//   * rank + A for every occupied orbit sits in registers (the pair count NN
//     is a template parameter, so the loops unroll completely), and the
//     suffix-sum differences that B needs, one pair per count of occupied
//     orbits above b, sit in the lane's slots of an LDS array; the lane then
//     takes its own omega - NN empty orbits from the top and, for each, reads
//     its pair of differences, computes all NN targets, issues all NN
//     gathers, then accumulates -- NN loads in flight per lane.  Every lane
//     runs the same number of hop blocks, so the occupation pattern causes no
//     divergence.
//
// Lanes of a wave hold consecutive ranks, which share their high orbits.
// Numbering orbits from the top makes every lane do the same physical hop at
// the same time on those shared orbits, so those gathers hit consecutive
// addresses.
//
// When n > omega - n the kernel works in the complementary space (holes as
// particles, COMP): the state ~s of rank dim-1-k has omega-n pairs, a hop O->E
// of s is the hop E->O of ~s, and V is symmetric, so the same code applies
// with ranks mirrored.  NN = min(n, omega-n) <= 20: a larger value would mean
// dim >= C(42, 21) ~ 5e11, beyond any GPU memory.
//
// Rank arithmetic is modular in R (uint32 whenever dim < 2^32): every target
// lies in [0, dim), so wrap-around in intermediate sums cancels.
#pragma once

#include <algorithm>
#include <type_traits>

#include "pd_internal.h"

namespace pd {
namespace sigma_detail {

constexpr int kThreads = 512;           // default workgroup size (and per-lane slot stride)
constexpr size_t kLdsPerCU = 160 * 1024;
// Dynamic LDS a workgroup may take: the CU's 160 KB less room for the
// kernels' static LDS (the tile index).
constexpr size_t kLdsUsable = kLdsPerCU - 1024;
constexpr int64_t kMaxGrid = 256 * 16;

template <typename R, typename T>
struct Params {
    int omega;
    int nn;        // pairs in the working space (n, or omega - n when mirrored)
    int ks;        // binomial table row stride (nn + 2)
    int64_t dim;
    int64_t ntiles;
    const T *__restrict__ x;
    T *__restrict__ y;
    const T *__restrict__ d;   // omega pair energies
    const T *__restrict__ V;   // omega x omega
    T dsum;                    // sum of d (for the mirrored diagonal)
    unsigned *sched;           // CoefBlock::sched: zero on entry and on exit
    int chunk;                 // tiles per XCD chunk (FP64 products on large spaces), 0: one tile per request
};

// Stages the binomial table C(p, k) * unit (p < omega, k < ks), the couplings and the
// pair energies into LDS; returns the three LDS arrays through the pointers.
template <typename R, typename T>
__device__ __forceinline__ void stage_tables(unsigned char *smem, int omega, int ks, const T *__restrict__ V,
                                             const T *__restrict__ d, R *&Ct, T *&Vs, T *&ds, R unit = 1) {
    Ct = reinterpret_cast<R *>(smem);
    const int ct_elems = omega * ks;
    Vs = reinterpret_cast<T *>(smem + ((ct_elems * (int)sizeof(R) + 15) & ~15));
    ds = Vs + omega * omega;
    for (int i = threadIdx.x; i < ct_elems; i += blockDim.x) {
        int p = i / ks, k = i - p * ks;
        Ct[i] = (R)g_binom.v[p][k] * unit;
    }
    for (int i = threadIdx.x; i < omega * omega; i += blockDim.x) Vs[i] = V[i];
    for (int i = threadIdx.x; i < omega; i += blockDim.x) ds[i] = d[i];
}

template <typename R, typename T>
__host__ __device__ constexpr size_t table_bytes(int omega, int ks) {
    return (((size_t)omega * ks * sizeof(R) + 15) & ~size_t(15)) + ((size_t)omega * omega + omega) * sizeof(T);
}

// Per-lane LDS scratch of sigma_row: 2 (NN + 1) rank words per thread.
template <typename R>
__host__ __device__ constexpr size_t prefix_bytes(int nn, int block) {
    return (size_t)(2 * nn + 2) * block * sizeof(R);
}

// Buffer resource over x for the byte-offset gathers (gfx9-family word 3).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t x_resource(const T *x, int64_t dim) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(x), (short)0, (int)(uint32_t)(dim * (int64_t)sizeof(T)),
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ T buffer_gather(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)byte_off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)byte_off, 0, 0));
}

// Truncated spaces (Sec. 3.5): x and y hold only the kept states.  A hop
// target is still found by its full-space rank; MAP turns that rank into the
// target's row, or drops the hop when the target was truncated away:
//   MAP 1: one 16-byte word per 64 full ranks (kept bits, kept count before
//          the word): row = base + popcount(bits below the rank);
//   MAP 2: binary search over the ascending kept ranks (the paper's search
//          for truncated spaces), all NN searches of a hop block in lockstep.
template <typename R>
struct TruncMap {
    const R *kranks = nullptr;
    const TruncWord *words = nullptr;
    int64_t kept = 0;
    int64_t self = 0;   // this row's index in the truncated space
};

template <typename R, typename T, int NN, int MAP>
__device__ __forceinline__ void map_gather(const TruncMap<R> &tm, const T *__restrict__ x, const R (&jt)[NN > 0 ? NN : 1],
                                           T (&xv)[NN > 0 ? NN : 1]) {
    if constexpr (MAP == 1) {
        TruncWord w[NN > 0 ? NN : 1];
#pragma unroll
        for (int r = 0; r < NN; ++r) w[r] = tm.words[(int64_t)(jt[r] >> 6)];
#pragma unroll
        for (int r = 0; r < NN; ++r) {
            const int sh = (int)(jt[r] & 63);
            const uint64_t below = w[r].bits & ((1ull << sh) - 1);
            const bool kept = (w[r].bits >> sh) & 1ull;
            xv[r] = kept ? x[(int64_t)w[r].base + __popcll(below)] : T(0);
        }
    } else {
        int64_t lo[NN > 0 ? NN : 1];
#pragma unroll
        for (int r = 0; r < NN; ++r) lo[r] = 0;
        for (int64_t len = tm.kept; len > 1;) {
            const int64_t half = len >> 1;
#pragma unroll
            for (int r = 0; r < NN; ++r) lo[r] = (tm.kranks[lo[r] + half] < jt[r]) ? lo[r] + half : lo[r];
            len -= half;
        }
#pragma unroll
        for (int r = 0; r < NN; ++r) {
            const int64_t pos = lo[r] + (tm.kranks[lo[r]] < jt[r] ? 1 : 0);
            xv[r] = (pos < tm.kept && tm.kranks[pos] == jt[r]) ? x[pos] : T(0);
        }
    }
}

// (H x)[row] for one row: NN pairs in the working space, COMP = mirrored.
// pre: this workgroup's prefix area of 2 (NN + 1) * pstride words (pstride >=
// blockDim.x); the lane uses entries [i * pstride + threadIdx.x] only.  xr: x_resource of x.
// BUF (32-bit ranks, FP32, dim * sizeof(T) < 2^32 only): every rank quantity is in
// units of sizeof(T) bytes -- Ct holds C(p, k) * sizeof(T) (stage_tables) and
// the lane's rank is scaled once -- so a target rank is directly the byte
// offset of a 32-bit-offset buffer load through xr (no 64-bit address
// arithmetic).  The greedy unranking stays exact: every compared entry is at
// most dim * sizeof(T) < 2^32.
// MAP != 0 (truncated space): row and dim are full-space, x is indexed by
// truncated rows (tm.self for the diagonal, map_gather for the hops).
// ISSUE_ALL: all NN gathers of a hop block are issued before the first of its
// multiply-adds (left to itself the compiler interleaves them four at a time,
// which leaves at most four loads in flight per lane).
template <typename W>
__device__ __forceinline__ int top_bit(W v) {
    if constexpr (sizeof(W) == 4)
        return 31 - __clz((int)v);
    else
        return 63 - __clzll((long long)v);
}

// S32: omega <= 32, so the state fits a 32-bit word and every bit scan and
// update is one instruction (measured 4% faster in FP32 and 1.4% in FP64 at
// 32 orbits, 17% in FP32 at 28).
template <typename R, typename T, int NN, bool COMP, bool BUF = false, int MAP = 0, bool ISSUE_ALL = false,
          bool S32 = false>
__device__ __forceinline__ T sigma_row(int64_t row, int64_t dim, int omega, int ks, const R *Ct, const T *Vs,
                                       const T *ds, T dsum, const T *__restrict__ x, R *pre, int pstride,
                                       __amdgpu_buffer_rsrc_t xr, const TruncMap<R> &tm = TruncMap<R>()) {
    using W = typename std::conditional<S32, uint32_t, uint64_t>::type;   // the state word
    static_assert(!(BUF && MAP), "byte-offset gathers index the full space");
    constexpr R U = BUF ? (R)sizeof(T) : (R)1;   // rank unit
    const R rk = (COMP ? (R)(dim - 1 - row) : (R)row) * U;

    // state of rank rk: greedy, orbits from the top.  With 32-bit ranks every
    // lane runs over all omega orbits (once the NN pairs are placed rem is 0
    // and C(p, 0) > 0 is never taken), so the loop needs no per-lane exit
    // test; the 64-bit-rank kernels keep the exit (without it the compiler
    // gave their mirrored forms ~80 more VGPRs).
    W s = 0;
    {
        R rem = rk;
        int k = NN;
        if constexpr (sizeof(R) == 4) {
            for (int p = omega - 1; p >= 0; --p) {
                const R c = Ct[p * ks + k];
                const bool take = c <= rem;
                rem -= take ? c : (R)0;
                k -= take ? 1 : 0;
                s |= take ? ((W)1 << p) : (W)0;
            }
        } else {
            for (int p = omega - 1; p >= 0 && k > 0; --p) {
                const R c = Ct[p * ks + k];
                if (c <= rem) {
                    s |= (W)1 << p;
                    rem -= c;
                    --k;
                }
            }
        }
    }

    // Occupied orbits numbered from the top (r = 0 highest).  rup/rdn: rank
    // plus the removed-orbit term of an up / down hop.  The suffix-sum
    // differences seen by an empty orbit with A occupied orbits above it,
    //   D0[A] = S_0 - S_m  and  D1[A] = S_p - S_0  (sums over those A orbits),
    // go to the lane's LDS slots, where each empty orbit reads its own A.
    R rup[NN > 0 ? NN : 1], rdn[NN > 0 ? NN : 1];
    int apos[NN > 0 ? NN : 1];
    T dacc = T(0);
    const int lane = threadIdx.x;
    {
        W occ = s;
        R s0 = 0, sm = 0, sp = 0;
#pragma unroll
        for (int r = 0; r < NN; ++r) {
            const int a = top_bit(occ);
            occ &= ~((W)1 << a);
            const int j = NN - r;
            const R c0 = Ct[a * ks + j], cm = Ct[a * ks + j - 1], cp = Ct[a * ks + j + 1];
            pre[r * pstride + lane] = s0 - sm;
            pre[(NN + 1 + r) * pstride + lane] = sp - s0;
            rup[r] = rk + (sm - s0 - c0);
            rdn[r] = rk + (s0 - sp - cp);
            apos[r] = a;
            s0 += c0;
            sm += cm;
            sp += cp;
            dacc += ds[a];
        }
        pre[NN * pstride + lane] = s0 - sm;
        pre[(2 * NN + 1) * pstride + lane] = sp - s0;
    }
    // Mirrored space: element dim - 1 - rank; fold the mirror into rup/rdn.
    if (COMP) {
#pragma unroll
        for (int r = 0; r < NN; ++r) {
            rup[r] = (R)(dim - 1) * U - rup[r];
            rdn[r] = (R)(dim - 1) * U - rdn[r];
        }
    }

    T acc = (COMP ? (dsum - dacc) : dacc) * x[MAP ? tm.self : row];
    if (NN == 0) return acc;
    // Every lane walks its own omega - NN empty orbits from the top, so all
    // lanes run the same number of hop blocks (no divergence on the
    // occupation pattern).  The e-th empty orbit b has A = (omega-1-b) - e
    // occupied orbits above it.
    const W full = omega >= (int)(8 * sizeof(W)) ? ~(W)0 : (((W)1 << omega) - 1);
    W E = ~s & full;
    const int ne = omega - NN;
    for (int e = 0; e < ne; ++e) {
        const int b = top_bit(E);
        E &= ~((W)1 << b);
        const int A = (omega - 1 - b) - e;
        const int t = NN - A;
        const R bup = pre[A * pstride + lane] + Ct[b * ks + t];
        const R bdn = pre[(NN + 1 + A) * pstride + lane] + Ct[b * ks + t + 1];
        const T *Vrow = Vs + b * omega;
        T xv[NN > 0 ? NN : 1];
        if constexpr (MAP == 0) {
#pragma unroll
            for (int r = 0; r < NN; ++r) {
                // r < A: a_r above b (down hop); otherwise below (up hop)
                const R jt = COMP ? ((r < A) ? (R)(rdn[r] - bdn) : (R)(rup[r] - bup))
                                  : ((r < A) ? (R)(rdn[r] + bdn) : (R)(rup[r] + bup));
                if constexpr (BUF)
                    xv[r] = buffer_gather<T>(xr, (uint32_t)jt);
                else
                    xv[r] = x[(int64_t)jt];
            }
            if constexpr (ISSUE_ALL) __builtin_amdgcn_sched_barrier(0);
        } else {
            R jt[NN > 0 ? NN : 1];
#pragma unroll
            for (int r = 0; r < NN; ++r)
                jt[r] = COMP ? ((r < A) ? (R)(rdn[r] - bdn) : (R)(rup[r] - bup))
                             : ((r < A) ? (R)(rdn[r] + bdn) : (R)(rup[r] + bup));
            map_gather<R, T, NN, MAP>(tm, x, jt, xv);
        }
#pragma unroll
        for (int r = 0; r < NN; ++r) acc += Vrow[apos[r]] * xv[r];
    }
    return acc;
}

// With at most 17 pairs the product keeps all NN gathers of a hop block in
// flight (ISSUE_ALL).  32-bit ranks: within 128 VGPRs, so 4 waves per SIMD,
// the occupancy the LDS allows (measured at 32 and 34 orbits: 6-11% faster in
// FP64, 7-9% in FP32; mirrored, 32 orbits and 17 pairs: 91.6 -> 79.8 ms
// FP64).  The mirrored FP64 kernel at 16 pairs spills 20-24 bytes per lane
// there; a copy of it outside the library ran 34 orbits, 18 pairs in 363
// against 515 ms, but the library's spaces that use it are refused
// (sigma_space_refused: an unexplained illegal memory access).  64-bit ranks: 3 waves
// per SIMD, without spills when not mirrored (35 orbits, 17 pairs: 1557 ->
// 1348 ms FP64, 803 -> 700 ms FP32); mirrored they spill up to 188 bytes per
// lane and ran 2.3-3.2x slower, so they keep the compiler's schedule.
template <typename R, bool COMP, int NN>
constexpr bool sigma_issue_all() {
    return NN <= 17 && (sizeof(R) == 4 || !COMP);
}
template <typename R, bool COMP, int NN>
constexpr int sigma_min_waves() {
    return sigma_issue_all<R, COMP, NN>() ? (sizeof(R) == 4 ? 4 : 3) : 1;
}

// FP64 products take tiles in per-XCD chunks (see the scheduler in sigma_kernel).
template <typename T>
constexpr bool sigma_xcd_chunks() {
    return sizeof(T) == 8;
}
constexpr int kMaxXcdChunk = 128;
constexpr int kMinXcdChunk = 16;

template <typename R, typename T, int NN, bool COMP, int BLOCK, bool BUF>
__global__ __launch_bounds__(BLOCK, (sigma_min_waves<R, COMP, NN>())) void sigma_kernel(Params<R, T> P) {
    constexpr bool kIssueAll = sigma_issue_all<R, COMP, NN>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int omega = P.omega, ks = P.ks;
    R *Ct;
    T *Vs, *ds;
    stage_tables<R, T>(smem, omega, ks, P.V, P.d, Ct, Vs, ds, BUF ? (R)sizeof(T) : (R)1);
    R *pre = reinterpret_cast<R *>(smem + ((table_bytes<R, T>(omega, ks) + 15) & ~size_t(15)));
    __syncthreads();
    const __amdgpu_buffer_rsrc_t xr = x_resource<T>(P.x, P.dim);   // used by the BUF gathers only

    const int64_t dim = P.dim;
    if (P.ntiles >= (int64_t)gridDim.x) {
        // Tiles are handed out in rank order, so the tiles in flight at any
        // moment are the most recently issued ones: one contiguous window of
        // ranks over the whole chip, whose hops gather from the same regions
        // of x (a static stride lets workgroups drift apart over hundreds of
        // tiles and spreads the window; one counter per XCD, each over its own
        // eighth of the ranks, keeps eight windows apart, and their targets
        // overflow the Infinity Cache: measured 7% slower in FP64).
        // FP64 on large spaces (P.chunk > 0): the global counter hands out
        // chunks of P.chunk tiles, each to one XCD (workgroup id mod 8 is the
        // XCD), whose workgroups take its tiles in order.  The eight XCDs
        // still share one window, and each XCD's L2 sees contiguous runs of
        // rows, whose nearby hops it then serves itself (4% faster in FP64 at
        // 32 and 34 orbits; FP32 gains nothing and keeps one tile per
        // request).  Small spaces keep one tile per request too: with short
        // chunks the refills come so often that the workgroups waiting on
        // them dominate (chunks of one tile made a 2.7e6-state product 20x
        // slower).
        __shared__ int64_t s_tile;
        const int64_t hi = P.ntiles;
        unsigned long long *xw = reinterpret_cast<unsigned long long *>(P.sched + 16);
        for (;;) {
            if (threadIdx.x == 0) {
                if (sigma_xcd_chunks<T>() && P.chunk > 0) {
                    // xw[xcd] = (global chunk + 1) << 32 | tiles taken from it.
                    // Whoever takes the tile one past its end (or the very
                    // first request) fetches the next chunk and installs it;
                    // requests that arrive meanwhile ask again.
                    const int S = P.chunk;
                    unsigned long long *w = xw + (blockIdx.x & 7);
                    for (;;) {
                        const unsigned long long v = atomicAdd(w, 1ull);
                        const unsigned c = (unsigned)(v >> 32), o = (unsigned)v;
                        if (c != 0 && o < (unsigned)S) {
                            s_tile = (int64_t)(c - 1) * S + o;
                            break;
                        }
                        if (c == 0 ? o == 0 : o == (unsigned)S) {
                            const unsigned g = atomicAdd(&P.sched[0], 1u);
                            atomicExch(w, ((unsigned long long)(g + 1) << 32) | 1ull);
                            s_tile = (int64_t)g * S;
                            break;
                        }
                    }
                } else {
                    s_tile = (int64_t)atomicAdd(&P.sched[0], 1u);
                }
            }
            __syncthreads();
            const int64_t tile = s_tile;
            __syncthreads();
            if (tile >= hi) break;
            const int64_t row = tile * BLOCK + threadIdx.x;
            if (row < dim) {
                if (sizeof(R) == 4 && omega <= 32)
                    P.y[row] = sigma_row<R, T, NN, COMP, BUF, 0, kIssueAll, sizeof(R) == 4>(
                        row, dim, omega, ks, Ct, Vs, ds, P.dsum, P.x, pre, BLOCK, xr);
                else
                    P.y[row] = sigma_row<R, T, NN, COMP, BUF, 0, kIssueAll>(row, dim, omega, ks, Ct, Vs, ds, P.dsum,
                                                                          P.x, pre, BLOCK, xr);
            }
        }
        // The last workgroup to finish clears the counters for the next launch.
        if (threadIdx.x == 0) {
            __threadfence();
            if (atomicAdd(&P.sched[8], 1u) == gridDim.x - 1) {
                atomicExch(&P.sched[0], 0u);
                if constexpr (sigma_xcd_chunks<T>())
                    for (int i = 0; i < 8; ++i) atomicExch(&xw[i], 0ull);
                atomicExch(&P.sched[8], 0u);
                __threadfence();
            }
        }
        return;
    }
    for (int64_t tile = blockIdx.x; tile < P.ntiles; tile += gridDim.x) {
        const int64_t row = tile * BLOCK + threadIdx.x;
        if (row >= dim) continue;
        P.y[row] = sigma_row<R, T, NN, COMP, BUF, 0, kIssueAll>(row, dim, omega, ks, Ct, Vs, ds, P.dsum, P.x, pre,
                                                              BLOCK, xr);
    }
}

// Dynamic LDS limit to set on an instantiation with NN pairs and BLOCK
// threads: the most any omega <= 62 can ask of it (tables plus per-lane
// slots), capped at what a CU holds.  One value per instantiation, so calls
// with different omegas, in any order and from any thread, agree on it.
template <typename R, typename T, int NN, int BLOCK>
constexpr size_t lds_limit() {
    const size_t need = ((table_bytes<R, T>(kMaxOmega, NN + 2) + 15) & ~size_t(15)) + prefix_bytes<R>(NN, BLOCK);
    return need < kLdsUsable ? need : kLdsUsable;
}

template <typename R, typename T, int NN, bool COMP, int BLOCK, bool BUF>
hipError_t launch_block(Params<R, T> P, size_t smem, hipStream_t stream) {
    // More than the default 64 KB of dynamic LDS needs the attribute.
    if (smem > 64 * 1024) {
        constexpr size_t lim = lds_limit<R, T, NN, BLOCK>();
        if (smem > lim) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sigma_kernel<R, T, NN, COMP, BLOCK, BUF>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim);
        if (e != hipSuccess) return e;
    }
    P.ntiles = (P.dim + BLOCK - 1) / BLOCK;
    int64_t grid = P.ntiles < kMaxGrid ? P.ntiles : kMaxGrid;
    if (grid >= 64) grid &= ~int64_t(7);  // a multiple of the XCD count
    // Chunks of up to 128 tiles, at least two per workgroup of the grid;
    // below 16 tiles a chunk (spaces under about 6.7e7 states with 512-row
    // tiles) every request takes one tile from the global counter.
    {
        const int64_t s = std::min<int64_t>(kMaxXcdChunk, P.ntiles / (2 * grid));
        P.chunk = s >= kMinXcdChunk ? (int)s : 0;
    }
    hipLaunchKernelGGL((sigma_kernel<R, T, NN, COMP, BLOCK, BUF>), dim3((unsigned)grid), dim3(BLOCK), smem, stream,
                       P);
    return hipGetLastError();
}

// The launch of a product: threads per workgroup, its dynamic LDS, and the
// LDS limit the kernel then runs under (the instantiation's attribute when
// the LDS exceeds the default 64 KB, else that default).
struct LaunchShape {
    int threads;
    size_t lds;
    size_t limit;
};

// Workgroups of 512 threads unless 256 keeps more waves resident: the LDS of
// a workgroup is the tables plus 2 (NN + 1) rank words per thread, and 160 KB
// per CU must hold whole workgroups.
template <typename R, typename T, int NN>
LaunchShape choose_shape(int omega, int ks) {
    const size_t tables = (table_bytes<R, T>(omega, ks) + 15) & ~size_t(15);
    const size_t s512 = tables + prefix_bytes<R>(NN, 512), s256 = tables + prefix_bytes<R>(NN, 256);
    const size_t waves512 = (kLdsUsable / s512) * 8, waves256 = std::min<size_t>((kLdsUsable / s256) * 4, 16);
    const size_t kDefault = 64 * 1024;
    if (waves256 > waves512) return {256, s256, s256 > kDefault ? lds_limit<R, T, NN, 256>() : kDefault};
    return {512, s512, s512 > kDefault ? lds_limit<R, T, NN, 512>() : kDefault};
}

template <typename R, typename T, int NN, bool COMP>
hipError_t launch_nn(const Params<R, T> &P, hipStream_t stream) {
    const LaunchShape sh = choose_shape<R, T, NN>(P.omega, P.ks);
    // Byte-offset buffer gathers (FP32, every byte offset of x within 32 bits;
    // measured slower than 64-bit global loads for FP64 gathers).
    constexpr bool kCanBuf = sizeof(R) == 4 && sizeof(T) == 4;
    const bool buf = kCanBuf && (uint64_t)P.dim * sizeof(T) < (uint64_t(1) << 32);
    if (sh.threads == 256)
        return buf ? launch_block<R, T, NN, COMP, 256, kCanBuf>(P, sh.lds, stream)
                   : launch_block<R, T, NN, COMP, 256, false>(P, sh.lds, stream);
    return buf ? launch_block<R, T, NN, COMP, 512, kCanBuf>(P, sh.lds, stream)
               : launch_block<R, T, NN, COMP, 512, false>(P, sh.lds, stream);
}

// The shape launch_nn takes for a space with nn pairs in the working space.
template <typename R, typename T>
bool shape_for(int omega, int nn, LaunchShape *out) {
    switch (nn) {
#define PD_NN_CASE(K) \
    case K: *out = choose_shape<R, T, K>(omega, K + 2); return true;
        PD_NN_CASE(0) PD_NN_CASE(1) PD_NN_CASE(2) PD_NN_CASE(3) PD_NN_CASE(4) PD_NN_CASE(5) PD_NN_CASE(6)
        PD_NN_CASE(7) PD_NN_CASE(8) PD_NN_CASE(9) PD_NN_CASE(10) PD_NN_CASE(11) PD_NN_CASE(12) PD_NN_CASE(13)
        PD_NN_CASE(14) PD_NN_CASE(15) PD_NN_CASE(16) PD_NN_CASE(17) PD_NN_CASE(18) PD_NN_CASE(19)
        PD_NN_CASE(20)
#undef PD_NN_CASE
        default: return false;
    }
}

template <typename R, typename T, bool COMP>
hipError_t dispatch_nn(const Params<R, T> &P, hipStream_t stream) {
    switch (P.nn) {
#define PD_NN_CASE(K) \
    case K: return launch_nn<R, T, K, COMP>(P, stream);
        PD_NN_CASE(0) PD_NN_CASE(1) PD_NN_CASE(2) PD_NN_CASE(3) PD_NN_CASE(4) PD_NN_CASE(5) PD_NN_CASE(6)
        PD_NN_CASE(7) PD_NN_CASE(8) PD_NN_CASE(9) PD_NN_CASE(10) PD_NN_CASE(11) PD_NN_CASE(12) PD_NN_CASE(13)
        PD_NN_CASE(14) PD_NN_CASE(15) PD_NN_CASE(16) PD_NN_CASE(17) PD_NN_CASE(18) PD_NN_CASE(19)
        PD_NN_CASE(20)
#undef PD_NN_CASE
        default: return hipErrorInvalidValue;
    }
}

// Truncated space: row i is the state of full rank kranks[i]; static tile
// order (no tile counters, so calls need no stream ordering).
template <typename R, typename T>
struct TruncParams {
    Params<R, T> P;       // P.dim = full dimension, P.ntiles over the kept rows
    const R *kranks;
    const TruncWord *words;
    int64_t kept;
};

template <typename R, typename T, int NN, bool COMP, int BLOCK, int MAP>
__global__ __launch_bounds__(BLOCK) void sigma_trunc_kernel(TruncParams<R, T> Q) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Params<R, T> &P = Q.P;
    const int omega = P.omega, ks = P.ks;
    R *Ct;
    T *Vs, *ds;
    stage_tables<R, T>(smem, omega, ks, P.V, P.d, Ct, Vs, ds);
    R *pre = reinterpret_cast<R *>(smem + ((table_bytes<R, T>(omega, ks) + 15) & ~size_t(15)));
    __syncthreads();
    const __amdgpu_buffer_rsrc_t xr = x_resource<T>(P.x, 1);   // unused (MAP gathers)
    TruncMap<R> tm;
    tm.kranks = Q.kranks;
    tm.words = Q.words;
    tm.kept = Q.kept;
    for (int64_t tile = blockIdx.x; tile < P.ntiles; tile += gridDim.x) {
        const int64_t i = tile * BLOCK + threadIdx.x;
        if (i >= Q.kept) continue;
        tm.self = i;
        P.y[i] = sigma_row<R, T, NN, COMP, false, MAP>((int64_t)Q.kranks[i], P.dim, omega, ks, Ct, Vs, ds, P.dsum,
                                                        P.x, pre, BLOCK, xr, tm);
    }
}

template <typename R, typename T, int NN, bool COMP>
hipError_t launch_trunc_nn(TruncParams<R, T> Q, int mode, hipStream_t stream) {
    constexpr int B = 256;
    const size_t smem = ((table_bytes<R, T>(Q.P.omega, Q.P.ks) + 15) & ~size_t(15)) + prefix_bytes<R>(NN, B);
    const void *fn = mode == kTruncBsearch ? reinterpret_cast<const void *>(&sigma_trunc_kernel<R, T, NN, COMP, B, 2>)
                                           : reinterpret_cast<const void *>(&sigma_trunc_kernel<R, T, NN, COMP, B, 1>);
    if (smem > 64 * 1024) {
        constexpr size_t lim = lds_limit<R, T, NN, B>();
        if (smem > lim) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim);
        if (e != hipSuccess) return e;
    }
    Q.P.ntiles = (Q.kept + B - 1) / B;
    const int64_t grid = Q.P.ntiles < kMaxGrid ? Q.P.ntiles : kMaxGrid;
    if (mode == kTruncBsearch)
        hipLaunchKernelGGL((sigma_trunc_kernel<R, T, NN, COMP, B, 2>), dim3((unsigned)grid), dim3(B), smem, stream, Q);
    else
        hipLaunchKernelGGL((sigma_trunc_kernel<R, T, NN, COMP, B, 1>), dim3((unsigned)grid), dim3(B), smem, stream, Q);
    return hipGetLastError();
}

template <typename R, typename T, bool COMP>
hipError_t dispatch_trunc_nn(const TruncParams<R, T> &Q, int mode, hipStream_t stream) {
    switch (Q.P.nn) {
#define PD_NN_CASE(K) \
    case K: return launch_trunc_nn<R, T, K, COMP>(Q, mode, stream);
        PD_NN_CASE(0) PD_NN_CASE(1) PD_NN_CASE(2) PD_NN_CASE(3) PD_NN_CASE(4) PD_NN_CASE(5) PD_NN_CASE(6)
        PD_NN_CASE(7) PD_NN_CASE(8) PD_NN_CASE(9) PD_NN_CASE(10) PD_NN_CASE(11) PD_NN_CASE(12) PD_NN_CASE(13)
        PD_NN_CASE(14) PD_NN_CASE(15) PD_NN_CASE(16) PD_NN_CASE(17) PD_NN_CASE(18) PD_NN_CASE(19)
        PD_NN_CASE(20)
#undef PD_NN_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename R, typename T>
hipError_t launch_trunc_typed(int omega, int n, const TruncSpace &tr, const T *d, const T *V, T dsum, const T *x,
                              T *y, hipStream_t stream) {
    TruncParams<R, T> Q;
    const bool comp = n > omega - n;
    Q.P.omega = omega;
    Q.P.nn = comp ? omega - n : n;
    Q.P.ks = Q.P.nn + 2;
    Q.P.dim = tr.full_dim;
    Q.P.ntiles = 0;
    Q.P.x = x;
    Q.P.y = y;
    Q.P.d = d;
    Q.P.V = V;
    Q.P.dsum = dsum;
    Q.P.sched = nullptr;
    Q.P.chunk = 0;
    Q.kranks = static_cast<const R *>(tr.kranks);
    Q.words = tr.words;
    Q.kept = tr.kept;
    return comp ? dispatch_trunc_nn<R, T, true>(Q, tr.index_mode, stream)
                : dispatch_trunc_nn<R, T, false>(Q, tr.index_mode, stream);
}

// y = H x with rank type R and value type T.
template <typename R, typename T>
hipError_t launch_typed(int omega, int n, int64_t dim, const T *d, const T *V, T dsum, const T *x, T *y,
                        unsigned *sched, hipStream_t stream) {
    Params<R, T> P;
    const bool comp = n > omega - n;
    P.omega = omega;
    P.nn = comp ? omega - n : n;
    P.ks = P.nn + 2;
    P.dim = dim;
    P.ntiles = (dim + kThreads - 1) / kThreads;
    P.x = x;
    P.y = y;
    P.d = d;
    P.V = V;
    P.dsum = dsum;
    P.sched = sched;
    P.chunk = 0;
    return comp ? dispatch_nn<R, T, true>(P, stream) : dispatch_nn<R, T, false>(P, stream);
}

}  // namespace sigma_detail
}  // namespace pd
