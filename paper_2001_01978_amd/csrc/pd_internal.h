// Internal declarations of the pairdiag HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <cstddef>
#include <mutex>

#include "pairdiag.h"

namespace pd {

// ---------------------------------------------------------------- binomials
// C(p, k) for 0 <= p, k < 64 with C = 0 for p < k (the paper's extension of
// Eq. extcmn), built at compile time by Pascal's rule.  All values fit uint64.
struct BinomTable {
    uint64_t v[64][64];
    constexpr BinomTable() : v() {
        for (int p = 0; p < 64; ++p) {
            v[p][0] = 1;
            for (int k = 1; k <= p; ++k) v[p][k] = v[p - 1][k - 1] + (k <= p - 1 ? v[p - 1][k] : 0);
        }
    }
};
static constexpr BinomTable kBinomHost{};
static __constant__ BinomTable g_binom = BinomTable();

inline uint64_t binom_host(int p, int k) {
    if (p < 0 || k < 0 || p > 63 || k > 63 || p < k) return 0;
    return kBinomHost.v[p][k];
}

// Coefficient block: pair energies and couplings in FP64 and FP32.
//   d[i] = 2 eps_i + V_ii (diagonal pair energy, Eq. diagonal)
//   V[b*omega + a] = V_ba (Eq. hamiltonian2), V_ii kept but unused by hops
constexpr int kMaxOmega = 62;
struct CoefBlock {
    double d64[64];
    double dsum64;
    double pad0[7];
    float d32[64];
    float dsum32;
    float pad1[15];
    double V64[kMaxOmega * kMaxOmega];
    float V32[kMaxOmega * kMaxOmega];
    // Tile counters of the sigma kernel: [0] the next tile (or chunk of
    // tiles), [8] finished workgroups, [16..31] one 64-bit word per XCD (its
    // current chunk and the tiles taken from it).  Zero between launches (the
    // last workgroup of a launch clears them), so launches that share a block
    // must be stream-ordered.
    uint32_t sched[32];
};
static_assert(offsetof(CoefBlock, sched) % 8 == 0, "the per-XCD words take 64-bit atomics");
constexpr size_t kCoefBytes = (sizeof(CoefBlock) + 255) & ~size_t(255);

// A basis handle carries kSigmaSlots coefficient blocks for pd_sigma, so
// products on several streams can use one handle at once: a call takes a
// block that is idle, or last used on its own stream (stream order protects
// it), and otherwise makes its stream wait for the block's last product.
constexpr int kSigmaSlots = 4;
constexpr size_t kHandleBlockBytes = kSigmaSlots * kCoefBytes;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
pd_status fail(pd_status s, const char *fmt, ...);
const char *last_error();
// PD_EINVAL unless p is device (or managed) memory; with bytes != 0, also
// unless [p, p + bytes) lies inside p's allocation.  No device work.
pd_status check_device_ptr(const void *p, const char *what, size_t bytes = 0);

#define PD_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::pd::fail(PD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Validates (omega, n, eps, V) and packs the coefficient block.
pd_status pack_coefficients(int omega, int n, const double *eps, const double *V, CoefBlock *out);

// ---------------------------------------------------------------- truncated spaces
// Sec. 3.5: a subset of the full (omega, n) space, kept in ascending order.
// Row i of a truncated vector is the state of full rank kranks[i].  The
// rank -> index map is one word per 64 full ranks: which of them are kept,
// and how many kept ranks precede the word.
struct alignas(16) TruncWord {
    uint64_t bits;
    uint64_t base;
};
enum { kTruncBitmap = 0, kTruncBsearch = 1 };
struct TruncSpace {
    int64_t full_dim;
    int64_t kept;
    const void *kranks;       // uint32 when full_dim < 2^32, else uint64
    const TruncWord *words;   // ceil(full_dim / 64)
    int index_mode;           // kTruncBitmap or kTruncBsearch (target index by binary search over kranks)
};
inline bool trunc_ranks32(int64_t full_dim) { return full_dim < (int64_t(1) << 32); }

}  // namespace pd

namespace pd {
// One coefficient block of a handle and what the host knows of its use.
struct SigmaSlot {
    CoefBlock *dev = nullptr;       // device block (coefficients + tile counters)
    CoefBlock host;                 // what dev holds, when has_coef
    int has_coef = 0;
    int used = 0;                   // a product has been issued on it
    hipStream_t last_stream = nullptr;
    hipEvent_t done = nullptr;      // recorded after its last product
};
}  // namespace pd

struct pd_basis_s {
    int omega;
    int n;
    int64_t dim;
    uint64_t *states;        // device, dim entries, or nullptr
    int device;
    pd::SigmaSlot slot[pd::kSigmaSlots];
    unsigned next_slot;      // round-robin victim when every slot is busy elsewhere
    std::mutex mu;           // guards slot[] and next_slot (pd_sigma from several threads)
    int truncated;           // 1: dim = trunc.kept rows of a truncated space
    pd::TruncSpace trunc;
};

namespace pd {

// ---------------------------------------------------------------- launchers
// basis.hip
hipError_t launch_basis_build(int omega, int n, int64_t dim, uint64_t *states, hipStream_t s);
hipError_t launch_basis_rank(int omega, int n, const uint64_t *states, int64_t count,
                             int64_t *ranks, hipStream_t s);
hipError_t launch_basis_unrank(int omega, int n, const int64_t *ranks, int64_t count,
                               uint64_t *states, hipStream_t s);

// Largest min(n, omega - n) sigma handles (register width of its hop loop).
constexpr int kMaxSigmaPairs = 20;
// Full-space products refused: mirrored spaces (n > omega - n) with 16 pairs
// in the working space and 32-bit ranks, i.e. omega 33, 34, 35 with n = omega
// - 16.  Their FP64 kernel (the library's only kernel that uses scratch: it
// spills 20-24 bytes per lane) made an illegal memory access on the device at omega = 34,
// n = 18, and the cause is not found: the row code, compiled for the host with
// every array it reads against an inaccessible page, touches nothing outside
// them on any row of the three spaces, so what remains is the compiled kernel
// or its launch.  They stay refused until the cause is shown.  Truncated
// products are not affected.
inline bool sigma_space_refused(int omega, int n) {
    const int nn = omega - n;
    return n > nn && nn == 16 && binom_host(omega, n) < (uint64_t(1) << 32);
}
// sigma.hip: y = H x for dtype dt using coefficients at coef (device).
// dsum64/dsum32: sum of all pair energies d_i (host copy of the block's dsum).
// tr: nullptr for the full space, else the truncated space (dim = tr->kept).
// Threads per workgroup, dynamic LDS and LDS limit of the product on a space
// (false when min(n, omega - n) has no kernel).
bool sigma_launch_shape(int omega, int n, pd_dtype dt, int *threads, int64_t *lds, int64_t *limit);
hipError_t launch_sigma(int omega, int n, int64_t dim, const CoefBlock *coef, pd_dtype dt,
                        const void *x, void *y, hipStream_t s, double dsum64, float dsum32,
                        const TruncSpace *tr = nullptr);

// vec.hip: Lanczos vector kernels.  Q holds columns of length dim with leading
// dimension ld (elements).  `partials` is scratch of partial_doubles() doubles.
int vec_grid();
size_t partial_doubles();
// Krylov columns are stored unnormalised: q_j = sc_j * Qt_j, sc_host[j] on the
// host.  p is FP32 (p_f32) or FP64 and stands for pf = sp * p; d_host[j] are
// coefficients of stored columns subtracted first: ps = pf - sum_j d_j Qt_j.
// out_dev[j] = q_j^T ps (j < ncols), out_dev[ncols] = ||ps||^2,
// out_dev[ncols + 1] = ||pf||^2.
// Q32 (all of these): null, or the FP32 store of columns j >= 1 (column j at
// Q32 + (j - 1) ld); column 0 is always FP64 at Q.  With Q32 the first FP32
// column must hold finite values even when ncols == 1 (it is read with weight 0).
hipError_t launch_project(const double *Q, int64_t ld, int ncols, int64_t dim, const void *p, bool p_f32, double sp,
                          const double *sc_host, const double *d_host, double *partials, double *out_dev,
                          hipStream_t s, const float *Q32 = nullptr);
// v = sp p - sum_j (d_j + c_dev[j] sc_j) Qt_j  ->  out (FP64, may be null) and
// out32 (FP32, may be null); out_dev[j] = q_j^T v (j < ncols), out_dev[ncols] =
// ||v||^2, both from the FP64 v.
hipError_t launch_update_project(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c_dev,
                                 const double *sc_host, const double *d_host, const void *p, bool p_f32, double sp,
                                 double *out, float *out32, double *partials, double *out_dev, hipStream_t s,
                                 const float *Q32 = nullptr);
// v -= sum_j c_dev[j] q_j in place (and out32); nrm2_dev[0] = ||v||^2.  With v
// null the vector is FP32 only and is updated in place in out32.
hipError_t launch_update_norm(const double *Q, int64_t ld, int ncols, int64_t dim, const double *c_dev,
                              const double *sc_host, double *v, float *out32, double *partials, double *nrm2_dev,
                              hipStream_t s, const float *Q32 = nullptr);
// Up to 64 doubles passed to a kernel by value.
struct SmallVec {
    double v[64];
};
// Thick restart, in place: Q[o] = sum_{j < ncols} Y_dev[j * k + o] Q[j] for o < k, then
// Q[k] = zs * Q[zcol] if zcol >= 0 (zcol >= k).  Y_dev: device, ncols x k row-major.
hipError_t launch_combine_many(double *Q, int64_t ld, int ncols, int k, int64_t dim, const double *Y_dev, int zcol,
                               double zs, hipStream_t s);
// out = sum_j y[j] Q[j] (j < ncols, y on the host); nrm2_dev[0] = ||out||^2, sum_dev[0] = sum(out).
hipError_t launch_combine(const double *Q, int64_t ld, int ncols, int64_t dim, const double *y_host,
                          double *out, double *partials, double *nrm2_dev, double *sum_dev,
                          hipStream_t s, const float *Q32 = nullptr);
// out = x * scale; optional FP32 copy out32.  out may equal x.
hipError_t launch_scale(const double *x, int64_t dim, double scale, double *out, float *out32,
                        hipStream_t s);
// nrm2/sum of a vector.
hipError_t launch_norm_sum(const double *x, int64_t dim, double *partials, double *nrm2_dev,
                           double *sum_dev, hipStream_t s);
hipError_t launch_fill_random(uint64_t seed, int64_t dim, double *out, hipStream_t s);
hipError_t launch_fill_unit(int64_t dim, int64_t index, double *out, hipStream_t s);
hipError_t launch_copy(const double *x, int64_t dim, double *out, hipStream_t s);
// occ[i] (device, omega doubles) = 2 sum_k psi_k^2 [bit i of state k].
// tr: as for launch_sigma (row k is the state of full rank tr->kranks[k]).
hipError_t launch_occupations(int omega, int n, int64_t dim, const double *psi, double *partials,
                              double *occ_dev, hipStream_t s, const TruncSpace *tr = nullptr);

// trunc.hip: selection of the kept states and construction of the map.
struct TruncCut {
    int64_t cut_bin;   // states whose bin <= cut_bin are kept
    int64_t kept;
};
// Diagonal bins: bin(s) = clamp(floor((diag(s) - dmin) * scale), 0, bins - 1),
// diag(s) = sum of d[q] over the occupied orbits q in ascending order (FP64).
struct DiagBins {
    double d[kMaxOmega];
    double dmin, scale;
    int64_t bins;
};
size_t trunc_hist_doubles(int64_t bins);
hipError_t launch_trunc_cut(int omega, int n, int64_t full_dim, const DiagBins &db, int64_t limit, uint64_t *hist,
                            uint64_t *partial, TruncCut *cut_dev, hipStream_t s);
size_t trunc_scan_words(int64_t full_dim);
constexpr int64_t kMaxTruncBins = int64_t(1) << 30;
// out[i] = kept full rank i as int64.
hipError_t launch_trunc_ranks64(const TruncSpace &tr, int64_t *out, hipStream_t s);
hipError_t launch_trunc_build(int omega, int n, int64_t full_dim, const DiagBins &db, int64_t cut_bin,
                              TruncWord *words, uint64_t *scan_tmp, void *kranks, int64_t cap, hipStream_t s);

// batched.hip
size_t batched_workspace_bytes(int count, const int *omega, const int *n, const pd_lanczos_opts *o);
pd_status batched_validate(int count, const int *omega, const int *n, const pd_lanczos_opts *o);
pd_status batched_run(int count, const int *omega, const int *n, const double *eps_packed, const double *V_packed,
                      const pd_lanczos_opts *o, int block, void *work, size_t work_bytes, double *E0_out,
                      double *occ_out, pd_lanczos_info *info_out, pd_batch_info *binfo, hipStream_t stream);

// mlp.hip
hipError_t launch_gemm_bf16(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                            float *C, int ldc, const float *bias, int epilogue, float *H, hipStream_t s);
hipError_t launch_mlp_loss(int count, const float *logits, const float *target, float *dl, float *partial,
                           float *loss, hipStream_t s);
hipError_t launch_gelu_back(int count, const float *z, float *g, hipStream_t s);
hipError_t launch_colsum(int M, int N, const float *G, float *db, hipStream_t s);
hipError_t launch_adam(int count, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_warm_expand(int omega, int n, int64_t dim, const float *logits, double lmax, double *psi,
                              hipStream_t s);

// probe.hip: streaming kernels of known byte count (achievable HBM bandwidth).
constexpr int kProbeMaxGrid = 65536;
// Workgroups of the streaming kernel `kind` over n floats (the read kernel
// writes one partial sum per workgroup).
int probe_grid(int kind, int64_t n);
hipError_t launch_stream_probe(int kind, bool nontemporal, const float *a, const float *b, float *c, int64_t n,
                               hipStream_t s);

// lanczos.cpp: the static workspace of pd_lanczos_ground_static.  *ptr: its
// device address on the current device (looked up once per device);
// *call_mu: the lock that serialises calls using it on that device.
constexpr size_t kStaticScratchBytes = PD_STATIC_SCRATCH_BYTES;
pd_status static_scratch(void **ptr, std::mutex **call_mu);

// tridiag.cpp: lowest eigenpair of the symmetric tridiagonal (alpha, beta).
int tridiag_lowest(int m, const double *alpha, const double *beta, double *theta, double *y);

}  // namespace pd
