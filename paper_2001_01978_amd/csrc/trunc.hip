// Truncation of the model space (Sec. 3.5).
//
// When C(omega, n) exceeds a dimension limit, the states with the highest
// diagonal elements (Eq. diagonal) are dropped: the diagonals are counted in
// `bins` equal bins between the smallest and the largest one, the bins are
// accumulated from the bottom, and the kept space is every state whose bin
// lies at or below the last bin at which the running count is still within the
// limit (bin 0 is always kept).  The kept states stay in the basis order.
//
// Every pass enumerates the full space the same way: one thread owns 64
// consecutive ranks, unranks the first (greedy inverse of the hash, Sec. 3.2)
// and steps to the next larger integer with the same popcount for the rest
// (the successor of Alg. conversion), so states are never stored.  A state's
// diagonal is summed over its occupied orbits in ascending order in FP64, and
// its bin is floor((diag - dmin) * scale) clamped to [0, bins).
//
// The map from full rank to kept row is one TruncWord per 64 ranks: the bits
// of the kept ranks and the number of kept ranks before the word (an
// exclusive scan of the bit counts).  The kept ranks are then expanded from
// the words into an ascending array.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int kT = 256;
constexpr int kChunk = 4096;              // histogram bins per partial sum
constexpr int kScanPer = kT * 4;          // map words per scan block
constexpr int64_t kMaxBlocks = 16384;

__device__ __forceinline__ uint64_t unrank_state(int omega, int n, uint64_t r) {
    uint64_t s = 0;
    int m = n;
    for (int p = omega - 1; p >= 0 && m > 0; --p) {
        const uint64_t c = g_binom.v[p][m];
        if (c <= r) {
            s |= 1ull << p;
            r -= c;
            --m;
        }
    }
    return s;
}

// Next larger integer with the same number of set bits (s != 0): the lowest
// run of ones moves its top bit up by one and the rest of the run to the bottom.
__device__ __forceinline__ uint64_t next_state(uint64_t s) {
    const uint64_t r = s + (s & (~s + 1));
    return (((r ^ s) >> 2) >> __builtin_ctzll(s)) | r;
}

// d: the pair energies staged in LDS.
__device__ __forceinline__ int64_t diag_bin(uint64_t s, const double *d, const DiagBins &db) {
    double acc = 0.0;
    for (uint64_t m = s; m; m &= m - 1) acc += d[__builtin_ctzll(m)];
    const double v = floor((acc - db.dmin) * db.scale);
    if (!(v > 0.0)) return 0;
    if (v >= (double)(db.bins - 1)) return db.bins - 1;
    return (int64_t)v;
}

__device__ __forceinline__ void stage_d(const DiagBins &db, int omega, double *d) {
    for (int i = threadIdx.x; i < omega; i += kT) d[i] = db.d[i];
    __syncthreads();
}

__device__ __forceinline__ uint64_t block_incl_scan(uint64_t v, uint64_t *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kT; o <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

inline unsigned blocks_for(int64_t items) {
    int64_t b = (items + kT - 1) / kT;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (unsigned)(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(kT) void zero_kernel(uint64_t *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < count; i += (int64_t)gridDim.x * kT) p[i] = 0;
}

__global__ __launch_bounds__(kT) void hist_kernel(int omega, int n, int64_t full_dim, DiagBins db, uint64_t *hist) {
    __shared__ double d[kMaxOmega];
    stage_d(db, omega, d);
    const int64_t W = (full_dim + 63) / 64;
    for (int64_t w = blockIdx.x * (int64_t)kT + threadIdx.x; w < W; w += (int64_t)gridDim.x * kT) {
        const int64_t r0 = w * 64;
        const int cnt = (int)(full_dim - r0 < 64 ? full_dim - r0 : 64);
        uint64_t s = unrank_state(omega, n, (uint64_t)r0);
        for (int j = 0; j < cnt; ++j) {
            atomicAdd(reinterpret_cast<unsigned long long *>(hist + diag_bin(s, d, db)), 1ull);
            if (j + 1 < cnt) s = next_state(s);
        }
    }
}

__global__ __launch_bounds__(kT) void chunk_sum_kernel(const uint64_t *hist, int64_t bins, uint64_t *partial) {
    __shared__ uint64_t sh[kT];
    const int64_t c0 = blockIdx.x * (int64_t)kChunk;
    uint64_t acc = 0;
    for (int k = threadIdx.x; k < kChunk; k += kT)
        if (c0 + k < bins) acc += hist[c0 + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// One workgroup: the chunk in which the running count first exceeds the
// limit, then the last bin inside it (or before it) still within the limit.
__global__ __launch_bounds__(kT) void find_cut_kernel(const uint64_t *hist, int64_t bins, const uint64_t *partial,
                                                      int64_t nchunks, uint64_t limit, TruncCut *out) {
    __shared__ uint64_t sh[kT];
    __shared__ int64_t s_chunk;
    __shared__ unsigned long long s_best1;   // best candidate bin + 1 (0: none)
    __shared__ uint64_t s_base, s_total, s_kept;
    if (threadIdx.x == 0) {
        s_chunk = -1;
        s_base = 0;
        s_best1 = 0;
    }
    __syncthreads();
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < nchunks; c0 += kT) {
        const int64_t c = c0 + threadIdx.x;
        const uint64_t v = c < nchunks ? partial[c] : 0;
        const uint64_t incl = carry + block_incl_scan(v, sh);
        if (c < nchunks && incl > limit && incl - v <= limit) {
            s_chunk = c;
            s_base = incl - v;
        }
        const uint64_t tot = sh[kT - 1];
        __syncthreads();
        carry += tot;
        if (s_chunk >= 0) break;
    }
    if (threadIdx.x == 0) s_total = carry;
    __syncthreads();
    if (s_chunk < 0) {   // everything within the limit
        if (threadIdx.x == 0) {
            out->cut_bin = bins - 1;
            out->kept = (int64_t)s_total;
        }
        return;
    }
    // 16 consecutive bins per thread
    constexpr int per = kChunk / kT;
    const int64_t b0 = s_chunk * kChunk + (int64_t)threadIdx.x * per;
    uint64_t own = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < bins) own += hist[b0 + k];
    const uint64_t excl = block_incl_scan(own, sh) - own;
    uint64_t cum = s_base + excl;
    int64_t cand = -1;
    uint64_t cand_cum = 0;
    for (int k = 0; k < per; ++k) {
        if (b0 + k >= bins) break;
        cum += hist[b0 + k];
        if (cum <= limit) {
            cand = b0 + k;
            cand_cum = cum;
        }
    }
    __syncthreads();
    if (cand >= 0) atomicMax(&s_best1, (unsigned long long)(cand + 1));
    __syncthreads();
    if (cand >= 0 && (unsigned long long)(cand + 1) == s_best1) s_kept = cand_cum;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_best1 > 0) {
            out->cut_bin = (int64_t)s_best1 - 1;
            out->kept = (int64_t)s_kept;
        } else if (s_chunk > 0) {   // the chunk's first bin already exceeds: cut before it
            out->cut_bin = s_chunk * kChunk - 1;
            out->kept = (int64_t)s_base;
        } else {                    // bin 0 alone exceeds the limit: keep bin 0
            out->cut_bin = 0;
            out->kept = (int64_t)hist[0];
        }
    }
}

__global__ __launch_bounds__(kT) void mark_kernel(int omega, int n, int64_t full_dim, DiagBins db, int64_t cut,
                                                  TruncWord *words) {
    __shared__ double d[kMaxOmega];
    stage_d(db, omega, d);
    const int64_t W = (full_dim + 63) / 64;
    for (int64_t w = blockIdx.x * (int64_t)kT + threadIdx.x; w < W; w += (int64_t)gridDim.x * kT) {
        const int64_t r0 = w * 64;
        const int cnt = (int)(full_dim - r0 < 64 ? full_dim - r0 : 64);
        uint64_t s = unrank_state(omega, n, (uint64_t)r0);
        uint64_t bits = 0;
        for (int j = 0; j < cnt; ++j) {
            if (diag_bin(s, d, db) <= cut) bits |= 1ull << j;
            if (j + 1 < cnt) s = next_state(s);
        }
        TruncWord t;
        t.bits = bits;
        t.base = (uint64_t)__popcll(bits);
        words[w] = t;
    }
}

// Exclusive scan of words[].base: per block, then the block totals (one
// workgroup), then the block offsets added back.
__global__ __launch_bounds__(kT) void scan_local_kernel(TruncWord *words, int64_t W, uint64_t *block_tot) {
    __shared__ uint64_t sh[kT];
    const int64_t w0 = blockIdx.x * (int64_t)kScanPer + (int64_t)threadIdx.x * 4;
    uint64_t c[4], sum = 0;
    for (int k = 0; k < 4; ++k) {
        c[k] = w0 + k < W ? words[w0 + k].base : 0;
        sum += c[k];
    }
    const uint64_t incl = block_incl_scan(sum, sh);
    uint64_t run = incl - sum;
    for (int k = 0; k < 4; ++k) {
        if (w0 + k < W) words[w0 + k].base = run;
        run += c[k];
    }
    if (threadIdx.x == kT - 1) block_tot[blockIdx.x] = incl;
}

__global__ __launch_bounds__(kT) void scan_tot_kernel(uint64_t *block_tot, int64_t nb) {
    __shared__ uint64_t sh[kT];
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kT) {
        const int64_t c = c0 + threadIdx.x;
        const uint64_t v = c < nb ? block_tot[c] : 0;
        const uint64_t incl = block_incl_scan(v, sh);
        if (c < nb) block_tot[c] = carry + incl - v;
        const uint64_t tot = sh[kT - 1];
        __syncthreads();
        carry += tot;
    }
}

__global__ __launch_bounds__(kT) void scan_add_kernel(TruncWord *words, int64_t W, const uint64_t *block_tot) {
    const uint64_t off = block_tot[blockIdx.x];
    const int64_t w0 = blockIdx.x * (int64_t)kScanPer + (int64_t)threadIdx.x * 4;
    for (int k = 0; k < 4; ++k)
        if (w0 + k < W) words[w0 + k].base += off;
}

// kranks holds `cap` entries; a selection that keeps more (a caller's info
// that does not match the cut) writes none past it and is rejected afterwards.
template <typename R>
__global__ __launch_bounds__(kT) void ranks_kernel(const TruncWord *words, int64_t W, R *kranks, uint64_t cap) {
    for (int64_t w = blockIdx.x * (int64_t)kT + threadIdx.x; w < W; w += (int64_t)gridDim.x * kT) {
        const TruncWord t = words[w];
        uint64_t bits = t.bits, pos = t.base;
        while (bits) {
            const int j = __builtin_ctzll(bits);
            bits &= bits - 1;
            if (pos < cap) kranks[pos] = (R)(w * 64 + j);
            ++pos;
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kT) void widen_kernel(const R *in, int64_t count, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < count; i += (int64_t)gridDim.x * kT)
        out[i] = (int64_t)in[i];
}

}  // namespace

size_t trunc_hist_doubles(int64_t bins) { return (size_t)bins + (size_t)((bins + kChunk - 1) / kChunk) + 2; }

hipError_t launch_trunc_cut(int omega, int n, int64_t full_dim, const DiagBins &db, int64_t limit, uint64_t *hist,
                            uint64_t *partial, TruncCut *cut_dev, hipStream_t s) {
    const int64_t nchunks = (db.bins + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(db.bins)), dim3(kT), 0, s, hist, db.bins);
    const int64_t W = (full_dim + 63) / 64;
    hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(W)), dim3(kT), 0, s, omega, n, full_dim, db, hist);
    hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)nchunks), dim3(kT), 0, s, (const uint64_t *)hist, db.bins,
                       partial);
    hipLaunchKernelGGL(find_cut_kernel, dim3(1), dim3(kT), 0, s, (const uint64_t *)hist, db.bins,
                       (const uint64_t *)partial, nchunks, (uint64_t)limit, cut_dev);
    return hipGetLastError();
}

size_t trunc_scan_words(int64_t full_dim) {
    const int64_t W = (full_dim + 63) / 64;
    return (size_t)((W + kScanPer - 1) / kScanPer);
}

hipError_t launch_trunc_build(int omega, int n, int64_t full_dim, const DiagBins &db, int64_t cut_bin,
                              TruncWord *words, uint64_t *scan_tmp, void *kranks, int64_t cap, hipStream_t s) {
    const int64_t W = (full_dim + 63) / 64;
    const int64_t nb = (int64_t)trunc_scan_words(full_dim);
    hipLaunchKernelGGL(mark_kernel, dim3(blocks_for(W)), dim3(kT), 0, s, omega, n, full_dim, db, cut_bin, words);
    hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nb), dim3(kT), 0, s, words, W, scan_tmp);
    hipLaunchKernelGGL(scan_tot_kernel, dim3(1), dim3(kT), 0, s, scan_tmp, nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(kT), 0, s, words, W, (const uint64_t *)scan_tmp);
    if (trunc_ranks32(full_dim))
        hipLaunchKernelGGL(ranks_kernel<uint32_t>, dim3(blocks_for(W)), dim3(kT), 0, s, (const TruncWord *)words, W,
                           static_cast<uint32_t *>(kranks), (uint64_t)cap);
    else
        hipLaunchKernelGGL(ranks_kernel<uint64_t>, dim3(blocks_for(W)), dim3(kT), 0, s, (const TruncWord *)words, W,
                           static_cast<uint64_t *>(kranks), (uint64_t)cap);
    return hipGetLastError();
}

hipError_t launch_trunc_ranks64(const TruncSpace &tr, int64_t *out, hipStream_t s) {
    if (tr.kept <= 0) return hipSuccess;
    if (trunc_ranks32(tr.full_dim))
        hipLaunchKernelGGL(widen_kernel<uint32_t>, dim3(blocks_for(tr.kept)), dim3(kT), 0, s,
                           static_cast<const uint32_t *>(tr.kranks), tr.kept, out);
    else
        hipLaunchKernelGGL(widen_kernel<uint64_t>, dim3(blocks_for(tr.kept)), dim3(kT), 0, s,
                           static_cast<const uint64_t *>(tr.kranks), tr.kept, out);
    return hipGetLastError();
}

}  // namespace pd
