/*
 * Plain CPU oracle for the seniority-zero pairing Hamiltonian (PairDiag method).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * Everything here follows the paper's definitions as literally as possible:
 *   - binomial numbers C^m_n with the extension C = 0 for n < m   (Sec. 3.1, Eq. extcmn)
 *   - basis by the '01' inversion iteration                        (Sec. 3.1, Alg. conversion)
 *   - index by binary search over the stored basis                 (Sec. 3.2)
 *   - index by the hash f(|i>) = 1 + sum_j C^j_{O_j - 1}           (Sec. 3.2, Eq. hash)
 *   - diagonal H_ii = sum_n (2 eps_n + V_nn) <i|S+_n S-_n|i>       (Sec. 3.3, Eq. diagonal)
 *   - off-diagonal <i|H|j> = V_EO for |j> = S+_E S-_O |i>          (Sec. 3.3)
 * Indices are 0-based here (paper index minus one).  All arithmetic is FP64.
 *
 * The hash variant of the row loop is the paper's fast path and is the one the
 * CPU baseline times; the binary-search variant is the independent index path
 * used for parity.
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXBITS 64

/* C^m_n of Eq. extcmn as a table cmn[n][m] (n objects, m chosen), built by
 * Pascal's rule; entries with n < m stay 0 (the paper's extension). */
static uint64_t cmn[OR_MAXBITS + 1][OR_MAXBITS + 1];
static int cmn_ready = 0;

static void cmn_init(void)
{
    if (cmn_ready) return;
    memset(cmn, 0, sizeof(cmn));
    for (int n = 0; n <= OR_MAXBITS; ++n) {
        cmn[n][0] = 1;
        for (int m = 1; m <= n; ++m)
            cmn[n][m] = cmn[n - 1][m - 1] + (m <= n - 1 ? cmn[n - 1][m] : 0);
    }
    cmn_ready = 1;
}

/* Eq. extcmn: C^m_n, 0 for n < m. */
uint64_t or_binom(int n, int m)
{
    cmn_init();
    if (n < 0 || m < 0 || n > OR_MAXBITS || m > OR_MAXBITS) return 0;
    if (n < m) return 0;
    return cmn[n][m];
}

/* Alg. conversion ('01' inversion): scan from the lowest bit; each set bit is
 * cleared; if the bit above it is clear, that bit is set and the scan stops;
 * otherwise the cleared bit is collected into the tail (which is refilled from
 * the lowest digit).  The paper prints the loop as i = 0, 2, ..., 61; the text
 * and the worked example need step 1, which is what is done here. */
uint64_t or_next_state(uint64_t in)
{
    uint64_t tail = 0;
    for (int i = 0; i <= 61; ++i) {
        if ((in >> i) & 1ull) {
            in &= ~(1ull << i);
            if (!((in >> (i + 1)) & 1ull)) {
                in |= 1ull << (i + 1);
                break;
            }
            tail = (tail << 1) | 1ull;
        }
    }
    return in + tail;
}

/* Sec. 3.1: start at the minimum 0..01..1 (n pairs in the lowest orbits) and
 * iterate until the maximum 1..10..0 has been produced.  Writes D = C^n_omega
 * states to out (caller sized) and returns the count, or -1 on bad input. */
int64_t or_basis_alg1(int omega, int n, uint64_t *out, int64_t cap)
{
    if (omega < 1 || omega > 62 || n < 0 || n > omega) return -1;
    uint64_t lo = (n == 0) ? 0ull : ((1ull << n) - 1ull);
    uint64_t hi = lo << (omega - n);
    int64_t k = 0;
    uint64_t s = lo;
    for (;;) {
        if (k >= cap) return -1;
        out[k++] = s;
        if (s == hi) break;
        s = or_next_state(s);
    }
    return k;
}

/* Sec. 3.2, Eq. hash: f(|i>) = 1 + sum_{j=1..m} C^j_{O_j - 1}, where O_j is the
 * 1-based orbit number of the j-th occupied bit counted from the lowest.
 * Returned 0-based: f - 1. */
int64_t or_hash(uint64_t s)
{
    cmn_init();
    int64_t f = 1;
    int j = 0;
    for (int orbit = 1; orbit <= 63; ++orbit) {
        if ((s >> (orbit - 1)) & 1ull) {
            ++j;
            f += (int64_t)or_binom(orbit - 1, j);
        }
    }
    return f - 1;
}

/* Inverse of the hash: the state whose f - 1 equals r, in the space of n pairs.
 * Greedy choice of O_n, O_{n-1}, ... as the largest orbit whose term still fits. */
uint64_t or_unhash(int64_t r, int n)
{
    uint64_t s = 0;
    int64_t rem = r;
    int top = 62;
    for (int j = n; j >= 1; --j) {
        int p = top;
        while (p >= 0 && (int64_t)or_binom(p, j) > rem) --p;
        if (p < 0) return ~0ull;
        s |= 1ull << p;
        rem -= (int64_t)or_binom(p, j);
        top = p - 1;
    }
    return rem == 0 ? s : ~0ull;
}

/* Sec. 3.2 binary search over the ascending basis; -1 if absent. */
int64_t or_index_bsearch(const uint64_t *basis, int64_t dim, uint64_t t)
{
    int64_t lo = 0, hi = dim - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (basis[mid] == t) return mid;
        if (basis[mid] < t) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* One row of y = H x (Sec. 3.3).  index_mode 0: binary search in basis;
 * index_mode 1: hash f; index_mode 2: binary search in a truncated basis
 * (Sec. 3.5), where a target that is not found was truncated away and its
 * hop is dropped.  V is omega x omega row-major. */
static double row_value(int omega, const double *eps, const double *V, uint64_t s,
                        const uint64_t *basis, int64_t dim, int index_mode,
                        const double *x, int64_t self, int *bad)
{
    double diag = 0.0;
    for (int i = 0; i < omega; ++i)
        if ((s >> i) & 1ull) diag += 2.0 * eps[i] + V[i * omega + i];
    double acc = diag * x[self];
    for (int O = 0; O < omega; ++O) {
        if (!((s >> O) & 1ull)) continue;
        for (int E = 0; E < omega; ++E) {
            if ((s >> E) & 1ull) continue;
            uint64_t t = (s & ~(1ull << O)) | (1ull << E);   /* S+_E S-_O |s> */
            int64_t j = index_mode == 1 ? or_hash(t) : or_index_bsearch(basis, dim, t);
            if (j < 0 && index_mode == 2) continue;
            if (j < 0 || j >= dim) { *bad = 1; continue; }
            acc += V[E * omega + O] * x[j];
        }
    }
    return acc;
}

/* y[r] = (H x)[r] for rows r in [row0, row1).  Returns 0, or -1 if a hop
 * target was not found (corrupt basis). */
int or_sigma_rows(int omega, int n, const double *eps, const double *V,
                  const uint64_t *basis, int64_t dim, int index_mode,
                  const double *x, double *y, int64_t row0, int64_t row1)
{
    (void)n;
    int bad = 0;
    cmn_init();
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : bad)
    for (int64_t r = row0; r < row1; ++r) {
        int b = 0;
        y[r - row0] = row_value(omega, eps, V, basis[r], basis, dim, index_mode, x, r, &b);
        bad |= b;
    }
    return bad ? -1 : 0;
}

/* Rows chosen by rank without a stored basis: state from the inverse hash,
 * targets from the hash.  For spot checks at sizes whose basis is not kept. */
int or_sigma_sampled(int omega, int n, const double *eps, const double *V,
                     int64_t dim, const double *x, const int64_t *rows, int64_t count,
                     double *y)
{
    int bad = 0;
    cmn_init();
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t q = 0; q < count; ++q) {
        int b = 0;
        uint64_t s = or_unhash(rows[q], n);
        if (s == ~0ull) { bad = 1; y[q] = 0.0; continue; }
        y[q] = row_value(omega, eps, V, s, NULL, dim, 1, x, rows[q], &b);
        bad |= b;
    }
    return bad ? -1 : 0;
}

/* The non-zero terms of row `row` (Sec. 3.3) without a stored basis: returns
 * the diagonal element, writes the n(omega-n) hop targets (hash of Sec. 3.2)
 * and their elements V_EO in the order O ascending, E ascending.  Returns the
 * number of hops in *count (-1 on a bad row). */
double or_row_terms(int omega, int n, const double *eps, const double *V, int64_t row,
                    int64_t *targets, double *coefs, int64_t *count)
{
    cmn_init();
    uint64_t s = or_unhash(row, n);
    if (s == ~0ull) { *count = -1; return 0.0; }
    double diag = 0.0;
    for (int i = 0; i < omega; ++i)
        if ((s >> i) & 1ull) diag += 2.0 * eps[i] + V[i * omega + i];
    int64_t q = 0;
    for (int O = 0; O < omega; ++O) {
        if (!((s >> O) & 1ull)) continue;
        for (int E = 0; E < omega; ++E) {
            if ((s >> E) & 1ull) continue;
            uint64_t t = (s & ~(1ull << O)) | (1ull << E);
            targets[q] = or_hash(t);
            coefs[q] = V[E * omega + O];
            ++q;
        }
    }
    *count = q;
    return diag;
}

/* y[r - r0] = (H x)[r] for r in [r0, r1) the way the paper's program runs:
 * states by the '01' inversion from the block start, targets by the hash.
 * Each thread takes a contiguous chunk and finds its first state from the
 * inverse hash.  Used for CPU timing. */
int or_sigma_block(int omega, int n, const double *eps, const double *V, int64_t dim,
                   const double *x, int64_t r0, int64_t r1, double *y)
{
    int bad = 0;
    cmn_init();
    const int64_t chunk = 16384;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t c0 = r0; c0 < r1; c0 += chunk) {
        int64_t c1 = c0 + chunk < r1 ? c0 + chunk : r1;
        uint64_t s = or_unhash(c0, n);
        if (s == ~0ull) { bad = 1; continue; }
        for (int64_t r = c0; r < c1; ++r) {
            int b = 0;
            y[r - r0] = row_value(omega, eps, V, s, NULL, dim, 1, x, r, &b);
            bad |= b;
            if (r + 1 < c1) s = or_next_state(s);
        }
    }
    return bad ? -1 : 0;
}

/* Explicit dense H (row-major dim x dim), zero-initialised by the caller. */
int or_dense_h(int omega, int n, const double *eps, const double *V,
               const uint64_t *basis, int64_t dim, double *H)
{
    (void)n;
    cmn_init();
    for (int64_t r = 0; r < dim; ++r) {
        uint64_t s = basis[r];
        double diag = 0.0;
        for (int i = 0; i < omega; ++i)
            if ((s >> i) & 1ull) diag += 2.0 * eps[i] + V[i * omega + i];
        H[r * dim + r] = diag;
        for (int O = 0; O < omega; ++O) {
            if (!((s >> O) & 1ull)) continue;
            for (int E = 0; E < omega; ++E) {
                if ((s >> E) & 1ull) continue;
                uint64_t t = (s & ~(1ull << O)) | (1ull << E);
                int64_t j = or_index_bsearch(basis, dim, t);
                if (j < 0) return -1;
                H[r * dim + j] += V[E * omega + O];
            }
        }
    }
    return 0;
}

/* <N_i> = 2 sum_k psi_k^2 [bit i of state k] (Sec. 4.3 output N_Occup). */
void or_occupations(int omega, const uint64_t *basis, int64_t dim, const double *psi,
                    double *occ)
{
    for (int i = 0; i < omega; ++i) occ[i] = 0.0;
    for (int64_t k = 0; k < dim; ++k) {
        double w = psi[k] * psi[k];
        for (int i = 0; i < omega; ++i)
            if ((basis[k] >> i) & 1ull) occ[i] += 2.0 * w;
    }
}

/* ---------------------------------------------------------------- Sec. 3.5
 * Bin of a state's diagonal element (Eq. diagonal, summed over the occupied
 * orbits in ascending order) among `bins` equal bins starting at dmin. */
static int64_t diag_bin(uint64_t s, const double *d, double dmin, double scale, int64_t bins)
{
    double acc = 0.0;
    for (int q = 0; q < 62; ++q)
        if ((s >> q) & 1ull) acc += d[q];
    double v = floor((acc - dmin) * scale);
    if (!(v > 0.0)) return 0;
    if (v >= (double)(bins - 1)) return bins - 1;
    return (int64_t)v;
}

/* Counts of the keys bin >> shift over the whole (omega, n) space, for keys in
 * [lo, lo + len): out[key - lo] (len <= 65536).  Every 64 ranks start from the
 * inverse hash and continue by '01' inversion; counts are per thread, then
 * added. */
int or_trunc_count(int omega, int n, const double *d, double dmin, double scale, int64_t bins, int shift,
                   int64_t lo, int64_t len, uint64_t *out)
{
    if (len < 1 || len > 65536) return -1;
    cmn_init();
    const int64_t dim = (int64_t)or_binom(omega, n), W = (dim + 63) / 64;
    memset(out, 0, (size_t)len * sizeof(uint64_t));
#pragma omp parallel
    {
        uint64_t *mine = (uint64_t *)calloc((size_t)len, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 256)
        for (int64_t w = 0; w < W; ++w) {
            const int64_t r0 = w * 64;
            const int cnt = (int)(dim - r0 < 64 ? dim - r0 : 64);
            uint64_t s = or_unhash(r0, n);
            for (int j = 0; j < cnt; ++j) {
                const int64_t key = diag_bin(s, d, dmin, scale, bins) >> shift;
                if (key >= lo && key < lo + len) mine[key - lo]++;
                if (j + 1 < cnt) s = or_next_state(s);
            }
        }
#pragma omp critical
        for (int64_t k = 0; k < len; ++k) out[k] += mine[k];
        free(mine);
    }
    return 0;
}

/* bits[w] bit j = 1 iff the state of rank 64 w + j lies in a bin <= cut. */
int or_trunc_bits(int omega, int n, const double *d, double dmin, double scale, int64_t bins, int64_t cut,
                  uint64_t *bits)
{
    cmn_init();
    const int64_t dim = (int64_t)or_binom(omega, n), W = (dim + 63) / 64;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t w = 0; w < W; ++w) {
        const int64_t r0 = w * 64;
        const int cnt = (int)(dim - r0 < 64 ? dim - r0 : 64);
        uint64_t s = or_unhash(r0, n), m = 0;
        for (int j = 0; j < cnt; ++j) {
            if (diag_bin(s, d, dmin, scale, bins) <= cut) m |= 1ull << j;
            if (j + 1 < cnt) s = or_next_state(s);
        }
        bits[w] = m;
    }
    return 0;
}

/* Rows of the truncated product for kept full ranks: the row's own index and
 * a target's index are the kept ranks below them (bits plus the exclusive
 * prefix count per word); targets outside the kept space are dropped.
 * Returns -1 if a listed rank is not kept. */
int or_trunc_sigma_sampled(int omega, int n, const double *eps, const double *V, const uint64_t *bits,
                           const int64_t *prefix, const int64_t *ranks, int64_t count, const double *x, double *y)
{
    int bad = 0;
    cmn_init();
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t q = 0; q < count; ++q) {
        const int64_t r = ranks[q];
        if (!((bits[r >> 6] >> (r & 63)) & 1ull)) { bad = 1; y[q] = 0.0; continue; }
        const int64_t self = prefix[r >> 6] + __builtin_popcountll(bits[r >> 6] & ((1ull << (r & 63)) - 1ull));
        const uint64_t s = or_unhash(r, n);
        double diag = 0.0;
        for (int i = 0; i < omega; ++i)
            if ((s >> i) & 1ull) diag += 2.0 * eps[i] + V[i * omega + i];
        double acc = diag * x[self];
        for (int O = 0; O < omega; ++O) {
            if (!((s >> O) & 1ull)) continue;
            for (int E = 0; E < omega; ++E) {
                if ((s >> E) & 1ull) continue;
                const int64_t t = or_hash((s & ~(1ull << O)) | (1ull << E));
                const uint64_t wd = bits[t >> 6];
                if (!((wd >> (t & 63)) & 1ull)) continue;
                acc += V[E * omega + O] * x[prefix[t >> 6] + __builtin_popcountll(wd & ((1ull << (t & 63)) - 1ull))];
            }
        }
        y[q] = acc;
    }
    (void)n;
    return bad ? -1 : 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
