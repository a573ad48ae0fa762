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
 *   - basis in ascending order (Tab. data, the order of Alg. conversion),
 *     successor = next larger integer with as many set bits       (Sec. 3.1)
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

/* Successor in the basis order.  Sec. 3.1 lists the states of n pairs in
 * ascending order (Tab. data, the order Alg. conversion visits them), so the
 * successor of s is the smallest integer above s with the same number of set
 * bits.  Written from that definition: let the lowest run of ones of s start
 * at bit p and hold L ones.  Any larger number with the same count must set a
 * clear bit above p; the smallest such change sets bit p + L (the first clear
 * bit above the run), clears the run, and puts the L - 1 ones left over on the
 * lowest bits 0 .. L-2.  Returns ~0 when no successor exists below 2^64. */
uint64_t or_next_state(uint64_t s)
{
    if (s == 0) return ~0ull;
    int p = 0;
    while (!((s >> p) & 1ull)) ++p;
    int L = 0;
    while (p + L < 64 && ((s >> (p + L)) & 1ull)) ++L;
    if (p + L >= 64) return ~0ull;
    uint64_t t = s;
    for (int i = p; i < p + L; ++i) t &= ~(1ull << i);
    t |= 1ull << (p + L);
    for (int i = 0; i < L - 1; ++i) t |= 1ull << i;
    return t;
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
 * states by the basis successor from the block start, targets by the hash.
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
 * inverse hash and continue by the basis successor; counts are per thread,
 * then added. */
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

/* Ascending full-space ranks of the kept states (bin <= cut) into out (cap
 * entries); returns their number, or -1 if cap is too small.  Ranks are
 * visited in chunks of 65536: a first pass counts the kept states of every
 * chunk, a running sum gives each chunk its first output position, a second
 * pass writes them.  States by the inverse hash at a chunk start, then the
 * basis successor. */
int64_t or_trunc_kept_ranks(int omega, int n, const double *d, double dmin, double scale, int64_t bins, int64_t cut,
                            int64_t *out, int64_t cap)
{
    cmn_init();
    const int64_t dim = (int64_t)or_binom(omega, n), chunk = 65536, nc = (dim + chunk - 1) / chunk;
    int64_t *start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    if (!start) return -1;
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t r0 = c * chunk, r1 = r0 + chunk < dim ? r0 + chunk : dim;
            int64_t pos = start[c], cnt = 0;
            uint64_t s = or_unhash(r0, n);
            for (int64_t r = r0; r < r1; ++r) {
                if (diag_bin(s, d, dmin, scale, bins) <= cut) {
                    if (pass == 1) out[pos++] = r;
                    ++cnt;
                }
                if (r + 1 < r1) s = or_next_state(s);
            }
            if (pass == 0) start[c + 1] = cnt;
        }
        if (pass == 0) {
            for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
            if (start[nc] > cap) {
                free(start);
                return -1;
            }
        }
    }
    const int64_t kept = start[nc];
    free(start);
    return kept;
}

/* Position of rank t in the ascending array a[0..len), or -1 (Sec. 3.2's
 * binary search, over the kept states of a truncated space as in Sec. 3.5). */
static int64_t find_rank(const int64_t *a, int64_t len, int64_t t)
{
    int64_t lo = 0, hi = len - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] == t) return mid;
        if (a[mid] < t) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Rows of the truncated product (H restricted to the kept states) for the
 * listed kept full ranks.  kept[0..nkept) holds the ascending full ranks of
 * the kept states; x and the rows are indexed by position in it.  The row's
 * own position and every hop target's are found by binary search (target
 * full ranks from the hash); targets not kept are dropped.  Returns -1 if a
 * listed rank is not kept. */
int or_trunc_sigma_sampled(int omega, int n, const double *eps, const double *V, const int64_t *kept,
                           int64_t nkept, const int64_t *ranks, int64_t count, const double *x, double *y)
{
    int bad = 0;
    cmn_init();
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t q = 0; q < count; ++q) {
        const int64_t r = ranks[q];
        const int64_t self = find_rank(kept, nkept, r);
        if (self < 0) { bad = 1; y[q] = 0.0; continue; }
        const uint64_t s = or_unhash(r, n);
        double diag = 0.0;
        for (int i = 0; i < omega; ++i)
            if ((s >> i) & 1ull) diag += 2.0 * eps[i] + V[i * omega + i];
        double acc = diag * x[self];
        for (int O = 0; O < omega; ++O) {
            if (!((s >> O) & 1ull)) continue;
            for (int E = 0; E < omega; ++E) {
                if ((s >> E) & 1ull) continue;
                const int64_t j = find_rank(kept, nkept, or_hash((s & ~(1ull << O)) | (1ull << E)));
                if (j < 0) continue;
                acc += V[E * omega + O] * x[j];
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
