// Lowest eigenpair of the m x m symmetric tridiagonal Lanczos matrix L of
// Alg. lanczos (diagonal alpha, off-diagonal beta), 1 <= m <= 64.  Shared by
// the host driver and the batched device solver.
//
// The paper obtains Ritz pairs by QR iteration (Sec. 3.4).  Only the lowest
// pair is needed, so this uses Sturm-sequence bisection for the eigenvalue
// (the number of negative pivots of L - x I equals the number of eigenvalues
// below x) and inverse iteration with a partially pivoted dense LU of
// L - theta I for the vector; both are backward stable.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace pd {

__host__ __device__ inline int tridiag_count_below(int m, const double *a, const double *b, double x) {
    int cnt = 0;
    double q = a[0] - x;
    const double tiny = 1e-300;
    if (q == 0.0) q = -tiny;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        q = a[i] - x - b[i - 1] * b[i - 1] / q;
        if (q == 0.0) q = -tiny;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// Solves A z = r in place (A dense m x m row-major, destroyed); partial
// pivoting; a pivot below `floor` is replaced by +-floor (A is singular to
// working precision when the shift is an exact eigenvalue, which inverse
// iteration wants).
__host__ __device__ inline void tridiag_dense_solve(int m, double *A, double *r, double floor) {
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int i = c + 1; i < m; ++i)
            if (fabs(A[i * m + c]) > fabs(A[piv * m + c])) piv = i;
        if (piv != c) {
            for (int j = 0; j < m; ++j) {
                double t = A[c * m + j];
                A[c * m + j] = A[piv * m + j];
                A[piv * m + j] = t;
            }
            double t = r[c];
            r[c] = r[piv];
            r[piv] = t;
        }
        double d = A[c * m + c];
        if (fabs(d) < floor) d = A[c * m + c] = (d < 0 ? -floor : floor);
        for (int i = c + 1; i < m; ++i) {
            double f = A[i * m + c] / d;
            if (f == 0.0) continue;
            for (int j = c; j < m; ++j) A[i * m + j] -= f * A[c * m + j];
            r[i] -= f * r[c];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = r[i];
        for (int j = i + 1; j < m; ++j) s -= A[i * m + j] * r[j];
        r[i] = s / A[i * m + i];
    }
}

// theta and unit y with y[0] >= 0 (the Ritz vector keeps q_1's sign).
// A: m*m doubles of scratch, v: m doubles of scratch.  Returns 0 or < 0.
__host__ __device__ inline int tridiag_lowest_work(int m, const double *alpha, const double *beta, double *theta,
                                                   double *y, double *A, double *v) {
    if (m < 1 || m > 64) return -1;
    if (m == 1) {
        *theta = alpha[0];
        y[0] = 1.0;
        return 0;
    }
    double lo = alpha[0], hi = alpha[0], norm = 0.0;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < m - 1 ? fabs(beta[i]) : 0.0);
        lo = fmin(lo, alpha[i] - r);
        hi = fmax(hi, alpha[i] + r);
        norm = fmax(norm, fabs(alpha[i]) + r);
    }
    lo -= 1e-12 * (norm + 1.0);
    hi += 1e-12 * (norm + 1.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (tridiag_count_below(m, alpha, beta, mid) >= 1) hi = mid; else lo = mid;
    }
    const double th = 0.5 * (lo + hi);
    *theta = th;
    for (int i = 0; i < m; ++i) v[i] = (1.0 + 0.01 * i) / sqrt((double)m);
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < m * m; ++i) A[i] = 0.0;
        for (int i = 0; i < m; ++i) {
            A[i * m + i] = alpha[i] - th;
            if (i + 1 < m) A[i * m + i + 1] = A[(i + 1) * m + i] = beta[i];
        }
        tridiag_dense_solve(m, A, v, 2.2e-16 * fmax(norm, 1e-300));
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += v[i] * v[i];
        s = sqrt(s);
        if (!(s > 0.0) || !isfinite(s)) return -2;
        for (int i = 0; i < m; ++i) v[i] /= s;
    }
    const double sg = v[0] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < m; ++i) y[i] = sg * v[i];
    return 0;
}

}  // namespace pd
