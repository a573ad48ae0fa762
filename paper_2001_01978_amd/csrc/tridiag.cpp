// Lowest eigenpair of the m x m symmetric tridiagonal Lanczos matrix L of
// Alg. lanczos (diagonal alpha, off-diagonal beta), m <= 64.
//
// The paper obtains Ritz pairs by QR iteration (Sec. 3.4).  Only the lowest
// pair is needed, so this uses Sturm-sequence bisection for the eigenvalue
// (the number of negative pivots of L - x I equals the number of eigenvalues
// below x) and inverse iteration with a partially pivoted dense LU of L - theta I
// for the vector; both are backward stable and the result is the same
// eigenpair.
#include <cmath>
#include <cstring>
#include <algorithm>

#include "pd_internal.h"

namespace pd {
namespace {

int count_below(int m, const double *a, const double *b, double x) {
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
// pivoting; a pivot below `floor` is replaced by it (A is singular to working
// precision when the shift is an exact eigenvalue, which inverse iteration wants).
void dense_solve(int m, double *A, double *r, double floor) {
    const double eps = floor;
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int i = c + 1; i < m; ++i)
            if (std::fabs(A[i * m + c]) > std::fabs(A[piv * m + c])) piv = i;
        if (piv != c) {
            for (int j = 0; j < m; ++j) std::swap(A[c * m + j], A[piv * m + j]);
            std::swap(r[c], r[piv]);
        }
        double d = A[c * m + c];
        if (std::fabs(d) < eps) d = A[c * m + c] = (d < 0 ? -eps : eps);
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

}  // namespace

int tridiag_lowest(int m, const double *alpha, const double *beta, double *theta, double *y) {
    if (m < 1 || m > 64) return -1;
    if (m == 1) {
        *theta = alpha[0];
        y[0] = 1.0;
        return 0;
    }
    double lo = alpha[0], hi = alpha[0], norm = 0.0;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(beta[i]) : 0.0);
        lo = std::min(lo, alpha[i] - r);
        hi = std::max(hi, alpha[i] + r);
        norm = std::max(norm, std::fabs(alpha[i]) + r);
    }
    // bisection for the smallest eigenvalue: count_below(lo) = 0 <= count_below(hi)
    lo -= 1e-12 * (norm + 1.0);
    hi += 1e-12 * (norm + 1.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(m, alpha, beta, mid) >= 1) hi = mid; else lo = mid;
    }
    const double th = 0.5 * (lo + hi);
    *theta = th;

    // inverse iteration
    double A[64 * 64];
    double v[64];
    for (int i = 0; i < m; ++i) v[i] = 1.0 / std::sqrt((double)m) * (1.0 + 0.01 * i);
    for (int pass = 0; pass < 3; ++pass) {
        std::memset(A, 0, sizeof(double) * m * m);
        for (int i = 0; i < m; ++i) {
            A[i * m + i] = alpha[i] - th;
            if (i + 1 < m) A[i * m + i + 1] = A[(i + 1) * m + i] = beta[i];
        }
        dense_solve(m, A, v, 2.2e-16 * std::max(norm, 1e-300));
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += v[i] * v[i];
        s = std::sqrt(s);
        if (!(s > 0.0) || !std::isfinite(s)) return -2;
        for (int i = 0; i < m; ++i) v[i] /= s;
    }
    // sign: first component non-negative (the Ritz vector keeps q_1's sign)
    double sg = v[0] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < m; ++i) y[i] = sg * v[i];
    return 0;
}

}  // namespace pd
