// Host entry of the tridiagonal eigensolver (algorithm in tridiag.h).
#include "pd_internal.h"
#include "tridiag.h"

namespace pd {

int tridiag_lowest(int m, const double *alpha, const double *beta, double *theta, double *y) {
    double A[64 * 64];
    double v[64];
    return tridiag_lowest_work(m, alpha, beta, theta, y, A, v);
}

}  // namespace pd
