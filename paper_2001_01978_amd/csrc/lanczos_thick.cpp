// Several lowest eigenpairs: thick-restart Lanczos (Wu and Simon), FP64.
//
// The paper needs only the first few states (Sec. 3.4) and restarts from the
// ground-state Ritz vector; several states need a restart that keeps more
// than one vector.  After a cycle of m steps, H Q = Q T + beta_m q_{m+1} e_m^T
// with T the projected matrix.  The k lowest Ritz pairs (theta_i, u_i = Q y_i)
// and q_{m+1} start the next cycle: H u_i = theta_i u_i + s_i q_{m+1} with
// s_i = beta_m (y_i)_m, so the new projected matrix begins as the arrowhead
//     [ diag(theta_1..theta_k)   s ]
//     [ s^T                  alpha ]
// and continues tridiagonally.  Every step is the step of the single-vector
// driver (recurrence terms subtracted before one classical Gram-Schmidt pass
// against all stored vectors, a second pass on the DGKS or rounding test);
// the first step of a cycle subtracts the couplings s_i u_i as well.  The
// projected matrix (at most 64 x 64) is diagonalised on the host by cyclic
// Jacobi rotations; the restart vectors are formed in place, row by row
// (launch_combine_many).
//
// Mixed precision (PD_F32) runs in two phases: thick restart with FP32
// products on FP32 copies of the columns until every wanted estimate is below
// 3e-6 (or, below 1e-4, stops falling), then, since the kept relations carry FP32 errors, a
// fresh FP64 run started from the sum of the wanted Ritz vectors.
//
// A pair counts as converged when its residual estimate
// |beta_m (y_i)_m| / |theta_i| is below tol; the returned values come from an
// explicit FP64 product per wanted vector (Rayleigh quotient and residual
// ||H u - E u|| / |E|, Eq. convergence).  A Krylov space built from one start
// vector holds one vector per distinct eigenvalue, so an exactly degenerate
// level is returned once.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <algorithm>

#include "pd_internal.h"

namespace pd {

namespace {

struct TLayout {
    size_t coef = 0, scal = 0, partials = 0, Y = 0, Q = 0, p = 0, x32 = 0, y32 = 0, total = 0;
    int64_t ld = 0;
    int m = 0;
};

constexpr int kScalars = 512;
constexpr int kOffC = 0, kOffC2 = 80, kOffNrm = 192, kOffSum = 193, kOffOcc = 256;
constexpr double kReorthEta = 0.70710678118654752;
constexpr double kReorthTau = 1.0 / 128.0;
constexpr int kMaxM = 64;

TLayout tlayout(int64_t dim, int krylov, int precision) {
    TLayout L;
    L.m = (int)std::min<int64_t>(krylov, dim);
    L.ld = (dim + 63) & ~int64_t(63);
    size_t off = 0;
    L.coef = off;
    off += kCoefBytes;
    L.scal = off;
    off += align256(kScalars * sizeof(double));
    L.partials = off;
    off += align256(partial_doubles() * sizeof(double));
    L.Y = off;
    off += align256(kMaxM * kMaxM * sizeof(double));
    L.Q = off;
    off += align256((size_t)(L.m + 1) * L.ld * sizeof(double));
    L.p = off;
    off += align256((size_t)L.ld * sizeof(double));
    if (precision == PD_F32) {
        L.x32 = off;
        off += align256((size_t)L.ld * sizeof(float));
        L.y32 = off;
        off += align256((size_t)L.ld * sizeof(float));
    }
    L.total = off;
    return L;
}

// Mixed precision: the FP32 phase ends when every wanted Ritz residual
// estimate is below this (well above the FP32 rounding of the products), or
// when the estimate stops falling.
constexpr double kSwitchTol = 3e-6;

// Eigenvalues (ascending) and eigenvectors (columns of Z, row-major n x n) of
// the symmetric matrix A (row-major) by cyclic Jacobi rotations.
void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; ++r) {   // A = J^T A J, columns p and q
                    const double arp = A[(size_t)r * n + p], arq = A[(size_t)r * n + q];
                    A[(size_t)r * n + p] = c * arp - s * arq;
                    A[(size_t)r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {   // rows p and q
                    const double apr = A[(size_t)p * n + r], aqr = A[(size_t)q * n + r];
                    A[(size_t)p * n + r] = c * apr - s * aqr;
                    A[(size_t)q * n + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < n; ++r) {
                    const double zrp = Z[(size_t)r * n + p], zrq = Z[(size_t)r * n + q];
                    Z[(size_t)r * n + p] = c * zrp - s * zrq;
                    Z[(size_t)r * n + q] = s * zrp + c * zrq;
                }
            }
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
    std::vector<double> Zs((size_t)n * n);
    w.resize(n);
    for (int c = 0; c < n; ++c) {
        w[c] = A[(size_t)order[c] * n + order[c]];
        for (int r = 0; r < n; ++r) Zs[(size_t)r * n + c] = Z[(size_t)r * n + order[c]];
    }
    Z.swap(Zs);
}

struct Dev {
    hipStream_t s;
    double *scal;
    double host[kScalars];
    hipError_t fetch(int off, int count) {
        hipError_t e = hipMemcpyAsync(host + off, scal + off, count * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
};

}  // namespace

int thick_keep(int nev, int m) { return std::min(m - 1, std::max(nev, nev + (m - nev) / 2)); }

size_t lanczos_eigs_workspace_bytes(int64_t dim, const pd_lanczos_opts *o) {
    return tlayout(dim, o->krylov, o->precision).total;
}

pd_status lanczos_eigs_run(pd_basis b, const CoefBlock &host_coef, int nev, const pd_lanczos_opts *o, void *work,
                           size_t work_bytes, double *E_out, double *psi, double *occ_out, double *res_out,
                           pd_lanczos_info *info_out, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const int omega = b->omega, n = b->n;
    const int64_t dim = b->dim;
    const TruncSpace *tr = b->truncated ? &b->trunc : nullptr;
    if (o->precision != PD_F64 && o->precision != PD_F32)
        return fail(PD_EINVAL, "several eigenpairs take precision PD_F64 or PD_F32");
    const TLayout L = tlayout(dim, o->krylov, o->precision);
    if (work_bytes < L.total) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, L.total);
    if (nev < 1 || nev > L.m || (L.m < dim && nev > L.m - 2))
        return fail(PD_EINVAL, "nev=%d needs krylov >= nev + 2 (krylov %d, dim %lld)", nev, o->krylov,
                    (long long)dim);
    unsigned char *base = static_cast<unsigned char *>(work);
    CoefBlock *coef = reinterpret_cast<CoefBlock *>(base + L.coef);
    double *scal = reinterpret_cast<double *>(base + L.scal);
    double *partials = reinterpret_cast<double *>(base + L.partials);
    double *Ydev = reinterpret_cast<double *>(base + L.Y);
    double *Q = reinterpret_cast<double *>(base + L.Q);
    double *p = reinterpret_cast<double *>(base + L.p);
    const bool mixed = o->precision == PD_F32 && o->mode == 0;
    float *x32 = mixed ? reinterpret_cast<float *>(base + L.x32) : nullptr;
    float *y32 = mixed ? reinterpret_cast<float *>(base + L.y32) : nullptr;
    const int64_t ld = L.ld;
    const int m = L.m;
    const int keep = thick_keep(nev, m);
    const double dsum64 = host_coef.dsum64;
    const float dsum32 = host_coef.dsum32;

    pd_lanczos_info info;
    std::memset(&info, 0, sizeof(info));
    {
        std::vector<double> dd(host_coef.d64, host_coef.d64 + omega);
        std::sort(dd.begin(), dd.end());
        double mm = 0.0;
        for (int i = 0; i < n; ++i) mm += dd[i];
        info.monopole_min = mm;
    }
    double dscale = 0.0;
    for (int i = 0; i < omega; ++i) dscale = std::max(dscale, std::fabs(host_coef.d64[i]));
    if (dscale == 0.0) dscale = 1.0;

    PD_HIP(hipMemcpyAsync(coef, &host_coef, sizeof(CoefBlock), hipMemcpyHostToDevice, s));
    PD_HIP(hipStreamSynchronize(s));
    Dev dev{s, scal, {}};

    // ---- start vector into column 0 (p is scratch)
    switch (o->start) {
        case PD_START_E1:
            PD_HIP(launch_fill_unit(dim, 0, p, s));
            break;
        case PD_START_RANDOM:
            PD_HIP(launch_fill_random(o->seed, dim, p, s));
            break;
        default:
            return fail(PD_EINVAL, "several eigenpairs take the E1 or RANDOM start");
    }
    PD_HIP(launch_norm_sum(p, dim, partials, scal + kOffNrm, scal + kOffSum, s));
    PD_HIP(dev.fetch(kOffNrm, 1));
    PD_HIP(launch_scale(p, dim, 1.0 / std::sqrt(dev.host[kOffNrm]), Q, nullptr, s));

    std::vector<double> alpha(m, 0.0), beta(m, 0.0), sc(m + 1, 1.0), d(kMaxM + 2, 0.0);
    std::vector<double> theta(m, 0.0), svec(m, 0.0), w, Z;
    int kk = 0;          // kept Ritz vectors at the start of the cycle
    bool converged = false;
    int cycle = 0, cycles_total = 0;
    // Phase 0 (mixed precision only): FP32 products on FP32 copies of the
    // columns until the estimates reach kSwitchTol.  The stored relations
    // H u_i = theta_i u_i + s_i q then carry FP32 errors, so phase 1 starts an
    // FP64 run afresh from the sum of the wanted Ritz vectors.
    for (int phase = mixed ? 0 : 1; phase < 2; ++phase) {
    const bool f32 = phase == 0;
    const double tol_phase = f32 ? std::max(o->tol, kSwitchTol) : o->tol;
    double best = INFINITY;
    int stall = 0;
    if (phase == 1 && mixed) {
        std::vector<double> ones(kk, 1.0);
        PD_HIP(launch_combine(Q, ld, kk, dim, ones.data(), p, partials, scal + kOffNrm, scal + kOffSum, s));
        PD_HIP(dev.fetch(kOffNrm, 1));
        PD_HIP(launch_scale(p, dim, 1.0 / std::sqrt(dev.host[kOffNrm]), Q, nullptr, s));
        kk = 0;
        std::fill(sc.begin(), sc.end(), 1.0);
        converged = false;
    }
    if (f32) PD_HIP(launch_scale(Q, dim, 1.0, Q, x32, s));
    for (cycle = 0;; ++cycle) {
        int m_eff = m;
        bool breakdown = false;
        for (int j = kk; j < m; ++j) {
            double *qj = Q + (size_t)j * ld;
            if (f32) {
                PD_HIP(launch_sigma(omega, n, dim, coef, PD_F32, x32, y32, s, dsum64, dsum32, tr));
                ++info.iterations_f32;
            } else {
                PD_HIP(launch_sigma(omega, n, dim, coef, PD_F64, qj, p, s, dsum64, dsum32, tr));
            }
            const void *pin = f32 ? static_cast<const void *>(y32) : static_cast<const void *>(p);
            ++info.iterations;
            const double sigma = j > kk ? alpha[j - 1] : (kk > 0 ? theta[0] : 0.0);
            std::fill(d.begin(), d.begin() + j + 1, 0.0);
            d[j] = sigma * sc[j];
            if (j > kk) d[j - 1] = beta[j - 1] * sc[j - 1];
            if (j == kk)
                for (int i = 0; i < kk; ++i) d[i] = svec[i] * sc[i];
            PD_HIP(launch_project(Q, ld, j + 1, dim, pin, f32, sc[j], sc.data(), d.data(), partials, scal + kOffC,
                                  s));
            double *dst = Q + (size_t)(j + 1) * ld;
            PD_HIP(launch_update_project(Q, ld, j + 1, dim, scal + kOffC, sc.data(), d.data(), pin, f32, sc[j], dst,
                                         f32 ? x32 : nullptr, partials, scal + kOffC2, s));
            PD_HIP(dev.fetch(kOffC, j + 3));
            PD_HIP(dev.fetch(kOffC2 + j + 1, 1));
            double nrm_v = dev.host[kOffC2 + j + 1];
            const double nrm_ps = dev.host[kOffC + j + 1], nrm_hq = dev.host[kOffC + j + 2];
            if (!(nrm_v >= kReorthEta * kReorthEta * nrm_ps && nrm_v >= kReorthTau * kReorthTau * nrm_hq)) {
                PD_HIP(launch_update_norm(Q, ld, j + 1, dim, scal + kOffC2, sc.data(), dst, f32 ? x32 : nullptr,
                                          partials, scal + kOffNrm, s));
                PD_HIP(dev.fetch(kOffNrm, 1));
                nrm_v = dev.host[kOffNrm];
                ++info.reorth_second_passes;
            }
            alpha[j] = sigma + dev.host[kOffC + j];
            beta[j] = std::sqrt(std::max(nrm_v, 0.0));
            double tnorm = 0.0;
            for (int i = 0; i < kk; ++i) tnorm = std::max(tnorm, std::fabs(theta[i]) + std::fabs(svec[i]));
            for (int i = kk; i <= j; ++i) tnorm = std::max(tnorm, std::fabs(alpha[i]) + beta[i]);
            if (beta[j] <= 1e-14 * std::max(tnorm, 1e-300)) {
                m_eff = j + 1;   // invariant subspace: the Ritz pairs are exact
                breakdown = true;
                break;
            }
            sc[j + 1] = 1.0 / beta[j];
        }
        // projected matrix: arrowhead of the kept pairs, then tridiagonal
        std::vector<double> T((size_t)m_eff * m_eff, 0.0);
        for (int i = 0; i < kk; ++i) {
            T[(size_t)i * m_eff + i] = theta[i];
            T[(size_t)i * m_eff + kk] = T[(size_t)kk * m_eff + i] = svec[i];
        }
        for (int j = kk; j < m_eff; ++j) {
            T[(size_t)j * m_eff + j] = alpha[j];
            if (j + 1 < m_eff) T[(size_t)j * m_eff + j + 1] = T[(size_t)(j + 1) * m_eff + j] = beta[j];
        }
        jacobi_eig(m_eff, T, w, Z);
        const double bl = breakdown ? 0.0 : beta[m_eff - 1];
        const int want = std::min(nev, m_eff);
        double rmax = 0.0;
        for (int i = 0; i < want; ++i)
            rmax = std::max(rmax, std::fabs(bl * Z[(size_t)(m_eff - 1) * m_eff + i]) /
                                      std::max(std::fabs(w[i]), 1e-3 * dscale));
        info.residual = rmax;
        converged = want == nev && rmax <= tol_phase;
        if (f32) {
            // near the FP32 floor the estimate has stopped falling: FP32 has
            // done what it can
            if (rmax < 0.7 * best) {
                best = rmax;
                stall = 0;
            } else if (rmax < 1e-4 && ++stall >= 3) {
                converged = want == nev;
            }
        }
        if (o->verbose)
            std::fprintf(stderr, "[pairdiag] thick cycle %d  E0=%.15g  E%d=%.15g  rho_max=%.3e  products=%d\n", cycle,
                         w[0], want - 1, w[want - 1], rmax, info.iterations);
        const bool last = converged || breakdown || o->mode == 1 || cycles_total + cycle >= o->max_restarts;
        const int newk = last ? want : std::min(keep, m_eff - 1);
        // restart vectors: u_o = sum_j Z[j][o] sc_j Qt_j (o < newk), then q_{m+1} at column newk
        std::vector<double> Yh((size_t)m_eff * newk);
        for (int j = 0; j < m_eff; ++j)
            for (int q = 0; q < newk; ++q) Yh[(size_t)j * newk + q] = Z[(size_t)j * m_eff + q] * sc[j];
        PD_HIP(hipMemcpyAsync(Ydev, Yh.data(), Yh.size() * sizeof(double), hipMemcpyHostToDevice, s));
        PD_HIP(launch_combine_many(Q, ld, m_eff, newk, dim, Ydev, last ? -1 : m_eff, last ? 0.0 : sc[m_eff], s));
        // the next cycle's first product reads the FP32 copy of column newk
        if (f32 && !last) PD_HIP(launch_scale(Q + (size_t)newk * ld, dim, 1.0, Q + (size_t)newk * ld, x32, s));
        PD_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < newk; ++i) {
            theta[i] = w[i];
            svec[i] = bl * Z[(size_t)(m_eff - 1) * m_eff + i];
            sc[i] = 1.0;
        }
        sc[newk] = 1.0;
        kk = newk;
        if (last) {
            if (breakdown && want == nev) converged = true;
            break;
        }
    }
    cycles_total += cycle + 1;
    if (f32 && !converged) break;   // phase 0 ran out of restarts
    }
    info.restarts = cycles_total - 1;

    // ---- explicit FP64 check of every wanted vector (columns 0..got-1); fewer
    // than nev only when the start vector's Krylov space is smaller than nev
    const int got = kk;
    bool all_ok = got == nev;
    double rmax = 0.0;
    for (int i = got; i < nev; ++i) {
        E_out[i] = NAN;
        if (res_out) res_out[i] = NAN;
    }
    for (int i = 0; i < got; ++i) {
        double *u = Q + (size_t)i * ld;
        PD_HIP(launch_norm_sum(u, dim, partials, scal + kOffNrm, scal + kOffSum, s));
        PD_HIP(dev.fetch(kOffNrm, 2));
        const double nrm = std::sqrt(dev.host[kOffNrm]);
        if (!(nrm > 0.0)) return fail(PD_EDEVICE, "Ritz vector %d vanished", i);
        const double sign = dev.host[kOffSum] < 0.0 ? -1.0 : 1.0;
        PD_HIP(launch_scale(u, dim, sign / nrm, u, nullptr, s));
        PD_HIP(launch_sigma(omega, n, dim, coef, PD_F64, u, p, s, dsum64, dsum32, tr));
        ++info.iterations;
        const double one = 1.0, th = theta[i];
        PD_HIP(launch_project(Q + (size_t)i * ld, ld, 1, dim, p, false, 1.0, &one, &th, partials, scal + kOffC, s));
        PD_HIP(dev.fetch(kOffC, 2));
        const double c0 = dev.host[kOffC], r2 = dev.host[kOffC + 1];
        const double Ei = th + c0;
        const double res = std::sqrt(std::max(r2 - c0 * c0, 0.0)) / std::max(std::fabs(Ei), 1e-3 * dscale);
        E_out[i] = Ei;
        if (res_out) res_out[i] = res;
        rmax = std::max(rmax, res);
        if (!(res <= o->tol)) all_ok = false;
        if (psi) PD_HIP(hipMemcpyAsync(psi + (size_t)i * dim, u, dim * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (occ_out) {
            PD_HIP(launch_occupations(omega, n, dim, u, partials, scal + kOffOcc, s, tr));
            PD_HIP(dev.fetch(kOffOcc, omega));
            for (int q = 0; q < omega; ++q) occ_out[(size_t)i * omega + q] = dev.host[kOffOcc + q];
        }
    }
    PD_HIP(hipStreamSynchronize(s));
    converged = converged && all_ok;
    info.converged = converged ? 1 : 0;
    info.residual = rmax;
    info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    if (!converged && o->mode == 0)
        return fail(PD_ENOCONV, "not converged after %d restarts (rho=%.3e)", cycle, rmax);
    return PD_OK;
}

}  // namespace pd
