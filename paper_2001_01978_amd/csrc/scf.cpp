// The exact pairing solution inside a self-consistent mean-field loop, the use
// the paper names for it in place of the BCS approximation (Sec. 1, Sec. 6).
//
// The mean field is synthetic (no Hartree-Fock code is linked here): the
// single-particle energies follow the pair occupations through a fixed
// matrix W, eps_i = eps0_i + sum_j W_ij <N_j> / 2.  Each iteration solves the
// ground state of Eq. hamiltonian2 with the current eps; the new field is
// compared with the one just used, and linear mixing gives the next one.
// From the second iteration on, the solve starts from the previous ground
// state (the caller's vector start of pd_lanczos_ground), which the change of
// the field barely moves.  Everything except the O(omega^2) field update runs
// in the library's kernels.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>
#include <algorithm>

#include "pd_internal.h"

using namespace pd;

extern "C" {

size_t pd_scf_workspace_bytes(pd_basis b, const pd_lanczos_opts *o) {
    const size_t lw = pd_lanczos_workspace_bytes(b, o);
    if (lw == 0) return 0;
    return align256((size_t)b->dim * sizeof(double)) + lw;
}

pd_status pd_scf_ground(pd_basis b, const double *eps0, const double *W, const double *V, const pd_scf_opts *so,
                        const pd_lanczos_opts *o, void *work_dev, size_t work_bytes, double *eps_out,
                        double *occ_out, double *E0, double *psi0_dev, pd_scf_info *info, hipStream_t stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!b) return fail(PD_EINVAL, "basis handle is NULL");
    if (!so || !o || !eps0 || !W || !V || !E0) return fail(PD_EINVAL, "so, o, eps0, W, V and E0 are required");
    if (!(so->mixing > 0.0 && so->mixing <= 1.0)) return fail(PD_EINVAL, "mixing must lie in (0, 1]");
    if (!(so->tol >= 0.0) || !std::isfinite(so->tol)) return fail(PD_EINVAL, "tol must be finite and >= 0");
    if (so->max_iter < 1) return fail(PD_EINVAL, "max_iter < 1");
    if (o->start == PD_START_USER) return fail(PD_EINVAL, "the first solve takes the E1, HF or RANDOM start");
    const int omega = b->omega;
    for (int i = 0; i < omega * omega; ++i)
        if (!std::isfinite(W[i])) return fail(PD_EINVAL, "W[%d] is not finite", i);
    const size_t need = pd_scf_workspace_bytes(b, o);
    if (need == 0) return fail(PD_EINVAL, "bad Lanczos options");
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    pd_status st0 = check_device_ptr(work_dev, "work_dev", need);
    if (st0 != PD_OK) return st0;
    if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");
    if (psi0_dev) {
        const char *a = reinterpret_cast<const char *>(psi0_dev), *w = static_cast<const char *>(work_dev);
        const size_t nb = (size_t)b->dim * sizeof(double);
        if ((st0 = check_device_ptr(psi0_dev, "psi0_dev", nb)) != PD_OK) return st0;
        if (a < w + work_bytes && w < a + nb) return fail(PD_EINVAL, "psi0_dev overlaps the workspace");
    }
    double *psi = static_cast<double *>(work_dev);
    const size_t pb = align256((size_t)b->dim * sizeof(double));
    void *lw = static_cast<unsigned char *>(work_dev) + pb;
    const size_t lw_bytes = work_bytes - pb;

    std::vector<double> eps(eps0, eps0 + omega), occ(omega), fresh(omega);
    pd_scf_info sum;
    std::memset(&sum, 0, sizeof(sum));
    sum.lanczos_converged = 1;
    double e0 = 0.0, change = INFINITY;
    int it = 0;
    for (it = 1; it <= so->max_iter; ++it) {
        pd_lanczos_opts ot = *o;
        const bool warm = it > 1 && so->reuse_psi;
        if (warm) {
            ot.start = PD_START_USER;
            ot.fallback = 0;
        }
        pd_lanczos_info li;
        pd_status st = pd_lanczos_ground(b, eps.data(), V, &ot, lw, lw_bytes, warm ? psi : nullptr, &e0, psi,
                                         occ.data(), &li, stream);
        if (st != PD_OK && st != PD_ENOCONV) return st;
        if (st == PD_ENOCONV) sum.lanczos_converged = 0;
        sum.products += li.iterations;
        if (it == 1) sum.products_first = li.iterations;
        sum.last_residual = li.residual;
        change = 0.0;
        for (int i = 0; i < omega; ++i) {
            double f = eps0[i];
            for (int j = 0; j < omega; ++j) f += W[(size_t)i * omega + j] * occ[j] * 0.5;
            fresh[i] = f;
            change = std::max(change, std::fabs(f - eps[i]));
        }
        if (change <= so->tol) break;
        if (it == so->max_iter) break;
        for (int i = 0; i < omega; ++i) eps[i] = (1.0 - so->mixing) * eps[i] + so->mixing * fresh[i];
    }
    sum.iterations = std::min(it, so->max_iter);
    sum.converged = change <= so->tol ? 1 : 0;
    sum.change = change;
    if (psi0_dev) {
        hipError_t e = hipMemcpyAsync(psi0_dev, psi, (size_t)b->dim * sizeof(double), hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(PD_EDEVICE, "psi copy: %s", hipGetErrorString(e));
    }
    *E0 = e0;
    if (eps_out) std::copy(eps.begin(), eps.end(), eps_out);
    if (occ_out) std::copy(occ.begin(), occ.end(), occ_out);
    sum.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = sum;
    if (!sum.converged) return fail(PD_ENOCONV, "self-consistency not reached in %d iterations (change %.3e)",
                                    sum.iterations, change);
    return PD_OK;
}

}  // extern "C"
