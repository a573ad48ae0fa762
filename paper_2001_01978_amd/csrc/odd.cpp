// Odd particle number in the blocking approximation (Sec. 2, Eq. hamiltonian3;
// the Block argument of the solver, Sec. 4.2; the N_Occup convention, Sec. 4.3).
//
// The unpaired particle sits on orbit b.  A pair can neither scatter into b
// (one of its two time-reversed states is taken) nor out of it (there is no
// pair there), and S+_b S-_b vanishes on it, so the seniority-one space is a
// direct sum of one block per b, and on block b
//     H_b = eps_b + H_even(n pairs on the omega - 1 orbits i != b),
// H_even being Eq. hamiltonian2 with eps and V restricted to i, j != b.
// Every block therefore has the same basis (n pairs on omega - 1 orbits);
// the blocks differ only in their coefficients.  block = 0 (all blocks, keep
// the lowest) is a batch of omega equal instances: when they fit the batched
// solver it runs them in one persistent launch, otherwise one basis handle is
// built in the workspace and the blocks are solved one after the other.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>
#include <algorithm>

#include "pd_internal.h"

namespace pd {
size_t lanczos_workspace_bytes(int64_t dim, const pd_lanczos_opts *o);
pd_status pack_coefficients(int omega, int n, const double *eps, const double *V, CoefBlock *out);
}  // namespace pd

using namespace pd;

namespace {

// Above this block dimension the one-at-a-time route is used: measured on
// MI355X with FP64 and 20 Krylov vectors, all blocks in one batched launch
// take 0.36 s against 0.69 s for 23 blocks of 705,432 states, 1.86 s against
// 1.96 s for 25 blocks of 2,704,156, and 4.23 s against 3.70 s for 26 blocks
// of 5,200,300 states.
constexpr int64_t kOddBatchedMaxDim = int64_t(1) << 22;

// Limits of the batched solver (batched.hip) for one reduced instance.
bool batched_fits(int om, int n, const pd_lanczos_opts *o) {
    return om >= 1 && om <= 32 && std::min(n, om - n) <= 12 && o->krylov >= 2 && o->krylov <= 32;
}

int resolve_route(int omega, int n, int block, int route, const pd_lanczos_opts *o) {
    if (block != 0) return PD_ODD_SEQUENTIAL;
    if (route != PD_ODD_AUTO) return route;
    const int om = omega - 1;
    if (batched_fits(om, n, o) && (int64_t)binom_host(om, n) <= kOddBatchedMaxDim) return PD_ODD_BATCHED;
    return PD_ODD_SEQUENTIAL;
}

// eps and V with orbit b left out (row-major, stride omega - 1).
void reduce_instance(int omega, const double *eps, const double *V, int b, double *eps_r, double *V_r) {
    const int om = omega - 1;
    int r = 0;
    for (int i = 0; i < omega; ++i) {
        if (i == b) continue;
        eps_r[r] = eps[i];
        int c = 0;
        for (int j = 0; j < omega; ++j)
            if (j != b) V_r[(size_t)r * om + c++] = V[(size_t)i * omega + j];
        ++r;
    }
}

// Smallest diagonal element of H_b (Monopole_Min of the blocked system): eps_b
// plus the n smallest pair energies 2 eps_i + V_ii with i != b.
double blocked_monopole(int omega, int n, const double *eps, const double *V, int b) {
    std::vector<double> d;
    d.reserve(omega);
    for (int i = 0; i < omega; ++i)
        if (i != b) d.push_back(2.0 * eps[i] + V[(size_t)i * omega + i]);
    std::sort(d.begin(), d.end());
    double s = eps[b];
    for (int k = 0; k < n; ++k) s += d[k];
    return s;
}

pd_status check_odd(int omega, int n, int block, int route, const pd_lanczos_opts *o) {
    if (omega < 2 || omega > kMaxOmega) return fail(PD_EINVAL, "odd system: omega=%d outside [2, %d]", omega, kMaxOmega);
    if (n < 0 || n > omega - 1) return fail(PD_EINVAL, "odd system: n=%d pairs outside [0, omega-1]", n);
    if (block < 0 || block > omega) return fail(PD_EINVAL, "block=%d outside [0, omega]", block);
    if (route < PD_ODD_AUTO || route > PD_ODD_BATCHED) return fail(PD_EINVAL, "route=%d", route);
    if (!o) return fail(PD_EINVAL, "opts is NULL");
    if (o->start == PD_START_USER) return fail(PD_EINVAL, "odd-system solves take no user start vector");
    if (route == PD_ODD_BATCHED) {
        if (block != 0) return fail(PD_EINVAL, "the batched route solves all blocks (block = 0)");
        if (!batched_fits(omega - 1, n, o))
            return fail(PD_ERANGE, "blocks of %d pairs on %d orbits (krylov %d) exceed the batched solver's limits", n,
                        omega - 1, o->krylov);
    }
    return PD_OK;
}

struct OddBatch {
    std::vector<int> om, n;
    std::vector<double> eps, V;
};

OddBatch make_batch(int omega, int n, const double *eps, const double *V) {
    OddBatch B;
    const int om = omega - 1;
    B.om.assign(omega, om);
    B.n.assign(omega, n);
    B.eps.resize((size_t)omega * om);
    B.V.resize((size_t)omega * om * om);
    for (int b = 0; b < omega; ++b)
        reduce_instance(omega, eps, V, b, B.eps.data() + (size_t)b * om, B.V.data() + (size_t)b * om * om);
    return B;
}

}  // namespace

extern "C" {

size_t pd_odd_workspace_bytes(int omega, int n, int block, int route, const pd_lanczos_opts *o) {
    if (check_odd(omega, n, block, route, o) != PD_OK) return 0;
    const int om = omega - 1;
    if (resolve_route(omega, n, block, route, o) == PD_ODD_BATCHED) {
        std::vector<int> oms(omega, om), ns(omega, n);
        return pd_batched_workspace_bytes(omega, oms.data(), ns.data(), o);
    }
    return align256(pd_basis_bytes(om, n, 0)) + lanczos_workspace_bytes((int64_t)binom_host(om, n), o);
}

pd_status pd_lanczos_ground_odd(int omega, int n, const double *eps, const double *V, int block, int route,
                                const pd_lanczos_opts *o, void *work_dev, size_t work_bytes, double *E,
                                int *block_out, double *E_blocks, double *occ, pd_lanczos_info *info,
                                hipStream_t stream) {
    const auto t0 = std::chrono::steady_clock::now();
    pd_status st = check_odd(omega, n, block, route, o);
    if (st != PD_OK) return st;
    if (!E) return fail(PD_EINVAL, "E is NULL");
    {
        // Whole-instance checks (finite, symmetric) before any block runs.
        std::unique_ptr<CoefBlock> blk(new (std::nothrow) CoefBlock);
        if (!blk) return fail(PD_ENOMEM, "host allocation failed");
        if ((st = pack_coefficients(omega, n, eps, V, blk.get())) != PD_OK) return st;
    }
    const int om = omega - 1;
    const int rt = resolve_route(omega, n, block, route, o);
    const size_t need = pd_odd_workspace_bytes(omega, n, block, route, o);
    if (need == 0) return fail(PD_EINVAL, "blocks of %d pairs on %d orbits: workspace size query failed", n, om);
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");

    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> Eb(omega, nan);
    std::vector<double> occ_best(om, 0.0);
    pd_lanczos_info tot;
    std::memset(&tot, 0, sizeof(tot));
    tot.converged = 1;
    tot.monopole_min = std::numeric_limits<double>::infinity();
    int best = -1;
    bool any_noconv = false;

    if (rt == PD_ODD_BATCHED) {
        OddBatch B = make_batch(omega, n, eps, V);
        std::vector<double> E0(omega), occ_all((size_t)omega * om);
        std::vector<pd_lanczos_info> inf(omega);
        st = pd_lanczos_ground_batched(omega, B.om.data(), B.n.data(), B.eps.data(), B.V.data(), o, 512, work_dev,
                                       work_bytes, E0.data(), occ_all.data(), inf.data(), nullptr, stream);
        if (st != PD_OK && st != PD_ENOCONV) return st;
        any_noconv = st == PD_ENOCONV;
        for (int b = 0; b < omega; ++b) {
            Eb[b] = eps[b] + E0[b];
            if (best < 0 || Eb[b] < Eb[best]) best = b;
            tot.iterations += inf[b].iterations;
            tot.restarts += inf[b].restarts;
            tot.converged &= inf[b].converged ? 1 : 0;
            tot.residual = std::max(tot.residual, inf[b].residual);
        }
        std::copy(occ_all.begin() + (size_t)best * om, occ_all.begin() + (size_t)(best + 1) * om, occ_best.begin());
    } else {
        const size_t basis_bytes = align256(pd_basis_bytes(om, n, 0));
        pd_basis bs = nullptr;
        if ((st = pd_basis_create(om, n, 0, work_dev, basis_bytes, stream, &bs)) != PD_OK) return st;
        void *lw = static_cast<unsigned char *>(work_dev) + basis_bytes;
        const size_t lw_bytes = work_bytes - basis_bytes;
        std::vector<double> eps_r(om), V_r((size_t)om * om), occ_r(om);
        const int b0 = block ? block - 1 : 0, b1 = block ? block : omega;
        for (int b = b0; b < b1; ++b) {
            reduce_instance(omega, eps, V, b, eps_r.data(), V_r.data());
            double e0 = 0.0;
            pd_lanczos_info bi;
            std::memset(&bi, 0, sizeof(bi));
            st = pd_lanczos_ground(bs, eps_r.data(), V_r.data(), o, lw, lw_bytes, nullptr, &e0, nullptr, occ_r.data(),
                                   &bi, stream);
            if (st != PD_OK && st != PD_ENOCONV) {
                pd_basis_destroy(bs);
                return st;
            }
            any_noconv |= st == PD_ENOCONV;
            Eb[b] = eps[b] + e0;
            if (best < 0 || Eb[b] < Eb[best]) {
                best = b;
                std::copy(occ_r.begin(), occ_r.begin() + om, occ_best.begin());
            }
            tot.iterations += bi.iterations;
            tot.iterations_f32 += bi.iterations_f32;
            tot.restarts += bi.restarts;
            tot.converged &= bi.converged ? 1 : 0;
            tot.residual = std::max(tot.residual, bi.residual);
            tot.sigma_seconds_f64 += bi.sigma_seconds_f64;
            tot.sigma_seconds_f32 += bi.sigma_seconds_f32;
            tot.reorth_second_passes += bi.reorth_second_passes;
        }
        pd_basis_destroy(bs);
    }

    for (int b = 0; b < omega; ++b)
        if (!std::isnan(Eb[b])) tot.monopole_min = std::min(tot.monopole_min, blocked_monopole(omega, n, eps, V, b));
    *E = Eb[best];
    if (block_out) *block_out = best + 1;
    if (E_blocks) std::copy(Eb.begin(), Eb.end(), E_blocks);
    if (occ) {
        // N_Occup of the chosen block: 1 on the blocked orbit (Sec. 4.3), the
        // pair occupations of the reduced problem on the others.
        int r = 0;
        for (int i = 0; i < omega; ++i) occ[i] = (i == best) ? 1.0 : occ_best[r++];
    }
    tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = tot;
    return any_noconv ? PD_ENOCONV : PD_OK;
}

}  // extern "C"
