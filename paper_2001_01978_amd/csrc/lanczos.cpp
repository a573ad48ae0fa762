// Restarted, fully reorthogonalised Lanczos driver (Sec. 3.4, Alg. lanczos).
//
// One cycle builds up to m = krylov orthonormal vectors q_1..q_m in the
// workspace.  Step k, three streaming passes at most:
//   1. ps = H q_k - sigma_k q_k - beta_{k-1} q_{k-1} on the fly, with sigma_k =
//      alpha_{k-1} (on the first step of a cycle: the Ritz value of the
//      previous cycle, 0 at the start, and no beta term): the recurrence of
//      Alg. lanczos with the estimate sigma_k in place of alpha_k; c = Q^T ps,
//      ||ps|| and ||H q_k||;
//   2. v = ps - Q c (Gram-Schmidt against every stored vector, which also
//      corrects alpha_k = sigma_k + c_k), with c' = Q^T v and ||v||;
//   3. v -= Q c' only when ||v|| < ||ps|| / sqrt(2) or ||v|| < ||H q_k|| / 128.
// A classical pass multiplies the orthogonality error already in Q by
// ||c|| / ||v|| and adds rounding of order u ||H q_k|| / ||v||; the first test
// (Daniel, Gragg, Kaufman and Stewart) keeps the factor <= 1, the second keeps
// the rounding below 128 u.  Subtracting the recurrence first makes c small,
// so the tests pass on most steps (without it c is dominated by alpha_k and
// the second pass is always needed).  beta_k = ||v||; q_{k+1} = v / beta_k is
// stored as v with the scale 1/beta_k, so no pass normalises it, and pass 2
// (or 3) also writes the FP32 copy for the next product.  The last step of a
// cycle needs only alpha_m.  After the cycle the lowest Ritz pair of the
// tridiagonal L = tridiag(beta, alpha, beta) gives psi = Q y, the start of the
// next cycle.  The first step of every cycle measures the residual of its
// start vector, |beta_1 / alpha_1| = ||H q - (q^T H q) q|| / |q^T H q|
// (Eq. convergence), and stops when it is below tol.
//
// Mixed precision: steps k >= 2 of a cycle run the product in FP32, and the
// Krylov columns q_2..q_m are stored in FP32 (the next product reads its
// column directly); precision value 2 keeps every column in FP64 and
// multiplies an FP32 copy instead.  Step 1 (the residual and alpha_1 = q^T H q of the restart
// vector) is always FP64 and q_1 is stored in FP64, so the FP32 error -- of
// the products and of the stored columns alike -- only enters the correction
// sum_{j>=2} y_j q_j, whose size shrinks with the residual; every dot
// product, norm and update is computed in FP64.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <algorithm>
#include <mutex>

#include "pd_internal.h"

namespace pd {

namespace {

struct Layout {
    size_t coef = 0, scal = 0, partials = 0, Q = 0, Q32 = 0, p = 0, w = 0, x32 = 0, y32 = 0, total = 0;
    int64_t ld = 0;
    int m = 0;
};

constexpr int kScalars = 512;  // doubles: c[66], c2[65], nrm2, sum, occ[64]
constexpr int kOffC = 0, kOffC2 = 80, kOffNrm = 192, kOffSum = 193, kOffOcc = 256;
// Thresholds of the second Gram-Schmidt pass (see the step description above).
constexpr double kReorthEta = 0.70710678118654752;   // 1/sqrt(2)
constexpr double kReorthTau = 1.0 / 128.0;
// precision value 2: FP32 products, every Krylov column stored in FP64
constexpr int kMixedF64Cols = 2;

Layout layout_for(int64_t dim, int krylov, int precision) {
    Layout L;
    L.m = (int)std::min<int64_t>(krylov, dim);
    L.ld = (dim + 63) & ~int64_t(63);
    size_t off = 0;
    L.coef = off;
    off += kCoefBytes;
    L.scal = off;
    off += align256(kScalars * sizeof(double));
    L.partials = off;
    off += align256(partial_doubles() * sizeof(double));
    L.Q = off;
    if (precision == PD_F32) {
        // q_1 in FP64, q_2..q_m in FP32
        off += align256((size_t)L.ld * sizeof(double));
        L.Q32 = off;
        off += align256((size_t)std::max(L.m - 1, 1) * L.ld * sizeof(float));
    } else {
        off += align256((size_t)L.m * L.ld * sizeof(double));
    }
    L.p = off;
    off += align256((size_t)L.ld * sizeof(double));
    L.w = off;
    off += align256((size_t)L.ld * sizeof(double));
    if (precision == kMixedF64Cols) {
        // FP64 columns: the FP32 product reads an FP32 copy of q_k
        L.x32 = off;
        off += align256((size_t)L.ld * sizeof(float));
    }
    if (precision == PD_F32 || precision == kMixedF64Cols) {
        L.y32 = off;
        off += align256((size_t)L.ld * sizeof(float));
    }
    L.total = off;
    return L;
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
    // one synchronisation for two ranges
    hipError_t fetch2(int off1, int count1, int off2, int count2) {
        hipError_t e = hipMemcpyAsync(host + off1, scal + off1, count1 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(host + off2, scal + off2, count2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }
};

}  // namespace

size_t lanczos_workspace_bytes(int64_t dim, const pd_lanczos_opts *o) {
    return layout_for(dim, o->krylov, o->precision).total;
}

// ---------------------------------------------------------------- static workspace
// The workspace of pd_lanczos_ground_static: a device array of fixed size in
// the library's code object, one copy per GPU.  Host code never passes the
// array's name to a kernel (in host code it only stands in for the symbol):
// its device address is looked up once per device and kept here.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_static_call_mu[kMaxDevices];
}  // namespace

pd_status static_scratch(void **ptr, std::mutex **call_mu) {
    int dev = 0;
    PD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PD_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PD_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *call_mu = &g_static_call_mu[dev];
    return PD_OK;
}

pd_status lanczos_run(pd_basis b, const CoefBlock &host_coef, const pd_lanczos_opts *o, void *work,
                      size_t work_bytes, const double *x0, double *E0_out, double *psi0, double *occ_out,
                      pd_lanczos_info *info_out, hipStream_t s, bool time_products) {
    auto t0 = std::chrono::steady_clock::now();
    const int omega = b->omega, n = b->n;
    const int64_t dim = b->dim;
    const TruncSpace *tr = b->truncated ? &b->trunc : nullptr;
    Layout L = layout_for(dim, o->krylov, o->precision);
    if (work_bytes < L.total)
        return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, L.total);
    unsigned char *base = static_cast<unsigned char *>(work);
    CoefBlock *coef = reinterpret_cast<CoefBlock *>(base + L.coef);
    double *scal = reinterpret_cast<double *>(base + L.scal);
    double *partials = reinterpret_cast<double *>(base + L.partials);
    double *Q = reinterpret_cast<double *>(base + L.Q);
    double *p = reinterpret_cast<double *>(base + L.p);
    double *w = reinterpret_cast<double *>(base + L.w);
    float *Q32 = o->precision == PD_F32 ? reinterpret_cast<float *>(base + L.Q32) : nullptr;
    float *x32 = o->precision == kMixedF64Cols ? reinterpret_cast<float *>(base + L.x32) : nullptr;
    float *y32 = o->precision != PD_F64 ? reinterpret_cast<float *>(base + L.y32) : nullptr;
    const int64_t ld = L.ld;
    const int m = L.m;
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
    // The vector kernels read FP32 column 2 (with zero weight) while only q_1
    // exists: it must hold finite values before its first write.
    if (Q32) PD_HIP(hipMemsetAsync(Q32, 0, (size_t)ld * sizeof(float), s));
    PD_HIP(hipStreamSynchronize(s));
    Dev dev{s, scal, {}};

    // ---- start vector into w
    switch (o->start) {
        case PD_START_E1:
            PD_HIP(launch_fill_unit(dim, 0, w, s));
            break;
        case PD_START_HF: {
            std::vector<int> idx(omega);
            for (int i = 0; i < omega; ++i) idx[i] = i;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int a, int c) { return host_coef.d64[a] < host_coef.d64[c]; });
            uint64_t st = 0;
            for (int i = 0; i < n; ++i) st |= 1ull << idx[i];
            int64_t r = 0;
            int j = 0;
            for (int q = 0; q < omega; ++q)
                if ((st >> q) & 1ull) r += (int64_t)binom_host(q, ++j);
            if (tr) {
                // Its row in the truncated space (the lowest diagonal is always kept).
                TruncWord wd;
                PD_HIP(hipMemcpyAsync(&wd, tr->words + (r >> 6), sizeof(wd), hipMemcpyDeviceToHost, s));
                PD_HIP(hipStreamSynchronize(s));
                const int sh = (int)(r & 63);
                if (!((wd.bits >> sh) & 1ull)) return fail(PD_EINVAL, "the HF state is not in the truncated space");
                r = (int64_t)wd.base + __builtin_popcountll(wd.bits & ((1ull << sh) - 1));
            }
            PD_HIP(launch_fill_unit(dim, r, w, s));
            break;
        }
        case PD_START_RANDOM:
            PD_HIP(launch_fill_random(o->seed, dim, w, s));
            break;
        case PD_START_USER:
            PD_HIP(launch_copy(x0, dim, w, s));
            break;
        default:
            return fail(PD_EINVAL, "unknown start %d", o->start);
    }
    PD_HIP(launch_norm_sum(w, dim, partials, scal + kOffNrm, scal + kOffSum, s));
    PD_HIP(dev.fetch(kOffNrm, 1));
    if (!(dev.host[kOffNrm] > 0.0) || !std::isfinite(dev.host[kOffNrm]))
        return fail(PD_EINVAL, "start vector has zero or non-finite norm");
    {
        double sc = 1.0 / std::sqrt(dev.host[kOffNrm]);
        PD_HIP(launch_scale(w, dim, sc, Q, nullptr, s));
    }

    // Fallback for a caller-supplied start: also try the RANDOM start (in w)
    // and keep the vector with the lower Rayleigh quotient (two FP64 products).
    if (o->start == PD_START_USER && o->fallback && m >= 2) {
        double rq[2];
        for (int t = 0; t < 2; ++t) {
            double *q = t == 0 ? Q : w;
            if (t == 1) {
                PD_HIP(launch_fill_random(o->seed, dim, w, s));
                PD_HIP(launch_norm_sum(w, dim, partials, scal + kOffNrm, scal + kOffSum, s));
                PD_HIP(dev.fetch(kOffNrm, 1));
                PD_HIP(launch_scale(w, dim, 1.0 / std::sqrt(dev.host[kOffNrm]), w, nullptr, s));
            }
            PD_HIP(launch_sigma(omega, n, dim, coef, PD_F64, q, p, s, dsum64, dsum32, tr));
            ++info.iterations;
            const double one = 1.0, zero = 0.0;
            PD_HIP(launch_project(q, ld, 1, dim, p, false, 1.0, &one, &zero, partials, scal + kOffC, s));
            PD_HIP(dev.fetch(kOffC, 1));
            rq[t] = dev.host[kOffC];
        }
        if (rq[1] < rq[0]) {
            PD_HIP(launch_scale(w, dim, 1.0, Q, nullptr, s));
            info.fallback_used = 1;
        }
    }

    // HIP events around every product: its device time, read after the step's sync
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    if (time_products) {
        PD_HIP(hipEventCreate(&ev.a));
        PD_HIP(hipEventCreate(&ev.b));
    }

    std::vector<double> alpha(m), beta(m), y(m), yy(m);
    // Column scales: q_j = sc[j] * (stored column j).  Columns are written
    // unnormalised by the Gram-Schmidt pass itself; 1/beta is kept here.
    std::vector<double> sc(m + 1, 1.0);
    // Part of the three-term recurrence subtracted before the projection:
    // sigma_k q_k + beta_{k-1} q_{k-1}, with sigma_k = alpha_{k-1} (the Ritz
    // value of the previous cycle at k = 0), as coefficients of stored columns.
    std::vector<double> d(m, 0.0);
    double theta = 0.0, residual = INFINITY, e0 = NAN;
    bool converged = false;
    bool final_check = false;  // this cycle only measures its start vector
    int cycle = 0;
    for (cycle = 0;; ++cycle) {
        int m_eff = m;
        sc[0] = 1.0;
        for (int k = 0; k < m; ++k) {
            double *qk = Q + (size_t)k * ld;
            const bool f32_step = y32 && k >= 1;
            // the product of the stored column k (FP32 column for FP32 steps); H q_k = sc[k] * it
            const void *pin = f32_step ? static_cast<const void *>(y32) : static_cast<const void *>(p);
            if (time_products) PD_HIP(hipEventRecord(ev.a, s));
            if (f32_step) {
                PD_HIP(launch_sigma(omega, n, dim, coef, PD_F32, Q32 ? Q32 + (size_t)(k - 1) * ld : x32, y32, s,
                                    dsum64, dsum32, tr));
                ++info.iterations_f32;
            } else {
                PD_HIP(launch_sigma(omega, n, dim, coef, PD_F64, qk, p, s, dsum64, dsum32, tr));
            }
            if (time_products) PD_HIP(hipEventRecord(ev.b, s));
            ++info.iterations;
            const double sp = sc[k];
            const double sigma = k > 0 ? alpha[k - 1] : theta;
            std::fill(d.begin(), d.begin() + k + 1, 0.0);
            d[k] = sigma * sc[k];
            if (k > 0) d[k - 1] = beta[k - 1] * sc[k - 1];
            // ps = H q_k - sigma q_k - beta_{k-1} q_{k-1}; c = Q^T ps (alpha_k = sigma + c_k),
            // ||ps||^2 and ||H q_k||^2
            PD_HIP(launch_project(Q, ld, k + 1, dim, pin, f32_step, sp, sc.data(), d.data(), partials,
                                  scal + kOffC, s, Q32));
            const bool store = k + 1 < m;      // q_{k+1} is needed (else only alpha_k, and beta_0 at k = 0)
            double nrm_v = 0.0;
            if (store || k == 0) {
                // v = H q_k - Q c, written as the next stored column (FP32 in mixed
                // precision; or into w), with c' = Q^T v, ||v||^2
                double *dst = store ? (Q32 ? nullptr : Q + (size_t)(k + 1) * ld) : w;
                float *dst32 = store ? (Q32 ? Q32 + (size_t)k * ld : x32) : nullptr;
                PD_HIP(launch_update_project(Q, ld, k + 1, dim, scal + kOffC, sc.data(), d.data(), pin, f32_step,
                                             sp, dst, dst32, partials, scal + kOffC2, s, Q32));
                PD_HIP(dev.fetch2(kOffC + k, 3, kOffC2 + k + 1, 1));
                nrm_v = dev.host[kOffC2 + k + 1];
                const double nrm_ps = dev.host[kOffC + k + 1], nrm_hq = dev.host[kOffC + k + 2];
                if (!(nrm_v >= kReorthEta * kReorthEta * nrm_ps && nrm_v >= kReorthTau * kReorthTau * nrm_hq)) {
                    // large cancellation: Gram-Schmidt once more, v -= Q c'
                    PD_HIP(launch_update_norm(Q, ld, k + 1, dim, scal + kOffC2, sc.data(), dst, dst32, partials,
                                              scal + kOffNrm, s, Q32));
                    PD_HIP(dev.fetch(kOffNrm, 1));
                    nrm_v = dev.host[kOffNrm];
                    ++info.reorth_second_passes;
                }
            } else {
                PD_HIP(dev.fetch(kOffC + k, 1));
            }
            if (time_products) {
                float ms = 0.0f;
                PD_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                (f32_step ? info.sigma_seconds_f32 : info.sigma_seconds_f64) += 1e-3 * ms;
            }
            alpha[k] = sigma + dev.host[kOffC + k];
            beta[k] = std::sqrt(std::max(nrm_v, 0.0));
            if (k == 0) {
                e0 = alpha[0];
                residual = beta[0] / std::max(std::fabs(alpha[0]), 1e-3 * dscale);
                if (o->verbose)
                    std::fprintf(stderr, "[pairdiag] cycle %d  E=%.15g  rho=%.3e  products=%d\n", cycle, e0,
                                 residual, info.iterations);
                if (residual <= o->tol) converged = true;
                if (converged || final_check) break;
            }
            if (!store) break;
            double tnorm = 0.0;
            for (int i = 0; i <= k; ++i) tnorm = std::max(tnorm, std::fabs(alpha[i]) + beta[i]);
            if (beta[k] <= 1e-14 * std::max(tnorm, 1e-300)) {
                m_eff = k + 1;  // invariant subspace: the Ritz pair is exact
                break;
            }
            sc[k + 1] = 1.0 / beta[k];
        }
        if (converged || final_check) break;
        if (tridiag_lowest(m_eff, alpha.data(), beta.data(), &theta, y.data()) != 0)
            return fail(PD_EDEVICE, "tridiagonal eigensolver failed (m=%d)", m_eff);
        for (int j = 0; j < m_eff; ++j) yy[j] = y[j] * sc[j];
        PD_HIP(launch_combine(Q, ld, m_eff, dim, yy.data(), w, partials, scal + kOffNrm, scal + kOffSum, s, Q32));
        PD_HIP(dev.fetch(kOffNrm, 1));
        double nr = std::sqrt(dev.host[kOffNrm]);
        if (!(nr > 0.0)) return fail(PD_EDEVICE, "Ritz vector vanished");
        PD_HIP(launch_scale(w, dim, 1.0 / nr, Q, nullptr, s));
        // Mode 1 (no restart) and the last allowed cycle only measure the Ritz vector next.
        if (o->mode == 1 || cycle >= o->max_restarts) final_check = true;
    }
    info.restarts = cycle;
    info.converged = converged ? 1 : 0;
    info.residual = residual;

    // ---- outputs from q_1 (normalised FP64 vector whose Rayleigh quotient is e0)
    PD_HIP(launch_norm_sum(Q, dim, partials, scal + kOffNrm, scal + kOffSum, s));
    PD_HIP(dev.fetch(kOffNrm, 2));
    double sign = dev.host[kOffSum] < 0.0 ? -1.0 : 1.0;
    if (psi0) PD_HIP(launch_scale(Q, dim, sign, psi0, nullptr, s));
    if (occ_out) {
        PD_HIP(launch_occupations(omega, n, dim, Q, partials, scal + kOffOcc, s, tr));
        PD_HIP(dev.fetch(kOffOcc, omega));
        for (int i = 0; i < omega; ++i) occ_out[i] = dev.host[kOffOcc + i];
    }
    PD_HIP(hipStreamSynchronize(s));
    *E0_out = e0;
    info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    if (!converged && o->mode == 0)
        return fail(PD_ENOCONV, "not converged after %d restarts (rho=%.3e)", cycle, residual);
    return PD_OK;
}

}  // namespace pd
