// C ABI entry points (include/pairdiag.h): argument validation, handle
// lifecycle and dispatch to the kernels.  No entry point allocates device
// memory; all of it comes from caller buffers sized by the *_bytes queries.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <memory>
#include <vector>
#include <algorithm>

#include "pd_internal.h"

namespace pd {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

pd_status fail(pd_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

const char *last_error() { return g_err; }

pd_status pack_coefficients(int omega, int n, const double *eps, const double *V, CoefBlock *out) {
    if (omega < 1 || omega > kMaxOmega) return fail(PD_EINVAL, "omega=%d outside [1, %d]", omega, kMaxOmega);
    if (n < 0 || n > omega) return fail(PD_EINVAL, "n=%d outside [0, omega]", n);
    if (!eps || !V) return fail(PD_EINVAL, "eps and V must be host arrays");
    std::memset(out, 0, sizeof(CoefBlock));
    for (int i = 0; i < omega; ++i)
        if (!std::isfinite(eps[i])) return fail(PD_EINVAL, "eps[%d] is not finite", i);
    for (int i = 0; i < omega; ++i)
        for (int j = 0; j < omega; ++j) {
            double v = V[i * omega + j];
            if (!std::isfinite(v)) return fail(PD_EINVAL, "V[%d][%d] is not finite", i, j);
            if (v != V[j * omega + i]) return fail(PD_EINVAL, "V is not symmetric at (%d, %d)", i, j);
        }
    double s64 = 0.0;
    float s32 = 0.0f;
    for (int i = 0; i < omega; ++i) {
        double d = 2.0 * eps[i] + V[i * omega + i];
        out->d64[i] = d;
        out->d32[i] = (float)d;
        s64 += d;
        s32 += (float)d;
    }
    out->dsum64 = s64;
    out->dsum32 = s32;
    for (int i = 0; i < omega * omega; ++i) {
        out->V64[i] = V[i];
        out->V32[i] = (float)V[i];
    }
    // V is stored with row stride omega: V[b*omega + a]
    return PD_OK;
}

size_t lanczos_workspace_bytes(int64_t dim, const pd_lanczos_opts *o);
size_t lanczos_eigs_workspace_bytes(int64_t dim, const pd_lanczos_opts *o);
pd_status lanczos_eigs_run(pd_basis b, const CoefBlock &host_coef, int nev, const pd_lanczos_opts *o, void *work,
                           size_t work_bytes, double *E_out, double *psi, double *occ_out, double *res_out,
                           pd_lanczos_info *info_out, hipStream_t s);
pd_status lanczos_run(pd_basis b, const CoefBlock &host_coef, const pd_lanczos_opts *o, void *work,
                      size_t work_bytes, const double *x0, double *E0_out, double *psi0, double *occ_out,
                      pd_lanczos_info *info_out, hipStream_t s, bool time_products = true);

namespace {

bool valid_space(int omega, int n) { return omega >= 1 && omega <= kMaxOmega && n >= 0 && n <= omega; }

// product: the caller runs full-space products on b (pd_warm_start does not).
pd_status check_sigma_range(pd_basis b, bool product = true) {
    int nn = std::min(b->n, b->omega - b->n);
    if (nn > kMaxSigmaPairs)
        return fail(PD_ERANGE, "min(n, omega-n)=%d exceeds %d (dim %lld)", nn, kMaxSigmaPairs, (long long)b->dim);
    if (product && !b->truncated && sigma_space_refused(b->omega, b->n))
        return fail(PD_ERANGE,
                    "omega=%d, n=%d: full-space products on mirrored spaces with 16 pairs and 32-bit ranks "
                    "(omega 33-35) are disabled (an unexplained illegal memory access)",
                    b->omega, b->n);
    return PD_OK;
}

}  // namespace

// Device memory check: turns host or foreign pointers, and device ranges that
// run past the end of their allocation, into PD_EINVAL before any kernel runs.
pd_status check_device_ptr(const void *p, const char *what, size_t bytes) {
    if (!p) return fail(PD_EINVAL, "%s is NULL", what);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PD_EINVAL, "%s is not device memory (%s)", what, hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(PD_EINVAL, "%s is not device memory", what);
    if (bytes) {
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        e = hipMemGetAddressRange(&base, &size, const_cast<void *>(p));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(PD_EINVAL, "%s: cannot query its allocation (%s)", what, hipGetErrorString(e));
        }
        const char *b0 = static_cast<const char *>(base), *pp = static_cast<const char *>(p);
        if (pp + bytes > b0 + size)
            return fail(PD_EINVAL, "%s: %zu bytes needed past %p, allocation ends %zu bytes after it", what, bytes,
                        p, (size_t)(b0 + size - pp));
    }
    return PD_OK;
}

namespace {

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

pd_status check_basis(pd_basis b) {
    if (!b) return fail(PD_EINVAL, "basis handle is NULL");
    return PD_OK;
}

// Entry points defined on the full space only.
pd_status check_full_basis(pd_basis b, const char *what) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (b->truncated) return fail(PD_EINVAL, "%s: not defined on a truncated basis", what);
    return PD_OK;
}

const TruncSpace *trunc_of(pd_basis b) { return b->truncated ? &b->trunc : nullptr; }

// Lowest and highest diagonal element (Monopole_Min and Monopole_Max): the
// state of the n orbits with the smallest (largest) pair energy, ties going
// to the lower (higher) orbit index, summed over its orbits in ascending
// order -- the order in which the truncation kernels sum every diagonal.
void diag_extremes(int omega, int n, const double *d, double *dmin, double *dmax) {
    std::vector<int> idx(omega);
    for (int i = 0; i < omega; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return d[a] < d[c]; });
    uint64_t lo = 0, hi = 0;
    for (int i = 0; i < n; ++i) {
        lo |= 1ull << idx[i];
        hi |= 1ull << idx[omega - 1 - i];
    }
    double a = 0.0, c = 0.0;
    for (int q = 0; q < omega; ++q) {
        if ((lo >> q) & 1ull) a += d[q];
        if ((hi >> q) & 1ull) c += d[q];
    }
    *dmin = a;
    *dmax = c;
}

DiagBins make_bins(int omega, const double *d, double dmin, double dmax, int64_t bins) {
    DiagBins db;
    std::memset(&db, 0, sizeof(db));
    for (int i = 0; i < omega; ++i) db.d[i] = d[i];
    db.dmin = dmin;
    db.scale = dmax > dmin ? (double)bins / (dmax - dmin) : 0.0;
    db.bins = bins;
    return db;
}

struct TruncLayout {
    size_t words, kranks, scan, total;
    int64_t W;
};
TruncLayout trunc_layout(int64_t full_dim, int64_t kept) {
    TruncLayout L;
    L.W = (full_dim + 63) / 64;
    size_t off = kHandleBlockBytes;
    L.words = off;
    off += align256((size_t)L.W * sizeof(TruncWord));
    L.kranks = off;
    off += align256((size_t)kept * (trunc_ranks32(full_dim) ? 4 : 8));
    L.scan = off;
    off += align256(trunc_scan_words(full_dim) * sizeof(uint64_t));
    L.total = off;
    return L;
}

// A handle over dev_buf (its first kHandleBlockBytes are the sigma slots) on
// the current device, with one event per slot; nullptr (message set) on failure.
void delete_handle(pd_basis b) {
    if (!b) return;
    for (int i = 0; i < kSigmaSlots; ++i)
        if (b->slot[i].done) (void)hipEventDestroy(b->slot[i].done);
    delete b;
}

pd_basis new_handle(void *dev_buf) {
    pd_basis b = new (std::nothrow) pd_basis_s;
    if (!b) {
        set_error("host allocation failed");
        return nullptr;
    }
    b->omega = b->n = 0;
    b->dim = 0;
    b->states = nullptr;
    b->next_slot = 0;
    b->truncated = 0;
    std::memset(&b->trunc, 0, sizeof(b->trunc));
    if (hipGetDevice(&b->device) != hipSuccess) b->device = 0;
    for (int i = 0; i < kSigmaSlots; ++i) {
        b->slot[i].dev = reinterpret_cast<CoefBlock *>(static_cast<unsigned char *>(dev_buf) + i * kCoefBytes);
        hipError_t e = hipEventCreateWithFlags(&b->slot[i].done, hipEventDisableTiming);
        if (e != hipSuccess) {
            b->slot[i].done = nullptr;
            set_error("hipEventCreateWithFlags: %s", hipGetErrorString(e));
            delete_handle(b);
            return nullptr;
        }
    }
    return b;
}

// The coefficient block a pd_sigma call on `stream` uses (caller holds b->mu).
// In order of preference: a block last used on this stream with the same
// coefficients, any block last used on this stream, an unused block, a block
// whose last product has finished; else the round-robin victim, after which
// `stream` waits for that block's last product.  A block whose product is
// still running on another stream is thus never rewritten or shared.
pd_status acquire_slot(pd_basis b, const CoefBlock &blk, hipStream_t stream, SigmaSlot **out) {
    SigmaSlot *same = nullptr, *idle = nullptr;
    for (int i = 0; i < kSigmaSlots; ++i) {
        SigmaSlot &s = b->slot[i];
        if (s.used && s.last_stream == stream) {
            if (s.has_coef && std::memcmp(&blk, &s.host, sizeof(CoefBlock)) == 0) {
                *out = &s;
                return PD_OK;
            }
            if (!same) same = &s;
        }
    }
    if (same) {
        *out = same;
        return PD_OK;
    }
    for (int i = 0; i < kSigmaSlots && !idle; ++i)
        if (!b->slot[i].used) idle = &b->slot[i];
    for (int i = 0; i < kSigmaSlots && !idle; ++i) {
        hipError_t q = hipEventQuery(b->slot[i].done);
        if (q == hipSuccess) idle = &b->slot[i];
        else if (q != hipErrorNotReady) return fail(PD_EDEVICE, "hipEventQuery: %s", hipGetErrorString(q));
    }
    if (!idle) {
        idle = &b->slot[b->next_slot++ % kSigmaSlots];
        hipError_t e = hipStreamWaitEvent(stream, idle->done, 0);
        if (e != hipSuccess) return fail(PD_EDEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
    }
    *out = idle;
    return PD_OK;
}

}  // namespace
}  // namespace pd

namespace pd {
namespace {
struct MlpLayout {
    size_t Z1, H1, Z2, H2, L, dL, G2, G1, part, loss, total;
};
bool valid_shape(const pd_mlp_shape *s) {
    return s && s->in >= 1 && s->h1 >= 1 && s->h2 >= 1 && s->out >= 1 && s->in <= 65536 && s->h1 <= 65536 &&
           s->h2 <= 65536 && s->out <= 65536;
}
MlpLayout mlp_layout(const pd_mlp_shape *s, int batch) {
    MlpLayout L;
    size_t off = 0;
    auto take = [&](size_t floats) {
        size_t o = off;
        off += align256(floats * sizeof(float));
        return o;
    };
    const size_t B = (size_t)batch;
    L.Z1 = take(B * s->h1);
    L.H1 = take(B * s->h1);
    L.Z2 = take(B * s->h2);
    L.H2 = take(B * s->h2);
    L.L = take(B * s->out);
    L.dL = take(B * s->out);
    L.G2 = take(B * s->h2);
    L.G1 = take(B * s->h1);
    L.part = take(64);
    L.loss = take(1);
    L.total = off;
    return L;
}
struct MlpParams {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
template <typename P>
P mlp_split(const pd_mlp_shape *s, P base, P *W1, P *b1, P *W2, P *b2, P *W3, P *b3) {
    P q = base;
    *W1 = q;
    q += (size_t)s->in * s->h1;
    *b1 = q;
    q += s->h1;
    *W2 = q;
    q += (size_t)s->h1 * s->h2;
    *b2 = q;
    q += s->h2;
    *W3 = q;
    q += (size_t)s->h2 * s->out;
    *b3 = q;
    q += s->out;
    return q;
}
hipError_t mlp_forward_impl(const pd_mlp_shape *s, const float *P, const float *X, int B, unsigned char *w,
                            const MlpLayout &L, float *logits, hipStream_t st) {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    mlp_split<const float *>(s, P, &W1, &b1, &W2, &b2, &W3, &b3);
    float *Z1 = (float *)(w + L.Z1), *H1 = (float *)(w + L.H1), *Z2 = (float *)(w + L.Z2), *H2 = (float *)(w + L.H2);
    hipError_t e = launch_gemm_bf16(false, false, B, s->h1, s->in, X, s->in, W1, s->h1, Z1, s->h1, b1, 2, H1, st);
    if (e == hipSuccess) e = launch_gemm_bf16(false, false, B, s->h2, s->h1, H1, s->h1, W2, s->h2, Z2, s->h2, b2, 2, H2, st);
    if (e == hipSuccess) e = launch_gemm_bf16(false, false, B, s->out, s->h2, H2, s->h2, W3, s->out, logits, s->out, b3, 1, nullptr, st);
    return e;
}
}  // namespace
}  // namespace pd

using namespace pd;

extern "C" {

const char *pd_version(void) { return "pairdiag-gfx950 0.1"; }

const char *pd_status_str(pd_status s) {
    switch (s) {
        case PD_OK: return "PD_OK";
        case PD_EINVAL: return "PD_EINVAL";
        case PD_ERANGE: return "PD_ERANGE";
        case PD_ENOMEM: return "PD_ENOMEM";
        case PD_EDEVICE: return "PD_EDEVICE";
        case PD_ENOCONV: return "PD_ENOCONV";
    }
    return "PD_UNKNOWN";
}

const char *pd_last_error(void) { return last_error(); }

int64_t pd_dimension(int omega, int n) {
    if (!valid_space(omega, n)) return 0;
    return (int64_t)binom_host(omega, n);
}

size_t pd_basis_bytes(int omega, int n, int store_states) {
    if (!valid_space(omega, n)) return 0;
    size_t b = kHandleBlockBytes;
    if (store_states) b += align256((size_t)binom_host(omega, n) * sizeof(uint64_t));
    return b;
}

pd_status pd_basis_create(int omega, int n, int store_states, void *dev_buf, size_t bytes, hipStream_t stream,
                          pd_basis *out) {
    if (!out) return fail(PD_EINVAL, "out is NULL");
    if (!valid_space(omega, n)) return fail(PD_EINVAL, "invalid space omega=%d n=%d", omega, n);
    size_t need = pd_basis_bytes(omega, n, store_states);
    if (bytes < need) return fail(PD_ENOMEM, "basis buffer %zu bytes, need %zu", bytes, need);
    pd_status st = check_device_ptr(dev_buf, "dev_buf", need);
    if (st != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return fail(PD_EINVAL, "dev_buf must be 256-byte aligned");
    pd_basis b = new_handle(dev_buf);
    if (!b) return fail(PD_EDEVICE, "handle creation: %s", last_error());
    b->omega = omega;
    b->n = n;
    b->dim = (int64_t)binom_host(omega, n);
    b->states = store_states ? reinterpret_cast<uint64_t *>(static_cast<unsigned char *>(dev_buf) + kHandleBlockBytes)
                             : nullptr;
    if (b->states) {
        hipError_t e = launch_basis_build(omega, n, b->dim, b->states, stream);
        if (e != hipSuccess) {
            delete_handle(b);
            return fail(PD_EDEVICE, "basis build: %s", hipGetErrorString(e));
        }
    }
    *out = b;
    return PD_OK;
}

void pd_basis_destroy(pd_basis b) { delete_handle(b); }

pd_status pd_basis_info(pd_basis b, int *omega, int *n, int64_t *dim) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (omega) *omega = b->omega;
    if (n) *n = b->n;
    if (dim) *dim = b->dim;
    return PD_OK;
}

const uint64_t *pd_basis_states(pd_basis b) { return b ? b->states : nullptr; }

pd_status pd_basis_rank(pd_basis b, const uint64_t *states_dev, int64_t count, int64_t *ranks_dev,
                        hipStream_t stream) {
    pd_status st = check_full_basis(b, "pd_basis_rank");
    if (st != PD_OK) return st;
    if (count < 0) return fail(PD_EINVAL, "count < 0");
    if (count == 0) return PD_OK;
    if ((st = check_device_ptr(states_dev, "states_dev", count * 8)) != PD_OK) return st;
    if ((st = check_device_ptr(ranks_dev, "ranks_dev", count * 8)) != PD_OK) return st;
    hipError_t e = launch_basis_rank(b->omega, b->n, states_dev, count, ranks_dev, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "rank: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_basis_unrank(pd_basis b, const int64_t *ranks_dev, int64_t count, uint64_t *states_dev,
                          hipStream_t stream) {
    pd_status st = check_full_basis(b, "pd_basis_unrank");
    if (st != PD_OK) return st;
    if (count < 0) return fail(PD_EINVAL, "count < 0");
    if (count == 0) return PD_OK;
    if ((st = check_device_ptr(states_dev, "states_dev", count * 8)) != PD_OK) return st;
    if ((st = check_device_ptr(ranks_dev, "ranks_dev", count * 8)) != PD_OK) return st;
    hipError_t e = launch_basis_unrank(b->omega, b->n, ranks_dev, count, states_dev, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "unrank: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_sigma(pd_basis b, const double *eps, const double *V, pd_dtype dt, const void *x_dev, void *y_dev,
                   hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (dt != PD_F64 && dt != PD_F32) return fail(PD_EINVAL, "dtype %d", (int)dt);
    if ((st = check_sigma_range(b)) != PD_OK) return st;
    CoefBlock blk;
    if ((st = pack_coefficients(b->omega, b->n, eps, V, &blk)) != PD_OK) return st;
    const size_t es = dt == PD_F64 ? 8 : 4;
    if ((st = check_device_ptr(x_dev, "x_dev", b->dim * es)) != PD_OK) return st;
    if ((st = check_device_ptr(y_dev, "y_dev", b->dim * es)) != PD_OK) return st;
    if (overlap(x_dev, b->dim * es, y_dev, b->dim * es)) return fail(PD_EINVAL, "x and y overlap");
    std::lock_guard<std::mutex> lock(b->mu);
    SigmaSlot *sl = nullptr;
    if ((st = acquire_slot(b, blk, stream, &sl)) != PD_OK) return st;
    // Upload only when the coefficients change; the copy completes before returning.
    if (!sl->has_coef || std::memcmp(&blk, &sl->host, sizeof(CoefBlock)) != 0) {
        sl->host = blk;
        sl->has_coef = 0;
        hipError_t e = hipMemcpyAsync(sl->dev, &sl->host, sizeof(CoefBlock), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(PD_EDEVICE, "coefficient upload: %s", hipGetErrorString(e));
        sl->has_coef = 1;
    }
    hipError_t e = launch_sigma(b->omega, b->n, b->dim, sl->dev, dt, x_dev, y_dev, stream, blk.dsum64, blk.dsum32,
                                trunc_of(b));
    if (e == hipSuccess) e = hipEventRecord(sl->done, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "sigma: %s", hipGetErrorString(e));
    sl->used = 1;
    sl->last_stream = stream;
    return PD_OK;
}

size_t pd_trunc_select_bytes(int omega, int n, int64_t bins) {
    if (!valid_space(omega, n) || bins < 1 || bins > kMaxTruncBins) return 0;
    return align256(trunc_hist_doubles(bins) * sizeof(uint64_t)) + 256;
}

pd_status pd_trunc_select(int omega, int n, const double *eps, const double *V, int64_t limit, int64_t bins,
                          void *work_dev, size_t work_bytes, pd_trunc_info *info, hipStream_t stream) {
    if (!info) return fail(PD_EINVAL, "info is NULL");
    if (!valid_space(omega, n)) return fail(PD_EINVAL, "invalid space omega=%d n=%d", omega, n);
    if (limit < 1) return fail(PD_EINVAL, "limit=%lld < 1", (long long)limit);
    if (bins < 1 || bins > kMaxTruncBins) return fail(PD_EINVAL, "bins=%lld outside [1, %lld]", (long long)bins,
                                                      (long long)kMaxTruncBins);
    std::unique_ptr<CoefBlock> blk(new (std::nothrow) CoefBlock);
    if (!blk) return fail(PD_ENOMEM, "host allocation failed");
    pd_status st = pack_coefficients(omega, n, eps, V, blk.get());
    if (st != PD_OK) return st;
    pd_trunc_info r;
    std::memset(&r, 0, sizeof(r));
    r.full_dim = (int64_t)binom_host(omega, n);
    r.limit = limit;
    r.bins = bins;
    diag_extremes(omega, n, blk->d64, &r.dmin, &r.dmax);
    const DiagBins db = make_bins(omega, blk->d64, r.dmin, r.dmax, bins);
    r.scale = db.scale;
    if (r.full_dim <= limit) {
        r.kept = r.full_dim;
        r.cut_bin = bins - 1;
    } else {
        const size_t need = pd_trunc_select_bytes(omega, n, bins);
        if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
        if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
        if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");
        uint64_t *hist = static_cast<uint64_t *>(work_dev);
        uint64_t *partial = hist + bins;
        TruncCut *cut_dev = reinterpret_cast<TruncCut *>(static_cast<unsigned char *>(work_dev) +
                                                         align256(trunc_hist_doubles(bins) * sizeof(uint64_t)));
        TruncCut cut;
        hipError_t e = launch_trunc_cut(omega, n, r.full_dim, db, limit, hist, partial, cut_dev, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&cut, cut_dev, sizeof(cut), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(PD_EDEVICE, "truncation histogram: %s", hipGetErrorString(e));
        r.cut_bin = cut.cut_bin;
        r.kept = cut.kept;
    }
    r.cutoff = r.scale > 0.0 ? r.dmin + (double)(r.cut_bin + 1) / r.scale : r.dmin;
    *info = r;
    return PD_OK;
}

size_t pd_basis_truncated_bytes(int omega, int n, const pd_trunc_info *info) {
    if (!info || !valid_space(omega, n) || info->full_dim != (int64_t)binom_host(omega, n) || info->kept < 1 ||
        info->kept > info->full_dim)
        return 0;
    return trunc_layout(info->full_dim, info->kept).total;
}

pd_status pd_basis_create_truncated(int omega, int n, const double *eps, const double *V, const pd_trunc_info *info,
                                    int index_mode, void *dev_buf, size_t bytes, hipStream_t stream, pd_basis *out) {
    if (!out || !info) return fail(PD_EINVAL, "out and info are required");
    if (!valid_space(omega, n)) return fail(PD_EINVAL, "invalid space omega=%d n=%d", omega, n);
    if (index_mode != PD_TRUNC_BITMAP && index_mode != PD_TRUNC_BSEARCH)
        return fail(PD_EINVAL, "index_mode=%d", index_mode);
    const int64_t full_dim = (int64_t)binom_host(omega, n);
    if (info->full_dim != full_dim || info->kept < 1 || info->kept > full_dim || info->bins < 1 ||
        info->bins > kMaxTruncBins || info->cut_bin < 0 || info->cut_bin >= info->bins)
        return fail(PD_EINVAL, "info does not describe a selection in this space");
    std::unique_ptr<CoefBlock> blk(new (std::nothrow) CoefBlock);
    if (!blk) return fail(PD_ENOMEM, "host allocation failed");
    pd_status st = pack_coefficients(omega, n, eps, V, blk.get());
    if (st != PD_OK) return st;
    double dmin, dmax;
    diag_extremes(omega, n, blk->d64, &dmin, &dmax);
    const DiagBins db = make_bins(omega, blk->d64, dmin, dmax, info->bins);
    if (dmin != info->dmin || dmax != info->dmax || db.scale != info->scale)
        return fail(PD_EINVAL, "eps and V differ from the ones the selection was made with");
    const TruncLayout L = trunc_layout(full_dim, info->kept);
    if (bytes < L.total) return fail(PD_ENOMEM, "basis buffer %zu bytes, need %zu", bytes, L.total);
    if ((st = check_device_ptr(dev_buf, "dev_buf", L.total)) != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return fail(PD_EINVAL, "dev_buf must be 256-byte aligned");
    unsigned char *base = static_cast<unsigned char *>(dev_buf);
    TruncWord *words = reinterpret_cast<TruncWord *>(base + L.words);
    void *kranks = base + L.kranks;
    uint64_t *scan = reinterpret_cast<uint64_t *>(base + L.scan);
    TruncWord last;
    hipError_t e = launch_trunc_build(omega, n, full_dim, db, info->cut_bin, words, scan, kranks, info->kept, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&last, words + (L.W - 1), sizeof(last), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "truncated basis: %s", hipGetErrorString(e));
    const int64_t built = (int64_t)(last.base + (uint64_t)__builtin_popcountll(last.bits));
    if (built != info->kept)
        return fail(PD_EINVAL, "selection keeps %lld states, info says %lld", (long long)built, (long long)info->kept);
    pd_basis b = new_handle(dev_buf);
    if (!b) return fail(PD_EDEVICE, "handle creation: %s", last_error());
    b->omega = omega;
    b->n = n;
    b->dim = info->kept;
    b->states = nullptr;
    b->truncated = 1;
    b->trunc.full_dim = full_dim;
    b->trunc.kept = info->kept;
    b->trunc.kranks = kranks;
    b->trunc.words = words;
    b->trunc.index_mode = index_mode == PD_TRUNC_BSEARCH ? kTruncBsearch : kTruncBitmap;
    *out = b;
    return PD_OK;
}

pd_status pd_basis_kept_ranks(pd_basis b, int64_t *ranks_dev, hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (!b->truncated) return fail(PD_EINVAL, "pd_basis_kept_ranks: the basis is not truncated");
    if ((st = check_device_ptr(ranks_dev, "ranks_dev", (size_t)b->dim * 8)) != PD_OK) return st;
    hipError_t e = launch_trunc_ranks64(b->trunc, ranks_dev, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "kept ranks: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_basis_truncation(pd_basis b, int *truncated, int64_t *full_dim) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (truncated) *truncated = b->truncated;
    if (full_dim) *full_dim = b->truncated ? b->trunc.full_dim : b->dim;
    return PD_OK;
}

void pd_lanczos_default_opts(pd_lanczos_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->krylov = 50;
    o->tol = 1e-10;
    o->max_restarts = 1000;
    o->mode = 0;
    o->start = PD_START_E1;
    o->seed = 0;
    o->precision = PD_F64;
    o->fallback = 0;
    o->verbose = 0;
}

static pd_status check_opts(const pd_lanczos_opts *o) {
    if (!o) return fail(PD_EINVAL, "opts is NULL");
    if (o->krylov < 2 || o->krylov > 64) return fail(PD_EINVAL, "krylov=%d outside [2, 64]", o->krylov);
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(PD_EINVAL, "tol must be finite and >= 0");
    if (o->max_restarts < 0) return fail(PD_EINVAL, "max_restarts < 0");
    if (o->mode != 0 && o->mode != 1) return fail(PD_EINVAL, "mode must be 0 or 1");
    if (o->start < PD_START_E1 || o->start > PD_START_USER) return fail(PD_EINVAL, "start=%d", o->start);
    if (o->precision < 0 || o->precision > 2) return fail(PD_EINVAL, "precision=%d", o->precision);
    return PD_OK;
}

size_t pd_lanczos_workspace_bytes(pd_basis b, const pd_lanczos_opts *o) {
    if (!b || check_opts(o) != PD_OK) return 0;
    return lanczos_workspace_bytes(b->dim, o);
}

pd_status pd_lanczos_ground(pd_basis b, const double *eps, const double *V, const pd_lanczos_opts *o,
                            void *work_dev, size_t work_bytes, const double *x0_dev, double *E0, double *psi0_dev,
                            double *occ, pd_lanczos_info *info, hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if ((st = check_opts(o)) != PD_OK) return st;
    if (!E0) return fail(PD_EINVAL, "E0 is NULL");
    if ((st = check_sigma_range(b)) != PD_OK) return st;
    CoefBlock blk;
    if ((st = pack_coefficients(b->omega, b->n, eps, V, &blk)) != PD_OK) return st;
    size_t need = lanczos_workspace_bytes(b->dim, o);
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");
    if (o->start == PD_START_USER) {
        if ((st = check_device_ptr(x0_dev, "x0_dev", b->dim * 8)) != PD_OK) return st;
    }
    if (psi0_dev) {
        if ((st = check_device_ptr(psi0_dev, "psi0_dev", b->dim * 8)) != PD_OK) return st;
        if (overlap(psi0_dev, b->dim * 8, work_dev, work_bytes)) return fail(PD_EINVAL, "psi0 overlaps workspace");
    }
    return lanczos_run(b, blk, o, work_dev, work_bytes, x0_dev, E0, psi0_dev, occ, info, stream);
}

pd_status pd_lanczos_ground_static(pd_basis b, const double *eps, const double *V, const pd_lanczos_opts *o,
                                   const double *x0_dev, double *E0, double *psi0_dev, double *occ,
                                   pd_lanczos_info *info, hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if ((st = check_opts(o)) != PD_OK) return st;
    if (!E0) return fail(PD_EINVAL, "E0 is NULL");
    if ((st = check_sigma_range(b)) != PD_OK) return st;
    CoefBlock blk;
    if ((st = pack_coefficients(b->omega, b->n, eps, V, &blk)) != PD_OK) return st;
    const size_t need = lanczos_workspace_bytes(b->dim, o);
    if (need > kStaticScratchBytes)
        return fail(PD_ERANGE, "workspace of %zu bytes exceeds the static %zu-byte array (use pd_lanczos_ground)",
                    need, kStaticScratchBytes);
    if (o->start == PD_START_USER) {
        if ((st = check_device_ptr(x0_dev, "x0_dev", b->dim * 8)) != PD_OK) return st;
    }
    if (psi0_dev) {
        if ((st = check_device_ptr(psi0_dev, "psi0_dev", b->dim * 8)) != PD_OK) return st;
    }
    void *work = nullptr;
    std::mutex *call_mu = nullptr;
    if ((st = static_scratch(&work, &call_mu)) != PD_OK) return st;
    std::lock_guard<std::mutex> lk(*call_mu);
    st = lanczos_run(b, blk, o, work, kStaticScratchBytes, x0_dev, E0, psi0_dev, occ, info, stream, false);
    // An early error return may leave work queued: let it finish before the
    // next call may reuse the array.
    if (st != PD_OK) (void)hipStreamSynchronize(stream);
    return st;
}

size_t pd_lanczos_eigs_workspace_bytes(pd_basis b, int nev, const pd_lanczos_opts *o) {
    if (!b || nev < 1 || check_opts(o) != PD_OK) return 0;
    return lanczos_eigs_workspace_bytes(b->dim, o);
}

pd_status pd_lanczos_eigs(pd_basis b, const double *eps, const double *V, int nev, const pd_lanczos_opts *o,
                          void *work_dev, size_t work_bytes, double *E, double *psi_dev, double *occ,
                          double *residuals, pd_lanczos_info *info, hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if ((st = check_opts(o)) != PD_OK) return st;
    if (!E) return fail(PD_EINVAL, "E is NULL");
    if (nev < 1 || nev > b->dim) return fail(PD_EINVAL, "nev=%d outside [1, dim=%lld]", nev, (long long)b->dim);
    if ((st = check_sigma_range(b)) != PD_OK) return st;
    CoefBlock blk;
    if ((st = pack_coefficients(b->omega, b->n, eps, V, &blk)) != PD_OK) return st;
    size_t need = lanczos_eigs_workspace_bytes(b->dim, o);
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");
    if (psi_dev) {
        const size_t pb = (size_t)nev * (size_t)b->dim * 8;
        if ((st = check_device_ptr(psi_dev, "psi_dev", pb)) != PD_OK) return st;
        if (overlap(psi_dev, pb, work_dev, work_bytes)) return fail(PD_EINVAL, "psi_dev overlaps workspace");
    }
    return lanczos_eigs_run(b, blk, nev, o, work_dev, work_bytes, E, psi_dev, occ, residuals, info, stream);
}

size_t pd_occupations_workspace_bytes(pd_basis b) {
    if (!b) return 0;
    return align256(partial_doubles() * sizeof(double)) + align256(64 * sizeof(double));
}

pd_status pd_occupations(pd_basis b, const double *psi_dev, void *work_dev, size_t work_bytes, double *occ_host,
                         hipStream_t stream) {
    pd_status st = check_basis(b);
    if (st != PD_OK) return st;
    if (!occ_host) return fail(PD_EINVAL, "occ_host is NULL");
    size_t need = pd_occupations_workspace_bytes(b);
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    if ((st = check_device_ptr(psi_dev, "psi_dev", b->dim * 8)) != PD_OK) return st;
    if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
    double *partials = static_cast<double *>(work_dev);
    double *occ_dev = reinterpret_cast<double *>(static_cast<unsigned char *>(work_dev) +
                                                 align256(partial_doubles() * sizeof(double)));
    hipError_t e = launch_occupations(b->omega, b->n, b->dim, psi_dev, partials, occ_dev, stream, trunc_of(b));
    if (e == hipSuccess) e = hipMemcpyAsync(occ_host, occ_dev, b->omega * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "occupations: %s", hipGetErrorString(e));
    return PD_OK;
}

size_t pd_batched_workspace_bytes(int count, const int *omega, const int *n, const pd_lanczos_opts *o) {
    if (check_opts(o) != PD_OK || batched_validate(count, omega, n, o) != PD_OK) return 0;
    return batched_workspace_bytes(count, omega, n, o);
}

pd_status pd_lanczos_ground_batched(int count, const int *omega, const int *n, const double *eps_packed,
                                    const double *V_packed, const pd_lanczos_opts *o, int block, void *work_dev,
                                    size_t work_bytes, double *E0_out, double *occ_out, pd_lanczos_info *info_out,
                                    pd_batch_info *binfo, hipStream_t stream) {
    pd_status st = check_opts(o);
    if (st != PD_OK) return st;
    if ((st = batched_validate(count, omega, n, o)) != PD_OK) return st;
    if (!eps_packed || !V_packed || !E0_out) return fail(PD_EINVAL, "eps_packed, V_packed and E0_out are required");
    if (block != 0 && block != 128 && block != 256 && block != 512) return fail(PD_EINVAL, "block=%d", block);
    size_t need = batched_workspace_bytes(count, omega, n, o);
    if (work_bytes < need) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, need);
    if ((st = check_device_ptr(work_dev, "work_dev", need)) != PD_OK) return st;
    if (reinterpret_cast<uintptr_t>(work_dev) & 255) return fail(PD_EINVAL, "work_dev must be 256-byte aligned");
    return batched_run(count, omega, n, eps_packed, V_packed, o, block, work_dev, work_bytes, E0_out, occ_out,
                       info_out, binfo, stream);
}

pd_status pd_warm_start(pd_basis b, const float *logits_dev, double *x0_dev, hipStream_t stream) {
    pd_status st = check_full_basis(b, "pd_warm_start");
    if (st != PD_OK) return st;
    if ((st = check_sigma_range(b, false)) != PD_OK) return st;
    if ((st = check_device_ptr(logits_dev, "logits_dev", b->omega * sizeof(float))) != PD_OK) return st;
    if ((st = check_device_ptr(x0_dev, "x0_dev", b->dim * sizeof(double))) != PD_OK) return st;
    float l[64];
    hipError_t e = hipMemcpyAsync(l, logits_dev, b->omega * sizeof(float), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "logits copy: %s", hipGetErrorString(e));
    double ls[64];
    for (int i = 0; i < b->omega; ++i) {
        if (!std::isfinite(l[i])) return fail(PD_EINVAL, "logit %d is not finite", i);
        ls[i] = l[i];
    }
    std::sort(ls, ls + b->omega, [](double a, double c) { return a > c; });
    double lmax = 0.0;
    for (int i = 0; i < b->n; ++i) lmax += ls[i];
    e = launch_warm_expand(b->omega, b->n, b->dim, logits_dev, lmax, x0_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "warm start: %s", hipGetErrorString(e));
    return PD_OK;
}


size_t pd_mlp_param_count(const pd_mlp_shape *s) {
    if (!valid_shape(s)) return 0;
    return (size_t)s->in * s->h1 + s->h1 + (size_t)s->h1 * s->h2 + s->h2 + (size_t)s->h2 * s->out + s->out;
}

size_t pd_mlp_workspace_bytes(const pd_mlp_shape *s, int batch) {
    if (!valid_shape(s) || batch < 1) return 0;
    return mlp_layout(s, batch).total;
}

pd_status pd_mlp_forward(const pd_mlp_shape *s, const float *params_dev, const float *X_dev, int batch, void *work_dev,
                         size_t work_bytes, float *logits_dev, hipStream_t stream) {
    if (!valid_shape(s) || batch < 1) return fail(PD_EINVAL, "bad network shape or batch");
    MlpLayout L = mlp_layout(s, batch);
    if (work_bytes < L.total) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, L.total);
    pd_status st;
    if ((st = check_device_ptr(params_dev, "params_dev", pd_mlp_param_count(s) * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(X_dev, "X_dev", (size_t)batch * s->in * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(work_dev, "work_dev", L.total)) != PD_OK) return st;
    if ((st = check_device_ptr(logits_dev, "logits_dev", (size_t)batch * s->out * 4)) != PD_OK) return st;
    hipError_t e = mlp_forward_impl(s, params_dev, X_dev, batch, (unsigned char *)work_dev, L, logits_dev, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "mlp forward: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_mlp_backward(const pd_mlp_shape *s, const float *params_dev, const float *X_dev, const float *target_dev,
                          int batch, void *work_dev, size_t work_bytes, float *grads_dev, float *loss_dev,
                          hipStream_t stream) {
    if (!valid_shape(s) || batch < 1) return fail(PD_EINVAL, "bad network shape or batch");
    MlpLayout L = mlp_layout(s, batch);
    if (work_bytes < L.total) return fail(PD_ENOMEM, "workspace %zu bytes, need %zu", work_bytes, L.total);
    const size_t np = pd_mlp_param_count(s);
    pd_status st;
    if ((st = check_device_ptr(params_dev, "params_dev", np * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(X_dev, "X_dev", (size_t)batch * s->in * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(target_dev, "target_dev", (size_t)batch * s->out * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(work_dev, "work_dev", L.total)) != PD_OK) return st;
    if ((st = check_device_ptr(grads_dev, "grads_dev", np * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(loss_dev, "loss_dev", 4)) != PD_OK) return st;
    unsigned char *w = (unsigned char *)work_dev;
    float *Lg = (float *)(w + L.L), *dL = (float *)(w + L.dL);
    hipError_t e = mlp_forward_impl(s, params_dev, X_dev, batch, w, L, Lg, stream);
    if (e == hipSuccess) e = launch_mlp_loss(batch * s->out, Lg, target_dev, dL, (float *)(w + L.part), loss_dev, stream);
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    mlp_split<const float *>(s, params_dev, &W1, &b1, &W2, &b2, &W3, &b3);
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    mlp_split<float *>(s, grads_dev, &gW1, &gb1, &gW2, &gb2, &gW3, &gb3);
    float *Z1 = (float *)(w + L.Z1), *H1 = (float *)(w + L.H1), *Z2 = (float *)(w + L.Z2), *H2 = (float *)(w + L.H2);
    float *G2 = (float *)(w + L.G2), *G1 = (float *)(w + L.G1);
    const int B = batch;
    // layer 3
    if (e == hipSuccess) e = launch_gemm_bf16(true, false, s->h2, s->out, B, H2, s->h2, dL, s->out, gW3, s->out, nullptr, 0, nullptr, stream);
    if (e == hipSuccess) e = launch_colsum(B, s->out, dL, gb3, stream);
    if (e == hipSuccess) e = launch_gemm_bf16(false, true, B, s->h2, s->out, dL, s->out, W3, s->out, G2, s->h2, nullptr, 0, nullptr, stream);
    if (e == hipSuccess) e = launch_gelu_back(B * s->h2, Z2, G2, stream);
    // layer 2
    if (e == hipSuccess) e = launch_gemm_bf16(true, false, s->h1, s->h2, B, H1, s->h1, G2, s->h2, gW2, s->h2, nullptr, 0, nullptr, stream);
    if (e == hipSuccess) e = launch_colsum(B, s->h2, G2, gb2, stream);
    if (e == hipSuccess) e = launch_gemm_bf16(false, true, B, s->h1, s->h2, G2, s->h2, W2, s->h2, G1, s->h1, nullptr, 0, nullptr, stream);
    if (e == hipSuccess) e = launch_gelu_back(B * s->h1, Z1, G1, stream);
    // layer 1
    if (e == hipSuccess) e = launch_gemm_bf16(true, false, s->in, s->h1, B, X_dev, s->in, G1, s->h1, gW1, s->h1, nullptr, 0, nullptr, stream);
    if (e == hipSuccess) e = launch_colsum(B, s->h1, G1, gb1, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "mlp backward: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_mlp_adam(int64_t count, float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int step,
                      float lr, float beta1, float beta2, float eps, hipStream_t stream) {
    if (count < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return fail(PD_EINVAL, "bad Adam arguments");
    pd_status st;
    if ((st = check_device_ptr(params_dev, "params_dev", count * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(grads_dev, "grads_dev", count * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(m_dev, "m_dev", count * 4)) != PD_OK) return st;
    if ((st = check_device_ptr(v_dev, "v_dev", count * 4)) != PD_OK) return st;
    hipError_t e = launch_adam((int)count, params_dev, grads_dev, m_dev, v_dev, lr, beta1, beta2, eps, step, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "adam: %s", hipGetErrorString(e));
    return PD_OK;
}

pd_status pd_sigma_launch_shape(int omega, int n, pd_dtype dt, int *threads, int64_t *lds_bytes,
                                int64_t *lds_limit_bytes) {
    if (!threads || !lds_bytes || !lds_limit_bytes) return fail(PD_EINVAL, "an output pointer is NULL");
    if (!valid_space(omega, n)) return fail(PD_EINVAL, "invalid space omega=%d n=%d", omega, n);
    if (dt != PD_F64 && dt != PD_F32) return fail(PD_EINVAL, "bad dtype %d", (int)dt);
    const int nn = std::min(n, omega - n);
    if (nn > kMaxSigmaPairs) return fail(PD_ERANGE, "min(n, omega-n)=%d exceeds %d", nn, kMaxSigmaPairs);
    if (!sigma_launch_shape(omega, n, dt, threads, lds_bytes, lds_limit_bytes))
        return fail(PD_ERANGE, "no product kernel for %d pairs", nn);
    return PD_OK;
}

int64_t pd_stream_probe_bytes(int kind, int64_t n) {
    if (n <= 0) return 0;
    switch (kind & ~PD_PROBE_NONTEMPORAL) {
        case PD_PROBE_READ: return 4 * n;
        case PD_PROBE_COPY: return 8 * n;
        case PD_PROBE_TRIAD: return 12 * n;
        case PD_PROBE_WRITE: return 4 * n;
    }
    return 0;
}

pd_status pd_stream_probe(int kind, const float *a_dev, const float *b_dev, float *c_dev, int64_t n,
                          hipStream_t stream) {
    const int k = kind & ~PD_PROBE_NONTEMPORAL;
    if (k < PD_PROBE_READ || k > PD_PROBE_WRITE) return fail(PD_EINVAL, "probe kind %d", kind);
    if (n <= 0 || n % 1024) return fail(PD_EINVAL, "n=%lld is not a positive multiple of 1024", (long long)n);
    const size_t nb = (size_t)n * 4;
    pd_status st;
    if (k != PD_PROBE_WRITE && (st = check_device_ptr(a_dev, "a_dev", nb)) != PD_OK) return st;
    if (k == PD_PROBE_TRIAD && (st = check_device_ptr(b_dev, "b_dev", nb)) != PD_OK) return st;
    if ((st = check_device_ptr(c_dev, "c_dev", k == PD_PROBE_READ ? (size_t)probe_grid(PD_PROBE_READ, n) * 4 : nb)) != PD_OK)
        return st;
    if (k != PD_PROBE_WRITE && overlap(a_dev, nb, c_dev, nb)) return fail(PD_EINVAL, "c overlaps a");
    if (k == PD_PROBE_TRIAD && overlap(b_dev, nb, c_dev, nb)) return fail(PD_EINVAL, "c overlaps b");
    hipError_t e = launch_stream_probe(k, (kind & PD_PROBE_NONTEMPORAL) != 0, a_dev, b_dev, c_dev, n, stream);
    if (e != hipSuccess) return fail(PD_EDEVICE, "stream probe: %s", hipGetErrorString(e));
    return PD_OK;
}

int pd_tridiag_lowest(int m, const double *alpha, const double *beta, double *theta, double *y) {
    if (!alpha || !theta || !y || (m > 1 && !beta)) return -1;
    return tridiag_lowest(m, alpha, beta, theta, y);
}

}  // extern "C"
