/*
 * pairdiag.h -- C ABI of the MI355X (gfx950) library for exact diagonalisation
 * of general pairing Hamiltonians in the seniority-zero space.
 *
 * The Hamiltonian is Eq. hamiltonian2 of Liu & Qi, "PairDiag: an exact
 * diagonalization program for solving general pairing Hamiltonians":
 *     H = sum_i (2 eps_i + V_ii) S+_i S-_i + sum_{i != j} V_ij S+_i S-_j
 * on omega doubly-degenerate orbits holding n pairs (the paper's m pairs in n
 * orbits, Sec. 3.1).  V is the paper's pairing matrix P_F taken literally
 * (attractive pairing has V_ij < 0).
 *
 * Conventions shared by every entry point:
 *   - Device memory is owned by the caller (any allocator; the Python binding
 *     uses torch tensors).  The library never allocates device memory; each
 *     object states the bytes it needs through a *_bytes query.  Host arrays
 *     are read during the call only.
 *   - Arguments are validated before any device work; invalid arguments
 *     return PD_EINVAL (or PD_ERANGE / PD_ENOMEM) and leave outputs untouched.
 *     A HIP failure returns PD_EDEVICE.  pd_last_error() gives a thread-local
 *     message for the last failure.
 *   - Work is issued on the given stream (0 = the null stream).  Entry points
 *     that return host scalars synchronise that stream before returning;
 *     the others are asynchronous and stream-ordered.
 *   - Basis ranks are 0-based: rank = f(|i>) - 1 with the hash of Sec. 3.2.
 *     The basis order is the ascending order of Tab. data and Alg. conversion.
 *   - Vectors are indexed by rank, length dim = C(omega, n) (Eq. extcmn).
 */
#ifndef PAIRDIAG_H
#define PAIRDIAG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PD_OK = 0,
    PD_EINVAL = 1,   /* bad argument (sizes, non-finite or non-symmetric V, null pointer) */
    PD_ERANGE = 2,   /* valid but unsupported size (e.g. dim does not fit the index type) */
    PD_ENOMEM = 3,   /* caller buffer smaller than the matching *_bytes query */
    PD_EDEVICE = 4,  /* HIP runtime error; see pd_last_error() */
    PD_ENOCONV = 5   /* iteration stopped before the tolerance; outputs hold the best iterate */
} pd_status;

typedef enum { PD_F64 = 0, PD_F32 = 1 } pd_dtype;

/* Start vectors of the Lanczos iteration (Sec. 3.4: the paper's default is e_1). */
typedef enum {
    PD_START_E1 = 0,      /* [1, 0, ..., 0]: the paper's Vector_Initialize */
    PD_START_HF = 1,      /* basis state with the n smallest 2 eps_i + V_ii */
    PD_START_RANDOM = 2,  /* x_k = 2 u_k - 1, u_k from SplitMix64 (seed, counter k) */
    PD_START_USER = 3     /* caller vector x0_dev (any norm, must be non-zero) */
} pd_start;

const char *pd_version(void);
const char *pd_status_str(pd_status s);
/* Thread-local description of the last non-OK status returned on this thread. */
const char *pd_last_error(void);

/* ------------------------------------------------------------------ basis
 * Sec. 3.1 (basis generation, Alg. conversion) and Sec. 3.2 (Eq. hash).
 * A basis handle describes the space (omega, n) and carries a small
 * coefficient block used by pd_sigma.  With store_states != 0 the library also
 * writes the ascending array of occupation bitstrings (uint64, bit i =
 * orbit i) into the caller buffer; sigma and the Lanczos driver never read it
 * (they recover states from ranks on the fly), so large spaces may skip it.
 * Limits: 1 <= omega <= 62, 0 <= n <= omega (Sec. 3.1: fewer than 63 orbits).
 */
typedef struct pd_basis_s *pd_basis;

/* Device bytes pd_basis_create needs; 0 for invalid (omega, n). */
size_t pd_basis_bytes(int omega, int n, int store_states);
/* Number of states C(omega, n); 0 for invalid (omega, n). */
int64_t pd_dimension(int omega, int n);
/* Builds the handle in *out.  dev_buf must stay valid while the handle lives. */
pd_status pd_basis_create(int omega, int n, int store_states, void *dev_buf, size_t bytes,
                          hipStream_t stream, pd_basis *out);
/* NULL-safe; never frees dev_buf. */
void pd_basis_destroy(pd_basis b);
pd_status pd_basis_info(pd_basis b, int *omega, int *n, int64_t *dim);
/* Device pointer of the stored state array (NULL if store_states was 0). */
const uint64_t *pd_basis_states(pd_basis b);
/* ranks_dev[q] = rank of states_dev[q], or -1 if it is not an n-pair state
 * of the omega orbits.  Both arrays are device memory of `count` entries. */
pd_status pd_basis_rank(pd_basis b, const uint64_t *states_dev, int64_t count,
                        int64_t *ranks_dev, hipStream_t stream);
/* states_dev[q] = state of rank ranks_dev[q]; ranks must lie in [0, dim). */
pd_status pd_basis_unrank(pd_basis b, const int64_t *ranks_dev, int64_t count,
                          uint64_t *states_dev, hipStream_t stream);

/* ------------------------------------------------------------------ truncation
 * Sec. 3.5: when C(omega, n) exceeds a dimension limit (Dimension_Limit), the
 * states with the highest diagonal elements (Eq. diagonal) are left out.
 * Every diagonal, summed over the occupied orbits in ascending order in FP64,
 * falls in one of `bins` equal bins between dmin and dmax (the paper uses
 * 1e8): bin = clamp(floor((diag - dmin) * scale), 0, bins - 1) with
 * scale = bins / (dmax - dmin) (0 if dmax == dmin).  dmin and dmax are the
 * diagonals of the n orbits with the smallest and the largest pair energy
 * 2 eps_i + V_ii (stable order, so ties go to the lower index for dmin and to
 * the higher index for dmax): Monopole_Min and Monopole_Max.  The bins are
 * accumulated from the bottom; the cut bin is the last one whose running count
 * is <= limit (bin 0 if bin 0 alone exceeds it), and a state is kept iff its
 * bin is <= the cut bin.  Kept states keep the basis order.
 *
 * pd_trunc_select computes the cut (a histogram pass over the full space on
 * the GPU; no device work if C(omega, n) <= limit).  work_dev: device, 256-byte
 * aligned, pd_trunc_select_bytes(omega, n, bins) bytes (8 bytes per bin);
 * bins in [1, 2^30].  Synchronises `stream`.
 *
 * pd_basis_create_truncated builds a basis handle over the kept states from
 * the same eps and V (PD_EINVAL if dmin, dmax or scale come out different):
 * its dimension is info->kept, and pd_sigma, pd_lanczos_ground and
 * pd_occupations act on the truncated space (H restricted to it: hops to
 * states left out are dropped).  A hop target is located by its full-space
 * rank (Sec. 3.2) and then mapped to its row: index_mode PD_TRUNC_BITMAP uses
 * one 16-byte word per 64 full ranks (which are kept, how many kept before);
 * PD_TRUNC_BSEARCH binary-searches the ascending kept ranks, as the paper
 * does for truncated spaces.  dev_buf: device, 256-byte aligned,
 * pd_basis_truncated_bytes(omega, n, info) bytes (full dim / 4 bytes for the
 * words, 4 or 8 bytes per kept state for its full rank: 4 when
 * C(omega, n) < 2^32).  pd_basis_rank, pd_basis_unrank and pd_warm_start
 * reject truncated handles.  Synchronises `stream`.
 *
 * pd_basis_kept_ranks: ranks_dev (device, dim int64) receives the full-space
 * rank of every kept state, ascending.  pd_basis_truncation: whether a handle
 * is truncated, and the full dimension. */
enum { PD_TRUNC_BITMAP = 0, PD_TRUNC_BSEARCH = 1 };
typedef struct {
    int64_t full_dim;  /* C(omega, n) */
    int64_t limit;     /* the dimension limit asked for */
    int64_t kept;      /* states kept (= full_dim when full_dim <= limit) */
    int64_t bins;
    int64_t cut_bin;   /* a state is kept iff its bin <= cut_bin */
    double dmin, dmax; /* lowest and highest diagonal element */
    double scale;      /* bins / (dmax - dmin), 0 if dmax == dmin */
    double cutoff;     /* upper edge of the cut bin, dmin + (cut_bin + 1) / scale (informative) */
} pd_trunc_info;
size_t pd_trunc_select_bytes(int omega, int n, int64_t bins);
pd_status pd_trunc_select(int omega, int n, const double *eps, const double *V, int64_t limit, int64_t bins,
                          void *work_dev, size_t work_bytes, pd_trunc_info *info, hipStream_t stream);
size_t pd_basis_truncated_bytes(int omega, int n, const pd_trunc_info *info);
pd_status pd_basis_create_truncated(int omega, int n, const double *eps, const double *V, const pd_trunc_info *info,
                                    int index_mode, void *dev_buf, size_t bytes, hipStream_t stream, pd_basis *out);
pd_status pd_basis_kept_ranks(pd_basis b, int64_t *ranks_dev, hipStream_t stream);
pd_status pd_basis_truncation(pd_basis b, int *truncated, int64_t *full_dim);

/* ------------------------------------------------------------------ sigma
 * y = H x, the matrix-free product of Sec. 3.3: every non-zero element is
 * generated from the pair hops |j> = S+_E S-_O |i> and located by its rank.
 * eps: host, omega doubles.  V: host, omega*omega doubles, row-major, exactly
 * symmetric and finite.  x, y: device vectors of dim elements of dtype dt
 * (PD_F64: double gathers and accumulation; PD_F32: float gathers, float
 * accumulation, coefficients rounded to float).  x and y must not overlap.
 * The handle's device buffer holds 4 coefficient blocks, each with the
 * kernel's tile counters.  A call takes a block that is unused, or
 * was last used on the same stream (stream order protects it), or whose last
 * product has finished; if every block is busy on other streams, `stream`
 * first waits for the oldest one's product.  So concurrent calls on one
 * handle from different streams and host threads are allowed and each
 * returns the complete product (at most 4 of them run truly in parallel).
 * When the coefficients differ from those the chosen block holds they are
 * uploaded on `stream` and the stream is synchronised; otherwise the call is
 * fully asynchronous.  pd_lanczos_ground keeps its own block in its
 * workspace.
 * PD_ERANGE, before any device work: min(n, omega - n) above 20; or a full
 * space with n = omega - 16 and omega 33, 34 or 35 (mirrored, 16 pairs,
 * 32-bit ranks), whose product is disabled: it made an illegal memory access
 * at omega = 34, n = 18 for a cause not yet found.  The same holds for the
 * Lanczos entry points and everything built on them (pd_scf_ground, the
 * odd-system blocks); truncated spaces are not affected.
 */
pd_status pd_sigma(pd_basis b, const double *eps, const double *V, pd_dtype dt,
                   const void *x_dev, void *y_dev, hipStream_t stream);

/* Launch shape of pd_sigma on the space (omega, n) in precision dt, without
 * running anything (an implementation detail, not a passage of the paper):
 * *threads = threads per workgroup (256 or 512), *lds_bytes = its dynamic
 * LDS, *lds_limit_bytes = the LDS limit the kernel runs under (the
 * instantiation's attribute above the default 64 KB, else that default);
 * pd_sigma's launch succeeds only when lds_bytes <= lds_limit_bytes.  The
 * shape is reported for the spaces pd_sigma refuses too.  Host only, no
 * device needed.  PD_EINVAL: bad space, dtype or NULL output;
 * PD_ERANGE: min(n, omega - n) above the largest kernel's pair count. */
pd_status pd_sigma_launch_shape(int omega, int n, pd_dtype dt, int *threads, int64_t *lds_bytes,
                                int64_t *lds_limit_bytes);

/* ------------------------------------------------------------------ Lanczos
 * Restarted, fully reorthogonalised Lanczos (Sec. 3.4, Alg. lanczos): Krylov
 * vectors are orthogonalised against all stored vectors (classical
 * Gram-Schmidt after the three-term recurrence, applied a second time when the
 * first pass leaves less than 1/sqrt(2) of the norm it started from, or less
 * than 1/128 of ||H q||), the lowest Ritz pair of the krylov x krylov
 * tridiagonal matrix comes from Sturm bisection and inverse iteration, and
 * the iteration restarts from the
 * ground-state Ritz vector.  Convergence (Eq. convergence): the restarted
 * vector q has rho = ||H q - (q^T H q) q|| / |q^T H q| <= tol; rho is computed
 * with an FP64 product.  mode 1 stops after the first cycle (no restart).
 * In mixed precision the FP64 refinement (an FP64 product of the restart
 * vector, which gives alpha_1 and the residual) runs at the start of every
 * cycle; there is no option to space it out (no refine_every).
 */
typedef struct {
    int krylov;        /* vectors per cycle (Lanc_Limit); 2..64; default 50 */
    double tol;        /* Lanc_Error; default 1e-10 */
    int max_restarts;  /* cycles after the first; default 1000 */
    int mode;          /* 0 restarted (default), 1 single cycle */
    int start;         /* pd_start; default PD_START_E1 */
    uint64_t seed;     /* PD_START_RANDOM stream */
    int fallback;      /* PD_START_USER only: 1 = also try the RANDOM start and keep the one
                          with the lower Rayleigh quotient (two extra products) */
    int precision;     /* PD_F64 (default) or PD_F32: FP32 products for Krylov steps
                          k >= 2 of every cycle, on Krylov vectors q_2..q_m stored in
                          FP32; the first step of each cycle and q_1, all dot products,
                          the recurrence, the reorthogonalisation arithmetic, the
                          tridiagonal solve and the Ritz vectors stay FP64 (the mixed
                          workspace is about half the FP64 one); 2: FP32 products as
                          for PD_F32, every Krylov vector stored in FP64 (the product
                          reads an FP32 copy of q_k; the FP64 workspace and more) */
    int verbose;       /* 1: one line per cycle on stderr */
} pd_lanczos_opts;

typedef struct {
    int iterations;      /* products H q (FP64 + FP32) */
    int iterations_f32;  /* of which FP32 */
    int restarts;        /* cycles after the first */
    int converged;       /* 1 if rho <= tol */
    double residual;     /* final rho */
    double monopole_min; /* smallest diagonal element (Monopole_Min, Sec. 4.3) */
    double seconds;      /* wall time of the call */
    double sigma_seconds_f64;  /* summed device time of the FP64 products (HIP events) */
    double sigma_seconds_f32;  /* summed device time of the FP32 products (HIP events) */
    int fallback_used;         /* 1 if the fallback replaced the caller's start vector */
    int reorth_second_passes;  /* steps whose Gram-Schmidt needed the second pass */
} pd_lanczos_info;

void pd_lanczos_default_opts(pd_lanczos_opts *o);
/* Device workspace bytes for pd_lanczos_ground with these options. */
size_t pd_lanczos_workspace_bytes(pd_basis b, const pd_lanczos_opts *o);
/* Ground state of H.  Outputs: *E0 (= q^T H q of the returned vector),
 * psi0_dev (device, dim doubles, optional: normalised, sum(psi) >= 0),
 * occ (host, omega doubles, optional: <N_i> = 2 <S+_i S-_i>, Sec. 4.3 N_Occup),
 * info (optional).  x0_dev: device start vector for PD_START_USER, else NULL.
 * Returns PD_ENOCONV (outputs filled) if max_restarts is reached first.
 * Synchronises `stream`. */
pd_status pd_lanczos_ground(pd_basis b, const double *eps, const double *V,
                            const pd_lanczos_opts *o, void *work_dev, size_t work_bytes,
                            const double *x0_dev, double *E0, double *psi0_dev, double *occ,
                            pd_lanczos_info *info, hipStream_t stream);

/* pd_lanczos_ground without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The workspace is a static device array
 * of PD_STATIC_SCRATCH_BYTES (256 MiB) inside the library, one per GPU, held
 * until the process ends.  The call allocates nothing (no device memory, no
 * events: info->sigma_seconds_f64/_f32 stay 0).  A problem whose
 * pd_lanczos_workspace_bytes exceeds the array returns PD_ERANGE before any
 * device work.  Every call on a GPU shares that GPU's array and leaves its
 * contents behind; the solver writes every part it reads first.  Calls
 * that overlap on one GPU would race on it: within this process a lock
 * serialises them (each call synchronises its stream before returning);
 * overlapping calls from other code that writes the array are not allowed.
 * psi0_dev must not point into the array.  Arguments, outputs and the other
 * errors as pd_lanczos_ground.  Synchronises `stream`. */
#define PD_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
pd_status pd_lanczos_ground_static(pd_basis b, const double *eps, const double *V, const pd_lanczos_opts *o,
                                   const double *x0_dev, double *E0, double *psi0_dev, double *occ,
                                   pd_lanczos_info *info, hipStream_t stream);

/* The nev lowest eigenpairs (the paper's "first few states", Sec. 3.4) by
 * thick-restart Lanczos, FP64: each cycle extends the kept Ritz vectors by
 * Krylov steps (the step of pd_lanczos_ground: recurrence subtracted, one
 * Gram-Schmidt pass against all stored vectors, a second on the DGKS or
 * rounding test) up to krylov vectors; the restart keeps the
 * min(krylov - 1, nev + (krylov - nev) / 2) lowest Ritz vectors and the
 * residual direction.  Stops when every wanted Ritz residual estimate is
 * <= tol; each returned pair is then checked with an explicit FP64 product:
 * E[i] is its Rayleigh quotient and residuals[i] = ||H u - E u|| / |E|.
 * Options: krylov >= nev + 2 (unless krylov >= dim), tol, max_restarts,
 * mode 1 = one cycle (FP64), start PD_START_E1 or PD_START_RANDOM (seed),
 * precision PD_F64, or PD_F32: FP32 products on FP32 copies of the columns
 * until every wanted estimate is below 3e-6 (or, below 1e-4, stops falling), then a fresh
 * FP64 run from the sum of the wanted Ritz vectors to tol (iterations counts
 * both, iterations_f32 the first).  A start vector's Krylov space holds one vector per
 * distinct eigenvalue: an exactly degenerate level appears once.
 * Outputs: E (host, nev doubles, ascending); psi_dev (optional, device,
 * nev x dim doubles, state i at psi_dev + i * dim, normalised, sum >= 0);
 * occ (optional, host, nev x omega); residuals (optional, host, nev);
 * info (iterations = products including the checks, restarts = cycles,
 * residual = the largest explicit residual).  Returns PD_ENOCONV (outputs
 * filled; NaN for pairs the Krylov space did not contain) if a pair misses
 * the tolerance.  Works on truncated handles.  Synchronises `stream`. */
size_t pd_lanczos_eigs_workspace_bytes(pd_basis b, int nev, const pd_lanczos_opts *o);
pd_status pd_lanczos_eigs(pd_basis b, const double *eps, const double *V, int nev, const pd_lanczos_opts *o,
                          void *work_dev, size_t work_bytes, double *E, double *psi_dev, double *occ,
                          double *residuals, pd_lanczos_info *info, hipStream_t stream);

/* The exact pairing solution inside a self-consistent mean-field loop, the
 * use the paper names for it in place of BCS (Sec. 1, Sec. 6).  The mean
 * field is synthetic: eps_i = eps0_i + sum_j W_ij <N_j> / 2 (W host,
 * omega x omega row-major, finite).  Iteration t solves the ground state of
 * Eq. hamiltonian2 with eps^(t) and V (pd_lanczos_ground with o; from the
 * second iteration on, with reuse_psi, started from the previous ground state),
 * forms eps_new = eps0 + W <N> / 2 and stops when max |eps_new - eps^(t)| <= tol,
 * else eps^(t+1) = (1 - mixing) eps^(t) + mixing eps_new.
 * o->start: E1, HF or RANDOM (the first solve).  work_dev: device, 256-byte
 * aligned, pd_scf_workspace_bytes(b, o) bytes.  Outputs (host): eps_out (the
 * eps of the last solve), occ_out (its <N_i>), *E0 (its ground-state energy);
 * psi0_dev (optional, device, dim doubles, outside the workspace) its ground
 * state; info.  Host or foreign pointers, short allocations, mixing outside
 * (0, 1], a non-finite W or a PD_START_USER start give PD_EINVAL (a short
 * work_bytes PD_ENOMEM) before any device work.
 * Returns PD_ENOCONV (outputs filled) if max_iter is reached first.
 * Synchronises `stream`. */
typedef struct {
    int max_iter;     /* iterations (solves) at most */
    double tol;       /* on max |eps_new - eps| */
    double mixing;    /* in (0, 1] */
    int reuse_psi;    /* 1: start every solve after the first from the previous ground state */
} pd_scf_opts;
typedef struct {
    int iterations;         /* solves */
    int converged;          /* 1 if the field change met tol */
    int products;           /* H q products over all solves */
    int products_first;     /* of the first solve */
    int lanczos_converged;  /* 1 if every solve met o->tol */
    double change;          /* max |eps_new - eps| of the last iteration */
    double last_residual;   /* rho of the last solve */
    double seconds;
} pd_scf_info;
size_t pd_scf_workspace_bytes(pd_basis b, const pd_lanczos_opts *o);
pd_status pd_scf_ground(pd_basis b, const double *eps0, const double *W, const double *V, const pd_scf_opts *so,
                        const pd_lanczos_opts *o, void *work_dev, size_t work_bytes, double *eps_out,
                        double *occ_out, double *E0, double *psi0_dev, pd_scf_info *info, hipStream_t stream);

/* <N_i> = 2 sum_k psi_k^2 [orbit i occupied in state k] for a device vector
 * psi (dim doubles, not renormalised); occ_host receives omega doubles.
 * work_dev needs pd_occupations_workspace_bytes(b).  Synchronises `stream`. */
size_t pd_occupations_workspace_bytes(pd_basis b);
pd_status pd_occupations(pd_basis b, const double *psi_dev, void *work_dev, size_t work_bytes,
                         double *occ_host, hipStream_t stream);

/* ------------------------------------------------------------------ batched
 * Many independent ground-state problems (as in a mean-field sweep that
 * replaces BCS by the exact solution, Sec. 1 and Sec. 6) solved in ONE
 * persistent kernel launch captured in a HIP graph: a device work queue hands
 * instances, largest first, to workgroups, and each workgroup runs the whole
 * restarted Lanczos iteration of pd_lanczos_ground for its instance (FP64,
 * random start with seed o->seed + instance index, tol / max_restarts / krylov
 * from o; krylov <= 32).  Limits per instance: omega <= 32, min(n, omega-n) <= 12
 * (instances with n > omega - n are solved as their particle-hole complement,
 * an exact identity: E0 = E0' + sum_i (2 eps_i + V_ii), <N_i> = 2 - <N_i>').
 * Inputs (host): omega[count], n[count]; eps_packed: the omega_i single-particle
 * energies of each instance back to back; V_packed: the omega_i x omega_i row-major
 * couplings back to back.  Outputs (host): E0_out[count]; occ_out (optional):
 * sum(omega_i) doubles, packed like eps; info_out (optional, per instance:
 * iterations, restarts, converged, residual); binfo (optional).
 * block: workgroup size 128, 256 or 512, or 0 to autotune it on a sample of the
 * batch (the choice is cached per batch shape for the life of the process;
 * batches of at most 32 instances, where the sample would be the whole batch,
 * take 512 untuned).  A cost model (work per product, team barrier overhead)
 * picks how many of the costliest instances are first solved by teams of
 * workgroups (grid = all compute units, split into 8 teams, or into the
 * smallest power of two of teams that covers them when fewer than 5 instances
 * go to teams) that split the rows and meet at a bounded-wait barrier; if a
 * wait times out (another kernel holding compute units) the call returns
 * PD_EDEVICE.  Without teams the grid is min(count, compute units).  The
 * workspace holds one Krylov slot of (krylov + 2) x (largest dimension)
 * doubles per team and one per workgroup sized for the largest instance left
 * to single workgroups (pd_batched_workspace_bytes): a batch that sends 5 or
 * more instances to teams, the largest of 2.26e8 states (omega = 32, 12
 * pairs), needs 8 such slots, more than one device holds at krylov 20; solve
 * such instances with pd_lanczos_ground.  Returns PD_ENOCONV if any
 * instance missed the tolerance (all outputs filled).  info_out[i].seconds is
 * the device time the instance took.
 * Synchronises `stream`. */
typedef struct {
    int block;             /* workgroup size used */
    int grid;              /* persistent workgroups (one per compute unit; at most count without teams) */
    int tuned;             /* 1 if this call ran the autotuner */
    int teams;             /* workgroup teams for the large instances (0: none) */
    int team_size;         /* workgroups per team */
    int large;             /* instances solved by teams */
    int converged;         /* instances that met the tolerance */
    long long total_iterations;
    double tune_seconds;
    double kernel_seconds; /* the graph launch, to completion */
    double seconds;        /* the whole call */
} pd_batch_info;

size_t pd_batched_workspace_bytes(int count, const int *omega, const int *n, const pd_lanczos_opts *o);
pd_status pd_lanczos_ground_batched(int count, const int *omega, const int *n, const double *eps_packed,
                                    const double *V_packed, const pd_lanczos_opts *o, int block,
                                    void *work_dev, size_t work_bytes, double *E0_out, double *occ_out,
                                    pd_lanczos_info *info_out, pd_batch_info *binfo, hipStream_t stream);

/* ------------------------------------------------------------------ odd mass
 * 2n + 1 particles in the blocking approximation (Sec. 2, Eq. hamiltonian3):
 * the unpaired particle on orbit b keeps pairs out of b, so the seniority-one
 * space is a direct sum of blocks b = 1..omega with
 *     H_b = eps_b + H(n pairs on the omega - 1 orbits other than b),
 * H being Eq. hamiltonian2 with eps and V restricted to those orbits.
 * block (the Block argument of Sec. 4.2): b in [1, omega] solves H_b only;
 * 0 solves every H_b and returns the lowest (ties: the smallest b).
 * route (block = 0 only; 0 for block != 0): PD_ODD_AUTO picks PD_ODD_BATCHED
 * when a block fits pd_lanczos_ground_batched (omega - 1 <= 32,
 * min(n, omega-1-n) <= 12, krylov <= 32) and has at most 2^22 states, else
 * PD_ODD_SEQUENTIAL.  BATCHED solves the omega blocks in one batched launch
 * (FP64, RANDOM starts with seed o->seed + b - 1, workgroup size 512);
 * SEQUENTIAL builds one basis of the reduced space in the workspace and runs
 * pd_lanczos_ground once per block with o as given.
 * Inputs (host): eps[omega] (single-particle energies), V[omega*omega]
 * (symmetric, finite), as for pd_lanczos_ground; omega in [2, 62];
 * n in [0, omega - 1] is the number of pairs (N_Pairs = n + 1/2).
 * o->start must not be PD_START_USER.
 * work_dev: device, 256-byte aligned, pd_odd_workspace_bytes(...) bytes.
 * Outputs (host): *E = the lowest solved E_b, eps_b included;
 * block_out (optional) its b (1-based); E_blocks (optional, omega doubles)
 * E_b of each block, NaN for blocks not solved; occ (optional, omega
 * doubles) the chosen block's <N_i>, with 1 on orbit b (Sec. 4.3, N_Occup);
 * info (optional) sums iterations, restarts, products and device times over
 * the blocks solved, residual = the largest, converged = all, monopole_min =
 * the smallest diagonal element over the solved blocks, seconds = the call.
 * Returns PD_ENOCONV (outputs filled) if a block missed the tolerance;
 * PD_ERANGE if the reduced space exceeds what sigma (or a forced batched
 * route) handles; PD_EINVAL / PD_ENOMEM on bad arguments or a short
 * workspace.  Synchronises `stream`. */
enum { PD_ODD_AUTO = 0, PD_ODD_SEQUENTIAL = 1, PD_ODD_BATCHED = 2 };
size_t pd_odd_workspace_bytes(int omega, int n, int block, int route, const pd_lanczos_opts *o);
pd_status pd_lanczos_ground_odd(int omega, int n, const double *eps, const double *V, int block, int route,
                                const pd_lanczos_opts *o, void *work_dev, size_t work_bytes, double *E,
                                int *block_out, double *E_blocks, double *occ, pd_lanczos_info *info,
                                hipStream_t stream);

/* ------------------------------------------------------------------ warm start
 * A small network maps an instance to one logit l_i per orbit; sigmoid(l_i)
 * estimates the half occupation <N_i>/2.  Taking it as the BCS v_i^2 gives
 * pair amplitudes v_i/u_i = exp(l_i/2), and the number-projected product state
 *     psi_k = prod_{i occupied in k} exp(l_i / 2)
 * is the start vector (computed as exp((sum_occ l_i - L)/2), L = sum of the n
 * largest l_i, so entries lie in (0, 1]; not normalised).
 * logits_dev: device, omega floats.  x0_dev: device, dim doubles.  Synchronises. */
pd_status pd_warm_start(pd_basis b, const float *logits_dev, double *x0_dev, hipStream_t stream);

/* Network: in -> h1 -> h2 -> out, GELU (tanh form) after the two hidden
 * layers, linear output.  Parameters: one FP32 device array, in this order:
 * W1 (in x h1, row-major), b1 (h1), W2 (h1 x h2), b2 (h2), W3 (h2 x out), b3 (out).
 * Activations are row-major (batch x features).  Products run on BF16 matrix
 * cores (operands rounded from FP32, FP32 accumulation).
 * Loss: mean over batch x out of (sigmoid(logit) - target)^2. */
typedef struct { int in, h1, h2, out; } pd_mlp_shape;
size_t pd_mlp_param_count(const pd_mlp_shape *s);
size_t pd_mlp_workspace_bytes(const pd_mlp_shape *s, int batch);
/* logits_dev: batch x out (device).  On return the workspace begins with
 * Z1 = X W1 + b1, the first layer's pre-activations (batch x h1 floats,
 * row-major). */
pd_status pd_mlp_forward(const pd_mlp_shape *s, const float *params_dev, const float *X_dev, int batch,
                         void *work_dev, size_t work_bytes, float *logits_dev, hipStream_t stream);
/* Forward, loss and backward: grads_dev (param_count floats) receives d loss / d params,
 * loss_dev (one float, device) the loss. */
pd_status pd_mlp_backward(const pd_mlp_shape *s, const float *params_dev, const float *X_dev,
                          const float *target_dev, int batch, void *work_dev, size_t work_bytes,
                          float *grads_dev, float *loss_dev, hipStream_t stream);
/* Adam (Kingma & Ba) with bias correction, step >= 1; m, v: state arrays of count floats. */
pd_status pd_mlp_adam(int64_t count, float *params_dev, const float *grads_dev, float *m_dev, float *v_dev,
                      int step, float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* ------------------------------------------------------------------ measurement
 * Achievable HBM bandwidth (not part of the method; the yardstick its
 * streaming kernels and its product are measured against).  One launch of a
 * streaming kernel over n floats with 16-byte vector accesses, every element
 * touched once, so the bytes it moves are exactly pd_stream_probe_bytes:
 *   PD_PROBE_READ   sums a; one partial sum per workgroup goes to c_dev[0..]   4 n bytes
 *   PD_PROBE_COPY   c = a                                                      8 n bytes
 *   PD_PROBE_TRIAD  c = a + 0.5 b                                             12 n bytes
 *   PD_PROBE_WRITE  c = 0.5                                                    4 n bytes
 * OR-ing PD_PROBE_NONTEMPORAL marks the accesses as streaming (no reuse).
 * a_dev, b_dev, c_dev: device float arrays of n elements (a unused by WRITE,
 * b used by TRIAD only; pass NULL for unused ones); c must not overlap a or b.
 * n: a positive multiple of 1024.  Asynchronous on `stream`.  PD_EINVAL on
 * a bad kind, n, pointer or overlap (no device work). */
enum { PD_PROBE_READ = 0, PD_PROBE_COPY = 1, PD_PROBE_TRIAD = 2, PD_PROBE_WRITE = 3, PD_PROBE_NONTEMPORAL = 16 };
int64_t pd_stream_probe_bytes(int kind, int64_t n);
pd_status pd_stream_probe(int kind, const float *a_dev, const float *b_dev, float *c_dev, int64_t n,
                          hipStream_t stream);

/* ------------------------------------------------------------------ host utility
 * Lowest eigenpair of the m x m symmetric tridiagonal matrix with diagonal
 * alpha[0..m) and off-diagonal beta[0..m-1) (the Lanczos matrix L of
 * Alg. lanczos), 1 <= m <= 64; y receives the unit eigenvector with y[0] >= 0.
 * Host arrays, no device work.  Returns 0, or a negative value on bad input. */
int pd_tridiag_lowest(int m, const double *alpha, const double *beta, double *theta, double *y);

#ifdef __cplusplus
}
#endif
#endif /* PAIRDIAG_H */
