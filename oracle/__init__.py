"""Oracle for the PairDiag method: plain, slow, obviously correct, CPU only.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU
library (the C part lives in pd_oracle.c and is built with gcc by build()).
Everything is FP64.

Functions and the passages they follow:
  binom, basis_alg1, next_state, hash_index, unhash,    Sec. 3.1-3.2, Eq. extcmn, Tab. data (ascending basis, the
    index_bsearch                                         order of Alg. conversion), Eq. hash, binary search
  sigma, sigma_sampled, row_terms, dense_h                Sec. 3.3, Eq. hamiltonian2, Eq. diagonal
  dense_ground                                            E0 as the lowest eigenvalue of the explicit H
  lanczos_ground                                          Sec. 3.4, Alg. lanczos, full reorthogonalisation,
                                                          restart with the ground Ritz vector, Eq. convergence
  lowest_eigenpairs                                       the first few states (Sec. 3.4): lowest eigenpairs of H
                                                          by a library eigensolver (dense, or ARPACK on sigma)
  occupations, monopole_min                               Sec. 4.3 outputs N_Occup and Monopole_Min
  blocked_instance, odd_ground                            Sec. 2 Eq. hamiltonian3 (blocking), Sec. 4.2 Block, Sec. 4.3 N_Occup
  scf_ground                                              Sec. 1 and 6: the exact solution inside a self-consistent
                                                          loop (synthetic mean field eps0 + W <N>/2, linear mixing)
  diagonals, trunc_select, sigma(index_mode=              Sec. 3.5 truncation (diagonal histogram, cut, binary
    'bsearch_truncated'), trunc_kept_ranks,               search in the truncated basis; for spaces too large to
    trunc_sigma_sampled                                   store: C histogram, the ascending kept ranks, sampled
                                                          rows with every index found by binary search in them)
  richardson_evb                                          constant-G check (Richardson equations, eigenvalue form)
  pbcs_vector                                             number-projected product start vector (warm start)
  mlp_*                                                   FP64 reference of the warm-start network

Parity status: every function here is pinned by a not-gpu test (paper tables,
closed forms, invariants, brute force), except the trained network weights,
which are not a function of the paper ("parity unpinned": judged by the
iterations they save).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_SO = os.path.join(_HERE, "_pd_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile pd_oracle.c with gcc (OpenMP over rows)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        P = ctypes.c_void_p
        L.or_binom.restype, L.or_binom.argtypes = u64, [i32, i32]
        L.or_next_state.restype, L.or_next_state.argtypes = u64, [u64]
        L.or_basis_alg1.restype, L.or_basis_alg1.argtypes = i64, [i32, i32, P, i64]
        L.or_hash.restype, L.or_hash.argtypes = i64, [u64]
        L.or_unhash.restype, L.or_unhash.argtypes = u64, [i64, i32]
        L.or_index_bsearch.restype, L.or_index_bsearch.argtypes = i64, [P, i64, u64]
        L.or_sigma_rows.restype = i32
        L.or_sigma_rows.argtypes = [i32, i32, P, P, P, i64, i32, P, P, i64, i64]
        L.or_sigma_sampled.restype = i32
        L.or_sigma_sampled.argtypes = [i32, i32, P, P, i64, P, P, i64, P]
        L.or_dense_h.restype, L.or_dense_h.argtypes = i32, [i32, i32, P, P, P, i64, P]
        L.or_trunc_count.restype = i32
        L.or_trunc_count.argtypes = [i32, i32, P, dbl, dbl, i64, i32, i64, i64, P]
        L.or_trunc_kept_ranks.restype = i64
        L.or_trunc_kept_ranks.argtypes = [i32, i32, P, dbl, dbl, i64, i64, P, i64]
        L.or_trunc_sigma_sampled.restype = i32
        L.or_trunc_sigma_sampled.argtypes = [i32, i32, P, P, P, i64, P, i64, P, P]
        L.or_sigma_block.restype = i32
        L.or_sigma_block.argtypes = [i32, i32, P, P, i64, P, i64, i64, P]
        L.or_row_terms.restype = dbl
        L.or_row_terms.argtypes = [i32, i32, P, P, i64, P, P, ctypes.POINTER(i64)]
        L.or_occupations.restype, L.or_occupations.argtypes = None, [i32, P, i64, P, P]
        L.or_num_threads.restype, L.or_num_threads.argtypes = i32, []
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- basis (Sec. 3.1-3.2)

def binom(n: int, m: int) -> int:
    """C^m_n of Eq. extcmn (0 for n < m)."""
    return int(lib().or_binom(n, m))


def next_state(s: int) -> int:
    return int(lib().or_next_state(s))


def basis_alg1(omega: int, n: int) -> np.ndarray:
    """All C^n_omega states in ascending order (Tab. data; the order Alg.
    conversion visits them), each the successor of the one before."""
    d = binom(omega, n)
    out = np.empty(d, dtype=np.uint64)
    got = lib().or_basis_alg1(omega, n, _p(out), d)
    if got != d:
        raise RuntimeError(f"basis generation produced {got} states, expected {d}")
    return out


def hash_index(s: int) -> int:
    """0-based f(|s>) - 1 of Eq. hash."""
    return int(lib().or_hash(int(s)))


def unhash(r: int, n: int) -> int:
    return int(lib().or_unhash(int(r), n))


def index_bsearch(basis: np.ndarray, t: int) -> int:
    return int(lib().or_index_bsearch(_p(basis), basis.size, int(t)))


# ---------------------------------------------------------------- H (Sec. 3.3)

def _check_h(omega, eps, V):
    eps = _f64(eps)
    V = _f64(V)
    assert eps.shape == (omega,) and V.shape == (omega, omega)
    return eps, V


def sigma(omega: int, n: int, eps, V, basis: np.ndarray, x, index_mode: str = "bsearch",
          rows: tuple[int, int] | None = None) -> np.ndarray:
    """y = H x over rows [r0, r1) (all rows by default).  index_mode 'bsearch'
    (independent path), 'hash' (the paper's fast path, used for timing) or
    'bsearch_truncated' (basis is a truncated space, Sec. 3.5: hops to states
    outside it are dropped)."""
    eps, V = _check_h(omega, eps, V)
    x = _f64(x)
    r0, r1 = rows if rows is not None else (0, basis.size)
    y = np.empty(r1 - r0)
    mode = {"bsearch": 0, "hash": 1, "bsearch_truncated": 2}[index_mode]
    rc = lib().or_sigma_rows(omega, n, _p(eps), _p(V), _p(basis), basis.size, mode, _p(x), _p(y), r0, r1)
    if rc != 0:
        raise RuntimeError("hop target missing from the basis")
    return y


def sigma_sampled(omega: int, n: int, eps, V, x, rows) -> np.ndarray:
    """(H x)[r] for the listed ranks r, with no stored basis (inverse hash + hash)."""
    eps, V = _check_h(omega, eps, V)
    x = _f64(x)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty(rows.size)
    rc = lib().or_sigma_sampled(omega, n, _p(eps), _p(V), binom(omega, n), _p(x), _p(rows),
                                rows.size, _p(y))
    if rc != 0:
        raise RuntimeError("bad row or hop target")
    return y


def sigma_block(omega: int, n: int, eps, V, x, r0: int, r1: int) -> np.ndarray:
    """(H x)[r0:r1] as the paper's program computes it: states one after the
    other by the basis successor, targets by the hash (no stored basis; x is
    the full vector)."""
    eps, V = _check_h(omega, eps, V)
    x = _f64(x)
    y = np.empty(r1 - r0)
    if lib().or_sigma_block(omega, n, _p(eps), _p(V), binom(omega, n), _p(x), r0, r1, _p(y)) != 0:
        raise RuntimeError("bad row range")
    return y


def row_terms(omega: int, n: int, eps, V, rows):
    """For each rank r: the diagonal H_rr, the hop targets and their elements
    (Sec. 3.3), from the hash alone.  Returns (diag[c], targets[c, K], coefs[c, K]),
    K = n(omega - n), so that (H x)[r] = diag*x[r] + sum(coefs * x[targets])."""
    eps, V = _check_h(omega, eps, V)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    K = n * (omega - n)
    diag = np.empty(rows.size)
    tg = np.empty((rows.size, max(K, 1)), dtype=np.int64)
    cf = np.empty((rows.size, max(K, 1)))
    cnt = ctypes.c_int64()
    for q, r in enumerate(rows):
        diag[q] = lib().or_row_terms(omega, n, _p(eps), _p(V), int(r), _p(tg[q]), _p(cf[q]), ctypes.byref(cnt))
        if cnt.value != K:
            raise RuntimeError(f"bad row {r}")
    return diag, tg[:, :K], cf[:, :K]


def dense_h(omega: int, n: int, eps, V, basis: np.ndarray | None = None) -> np.ndarray:
    eps, V = _check_h(omega, eps, V)
    if basis is None:
        basis = basis_alg1(omega, n)
    d = basis.size
    if d > 13000:
        raise ValueError("dense H only for small spaces")
    H = np.zeros((d, d))
    if lib().or_dense_h(omega, n, _p(eps), _p(V), _p(basis), d, _p(H)) != 0:
        raise RuntimeError("hop target missing from the basis")
    return H


def occupations(omega: int, basis: np.ndarray, psi) -> np.ndarray:
    """<N_i> = 2 <S+_i S-_i> (Sec. 4.3, N_Occup)."""
    psi = _f64(psi)
    occ = np.empty(omega)
    lib().or_occupations(omega, _p(basis), basis.size, _p(psi), _p(occ))
    return occ


def monopole_min(omega: int, n: int, eps, V) -> float:
    """Minimum diagonal element (Monopole_Min, the Hartree-Fock energy):
    the sum of the n smallest pair energies 2 eps_i + V_ii (Eq. diagonal)."""
    eps, V = _check_h(omega, eps, V)
    d = np.sort(2.0 * eps + np.diag(V))
    return float(d[:n].sum())


def _normalise_sign(psi: np.ndarray) -> np.ndarray:
    psi = psi / np.linalg.norm(psi)
    return -psi if psi.sum() < 0 else psi


def dense_ground(omega: int, n: int, eps, V):
    """E0, psi0 and <N_i> from the explicit matrix (library eigensolver)."""
    basis = basis_alg1(omega, n)
    H = dense_h(omega, n, eps, V, basis)
    w, Z = np.linalg.eigh(H)
    psi = _normalise_sign(Z[:, 0])
    return float(w[0]), psi, occupations(omega, basis, psi), w


# ---------------------------------------------------------------- Lanczos (Sec. 3.4)

def lanczos_ground(omega: int, n: int, eps, V, krylov: int = 50, tol: float = 1e-10,
                   max_restarts: int = 200, start=None, restart: bool = True,
                   basis: np.ndarray | None = None, index_mode: str = "bsearch"):
    """Restarted Lanczos of Alg. lanczos with Gram-Schmidt against all stored
    vectors (applied twice), Ritz pairs of the tridiagonal L, restart from the
    ground-state Ritz vector, stop when |beta_1/alpha_1| <= tol (Eq. convergence).

    start: None -> [1, 0, ..., 0] (the paper's default), else a vector.
    Returns dict(E0, psi, occ, iterations, restarts, residual)."""
    eps, V = _check_h(omega, eps, V)
    if basis is None:
        basis = basis_alg1(omega, n)
    d = basis.size
    H = lambda v: sigma(omega, n, eps, V, basis, v, index_mode)
    if start is None:
        p = np.zeros(d)
        p[0] = 1.0
    else:
        p = _f64(start).copy()
    m = min(krylov, d)
    iterations = 0
    residual = math.inf
    theta = math.nan
    for cycle in range(max_restarts + 1):
        Q = np.zeros((m, d))
        alpha = np.zeros(m)
        beta = np.zeros(m)
        k_used = m
        for i in range(m):
            Q[i] = p / np.linalg.norm(p)
            p = H(Q[i])
            iterations += 1
            alpha[i] = Q[i] @ p
            p = p - alpha[i] * Q[i] - (beta[i - 1] * Q[i - 1] if i > 0 else 0.0)
            for _ in range(2):
                p = p - Q[: i + 1].T @ (Q[: i + 1] @ p)
            beta[i] = np.linalg.norm(p)
            if i == 0:
                residual = beta[0] / max(abs(alpha[0]), 1e-300)
                if cycle > 0 and residual <= tol:
                    theta = alpha[0]
                    psi = Q[0]
                    return _finish(omega, basis, psi, theta, iterations, cycle, residual)
            if beta[i] <= 1e-14 * max(abs(alpha[i]), 1.0):
                k_used = i + 1
                break
        T = np.diag(alpha[:k_used]) + np.diag(beta[: k_used - 1], 1) + np.diag(beta[: k_used - 1], -1)
        w, Z = np.linalg.eigh(T)
        theta = w[0]
        psi = Q[:k_used].T @ Z[:, 0]
        if k_used < m or not restart:
            r = H(psi / np.linalg.norm(psi))
            t = psi / np.linalg.norm(psi)
            residual = np.linalg.norm(r - (t @ r) * t) / abs(t @ r)
            return _finish(omega, basis, psi, t @ r, iterations, cycle, residual)
        p = psi
    return _finish(omega, basis, psi, theta, iterations, max_restarts, residual)


def lowest_eigenpairs(omega: int, n: int, eps, V, nev: int, dense_limit: int = 6000):
    """The nev lowest eigenvalues of H with eigenvectors (normalised, sum >= 0)
    and their N_Occup: the definition, by a library eigensolver -- dense eigh
    up to dense_limit states, otherwise ARPACK (scipy eigsh, smallest
    algebraic) on a linear operator that applies the oracle's own product."""
    eps, V = _check_h(omega, eps, V)
    basis = basis_alg1(omega, n)
    d = basis.size
    if d <= dense_limit:
        w, Z = np.linalg.eigh(dense_h(omega, n, eps, V, basis))
        w, Z = w[:nev], Z[:, :nev]
    else:
        from scipy.sparse.linalg import LinearOperator, eigsh
        op = LinearOperator((d, d), matvec=lambda v: sigma(omega, n, eps, V, basis, np.ravel(v)), dtype=np.float64)
        w, Z = eigsh(op, k=nev, which="SA", tol=1e-13, v0=np.ones(d), ncv=max(2 * nev + 20, 40))
        order = np.argsort(w)
        w, Z = w[order], Z[:, order]
    Z = np.stack([_normalise_sign(Z[:, i]) for i in range(nev)], axis=1)
    occ = np.stack([occupations(omega, basis, Z[:, i]) for i in range(nev)])
    return w, Z, occ


def _finish(omega, basis, psi, theta, iterations, restarts, residual):
    psi = _normalise_sign(psi)
    return dict(E0=float(theta), psi=psi, occ=occupations(omega, basis, psi),
                iterations=iterations, restarts=restarts, residual=float(residual))


# ---------------------------------------------------------------- truncation (Sec. 3.5)

def diagonals(omega: int, eps, V, basis: np.ndarray) -> np.ndarray:
    """Diagonal element of every state (Eq. diagonal), summed over the occupied
    orbits in ascending order."""
    eps, V = _check_h(omega, eps, V)
    d = 2.0 * eps + np.diag(V)
    acc = np.zeros(basis.size)
    for q in range(omega):
        occ = ((basis >> np.uint64(q)) & np.uint64(1)).astype(bool)
        acc[occ] += d[q]
    return acc


def trunc_select(omega: int, n: int, eps, V, limit: int, bins: int = 10**8, method: str = "auto"):
    """The truncation of Sec. 3.5.  If C(omega, n) exceeds `limit`, the
    diagonal elements are counted in `bins` equal bins from the smallest to the
    largest diagonal (Monopole_Min to Monopole_Max), the bins are accumulated
    from the bottom, and the states in the bins up to the last one whose
    running count is still within the limit are kept (bin 0 in any case).
    The extreme diagonals are those of the n orbits with the smallest and the
    largest pair energy (stable order of 2 eps_i + V_ii).
    method: 'numpy' (stored basis, vectorised), 'c' (bins counted by rank in C,
    for spaces too large to store; states and ranks are then None) or 'auto'.
    Returns dict(full_dim, kept, cut_bin, dmin, dmax, scale, states, ranks)."""
    eps, V = _check_h(omega, eps, V)
    full = binom(omega, n)
    d = 2.0 * eps + np.diag(V)
    order = np.argsort(d, kind="stable")
    def extreme(orbits):
        acc = 0.0
        for q in sorted(int(i) for i in orbits):
            acc += d[q]
        return acc
    dmin = extreme(order[:n])
    dmax = extreme(order[omega - n:])
    scale = bins / (dmax - dmin) if dmax > dmin else 0.0
    if method == "c" or (method == "auto" and full > 4_000_000):
        if full <= limit:
            return dict(full_dim=full, kept=full, cut_bin=bins - 1, dmin=dmin, dmax=dmax, scale=scale,
                        states=None, ranks=None)
        dd = np.zeros(62)
        dd[:omega] = d
        # The running count in two levels: chunks of 4096 bins, then the bins
        # of the chunk in which it first exceeds the limit.
        def count(shift, lo, length):
            out = np.zeros(length, dtype=np.uint64)
            if lib().or_trunc_count(omega, n, _p(dd), dmin, scale, bins, shift, lo, length,
                                    out.ctypes.data_as(ctypes.c_void_p)) != 0:
                raise RuntimeError("bad count range")
            return out.astype(np.int64)
        nchunks = (bins + 4095) // 4096
        coarse = np.concatenate([count(12, lo, min(65536, nchunks - lo)) for lo in range(0, nchunks, 65536)])
        ccum = np.cumsum(coarse)
        c = int(np.searchsorted(ccum, limit, side="right"))   # first chunk whose running count exceeds limit
        base = int(ccum[c - 1]) if c > 0 else 0
        fine_cum = base + np.cumsum(count(0, c * 4096, min(4096, bins - c * 4096)))
        k = int(np.searchsorted(fine_cum, limit, side="right")) - 1
        if k >= 0:
            cut, kept = c * 4096 + k, int(fine_cum[k])
        elif c > 0:
            cut, kept = c * 4096 - 1, base
        else:
            cut, kept = 0, int(fine_cum[0])
        return dict(full_dim=full, kept=kept, cut_bin=cut, dmin=dmin, dmax=dmax, scale=scale,
                    states=None, ranks=None)
    basis = basis_alg1(omega, n)
    if full <= limit:
        return dict(full_dim=full, kept=full, cut_bin=bins - 1, dmin=dmin, dmax=dmax, scale=scale,
                    states=basis, ranks=np.arange(full))
    v = np.floor((diagonals(omega, eps, V, basis) - dmin) * scale)
    b = np.where(v > 0.0, np.minimum(v, bins - 1), 0.0).astype(np.int64)
    cum = np.cumsum(np.bincount(b, minlength=bins))
    cut = max(int(np.searchsorted(cum, limit, side="right")) - 1, 0)
    keep = b <= cut
    return dict(full_dim=full, kept=int(keep.sum()), cut_bin=cut, dmin=dmin, dmax=dmax, scale=scale,
                states=basis[keep], ranks=np.nonzero(keep)[0])


# ---------------------------------------------------------------- self-consistent loop (Sec. 1, Sec. 6)

def scf_ground(omega: int, n: int, eps0, W, V, mixing: float = 0.5, tol: float = 1e-10, max_iter: int = 200):
    """The exact pairing solution inside a self-consistent mean-field loop, the
    use the paper names for it in place of BCS.  The mean field is synthetic:
    eps_i = eps0_i + sum_j W_ij <N_j> / 2.  Iteration t solves the pairing
    ground state with eps^(t) (dense), forms eps_new = eps0 + W occ / 2, stops
    when max |eps_new - eps^(t)| <= tol, else mixes
    eps^(t+1) = (1 - mixing) eps^(t) + mixing eps_new.
    Returns dict(eps, occ, E0, iterations, change) for the last solve."""
    eps0, V = _check_h(omega, eps0, V)
    W = _f64(W)
    eps = eps0.copy()
    for it in range(1, max_iter + 1):
        E0, _, occ, _ = dense_ground(omega, n, eps, V)
        new = eps0 + W @ occ / 2.0
        change = float(np.max(np.abs(new - eps)))
        if change <= tol:
            return dict(eps=eps, occ=occ, E0=E0, iterations=it, change=change)
        eps = (1.0 - mixing) * eps + mixing * new
    return dict(eps=eps, occ=occ, E0=E0, iterations=max_iter, change=change)


def trunc_kept_ranks(omega: int, n: int, eps, V, sel, bins: int = 10**8) -> np.ndarray:
    """Ascending full-space ranks of the states a selection from trunc_select
    keeps (bin <= cut), recomputed state by state in C."""
    eps, V = _check_h(omega, eps, V)
    d = np.zeros(62)
    d[:omega] = 2.0 * eps + np.diag(V)
    out = np.empty(int(sel["kept"]), dtype=np.int64)
    got = lib().or_trunc_kept_ranks(omega, n, _p(d), sel["dmin"], sel["scale"], bins, sel["cut_bin"],
                                    out.ctypes.data_as(ctypes.c_void_p), out.size)
    if got != out.size:
        raise RuntimeError(f"selection keeps {got} states, expected {out.size}")
    return out


def trunc_sigma_sampled(omega: int, n: int, eps, V, kept, ranks, x) -> np.ndarray:
    """Rows of the truncated product (H restricted to the kept states) for the
    listed kept full ranks.  kept: ascending kept full ranks (x is indexed by
    position in it); each row's position and each target's are found by
    binary search in kept (Sec. 3.2, Sec. 3.5), targets not kept dropped."""
    eps, V = _check_h(omega, eps, V)
    x = _f64(x)
    kept = np.ascontiguousarray(kept, dtype=np.int64)
    ranks = np.ascontiguousarray(ranks, dtype=np.int64)
    y = np.empty(ranks.size)
    rc = lib().or_trunc_sigma_sampled(omega, n, _p(eps), _p(V), kept.ctypes.data_as(ctypes.c_void_p), kept.size,
                                      _p(ranks), ranks.size, _p(x), _p(y))
    if rc != 0:
        raise RuntimeError("a listed rank is not kept")
    return y


# ---------------------------------------------------------------- odd mass (Sec. 2, Eq. hamiltonian3)

def blocked_instance(omega: int, eps, V, b: int):
    """eps and V of H_b's pair part: orbit b (0-based) removed (Eq. hamiltonian3)."""
    eps, V = _check_h(omega, eps, V)
    keep = [i for i in range(omega) if i != b]
    return eps[keep].copy(), V[np.ix_(keep, keep)].copy()


def odd_ground(omega: int, n: int, eps, V, block: int = 0, solver: str = "dense", **lanczos_kw):
    """2n+1 particles, blocking approximation.  H_b = eps_b + the pair
    Hamiltonian of Eq. hamiltonian2 on the omega-1 orbits other than b.
    block (Sec. 4.2, Block): b in 1..omega solves that block; 0 solves all
    and keeps the lowest.  N_Occup (Sec. 4.3): 1 on the blocked orbit.
    solver: 'dense' (explicit matrix) or 'lanczos' (the oracle's Lanczos).
    Returns dict(E, block, E_blocks, occ) with E_blocks NaN where not solved."""
    eps, V = _check_h(omega, eps, V)
    if not (omega >= 2 and 0 <= n <= omega - 1 and 0 <= block <= omega):
        raise ValueError("odd system needs omega >= 2, 0 <= n <= omega-1, 0 <= block <= omega")
    blocks = range(omega) if block == 0 else [block - 1]
    E_blocks = np.full(omega, np.nan)
    occ_blocks = {}
    for b in blocks:
        eps_b, V_b = blocked_instance(omega, eps, V, b)
        if solver == "dense":
            e0, _, occ_b, _ = dense_ground(omega - 1, n, eps_b, V_b)
        else:
            r = lanczos_ground(omega - 1, n, eps_b, V_b, **lanczos_kw)
            e0, occ_b = r["E0"], r["occ"]
        E_blocks[b] = eps[b] + e0
        occ_blocks[b] = occ_b
    best = min(blocks, key=lambda b: (E_blocks[b], b))
    occ = np.insert(occ_blocks[best], best, 1.0)
    return dict(E=float(E_blocks[best]), block=best + 1, E_blocks=E_blocks, occ=occ)


# ---------------------------------------------------------------- Richardson (constant G)

def richardson_evb(eps, g: float, n: int, steps: int = 400, newton_iters: int = 30) -> float:
    """Ground-state energy (and the u_i) for eps_i distinct and constant V_ij = -g,
    i.e. pair energies e_i = 2 eps_i, from the Richardson equations in eigenvalue form.

    Unknowns u_i = g sum_alpha 1/(e_i - E_alpha) satisfy
        u_i^2 = u_i + g sum_{j != i} (u_i - u_j)/(e_i - e_j),     sum_i u_i = n,
    and E0 = sum_i e_i u_i - g n (Omega - n + 1).
    Continued in g from 0 (u = 1 on the n lowest levels) with Newton steps."""
    e = 2.0 * _f64(eps)
    omega = e.size
    order = np.argsort(e)
    u = np.zeros(omega)
    u[order[:n]] = 1.0
    diff = e[:, None] - e[None, :]
    np.fill_diagonal(diff, np.inf)
    inv = 1.0 / diff                     # 1/(e_i - e_j), 0 on the diagonal
    for s in range(1, steps + 1):
        gs = g * s / steps
        for _ in range(newton_iters):
            du = u[:, None] - u[None, :]
            F = u * u - u - gs * (du * inv).sum(axis=1)
            J = gs * inv.copy()
            np.fill_diagonal(J, 2.0 * u - 1.0 - gs * inv.sum(axis=1))
            step = np.linalg.solve(J, -F)
            u = u + step
            if np.max(np.abs(step)) < 1e-15:
                break
    return float(e @ u - g * n * (omega - n + 1)), u


# ---------------------------------------------------------------- warm start

def pbcs_vector(omega: int, n: int, logits, basis: np.ndarray | None = None) -> np.ndarray:
    """Number-projected product state: psi_k proportional to prod_{i in occ(k)} z_i,
    z_i = exp(l_i / 2), normalised, computed term by term in log space."""
    if basis is None:
        basis = basis_alg1(omega, n)
    l = _f64(logits)
    bits = ((basis[:, None] >> np.arange(omega, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.float64)
    logpsi = 0.5 * (bits @ l)
    psi = np.exp(logpsi - logpsi.max())
    return psi / np.linalg.norm(psi)


def gelu_tanh(x):
    """GELU, tanh form (Hendrycks & Gimpel 2016)."""
    c = math.sqrt(2.0 / math.pi)
    return 0.5 * x * (1.0 + np.tanh(c * (x + 0.044715 * x ** 3)))


def gelu_tanh_grad(x):
    c = math.sqrt(2.0 / math.pi)
    t = np.tanh(c * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * c * (1.0 + 3 * 0.044715 * x * x)


def mlp_forward(params, X):
    """X (B x in) -> logits (B x out); params = [W1, b1, W2, b2, W3, b3], W as (in x out).
    Hidden layers use GELU, the output layer is linear."""
    W1, b1, W2, b2, W3, b3 = [_f64(p) for p in params]
    X = _f64(X)
    z1 = X @ W1 + b1
    h1 = gelu_tanh(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu_tanh(z2)
    out = h2 @ W3 + b3
    return out, (X, z1, h1, z2, h2)


def mlp_loss(logits, target_half_occ):
    """mean over all entries of (sigmoid(l) - <N_i>/2)^2."""
    s = 1.0 / (1.0 + np.exp(-_f64(logits)))
    r = s - _f64(target_half_occ)
    return float(np.mean(r * r)), 2.0 * r * s * (1.0 - s) / r.size


def mlp_backward(params, cache, dout):
    W1, b1, W2, b2, W3, b3 = [_f64(p) for p in params]
    X, z1, h1, z2, h2 = cache
    dW3 = h2.T @ dout
    db3 = dout.sum(axis=0)
    dh2 = dout @ W3.T
    dz2 = dh2 * gelu_tanh_grad(z2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * gelu_tanh_grad(z1)
    dW1 = X.T @ dz1
    db1 = dz1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]
