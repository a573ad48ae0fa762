"""Pins of the truncation oracle (Sec. 3.5): the kept space against a plain
sort of the diagonal elements, the truncated product against the full matrix
restricted to the kept states, and the variational and nesting properties a
truncated ground state must have."""
from __future__ import annotations

import math

import numpy as np
import pytest


def _inst(omega, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.0, omega, omega)
    G = 0.3 * (1.0 + 0.2 * rng.uniform(size=(omega, omega)))
    return eps, -0.5 * (G + G.T)


def _diag_brute(omega, eps, V, states):
    """Eq. diagonal state by state with Python integers (independent of the
    vectorised oracle)."""
    d = 2.0 * eps + np.diag(V)
    out = []
    for s in states:
        s = int(s)
        acc = 0.0
        for q in range(omega):
            if (s >> q) & 1:
                acc += d[q]
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("omega,n,seed", [(12, 6, 0), (14, 5, 1), (13, 9, 2)])
def test_fine_bins_keep_exactly_the_lowest_diagonals(oracle_mod, omega, n, seed):
    # With 1e8 bins every bin holds at most one of these distinct diagonals, so
    # the kept space is exactly the `limit` states of lowest diagonal.
    eps, V = _inst(omega, seed)
    basis = oracle_mod.basis_alg1(omega, n)
    diag = _diag_brute(omega, eps, V, basis)
    assert len(np.unique(diag)) == diag.size
    for limit in (1, 7, basis.size // 3, basis.size - 1):
        t = oracle_mod.trunc_select(omega, n, eps, V, limit, bins=10**8)
        assert t["kept"] == limit
        lowest = np.sort(np.argsort(diag, kind="stable")[:limit])
        np.testing.assert_array_equal(t["ranks"], lowest)
        np.testing.assert_array_equal(t["states"], basis[lowest])
        assert t["dmin"] == diag.min() and t["dmax"] == diag.max()


@pytest.mark.parametrize("bins", [7, 100, 4096])
def test_coarse_bins_cut_is_monotone_and_maximal(oracle_mod, bins):
    omega, n = 14, 6
    eps, V = _inst(omega, 3)
    basis = oracle_mod.basis_alg1(omega, n)
    diag = _diag_brute(omega, eps, V, basis)
    for limit in (5, 300, 1500, 2900):
        t = oracle_mod.trunc_select(omega, n, eps, V, limit, bins=bins)
        keep = np.zeros(basis.size, bool)
        keep[t["ranks"]] = True
        # a cut in the diagonal: everything kept lies at or below everything dropped
        if (~keep).any():
            assert diag[keep].max() <= diag[~keep].min()
        if t["kept"] <= limit:
            # maximal: the next non-empty bin would overflow the limit
            nxt = diag[~keep]
            if nxt.size:
                nb = np.floor((nxt - diag.min()) * t["scale"])
                first = nb.min()
                assert t["kept"] + np.count_nonzero(nb == first) > limit
        else:
            assert t["cut_bin"] == 0   # only bin 0, which alone exceeds the limit
        assert t["kept"] == keep.sum()


def test_no_truncation_within_limit_and_degenerate_diagonals(oracle_mod):
    omega, n = 10, 4
    eps, V = _inst(omega, 4)
    t = oracle_mod.trunc_select(omega, n, eps, V, math.comb(omega, n))
    assert t["kept"] == t["full_dim"] == 210
    np.testing.assert_array_equal(t["ranks"], np.arange(210))
    # equal pair energies: one diagonal value, everything in bin 0, kept whole
    flat = oracle_mod.trunc_select(omega, n, np.zeros(omega), -0.3 * np.ones((omega, omega)), 10)
    assert flat["scale"] == 0.0 and flat["cut_bin"] == 0 and flat["kept"] == 210


def test_truncated_sigma_is_the_restricted_matrix(oracle_mod):
    omega, n = 11, 5
    eps, V = _inst(omega, 5)
    H = oracle_mod.dense_h(omega, n, eps, V)
    t = oracle_mod.trunc_select(omega, n, eps, V, 200, bins=1000)
    keep = t["ranks"]
    x = np.random.default_rng(0).standard_normal(keep.size)
    y = oracle_mod.sigma(omega, n, eps, V, t["states"], x, index_mode="bsearch_truncated")
    np.testing.assert_allclose(y, H[np.ix_(keep, keep)] @ x, rtol=1e-13, atol=1e-12)
    with pytest.raises(RuntimeError):
        oracle_mod.sigma(omega, n, eps, V, t["states"], x, index_mode="bsearch")


def test_truncated_ground_state_variational_and_nested(oracle_mod):
    omega, n = 12, 6
    eps, V = _inst(omega, 6)
    H = oracle_mod.dense_h(omega, n, eps, V)
    E_full = np.linalg.eigvalsh(H)[0]
    prev = math.inf
    for limit in (50, 200, 500, 924):
        t = oracle_mod.trunc_select(omega, n, eps, V, limit, bins=10**6)
        k = t["ranks"]
        E = np.linalg.eigvalsh(H[np.ix_(k, k)])[0]
        assert E >= E_full - 1e-12 and E <= prev + 1e-12
        prev = E
        r = oracle_mod.lanczos_ground(omega, n, eps, V, krylov=30, tol=1e-11, basis=t["states"],
                                      index_mode="bsearch_truncated")
        assert r["E0"] == pytest.approx(E, abs=1e-9)
        assert r["occ"].sum() == pytest.approx(2 * n, abs=1e-9)
    assert prev == pytest.approx(E_full, abs=1e-12)


@pytest.mark.parametrize("omega,n,limit,bins", [(14, 7, 1500, 10**8), (16, 6, 3000, 4096), (15, 10, 100, 7),
                                                (18, 9, 20000, 10**6)])
def test_c_histogram_path_matches_numpy_path(oracle_mod, omega, n, limit, bins):
    eps, V = _inst(omega, omega + n)
    a = oracle_mod.trunc_select(omega, n, eps, V, limit, bins, method="numpy")
    c = oracle_mod.trunc_select(omega, n, eps, V, limit, bins, method="c")
    for k in ("full_dim", "kept", "cut_bin", "dmin", "dmax", "scale"):
        assert a[k] == c[k], k
    kept = oracle_mod.trunc_kept_ranks(omega, n, eps, V, c, bins)
    np.testing.assert_array_equal(kept, a["ranks"])
    x = np.random.default_rng(1).standard_normal(a["kept"])
    rows = a["ranks"][:: max(1, a["kept"] // 300)]
    y = oracle_mod.trunc_sigma_sampled(omega, n, eps, V, kept, rows, x)
    y_all = oracle_mod.sigma(omega, n, eps, V, a["states"], x, index_mode="bsearch_truncated")
    idx = np.searchsorted(a["ranks"], rows)
    np.testing.assert_allclose(y, y_all[idx], rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("limit,bins", [(1, 10**8), (1, 5), (40, 4096), (700, 10**6), (2000, 9000)])
def test_c_histogram_path_edges_with_ties(oracle_mod, limit, bins):
    # coarse dyadic pair energies: many equal diagonals, so whole bins (and whole
    # 4096-bin chunks) cross the limit at once
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2001_01978_amd import inputs
    omega, n = 16, 7
    _, _, eps, V = inputs.dyadic_instance(omega, n, seed=4)
    a = oracle_mod.trunc_select(omega, n, eps, V, limit, bins, method="numpy")
    c = oracle_mod.trunc_select(omega, n, eps, V, limit, bins, method="c")
    assert (a["kept"], a["cut_bin"]) == (c["kept"], c["cut_bin"])
