"""Pins of the oracle's lowest eigenpairs: the quasi-spin spectrum of the
degenerate shell with its multiplicities, ARPACK against the dense solver,
and the eigen-equation itself."""
from __future__ import annotations

import math

import numpy as np
import pytest


def quasispin_levels(omega, n, g):
    """eps = 0, V_ij = -g (all i, j): H = -g S+ S- with S+ = sum_i S+_i.  The
    n-pair space splits into quasi-spin multiplets S = omega/2 - nu,
    nu = 0..min(n, omega - n), each C(omega, nu) - C(omega, nu - 1) times, with
    E = -g [S (S + 1) - S_z (S_z - 1)], S_z = n - omega/2."""
    out = []
    sz = n - omega / 2
    for nu in range(min(n, omega - n) + 1):
        S = omega / 2 - nu
        mult = math.comb(omega, nu) - (math.comb(omega, nu - 1) if nu > 0 else 0)
        out += [-g * (S * (S + 1) - sz * (sz - 1))] * mult
    return np.sort(np.array(out))


@pytest.mark.parametrize("omega,n,g", [(8, 4, 0.5), (9, 3, 0.3), (10, 7, 1.0)])
def test_degenerate_shell_spectrum_with_multiplicities(oracle_mod, omega, n, g):
    H = oracle_mod.dense_h(omega, n, np.zeros(omega), -g * np.ones((omega, omega)))
    np.testing.assert_allclose(np.linalg.eigvalsh(H), quasispin_levels(omega, n, g), atol=1e-11)
    w, Z, occ = oracle_mod.lowest_eigenpairs(omega, n, np.zeros(omega), -g * np.ones((omega, omega)), 3)
    np.testing.assert_allclose(w, quasispin_levels(omega, n, g)[:3], atol=1e-11)


def test_arpack_matches_dense_and_solves_the_eigen_equation(oracle_mod):
    omega, n = 14, 7
    rng = np.random.default_rng(2)
    eps = rng.uniform(0, omega, omega)
    G = 0.3 * (1 + 0.2 * rng.uniform(size=(omega, omega)))
    V = -0.5 * (G + G.T)
    wd, Zd, od = oracle_mod.lowest_eigenpairs(omega, n, eps, V, 5)
    wa, Za, oa = oracle_mod.lowest_eigenpairs(omega, n, eps, V, 5, dense_limit=0)
    np.testing.assert_allclose(wa, wd, rtol=1e-12)
    np.testing.assert_allclose(np.abs(np.sum(Za * Zd, axis=0)), 1.0, atol=1e-9)
    np.testing.assert_allclose(oa, od, atol=1e-8)
    basis = oracle_mod.basis_alg1(omega, n)
    for i in range(5):
        r = oracle_mod.sigma(omega, n, eps, V, basis, Zd[:, i]) - wd[i] * Zd[:, i]
        assert np.linalg.norm(r) <= 1e-11 * abs(wd[i])
        assert occ_sum_ok(od[i], n)


def occ_sum_ok(occ, n):
    return abs(occ.sum() - 2 * n) < 1e-9 and (occ >= -1e-12).all() and (occ <= 2 + 1e-12).all()
