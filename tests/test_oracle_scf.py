"""Pins of the self-consistent loop oracle: no field gives one plain solve,
the result is a fixed point of the field, the degenerate shell with a uniform
field has a closed form, and the fixed point does not depend on the mixing."""
from __future__ import annotations

import numpy as np
import pytest


def _inst(omega, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.0, omega, omega)
    G = 0.3 * (1.0 + 0.2 * rng.uniform(size=(omega, omega)))
    W = 0.4 * rng.uniform(size=(omega, omega))
    return eps, -0.5 * (G + G.T), 0.5 * (W + W.T)


def test_no_field_is_one_solve(oracle_mod):
    eps, V, _ = _inst(9, 0)
    r = oracle_mod.scf_ground(9, 4, eps, np.zeros((9, 9)), V)
    E0, _, occ, _ = oracle_mod.dense_ground(9, 4, eps, V)
    assert r["iterations"] == 1 and r["E0"] == E0
    np.testing.assert_array_equal(r["occ"], occ)


@pytest.mark.parametrize("omega,n,seed", [(9, 4, 1), (10, 3, 2), (8, 6, 3)])
def test_fixed_point_and_mixing_independence(oracle_mod, omega, n, seed):
    eps0, V, W = _inst(omega, seed)
    a = oracle_mod.scf_ground(omega, n, eps0, W, V, mixing=0.5, tol=1e-12)
    b = oracle_mod.scf_ground(omega, n, eps0, W, V, mixing=0.3, tol=1e-12)
    assert a["change"] <= 1e-12 and a["iterations"] > 2
    # self-consistency: the field of the returned occupations is the returned field
    np.testing.assert_allclose(eps0 + W @ a["occ"] / 2, a["eps"], atol=1e-11)
    np.testing.assert_allclose(a["eps"], b["eps"], atol=1e-10)
    np.testing.assert_allclose(a["occ"], b["occ"], atol=1e-10)
    assert a["E0"] == pytest.approx(oracle_mod.dense_ground(omega, n, a["eps"], V)[0], abs=1e-12)


def test_degenerate_shell_uniform_field_closed_form(oracle_mod):
    # eps0 = 0, V_ij = -g, W_ij = w: by symmetry <N_i> = 2n/omega, so eps_i = w n
    # for every i, and E0 = 2 n (w n) - g n (omega - n + 1).
    omega, n, g, w = 10, 4, 0.3, 0.2
    r = oracle_mod.scf_ground(omega, n, np.zeros(omega), w * np.ones((omega, omega)),
                              -g * np.ones((omega, omega)), mixing=1.0, tol=1e-12)
    np.testing.assert_allclose(r["occ"], 2 * n / omega, atol=1e-12)
    np.testing.assert_allclose(r["eps"], w * n, atol=1e-12)
    assert r["E0"] == pytest.approx(2 * n * w * n - g * n * (omega - n + 1), abs=1e-11)
