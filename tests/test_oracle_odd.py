"""Pins of the odd-system oracle (blocking approximation, Sec. 2 Eq. hamiltonian3)
and, on the way, of the even Hamiltonian (Eq. hamiltonian2), against the
fermion Hamiltonian of Eq. hamiltonian1 built from scratch in the Fock space of
the 2*omega single-particle states.

The Fock construction below shares nothing with the oracle: modes 2i and 2i+1
are the time-reversed states i and i-bar, operators act by Jordan-Wigner bit
rules, and H = sum_p eps_p n_p + sum_{ii'} V_ii' a+_i a+_ibar a_i'bar a_i'.
Seniority (the number of orbits holding exactly one particle) is conserved,
so the seniority-zero sector of 2n particles must have the spectrum of the
pair Hamiltonian, and the seniority-one sector of 2n+1 particles the spectra
of all blocked Hamiltonians H_b, each twice (the odd particle in b or b-bar).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest


def _annihilate(s: int, p: int):
    if not (s >> p) & 1:
        return None
    sign = -1.0 if bin(s & ((1 << p) - 1)).count("1") % 2 else 1.0
    return sign, s ^ (1 << p)


def _create(s: int, p: int):
    if (s >> p) & 1:
        return None
    sign = -1.0 if bin(s & ((1 << p) - 1)).count("1") % 2 else 1.0
    return sign, s | (1 << p)


def _apply(ops, s):
    """ops: [(mode, is_creation)] written left to right as in the operator
    product; applied right to left.  Returns (coefficient, state) or None."""
    c = 1.0
    for mode, dag in reversed(ops):
        r = (_create if dag else _annihilate)(s, mode)
        if r is None:
            return None
        c *= r[0]
        s = r[1]
    return c, s


def _seniority(s: int, omega: int) -> int:
    return sum(((s >> (2 * i)) & 1) != ((s >> (2 * i + 1)) & 1) for i in range(omega))


def fock_sector(omega: int, eps, V, particles: int, seniority: int):
    """Eq. hamiltonian1 restricted to one particle number and seniority.
    Returns (H, states, leak) where leak is the largest |element| that H sends
    out of the sector (zero if seniority is conserved)."""
    states = [s for s in range(1 << (2 * omega))
              if bin(s).count("1") == particles and _seniority(s, omega) == seniority]
    index = {s: k for k, s in enumerate(states)}
    H = np.zeros((len(states), len(states)))
    leak = 0.0
    for col, s in enumerate(states):
        out = {}
        for p in range(2 * omega):
            if (s >> p) & 1:
                out[s] = out.get(s, 0.0) + eps[p // 2]
        for i in range(omega):
            for j in range(omega):
                r = _apply([(2 * i, True), (2 * i + 1, True), (2 * j + 1, False), (2 * j, False)], s)
                if r is not None:
                    out[r[1]] = out.get(r[1], 0.0) + V[i, j] * r[0]
        for t, v in out.items():
            if t in index:
                H[index[t], col] += v
            else:
                leak = max(leak, abs(v))
    return H, states, leak


def _inst(omega, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.0, omega, omega)
    G = 0.3 * (1.0 + 0.2 * rng.uniform(size=(omega, omega)))
    G = 0.5 * (G + G.T)
    return eps, -G


@pytest.mark.parametrize("omega,n,seed", [(4, 2, 0), (5, 2, 1), (5, 3, 2)])
def test_even_pair_hamiltonian_matches_fock_seniority_zero(oracle_mod, omega, n, seed):
    eps, V = _inst(omega, seed)
    H, _, leak = fock_sector(omega, eps, V, 2 * n, 0)
    assert leak == 0.0
    w_fock = np.linalg.eigvalsh(H)
    w_pair = np.linalg.eigvalsh(oracle_mod.dense_h(omega, n, eps, V))
    assert len(w_fock) == math.comb(omega, n)
    np.testing.assert_allclose(w_fock, w_pair, rtol=0, atol=1e-12)


@pytest.mark.parametrize("omega,n,seed", [(4, 1, 3), (5, 2, 4), (5, 1, 5), (6, 2, 6)])
def test_blocked_spectra_match_fock_seniority_one(oracle_mod, omega, n, seed):
    eps, V = _inst(omega, seed)
    H, states, leak = fock_sector(omega, eps, V, 2 * n + 1, 1)
    assert leak == 0.0
    assert len(states) == omega * 2 * math.comb(omega - 1, n)
    w_fock, Z = np.linalg.eigh(H)
    parts = []
    for b in range(omega):
        eb, Vb = oracle_mod.blocked_instance(omega, eps, V, b)
        parts.append(eps[b] + np.linalg.eigvalsh(oracle_mod.dense_h(omega - 1, n, eb, Vb)))
    w_blocks = np.sort(np.concatenate(parts + parts))
    np.testing.assert_allclose(w_fock, w_blocks, rtol=0, atol=1e-12)

    r = oracle_mod.odd_ground(omega, n, eps, V)
    assert r["E"] == pytest.approx(w_fock[0], abs=1e-12)
    # The lowest level is doubly degenerate (odd particle in b or b-bar); the
    # occupations of the average over that pair do not depend on the basis
    # eigh picked inside it.
    assert w_fock[1] - w_fock[0] < 1e-10 and w_fock[2] - w_fock[0] > 1e-8
    occ = np.zeros(omega)
    for k in range(2):
        for amp, s in zip(Z[:, k], states):
            for p in range(2 * omega):
                if (s >> p) & 1:
                    occ[p // 2] += 0.5 * amp * amp
    np.testing.assert_allclose(r["occ"], occ, atol=1e-10)
    assert r["occ"][r["block"] - 1] == 1.0


@pytest.mark.parametrize("omega,n,g", [(6, 2, 0.4), (7, 3, 0.25), (8, 4, 1.0), (9, 1, 0.5)])
def test_odd_degenerate_shell_seniority_formula(oracle_mod, omega, n, g):
    # eps = 0, V_ij = -g: E(N, v) = -g/4 (N - v)(2 omega - N - v + 2); N = 2n+1, v = 1.
    N = 2 * n + 1
    r = oracle_mod.odd_ground(omega, n, np.zeros(omega), -g * np.ones((omega, omega)))
    assert r["E"] == pytest.approx(-g / 4 * (N - 1) * (2 * omega - N - 1 + 2), abs=1e-11)
    np.testing.assert_allclose(r["E_blocks"], r["E"], atol=1e-11)


def test_odd_block_modes_and_edges(oracle_mod):
    omega = 7
    eps, V = _inst(omega, 11)
    every = oracle_mod.odd_ground(omega, 3, eps, V, block=0)
    for b in range(1, omega + 1):
        one = oracle_mod.odd_ground(omega, 3, eps, V, block=b)
        assert one["block"] == b
        assert one["E"] == pytest.approx(every["E_blocks"][b - 1], abs=1e-12)
        assert np.isnan(np.delete(one["E_blocks"], b - 1)).all()
    assert every["E"] == pytest.approx(np.min(every["E_blocks"]), abs=0)
    assert every["block"] == int(np.argmin(every["E_blocks"])) + 1
    # no pairs: the odd particle sits on the lowest level
    r0 = oracle_mod.odd_ground(omega, 0, eps, V)
    assert r0["E"] == pytest.approx(eps.min()) and r0["block"] == int(np.argmin(eps)) + 1
    np.testing.assert_allclose(np.delete(r0["occ"], r0["block"] - 1), 0.0)
    # all other orbits full: diagonal only
    rf = oracle_mod.odd_ground(omega, omega - 1, eps, V)
    d = 2 * eps + np.diag(V)
    full = [eps[b] + d.sum() - d[b] for b in range(omega)]
    np.testing.assert_allclose(rf["E_blocks"], full, atol=1e-12)
    np.testing.assert_allclose(rf["occ"], np.where(np.arange(omega) == rf["block"] - 1, 1.0, 2.0))


def test_odd_lanczos_solver_matches_dense(oracle_mod):
    omega = 9
    eps, V = _inst(omega, 12)
    a = oracle_mod.odd_ground(omega, 4, eps, V)
    b = oracle_mod.odd_ground(omega, 4, eps, V, solver="lanczos", krylov=30, tol=1e-12)
    np.testing.assert_allclose(b["E_blocks"], a["E_blocks"], rtol=1e-12)
    np.testing.assert_allclose(b["occ"], a["occ"], atol=1e-8)
    assert a["block"] == b["block"]


def test_fock_builder_sign_rules():
    # anticommutation on two modes: a_0 a+_1 = - a+_1 a_0 on |1 0> (mode 0 occupied)
    s = 0b01
    left = _apply([(0, False), (1, True)], s)
    right = _apply([(1, True), (0, False)], s)
    assert left[1] == right[1] and left[0] == -right[0]
    # a+_p a_p is the number operator on every basis state of 3 modes
    for s, p in itertools.product(range(8), range(3)):
        r = _apply([(p, True), (p, False)], s)
        assert (r is not None) == bool((s >> p) & 1)
        if r is not None:
            assert r == (1.0, s)
