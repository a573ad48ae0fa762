"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
value the paper prints, a closed form, an invariant, a library routine on a
special case, or brute force on tiny inputs.  CPU only.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2001_01978_amd import inputs


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ binomials / dimensions

def test_binom_extcmn_against_math_comb(oracle_mod):
    # Eq. extcmn, including the zero extension for n < m.
    for n in range(0, 63):
        for m in range(0, 63):
            want = math.comb(n, m) if n >= m else 0
            assert oracle_mod.binom(n, m) == want


def test_config_dimensions(oracle_mod):
    assert oracle_mod.binom(4, 2) == 6
    assert oracle_mod.binom(16, 8) == 12870
    assert oracle_mod.binom(24, 12) == 2704156
    assert oracle_mod.binom(28, 14) == 40116600
    assert oracle_mod.binom(32, 16) == 601080390
    assert oracle_mod.binom(34, 17) == 2333606220


def test_hspa_dimensions(oracle_mod, golden_dir):
    tab = _load(golden_dir, "paper_table_hspa.json")
    for row in tab["rows"]:
        d = oracle_mod.binom(row["omega"], tab["n"])
        # the table prints 2 significant digits
        assert abs(d - row["dim_approx"]) <= 0.051 * row["dim_approx"], (row, d)


# ------------------------------------------------------------------ basis (Alg. conversion)

def test_table_data(oracle_mod, golden_dir):
    tab = _load(golden_dir, "paper_table_data.json")
    b = oracle_mod.basis_alg1(tab["omega"], tab["n"])
    assert b.size == len(tab["rows"])
    for idx, binary, dec in tab["rows"]:
        assert int(b[idx - 1]) == int(binary, 2) == dec


def test_alg1_walkthrough(oracle_mod, golden_dir):
    seq = [int(s, 2) for s in _load(golden_dir, "paper_alg1_walkthrough.json")["sequence"]]
    s = seq[0]
    for want in seq[1:]:
        s = oracle_mod.next_state(s)
        assert s == want


def test_successor_is_next_integer_with_equal_popcount(oracle_mod):
    # The successor's definition checked by exhaustive search: for every
    # s < 2^13 with at least one set bit, the smallest t > s with as many ones.
    nxt = {}
    by_count = {}
    for t in range(1, 1 << 14):
        by_count.setdefault(bin(t).count("1"), []).append(t)
    for k, ts in by_count.items():
        for a, b in zip(ts, ts[1:]):
            nxt[a] = b
    for s in range(1, 1 << 13):
        assert oracle_mod.next_state(s) == nxt[s], s
    # near the top of a 62-orbit space
    top = ((1 << 5) - 1) << 56
    assert oracle_mod.next_state(top) == (1 << 61) | ((1 << 4) - 1)


@pytest.mark.parametrize("omega", range(1, 15))
def test_basis_brute_force(oracle_mod, omega):
    # all n-subsets of omega orbits as bitmasks, sorted ascending
    for n in range(0, omega + 1):
        brute = sorted(sum(1 << p for p in c) for c in itertools.combinations(range(omega), n))
        b = oracle_mod.basis_alg1(omega, n)
        assert [int(v) for v in b] == brute


def test_basis_properties_larger(oracle_mod):
    for omega, n in [(20, 10), (22, 7), (24, 12), (40, 3), (62, 2), (62, 61)]:
        b = oracle_mod.basis_alg1(omega, n)
        assert b.size == math.comb(omega, n)
        assert np.all(np.diff(b.astype(np.uint64)) > 0)
        pc = np.array([bin(int(v)).count("1") for v in b[:: max(1, b.size // 5000)]])
        assert np.all(pc == n)
        assert int(b.max()) < (1 << omega)


# ------------------------------------------------------------------ index search (Sec. 3.2)

def test_hash_examples(oracle_mod, golden_dir):
    ex = _load(golden_dir, "paper_hash_examples.json")
    for binary, f in ex["f"]:
        assert oracle_mod.hash_index(int(binary, 2)) + 1 == f


@pytest.mark.parametrize("omega,n", [(4, 2), (10, 5), (13, 4), (16, 8), (18, 11)])
def test_hash_and_bsearch_equal_position(oracle_mod, omega, n):
    b = oracle_mod.basis_alg1(omega, n)
    for k in range(0, b.size, max(1, b.size // 3000)):
        s = int(b[k])
        assert oracle_mod.hash_index(s) == k
        assert oracle_mod.index_bsearch(b, s) == k
        assert oracle_mod.unhash(k, n) == s
    assert oracle_mod.index_bsearch(b, int(b[-1]) + 1) == -1


def test_unhash_large_round_trip(oracle_mod):
    rng = np.random.default_rng(5)
    for omega, n in [(34, 17), (40, 20), (62, 31), (62, 1)]:
        d = math.comb(omega, n)
        for r in list(rng.integers(0, d, 200)) + [0, d - 1]:
            s = oracle_mod.unhash(int(r), n)
            assert bin(s).count("1") == n and s < (1 << omega)
            assert oracle_mod.hash_index(s) == int(r)


def test_complement_invariant(oracle_mod):
    # s -> s XOR (2^omega - 1) maps rank k of (omega, n) to rank D-1-k of (omega, omega-n)
    for omega, n in [(9, 4), (12, 5), (16, 8)]:
        b = oracle_mod.basis_alg1(omega, n)
        full = (1 << omega) - 1
        d = b.size
        for k in range(0, d, max(1, d // 500)):
            assert oracle_mod.hash_index(int(b[k]) ^ full) == d - 1 - k


# ------------------------------------------------------------------ Hamiltonian (Sec. 3.3)

def test_worked_6x6(oracle_mod, golden_dir):
    ex = _load(golden_dir, "paper_matrix_6x6.json")
    om, n = ex["omega"], ex["n"]
    eps = np.array(ex["eps"], float)
    V = np.full((om, om), ex["V_const"])
    H = oracle_mod.dense_h(om, n, eps, V)
    assert np.allclose(H, np.array(ex["H"]), atol=1e-14, rtol=0)
    nz = sorted(j + 1 for j in range(1, 6) if H[0, j] != 0.0)
    assert nz == sorted(ex["row1_offdiag_1based"])


def _rand_inst(omega, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0, omega, omega)
    G = rng.uniform(0.1, 0.6, (omega, omega))
    V = -(G + G.T) / 2
    return eps, V


@pytest.mark.parametrize("omega,n", [(6, 3), (9, 2), (10, 6), (12, 6)])
def test_h_counts_trace_frobenius(oracle_mod, omega, n):
    eps, V = _rand_inst(omega, omega * 100 + n)
    H = oracle_mod.dense_h(omega, n, eps, V)
    d = math.comb(omega, n)
    off = H - np.diag(np.diag(H))
    # symmetric
    assert np.array_equal(H, H.T)
    # n(omega-n) off-diagonal hops per row (all V_ij != 0 here), Sec. 3.3
    assert np.all((off != 0).sum(axis=1) == n * (omega - n))
    # total off-diagonal nonzeros, Eq. elements in the paper's letters (n orbits, m pairs)
    nn, m = omega, n
    assert (off != 0).sum() == math.factorial(nn) // (math.factorial(m - 1) * math.factorial(nn - m - 1))
    # trace = C(omega-1, n-1) * sum_i (2 eps_i + V_ii)
    assert math.isclose(np.trace(H), math.comb(omega - 1, n - 1) * np.sum(2 * eps + np.diag(V)), rel_tol=1e-12)
    # sum of squared off-diagonal elements = C(omega-2, n-1) * sum_{i != j} V_ij^2
    offv = V - np.diag(np.diag(V))
    assert math.isclose((off ** 2).sum(), math.comb(omega - 2, n - 1) * (offv ** 2).sum(), rel_tol=1e-12)


def test_sigma_equals_dense_matvec_and_hash_path(oracle_mod):
    omega, n = 12, 5
    eps, V = _rand_inst(omega, 7)
    b = oracle_mod.basis_alg1(omega, n)
    H = oracle_mod.dense_h(omega, n, eps, V, b)
    x = inputs.random_vector(3, b.size)
    y1 = oracle_mod.sigma(omega, n, eps, V, b, x, "bsearch")
    y2 = oracle_mod.sigma(omega, n, eps, V, b, x, "hash")
    assert np.allclose(y1, H @ x, rtol=1e-13, atol=1e-12)
    assert np.array_equal(y1, y2)
    rows = np.array([0, 1, 17, b.size // 2, b.size - 1])
    y3 = oracle_mod.sigma_sampled(omega, n, eps, V, x, rows)
    assert np.array_equal(y3, y1[rows])
    y4 = oracle_mod.sigma(omega, n, eps, V, b, x, "hash", rows=(5, 50))
    assert np.array_equal(y4, y1[5:50])
    y5 = oracle_mod.sigma_block(omega, n, eps, V, x, 3, b.size)
    assert np.array_equal(y5, y1[3:])


def test_row_terms_reproduce_dense_rows(oracle_mod):
    omega, n = 11, 4
    eps, V = _rand_inst(omega, 17)
    H = oracle_mod.dense_h(omega, n, eps, V)
    rows = np.array([0, 3, 100, 329])
    diag, tg, cf = oracle_mod.row_terms(omega, n, eps, V, rows)
    for q, r in enumerate(rows):
        row = np.zeros(H.shape[0])
        row[r] += diag[q]
        np.add.at(row, tg[q], cf[q])
        assert np.array_equal(row, H[r])


def test_sigma_dyadic_exact(oracle_mod):
    omega, n, eps, V = inputs.dyadic_instance(11, 4, 9)
    b = oracle_mod.basis_alg1(omega, n)
    x = inputs.dyadic_vector(2, b.size)
    H = oracle_mod.dense_h(omega, n, eps, V, b)
    y = oracle_mod.sigma(omega, n, eps, V, b, x)
    assert np.array_equal(y, H @ x)          # every partial sum is exact


# ------------------------------------------------------------------ E0 closed forms

def test_e0_no_pairing(oracle_mod):
    omega, n = 10, 4
    eps = np.array([3.0, -1.0, 2.5, 0.5, 7.0, 1.25, -2.0, 4.0, 6.0, 0.0])
    V = np.zeros((omega, omega))
    E0, psi, occ, _ = oracle_mod.dense_ground(omega, n, eps, V)
    assert math.isclose(E0, np.sort(2 * eps)[:n].sum(), abs_tol=1e-12)


def test_e0_diagonal_only(oracle_mod):
    omega, n = 9, 4
    eps, V = _rand_inst(omega, 11)
    Vd = np.diag(np.diag(V))
    E0, *_ = oracle_mod.dense_ground(omega, n, eps, Vd)
    assert math.isclose(E0, np.sort(2 * eps + np.diag(Vd))[:n].sum(), abs_tol=1e-12)
    assert math.isclose(oracle_mod.monopole_min(omega, n, eps, V), np.sort(2 * eps + np.diag(V))[:n].sum())
    b = oracle_mod.basis_alg1(omega, n)
    H = oracle_mod.dense_h(omega, n, eps, V, b)
    assert math.isclose(oracle_mod.monopole_min(omega, n, eps, V), np.diag(H).min(), rel_tol=1e-14)


@pytest.mark.parametrize("omega,n,g", [(8, 4, 0.3), (10, 3, 0.7), (12, 6, 0.25)])
def test_degenerate_shell(oracle_mod, omega, n, g):
    e = 1.5
    eps = np.full(omega, e)
    V = np.full((omega, omega), -g)
    E0, psi, occ, _ = oracle_mod.dense_ground(omega, n, eps, V)
    assert math.isclose(E0, 2 * n * e - g * n * (omega - n + 1), abs_tol=1e-12)
    assert np.allclose(psi, 1 / math.sqrt(psi.size), atol=1e-12)
    assert np.allclose(occ, 2 * n / omega, atol=1e-12)


def test_one_pair_is_orbit_matrix(oracle_mod):
    omega = 9
    eps, V = _rand_inst(omega, 4)
    E0, *_ = oracle_mod.dense_ground(omega, 1, eps, V)
    assert math.isclose(E0, np.linalg.eigvalsh(2 * np.diag(eps) + V)[0], abs_tol=1e-12)


def test_two_level_closed_form(oracle_mod):
    e1, e2, g = 0.7, 2.9, 0.45
    E0, *_ = oracle_mod.dense_ground(2, 1, np.array([e1, e2]) / 2, np.full((2, 2), -g))
    want = (e1 + e2) / 2 - g - math.sqrt(g * g + (e2 - e1) ** 2 / 4)
    assert math.isclose(E0, want, abs_tol=1e-13)


def test_particle_hole(oracle_mod):
    omega, n = 9, 3
    eps, V = _rand_inst(omega, 21)
    d = 2 * eps + np.diag(V)
    _, _, _, w1 = oracle_mod.dense_ground(omega, n, eps, V)
    _, _, _, w2 = oracle_mod.dense_ground(omega, omega - n, -eps - np.diag(V), V)
    assert np.allclose(np.sort(w1), np.sort(d.sum() + w2), atol=1e-11)


# ------------------------------------------------------------------ paper tables

def test_table_lapack_dense_and_lanczos(oracle_mod, golden_dir):
    tab = _load(golden_dir, "paper_table_lapack.json")
    om, n = tab["omega"], tab["n"]
    for k, row in enumerate(tab["rows"]):
        eps, V = inputs.equal_spacing(om, -row["G"], float_g=True)
        r = oracle_mod.lanczos_ground(om, n, eps, V, krylov=50, tol=1e-12)
        assert abs(r["E0"] - row["E_lapack"]) <= 2e-12, (row, r["E0"])
        assert abs(r["E0"] - row["E_pairdiag"]) <= 2e-12, (row, r["E0"])
        if k == 0:
            # exact-double G is off the table by more than its printed digits (reading of G rounding)
            eps2, V2 = inputs.equal_spacing(om, -row["G"], float_g=False)
            r2 = oracle_mod.lanczos_ground(om, n, eps2, V2, krylov=50, tol=1e-12)
            assert abs(r2["E0"] - row["E_lapack"]) > 1e-9


def test_table_hspa_richardson(oracle_mod, golden_dir):
    tab = _load(golden_dir, "paper_table_hspa.json")
    n, g = tab["n"], -tab["G"]
    for row in tab["rows"]:
        eps = np.arange(1, row["omega"] + 1, dtype=float)
        E, u = oracle_mod.richardson_evb(eps, g, n)
        assert abs(E - row["E_richardson"]) <= 6e-8, (row, E)
        assert math.isclose(u.sum(), n, abs_tol=1e-9)
        Ef, _ = oracle_mod.richardson_evb(eps, float(np.float32(g)), n)
        assert abs(Ef - row["E_pairdiag"]) <= 6e-8, (row, Ef)


@pytest.mark.parametrize("omega,n,g", [(10, 5, 0.4), (12, 4, 0.9), (13, 6, 0.2), (14, 7, 1.3)])
def test_richardson_vs_dense_equal_spacing(oracle_mod, omega, n, g):
    eps = np.arange(1, omega + 1, dtype=float)
    E, _ = oracle_mod.richardson_evb(eps, g, n)
    E0, *_ = oracle_mod.dense_ground(omega, n, eps, np.full((omega, omega), -g))
    assert abs(E - E0) <= 1e-10 * abs(E0)


def test_richardson_vs_dense_random_levels(oracle_mod):
    rng = np.random.default_rng(3)
    omega, n, g = 11, 5, 0.35
    eps = np.sort(rng.uniform(0, 6, omega))
    E, _ = oracle_mod.richardson_evb(eps, g, n)
    E0, *_ = oracle_mod.dense_ground(omega, n, eps, np.full((omega, omega), -g))
    assert abs(E - E0) <= 1e-10 * abs(E0)


# ------------------------------------------------------------------ Lanczos and outputs

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lanczos_vs_dense_random(oracle_mod, seed):
    omega, n = 13, 6
    eps, V = _rand_inst(omega, 40 + seed)
    E0, psi0, occ0, _ = oracle_mod.dense_ground(omega, n, eps, V)
    r = oracle_mod.lanczos_ground(omega, n, eps, V, krylov=20, tol=1e-11)
    assert abs(r["E0"] - E0) <= 1e-12 * abs(E0)
    assert np.allclose(r["psi"], psi0, atol=1e-9)
    assert np.allclose(r["occ"], occ0, atol=1e-9)
    assert r["restarts"] >= 1


def test_lanczos_start_independent_and_mode1_variational(oracle_mod):
    omega, n = 12, 6
    eps, V = _rand_inst(omega, 77)
    E0, *_ = oracle_mod.dense_ground(omega, n, eps, V)
    b = oracle_mod.basis_alg1(omega, n)
    r = oracle_mod.lanczos_ground(omega, n, eps, V, krylov=15, tol=1e-11,
                                  start=inputs.random_vector(9, b.size))
    assert abs(r["E0"] - E0) <= 1e-12 * abs(E0)
    prev = math.inf
    for m in (3, 6, 10, 16):
        r1 = oracle_mod.lanczos_ground(omega, n, eps, V, krylov=m, restart=False)
        assert r1["E0"] >= E0 - 1e-12 and r1["E0"] <= prev + 1e-12
        prev = r1["E0"]


def test_perron_frobenius_and_particle_number(oracle_mod):
    omega, n = 12, 5
    eps, V = _rand_inst(omega, 8)
    E0, psi, occ, _ = oracle_mod.dense_ground(omega, n, eps, V)
    assert np.all(psi > 0)
    assert math.isclose(occ.sum(), 2 * n, abs_tol=1e-12)
    assert np.all(occ >= 0) and np.all(occ <= 2)


def test_hellmann_feynman_occupations(oracle_mod):
    omega, n = 10, 4
    eps, V = _rand_inst(omega, 31)
    E0, psi, occ, _ = oracle_mod.dense_ground(omega, n, eps, V)
    h = 1e-5
    for i in range(omega):
        ep, em = eps.copy(), eps.copy()
        ep[i] += h
        em[i] -= h
        dE = (oracle_mod.dense_ground(omega, n, ep, V)[0] - oracle_mod.dense_ground(omega, n, em, V)[0]) / (2 * h)
        assert abs(dE - occ[i]) <= 1e-7


def test_orbit_permutation_invariance(oracle_mod):
    omega, n = 10, 5
    eps, V = _rand_inst(omega, 12)
    perm = np.random.default_rng(1).permutation(omega)
    E0, _, occ, _ = oracle_mod.dense_ground(omega, n, eps, V)
    E1, _, occ1, _ = oracle_mod.dense_ground(omega, n, eps[perm], V[np.ix_(perm, perm)])
    assert abs(E0 - E1) <= 1e-12 * abs(E0)
    assert np.allclose(occ[perm], occ1, atol=1e-10)


# ------------------------------------------------------------------ warm-start pieces

def test_pbcs_constant_logits_uniform(oracle_mod):
    psi = oracle_mod.pbcs_vector(10, 4, np.full(10, 0.37))
    assert np.allclose(psi, 1 / math.sqrt(psi.size), atol=1e-15)


def test_pbcs_brute_product(oracle_mod):
    omega, n = 6, 3
    l = np.array([0.3, -1.2, 2.0, 0.0, 5.5, -3.0])
    b = oracle_mod.basis_alg1(omega, n)
    want = np.array([math.prod(math.exp(l[i] / 2) for i in range(omega) if (int(s) >> i) & 1) for s in b])
    want /= np.linalg.norm(want)
    assert np.allclose(oracle_mod.pbcs_vector(omega, n, l, b), want, rtol=1e-13)


def test_mlp_reference_gradients_finite_difference(oracle_mod):
    rng = np.random.default_rng(0)
    dims = [7, 6, 5, 4]
    params = []
    for a, c in zip(dims[:-1], dims[1:]):
        params += [rng.normal(0, 0.5, (a, c)), rng.normal(0, 0.1, c)]
    X = rng.normal(size=(3, dims[0]))
    T = rng.uniform(0, 1, (3, dims[-1]))

    def loss(ps):
        out, _ = oracle_mod.mlp_forward(ps, X)
        return oracle_mod.mlp_loss(out, T)[0]

    out, cache = oracle_mod.mlp_forward(params, X)
    _, dout = oracle_mod.mlp_loss(out, T)
    grads = oracle_mod.mlp_backward(params, cache, dout)
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp = loss(params)
            flat[idx] = old - h
            lm = loss(params)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - gflat[idx]) <= 1e-8 + 1e-6 * abs(gflat[idx])


def test_gelu_reference_matches_erf_form_closely(oracle_mod):
    x = np.linspace(-5, 5, 101)
    erf_form = 0.5 * x * (1 + np.vectorize(math.erf)(x / math.sqrt(2)))
    assert np.max(np.abs(oracle_mod.gelu_tanh(x) - erf_form)) < 1e-3
