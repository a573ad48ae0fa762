"""GPU parity of the lowest eigenpairs (thick-restart Lanczos,
pd_lanczos_eigs) against the oracle's lowest_eigenpairs: energies within
1e-10 relative, explicit residuals within the tolerance, eigenvectors up to
sign within 1e-7, occupations within 1e-8."""
import math

import numpy as np
import pytest

from paper_2001_01978_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdg():
    import torch
    assert torch.cuda.is_available()
    from paper_2001_01978_amd import pairdiag
    pairdiag.load()
    return pairdiag


def _check(r, w, Z, occ, rtol=1e-10, vtol=1e-7, otol=1e-8):
    nev = len(w)
    assert r.converged and r.status == 0
    np.testing.assert_allclose(r.E, w, rtol=rtol, atol=rtol)
    assert (r.residuals <= 1e-10).all()
    psi = r.psi.cpu().numpy()
    for i in range(nev):
        ov = abs(float(psi[i] @ Z[:, i]))
        assert ov == pytest.approx(1.0, abs=vtol), (i, ov)
    np.testing.assert_allclose(r.occ, occ, atol=otol)


@pytest.mark.parametrize("om,n,nev,krylov", [(12, 6, 4, 20), (13, 4, 6, 24), (14, 9, 3, 16), (10, 5, 1, 12),
                                             (16, 8, 8, 40)])
def test_eigs_vs_oracle_dense(pdg, oracle_mod, om, n, nev, krylov):
    _, _, eps, V = inputs.c5_instance(om, n, seed=om * 7 + nev)
    print(f"eigs om={om} n={n} nev={nev}", flush=True)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.lanczos_eigs(b, eps, V, nev, krylov=krylov, tol=1e-11, seed=2)
    _check(r, *oracle_mod.lowest_eigenpairs(om, n, eps, V, nev))


def test_eigs_space_smaller_than_krylov_is_exact(pdg, oracle_mod):
    om, n = 6, 3
    _, _, eps, V = inputs.c5_instance(om, n, seed=1)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.lanczos_eigs(b, eps, V, 5, krylov=30, tol=1e-11)
    _check(r, *oracle_mod.lowest_eigenpairs(om, n, eps, V, 5))
    r1 = pdg.lanczos_eigs(pdg.Basis(1, 1, store_states=False), np.array([0.5]), np.array([[-0.2]]), 1, krylov=4)
    assert r1.E[0] == pytest.approx(0.8, abs=1e-15)


def test_eigs_degenerate_shell_gives_distinct_quasispin_levels(pdg):
    om, n, g = 14, 6, 0.3
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.lanczos_eigs(b, np.zeros(om), -g * np.ones((om, om)), 4, krylov=20, tol=1e-12)
    sz = n - om / 2
    levels = [-g * ((om / 2 - nu) * (om / 2 - nu + 1) - sz * (sz - 1)) for nu in range(4)]
    np.testing.assert_allclose(r.E, levels, rtol=1e-11)


def test_eigs_larger_vs_oracle_arpack(pdg, oracle_mod):
    om, n, nev = 20, 8, 4
    _, _, eps, V = inputs.c5_instance(om, n, seed=3)
    print("eigs om=20 n=8 vs ARPACK", flush=True)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.lanczos_eigs(b, eps, V, nev, krylov=30, tol=1e-10, seed=1)
    _check(r, *oracle_mod.lowest_eigenpairs(om, n, eps, V, nev), rtol=1e-10, vtol=1e-6, otol=1e-7)


def test_eigs_nev1_matches_ground_state(pdg):
    om, n = 18, 9
    _, _, eps, V = inputs.c5_instance(om, n, seed=4)
    b = pdg.Basis(om, n, store_states=False)
    g = pdg.lanczos_ground(b, eps, V, krylov=20, tol=1e-11, start="random")
    r = pdg.lanczos_eigs(b, eps, V, 1, krylov=20, tol=1e-11)
    assert r.E[0] == pytest.approx(g.E0, rel=1e-12)
    np.testing.assert_allclose(r.psi[0].cpu().numpy(), g.psi.cpu().numpy(), atol=1e-7)
    np.testing.assert_allclose(r.occ[0], g.occ, atol=1e-9)


def test_eigs_on_truncated_space(pdg, oracle_mod):
    om, n, limit = 14, 7, 1500
    _, _, eps, V = inputs.c5_instance(om, n, seed=5)
    ref = oracle_mod.trunc_select(om, n, eps, V, limit, 10**8)
    H = oracle_mod.dense_h(om, n, eps, V)
    k = ref["ranks"]
    w = np.linalg.eigvalsh(H[np.ix_(k, k)])[:3]
    b = pdg.Basis.truncated(om, n, eps, V, limit, 10**8)
    r = pdg.lanczos_eigs(b, eps, V, 3, krylov=20, tol=1e-11)
    assert r.converged
    np.testing.assert_allclose(r.E, w, rtol=1e-10)


def test_eigs_argument_errors(pdg):
    om, n = 10, 5
    _, _, eps, V = inputs.c5_instance(om, n, seed=6)
    b = pdg.Basis(om, n, store_states=False)
    for kw in (dict(krylov=6, nev=5), dict(krylov=20, nev=3, start="hf")):
        nev = kw.pop("nev")
        with pytest.raises(pdg.PairDiagError):
            pdg.lanczos_eigs(b, eps, V, nev, **kw)


@pytest.mark.parametrize("om,n,nev", [(16, 8, 1), (16, 8, 4), (20, 9, 3)])
def test_eigs_mixed_precision(pdg, oracle_mod, om, n, nev):
    # FP32 phase, then FP64 to the tolerance: the same pairs as FP64 alone
    _, _, eps, V = inputs.c5_instance(om, n, seed=om + 3 * nev)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.lanczos_eigs(b, eps, V, nev, krylov=24, tol=1e-10, seed=3, precision="f32")
    assert r.iterations_f32 > 0 and r.iterations > r.iterations_f32
    _check(r, *oracle_mod.lowest_eigenpairs(om, n, eps, V, nev), rtol=1e-10, vtol=1e-6, otol=1e-7)


def test_eigs_full_size_sampled(pdg, oracle_mod):
    """The benchmark's four lowest states as they are timed: Omega=32, n=16
    (6.0e8 states), seed-0 instance, krylov 20, tol 1e-10, FP64.  For each
    pair the eigen-equation on sampled rows with the oracle's own hop
    enumeration, |(H psi)_r - E psi_r| <= res |E|; orthonormal vectors; the
    ground state alone without a negative component (Perron-Frobenius), the
    others with both signs."""
    import torch
    om, n, nev = 32, 16, 4
    _, _, eps, V = inputs.c5_instance(om, n, seed=0)
    b = pdg.Basis(om, n, store_states=False)
    print("full-size eigenpairs omega=32 n=16 nev=4", flush=True)
    r = pdg.lanczos_eigs(b, eps, V, nev, krylov=20, tol=1e-10, seed=1)
    assert r.converged and (r.residuals <= 1e-10).all()
    assert np.all(np.diff(r.E) > 0)
    psi = r.psi
    G = (psi @ psi.T).cpu().numpy()
    np.testing.assert_allclose(G, np.eye(nev), atol=1e-10)
    big = [float(psi[i].abs().max()) for i in range(nev)]
    assert int((psi[0] < -1e-6 * big[0]).sum()) == 0
    for i in range(1, nev):
        assert int((psi[i] < -1e-6 * big[i]).sum()) > 0 and int((psi[i] > 1e-6 * big[i]).sum()) > 0
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([rng.integers(0, b.dim, 2000), np.arange(0, 50), np.arange(b.dim - 50, b.dim)]))
    diag, tg, cf = oracle_mod.row_terms(om, n, eps, V, rows)
    ri = torch.tensor(rows, device=psi.device)
    ti = torch.tensor(tg.reshape(-1), device=psi.device)
    for i in range(nev):
        pr = psi[i][ri].cpu().numpy()
        pt = psi[i][ti].cpu().numpy().reshape(tg.shape)
        hpsi = diag * pr + (cf * pt).sum(axis=1)
        assert np.all(np.abs(hpsi - r.E[i] * pr) <= r.residuals[i] * abs(r.E[i]) + 1e-13), i
    np.testing.assert_allclose(r.occ.sum(axis=1), 2 * n, atol=1e-8)
