"""GPU parity of the self-consistent loop (pd_scf_ground) against the oracle's
scf_ground: the converged field and occupations within 1e-7, E0 within 1e-9
relative; the degenerate-shell closed form; the same fixed point with and
without the previous-solution start, with fewer products with it."""
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


def _field(omega, seed, scale=0.4):
    u = inputs.uniform01(seed, 0, omega * omega).reshape(omega, omega)
    return scale * 0.5 * (u + u.T)


@pytest.mark.parametrize("om,n", [(9, 4), (10, 3), (8, 6), (12, 6)])
def test_scf_vs_oracle(pdg, oracle_mod, om, n):
    _, _, eps0, V = inputs.c5_instance(om, n, seed=om)
    W = _field(om, om + 100)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.scf_ground(b, eps0, W, V, mixing=0.5, tol=1e-9, krylov=20, start="random")
    ref = oracle_mod.scf_ground(om, n, eps0, W, V, mixing=0.5, tol=1e-11)
    assert r.status == 0 and r.info["converged"] and r.info["iterations"] > 2
    np.testing.assert_allclose(r.eps, ref["eps"], atol=1e-7)
    np.testing.assert_allclose(r.occ, ref["occ"], atol=1e-7)
    assert abs(r.E0 - ref["E0"]) <= 1e-9 * abs(ref["E0"])


def test_scf_degenerate_shell_closed_form(pdg):
    om, n, g, w = 12, 5, 0.3, 0.2
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.scf_ground(b, np.zeros(om), w * np.ones((om, om)), -g * np.ones((om, om)), mixing=1.0, tol=1e-10,
                       krylov=20, start="random")
    np.testing.assert_allclose(r.occ, 2 * n / om, atol=1e-9)
    np.testing.assert_allclose(r.eps, w * n, atol=1e-9)
    assert r.E0 == pytest.approx(2 * n * w * n - g * n * (om - n + 1), rel=1e-10)


def test_scf_previous_solution_start_same_fixed_point_fewer_products(pdg):
    om, n = 20, 10
    _, _, eps0, V = inputs.c5_instance(om, n, seed=3)
    W = _field(om, 7, 0.3)
    b = pdg.Basis(om, n, store_states=False)
    kw = dict(mixing=0.6, tol=1e-8, krylov=20, start="random")
    a = pdg.scf_ground(b, eps0, W, V, reuse_psi=True, **kw)
    c = pdg.scf_ground(b, eps0, W, V, reuse_psi=False, **kw)
    assert a.info["converged"] and c.info["converged"]
    np.testing.assert_allclose(a.eps, c.eps, atol=1e-7)
    np.testing.assert_allclose(a.occ, c.occ, atol=1e-7)
    # self-consistency of the returned pair
    np.testing.assert_allclose(eps0 + W @ a.occ / 2, a.eps, atol=1e-7)
    assert a.info["products"] < c.info["products"]


def test_scf_no_field_is_one_solve_and_errors(pdg):
    om, n = 10, 5
    _, _, eps0, V = inputs.c5_instance(om, n, seed=4)
    b = pdg.Basis(om, n, store_states=False)
    r = pdg.scf_ground(b, eps0, np.zeros((om, om)), V, krylov=20, start="random")
    g = pdg.lanczos_ground(b, eps0, V, krylov=20, start="random")
    assert r.info["iterations"] == 1 and r.E0 == pytest.approx(g.E0, rel=1e-14)
    with pytest.raises(pdg.PairDiagError):
        pdg.scf_ground(b, eps0, np.zeros((om, om)), V, mixing=0.0)
    with pytest.raises(pdg.PairDiagError):
        pdg.scf_ground(b, eps0, np.full((om, om), np.nan), V)
    m = pdg.scf_ground(b, eps0, _field(om, 9), V, max_iter=2, tol=0.0, krylov=20, start="random")
    assert m.status == pdg.PD_ENOCONV and m.info["iterations"] == 2 and not m.info["converged"]


def test_scf_benchmark_size(pdg, oracle_mod):
    """The benchmark's loop: Omega=24, n=12 (2.7e6 states), seed-0 instance,
    W = 0.3 (U + U^T)/2 (stream 5), mixing 0.6, field tol 1e-8, solves to
    1e-11.  Both starts reach the same fixed point; the returned field is that
    of the returned occupations; the final ground state satisfies the
    eigen-equation of the final field on sampled rows (the oracle's hop
    enumeration)."""
    import torch
    om, n = 24, 12
    _, _, eps0, V = inputs.c5_instance(om, n, seed=0)
    W = _field(om, 5, 0.3)
    b = pdg.Basis(om, n, store_states=False)
    kw = dict(mixing=0.6, tol=1e-8, krylov=20, start="random", lanczos_tol=1e-11)
    a = pdg.scf_ground(b, eps0, W, V, reuse_psi=True, want_psi=True, **kw)
    c = pdg.scf_ground(b, eps0, W, V, reuse_psi=False, **kw)
    assert a.info["converged"] and c.info["converged"] and a.info["lanczos_converged"]
    assert a.info["products"] < c.info["products"]
    np.testing.assert_allclose(eps0 + W @ a.occ / 2, a.eps, atol=1e-8)
    np.testing.assert_allclose(a.eps, c.eps, atol=1e-7)
    np.testing.assert_allclose(a.occ, c.occ, atol=1e-7)
    assert abs(a.E0 - c.E0) <= 1e-9 * abs(c.E0)
    assert abs(a.occ.sum() - 2 * n) <= 1e-8
    psi = a.psi
    rows = np.unique(np.random.default_rng(13).integers(0, b.dim, 2000))
    diag, tg, cf = oracle_mod.row_terms(om, n, a.eps, V, rows)
    pr = psi[torch.tensor(rows, device=psi.device)].cpu().numpy()
    pt = psi[torch.tensor(tg.reshape(-1), device=psi.device)].cpu().numpy().reshape(tg.shape)
    hpsi = diag * pr + (cf * pt).sum(axis=1)
    assert np.all(np.abs(hpsi - a.E0 * pr) <= 1e-11 * abs(a.E0) + 1e-13)


def test_scf_rejects_host_pointers_before_device_work(pdg):
    import ctypes
    om, n = 10, 5
    _, _, eps0, V = inputs.c5_instance(om, n, seed=4)
    W = _field(om, 9)
    b = pdg.Basis(om, n, store_states=False)
    L = pdg.load()
    o = pdg.make_opts(krylov=20, start="random")
    so = pdg.ScfOpts(max_iter=50, tol=1e-8, mixing=0.5, reuse_psi=1)
    nb = L.pd_scf_workspace_bytes(b.handle, ctypes.byref(o))
    buf, off = pdg.device_buffer(nb)
    eps, occ, e0 = np.empty(om), np.empty(om), ctypes.c_double()
    host = np.zeros(b.dim)
    args = (b.handle, pdg._hp(eps0), pdg._hp(W), pdg._hp(V), ctypes.byref(so), ctypes.byref(o))
    st = L.pd_scf_ground(*args, ctypes.c_void_p(buf.data_ptr() + off), nb, pdg._hp(eps), pdg._hp(occ),
                         ctypes.byref(e0), pdg._hp(host), None, None)
    assert st == pdg.PD_EINVAL                      # psi0_dev on the host
    hw = np.zeros(nb // 8 + 1)
    st = L.pd_scf_ground(*args, pdg._hp(hw), nb, pdg._hp(eps), pdg._hp(occ), ctypes.byref(e0), None, None, None)
    assert st == pdg.PD_EINVAL                      # workspace on the host
    st = L.pd_scf_ground(*args, ctypes.c_void_p(buf.data_ptr() + off), nb, pdg._hp(eps), pdg._hp(occ),
                         ctypes.byref(e0), None, None, None)
    assert st == pdg.PD_OK
