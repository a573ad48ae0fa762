"""GPU parity: the HIP path (through the C ABI) against the oracle.

Basis and ranks are compared bit for bit.  Sigma is compared element by
element: bit-exact on dyadic inputs (every product and partial sum is exact,
so summation order cannot matter), and within a rounding bound on random
inputs.  At the full workload sizes sigma is checked on sampled rows that the
oracle computes one by one.
"""
import math

import numpy as np
import pytest

from paper_2001_01978_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pdg():
    from paper_2001_01978_amd import pairdiag
    pairdiag.load()
    return pairdiag


def _host_u64(t):
    return t.cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------ basis

SMALL_SPACES = [(om, n) for om in range(1, 17) for n in range(0, om + 1)]


def test_basis_bit_exact_all_small_spaces(torch_cuda, pdg, oracle_mod):
    for om, n in SMALL_SPACES:
        b = pdg.Basis(om, n)
        got = _host_u64(b.states())
        want = oracle_mod.basis_alg1(om, n)
        assert np.array_equal(got, want), (om, n)


@pytest.mark.parametrize("om,n", [(20, 10), (24, 12), (26, 7), (62, 2), (62, 60), (28, 14)])
def test_basis_bit_exact_larger(torch_cuda, pdg, oracle_mod, om, n):
    b = pdg.Basis(om, n)
    got = _host_u64(b.states())
    want = oracle_mod.basis_alg1(om, n)
    assert got.size == want.size == math.comb(om, n)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("om,n", [(16, 8), (34, 17), (40, 9), (62, 31), (62, 1), (35, 17)])
def test_rank_unrank_vs_hash(torch_cuda, pdg, oracle_mod, om, n):
    torch = torch_cuda
    b = pdg.Basis(om, n, store_states=False)
    d = math.comb(om, n)
    rng = np.random.default_rng(om * 64 + n)
    ranks = np.unique(np.concatenate([rng.integers(0, d, 4000), [0, d - 1]]))
    states = _host_u64(b.unrank(torch.tensor(ranks, device="cuda")))
    for r, s in zip(ranks[:600], states[:600]):
        assert oracle_mod.unhash(int(r), n) == int(s)
        assert oracle_mod.hash_index(int(s)) == int(r)
    back = b.rank(torch.tensor(states.view(np.int64), device="cuda")).cpu().numpy()
    assert np.array_equal(back, ranks)


def test_rank_rejects_foreign_states(torch_cuda, pdg):
    torch = torch_cuda
    b = pdg.Basis(10, 4, store_states=False)
    bad = np.array([0b111, 0b11111, 1 << 10 | 0b111, 0b1111], dtype=np.uint64)
    r = b.rank(torch.tensor(bad.view(np.int64), device="cuda")).cpu().numpy()
    assert list(r[:3]) == [-1, -1, -1] and r[3] == 0


# ------------------------------------------------------------------ sigma

SIGMA_SPACES = [(4, 2), (1, 0), (1, 1), (2, 1), (5, 0), (5, 5), (9, 1), (9, 8), (12, 5), (12, 7),
                (13, 6), (16, 8), (18, 3), (18, 15), (20, 10), (22, 11), (40, 3), (62, 2), (62, 61),
                (30, 5), (33, 7), (24, 12)]


@pytest.mark.parametrize("om,n", SIGMA_SPACES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sigma_dyadic_bit_exact(torch_cuda, pdg, oracle_mod, om, n, dtype):
    torch = torch_cuda
    omega, n, eps, V = inputs.dyadic_instance(om, n, seed=om * 100 + n)
    d = math.comb(om, n)
    basis = oracle_mod.basis_alg1(om, n)
    x = inputs.dyadic_vector(om + n, d, bits=6 if dtype == "f32" else 8)
    want = oracle_mod.sigma(om, n, eps, V, basis, x)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = pdg.Basis(om, n, store_states=False)
    xt = torch.tensor(x, dtype=tdt, device="cuda")
    y = b.sigma(eps, V, xt).cpu().numpy().astype(np.float64)
    assert np.array_equal(y, want), (om, n, dtype, np.abs(y - want).max())


@pytest.mark.parametrize("om,n", [(16, 8), (20, 7), (21, 14), (24, 12)])
def test_sigma_random_f64_and_f32(torch_cuda, pdg, oracle_mod, om, n):
    torch = torch_cuda
    rng = np.random.default_rng(om + 7 * n)
    eps = rng.uniform(0, om, om)
    G = rng.uniform(0.1, 0.6, (om, om))
    V = -(G + G.T) / 2
    d = math.comb(om, n)
    basis = oracle_mod.basis_alg1(om, n)
    x = inputs.random_vector(5, d)
    want = oracle_mod.sigma(om, n, eps, V, basis, x)
    # |H| |x| bounds the rounding of any summation order
    absx = oracle_mod.sigma(om, n, np.abs(eps), np.abs(V), basis, np.abs(x))
    b = pdg.Basis(om, n, store_states=False)
    y64 = b.sigma(eps, V, torch.tensor(x, device="cuda")).cpu().numpy()
    K = n * (om - n) + 1
    assert np.all(np.abs(y64 - want) <= 2 * K * 2.0 ** -53 * absx + 1e-300)
    x32 = x.astype(np.float32)
    want32 = oracle_mod.sigma(om, n, eps, V, basis, x32.astype(np.float64))
    y32 = b.sigma(eps, V, torch.tensor(x32, device="cuda")).cpu().numpy().astype(np.float64)
    # float coefficients (relative 2^-24 each) plus float accumulation
    assert np.all(np.abs(y32 - want32) <= (2 * K + 4) * 2.0 ** -24 * absx)


def test_sigma_repeated_launches_cover_every_row(torch_cuda, pdg, oracle_mod):
    """Omega=24, n=12 (5,282 tiles of 512 rows, more than the grid's
    workgroups: tiles come from the tile counter): every launch writes every
    row, whatever ran before on the same basis."""
    torch = torch_cuda
    om, n, eps, V = inputs.dyadic_instance(24, 12, seed=77)
    d = math.comb(om, n)
    x = inputs.dyadic_vector(om + n, d, bits=6)
    want = oracle_mod.sigma(om, n, eps, V, oracle_mod.basis_alg1(om, n), x)
    b = pdg.Basis(om, n, store_states=False)
    for dt in (torch.float64, torch.float32, torch.float32, torch.float64):
        xt = torch.tensor(x, dtype=dt, device="cuda")
        y = torch.full_like(xt, float("nan"))
        b.sigma(eps, V, xt, y)
        assert np.array_equal(y.cpu().numpy().astype(np.float64), want), dt


def test_sigma_matches_paper_6x6(torch_cuda, pdg, oracle_mod, golden_dir):
    import json, os
    torch = torch_cuda
    ex = json.load(open(os.path.join(golden_dir, "paper_matrix_6x6.json")))
    eps = np.array(ex["eps"], float)
    V = np.full((4, 4), ex["V_const"])
    H = np.array(ex["H"])
    b = pdg.Basis(4, 2)
    for j in range(6):
        e = torch.zeros(6, dtype=torch.float64, device="cuda")
        e[j] = 1.0
        col = b.sigma(eps, V, e).cpu().numpy()
        assert np.allclose(col, H[:, j], atol=1e-15, rtol=0)


def _sampled_rows(d, count, seed):
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.integers(0, d, count), np.arange(0, 300), np.arange(d - 300, d)]))
    return rows


def _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x_dev, rows):
    """(H x)[rows] with x read from the device only where the rows need it."""
    import torch
    diag, tg, cf = oracle_mod.row_terms(om, n, eps, V, rows)
    xr = x_dev[torch.tensor(rows, device=x_dev.device)].cpu().numpy().astype(np.float64)
    xt = x_dev[torch.tensor(tg.reshape(-1), device=x_dev.device)].cpu().numpy().astype(np.float64).reshape(tg.shape)
    want = diag * xr + (cf * xt).sum(axis=1)
    bound = np.abs(diag * xr) + (np.abs(cf) * np.abs(xt)).sum(axis=1)
    return want, bound


def test_sigma_full_size_omega28_sampled_f64(torch_cuda, pdg, oracle_mod):
    """Full 40,116,600-state space (Omega=28, n=14), the launch the bench times."""
    torch = torch_cuda
    om, n, eps, V = inputs.c2b_instance(0)
    d = math.comb(om, n)
    b = pdg.Basis(om, n, store_states=False)
    x = torch.empty(d, dtype=torch.float64, device="cuda")
    x.uniform_(-1, 1, generator=torch.Generator(device="cuda").manual_seed(3))
    y = b.sigma(eps, V, x)
    rows = _sampled_rows(d, 20000, 1)
    want, bound = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy()
    K = n * (om - n) + 1
    assert np.all(np.abs(got - want) <= 2 * K * 2.0 ** -53 * bound)


@pytest.mark.parametrize("om,n", [(28, 14), (32, 16), (34, 17)])
def test_sigma_full_size_dyadic_exact_sampled(torch_cuda, pdg, oracle_mod, om, n):
    """FP64 and FP32 at Omega=28 (4.0e7 states), Omega=32 (6.0e8 states, the
    benchmark's space and launch) and Omega=34 (2.3e9 states; FP64 there runs
    256-thread workgroups): exact on sampled rows, and every row written (the
    FP64 launches at 32 and 34 orbits hand out tiles in per-XCD chunks)."""
    torch = torch_cuda
    _, _, eps, V = inputs.dyadic_instance(om, n, 5)
    d = math.comb(om, n)
    b = pdg.Basis(om, n, store_states=False)
    dts = (torch.float64, torch.float32)
    for dt in dts:
        x = torch.randint(-63, 64, (d,), dtype=dt, device="cuda")
        y = torch.full_like(x, float("nan"))
        b.sigma(eps, V, x, y)
        assert not bool(torch.isnan(y).any()), (dt, "a row was not written")
        rows = _sampled_rows(d, 4000, 2)
        want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
        got = y[torch.tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
        assert np.array_equal(got, want), dt
        del x, y
        torch.cuda.empty_cache()


def test_sigma_chunked_schedule_every_row(torch_cuda, pdg, oracle_mod):
    """Omega=30, n=15 (1.55e8 states, 302,964 tiles: FP64 tiles go out in
    per-XCD chunks of 36): launches in a row, FP32 launches (one tile per
    request) between them, and two streams sharing the handle; every launch
    writes every row, all launches agree bit for bit, and sampled rows equal
    the oracle exactly."""
    torch = torch_cuda
    om, n, eps, V = inputs.dyadic_instance(30, 15, 11)
    d = math.comb(om, n)
    b = pdg.Basis(om, n, store_states=False)
    x = torch.randint(-63, 64, (d,), dtype=torch.float64, device="cuda")
    x32 = x.float()
    ref = None
    for dt in (torch.float64, torch.float32, torch.float64, torch.float64):
        xi = x if dt == torch.float64 else x32
        y = torch.full_like(xi, float("nan"))
        b.sigma(eps, V, xi, y)
        assert not bool(torch.isnan(y).any()), (dt, "a row was not written")
        if ref is None:
            ref = y
        else:
            assert torch.equal(y.double(), ref), dt
        del y
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    ys = []
    for k in range(4):
        st = streams[k % 2]
        with torch.cuda.stream(st):
            y = torch.full_like(x, float("nan"))
            b.sigma(eps, V, x, y, stream=st)
            ys.append(y)
    torch.cuda.synchronize()
    for y in ys:
        assert torch.equal(y, ref)
    rows = _sampled_rows(d, 2000, 4)
    want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = ref[torch.tensor(rows, device="cuda")].cpu().numpy()
    assert np.array_equal(got, want)
    del x, x32, ys, ref
    torch.cuda.empty_cache()


def test_sigma_most_pairs_that_fit(torch_cuda, pdg, oracle_mod):
    """Omega=36, n=18: 9.1e9 states, 18 pairs (the most whose vectors fit the
    device: 19 pairs need at least C(38, 19) = 3.5e10 states), 64-bit ranks,
    FP32 vectors of 36 GB: exact on sampled rows, every row written."""
    import gc
    torch = torch_cuda
    gc.collect()
    torch.cuda.empty_cache()
    om, n, eps, V = inputs.dyadic_instance(36, 18, 12)
    d = math.comb(om, n)
    b = pdg.Basis(om, n, store_states=False)
    x = torch.randint(-63, 64, (d,), dtype=torch.float32, device="cuda")
    y = torch.full_like(x, float("nan"))
    b.sigma(eps, V, x, y)
    written = not bool(torch.isnan(y).any())
    rows = _sampled_rows(d, 800, 7)
    want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    del x, y
    torch.cuda.empty_cache()
    assert written, "a row was not written"
    assert np.array_equal(got, want)


@pytest.mark.parametrize("om,n,dtype", [(32, 17, "f64"), (32, 17, "f32"), (35, 18, "f32")])
def test_sigma_mirrored_full_size_sampled(torch_cuda, pdg, oracle_mod, om, n, dtype):
    """n > Omega/2 at full size: the mirrored kernel (holes as particles,
    ranks dim-1-k) on 5.65e8 states (32 orbits, 17 pairs; FP64 takes the
    per-XCD chunk schedule) and on 4.5e9 states (35 orbits, 18 pairs, 64-bit
    ranks): exact on sampled rows, every row written."""
    import gc
    torch = torch_cuda
    gc.collect()
    torch.cuda.empty_cache()
    _, _, eps, V = inputs.dyadic_instance(om, n, 9)
    d = math.comb(om, n)
    assert n > om - n
    b = pdg.Basis(om, n, store_states=False)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    x = torch.randint(-63, 64, (d,), dtype=tdt, device="cuda")
    y = torch.full_like(x, float("nan"))
    b.sigma(eps, V, x, y)
    written = not bool(torch.isnan(y).any())
    rows = _sampled_rows(d, 1500, 6)
    want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    del x, y
    torch.cuda.empty_cache()
    assert written, "a row was not written"
    assert np.array_equal(got, want)


@pytest.mark.skip(reason="disabled in the library: the product on this space (mirrored, 16 pairs, 32-bit ranks) "
                         "made an illegal memory access at Omega=34, n=18 and its cause is not found; pd_sigma "
                         "refuses it with PD_ERANGE (test_sigma_refuses_disabled_mirrored_spaces)")
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sigma_mirrored_16_pairs_rank32_full_size_sampled(torch_cuda, pdg, oracle_mod, dtype):
    """Omega=34, n=18 (2.2e9 states, mirrored: 16 holes, 32-bit ranks):
    exact on sampled rows, every row written."""
    torch = torch_cuda
    om, n = 34, 18
    _, _, eps, V = inputs.dyadic_instance(om, n, 9)
    d = math.comb(om, n)
    b = pdg.Basis(om, n, store_states=False)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    x = torch.randint(-63, 64, (d,), dtype=tdt, device="cuda")
    y = torch.full_like(x, float("nan"))
    b.sigma(eps, V, x, y)
    written = not bool(torch.isnan(y).any())
    rows = _sampled_rows(d, 1500, 6)
    want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    del x, y
    torch.cuda.empty_cache()
    assert written, "a row was not written"
    assert np.array_equal(got, want)


@pytest.mark.parametrize("om,n", [(33, 17), (34, 18), (35, 19)])
def test_sigma_refuses_disabled_mirrored_spaces(torch_cuda, pdg, om, n):
    """The full-space products the library disables (mirrored, 16 pairs,
    32-bit ranks) are refused with PD_ERANGE before any device work, by
    pd_sigma and pd_lanczos_ground alike; the neighbouring mirrored spaces
    keep their kernels (checked by the tests above)."""
    import ctypes
    L = pdg.load()
    assert math.comb(om, n) < 2 ** 32 and om - n == 16
    _, _, eps, V = inputs.c5_instance(om, n, seed=0)
    b = pdg.Basis(om, n, store_states=False)
    st = L.pd_sigma(b.handle, pdg._hp(eps), pdg._hp(V), pdg.PD_F64, None, None, None)
    assert st == pdg.PD_ERANGE and b"disabled" in L.pd_last_error()
    st = L.pd_sigma(b.handle, pdg._hp(eps), pdg._hp(V), pdg.PD_F32, None, None, None)
    assert st == pdg.PD_ERANGE
    o = pdg.make_opts(krylov=20)
    E = ctypes.c_double()
    st = L.pd_lanczos_ground(b.handle, pdg._hp(eps), pdg._hp(V), ctypes.byref(o), None, 0, None, ctypes.byref(E),
                             None, None, None, None)
    assert st == pdg.PD_ERANGE and b"disabled" in L.pd_last_error()
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sigma_rank64_path_sampled(torch_cuda, pdg, oracle_mod, dtype):
    """dim = C(35,17) = 4.5e9 > 2^32: 64-bit rank arithmetic; FP32 (18 GB
    vectors) and FP64 (36 GB vectors, where 512-thread workgroups would need
    all but 1 KB of a CU's LDS and 256-thread ones are taken): exact on
    sampled rows, every row written."""
    import gc
    torch = torch_cuda
    gc.collect()
    torch.cuda.empty_cache()
    om, n, eps, V = inputs.dyadic_instance(35, 17, 8)
    d = math.comb(om, n)
    assert d > 2 ** 32
    b = pdg.Basis(om, n, store_states=False)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    x = torch.randint(-63, 64, (d,), dtype=tdt, device="cuda")
    y = torch.full_like(x, float("nan"))
    b.sigma(eps, V, x, y)
    written = not bool(torch.isnan(y).any())
    rows = _sampled_rows(d, 1500, 3)
    want, _ = _oracle_rows_on_device_x(oracle_mod, om, n, eps, V, x, rows)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    del x, y
    torch.cuda.empty_cache()
    assert written, "a row was not written"
    assert np.array_equal(got, want)
