"""Host-side checks of the C ABI library: it loads without a GPU, exports every
symbol declared in include/pairdiag.h, and its host-only logic (sizes,
validation that happens before any device work, the tridiagonal eigensolver)
behaves.  No compute call touches a device here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2001_01978_amd import inputs
from paper_2001_01978_amd import pairdiag as pdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "pairdiag.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = pdg.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(pdg.SIGNATURES), set(declared) ^ set(pdg.SIGNATURES)


def test_version_and_status_strings():
    L = pdg.load()
    assert L.pd_version().startswith(b"pairdiag")
    for s, name in enumerate(["PD_OK", "PD_EINVAL", "PD_ERANGE", "PD_ENOMEM", "PD_EDEVICE", "PD_ENOCONV"]):
        assert L.pd_status_str(s).decode() == name


def test_dimension_and_sizes():
    L = pdg.load()
    for om in range(1, 63):
        for n in (0, 1, om // 3, om // 2, om):
            assert pdg.dimension(om, n) == math.comb(om, n)
    assert pdg.dimension(0, 0) == 0 and pdg.dimension(63, 2) == 0 and pdg.dimension(10, 11) == 0
    assert L.pd_basis_bytes(10, 11, 1) == 0
    b0 = L.pd_basis_bytes(28, 14, 0)
    b1 = L.pd_basis_bytes(28, 14, 1)
    assert b0 > 0 and b1 - b0 >= 8 * 40116600 and b1 % 256 == 0


def test_basis_create_rejects_bad_space_before_device_work():
    L = pdg.load()
    h = ctypes.c_void_p()
    assert L.pd_basis_create(70, 3, 0, None, 0, None, ctypes.byref(h)) == pdg.PD_EINVAL
    assert L.pd_basis_create(10, 4, 1, None, 10, None, ctypes.byref(h)) == pdg.PD_ENOMEM
    assert b"need" in L.pd_last_error()


@pytest.mark.parametrize("m", [1, 2, 3, 7, 20, 50, 64])
def test_tridiag_lowest_against_library_eigh(m):
    rng = np.random.default_rng(m)
    a = rng.normal(size=m) * 3
    b = rng.normal(size=max(m - 1, 0))
    th, y = pdg.tridiag_lowest(a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    w, Z = np.linalg.eigh(T)
    assert abs(th - w[0]) <= 1e-13 * max(1.0, np.abs(w).max())
    z = Z[:, 0] * (1 if Z[0, 0] >= 0 else -1)
    assert np.allclose(y, z, atol=1e-10)
    assert abs(np.linalg.norm(y) - 1) < 1e-14


def test_tridiag_lowest_degenerate_offdiagonal():
    a = np.array([3.0, 1.0, 2.0, 1.5])
    b = np.array([0.0, 0.0, 0.0])
    th, y = pdg.tridiag_lowest(a, b)
    assert th == pytest.approx(1.0, abs=1e-14)
    assert abs(abs(y[1]) - 1.0) < 1e-12


def test_splitmix64_published_value():
    # SplitMix64 from state 0: the first output is 0xE220A8397B1DCDAF
    assert int(inputs.splitmix64(0, 0, 1)[0]) == 0xE220A8397B1DCDAF
    u = inputs.uniform01(123, 0, 100000)
    assert 0 <= u.min() and u.max() < 1 and abs(u.mean() - 0.5) < 0.01


def test_instance_recipes_shapes_and_signs():
    om, n, eps, V = inputs.c1_instance(0)
    assert (om, n) == (16, 8) and np.all(np.diff(eps) >= 0) and eps.max() < 10
    assert np.array_equal(V, V.T) and np.all(V < 0) and np.all(-V <= 0.3 * 1.2 + 1e-15)
    for seed in range(50):
        om, n, eps, V = inputs.family3_instance(seed)
        assert 10 <= om <= 24 and math.ceil(om / 4) <= n <= om // 2
        assert np.array_equal(V, V.T) and np.all(V < 0)


@pytest.mark.parametrize("om,n,bins", [(10, 5, 1000), (12, 4, 10**8), (9, 0, 7), (9, 9, 5), (14, 7, 3), (7, 3, 1)])
def test_trunc_select_without_a_cut_runs_on_the_host(oracle_mod, om, n, bins):
    """When the space fits the limit, pd_trunc_select needs no device: the
    extreme diagonals (n lowest / highest pair energies, stable order) and the
    bin scale against the oracle, bit for bit, and every state kept."""
    L = pdg.load()
    _, _, eps, V = inputs.c5_instance(om, n, seed=om + n)
    full = math.comb(om, n)
    info = pdg.TruncInfo()
    st = L.pd_trunc_select(om, n, pdg._hp(eps), pdg._hp(V), full, bins, None, 0, ctypes.byref(info), None)
    assert st == pdg.PD_OK, L.pd_last_error()
    ref = oracle_mod.trunc_select(om, n, eps, V, full, bins, method="numpy")
    assert (info.full_dim, info.kept, info.cut_bin, info.bins, info.limit) == (full, full, bins - 1, bins, full)
    assert info.dmin == ref["dmin"] and info.dmax == ref["dmax"] and info.scale == ref["scale"]
    if ref["scale"] > 0:
        assert info.cutoff == ref["dmin"] + bins / ref["scale"]
    else:
        assert info.cutoff == ref["dmin"]


def test_new_entry_points_reject_bad_arguments_before_device_work():
    L = pdg.load()
    om, n = 10, 4
    _, _, eps, V = inputs.c5_instance(om, n, seed=3)
    o = pdg.make_opts(krylov=20, start="random")
    E, blk = ctypes.c_double(), ctypes.c_int()

    def odd(omega, nn, block, route, opts=o):
        return L.pd_lanczos_ground_odd(omega, nn, pdg._hp(eps), pdg._hp(V), block, route, ctypes.byref(opts),
                                       None, 0, ctypes.byref(E), ctypes.byref(blk), None, None, None, None)
    assert odd(1, 0, 0, 0) == pdg.PD_EINVAL                 # omega < 2
    assert odd(om, om, 0, 0) == pdg.PD_EINVAL               # n > omega - 1 pairs
    assert odd(om, n, om + 1, 0) == pdg.PD_EINVAL           # block outside [0, omega]
    assert odd(om, n, 0, 3) == pdg.PD_EINVAL                # unknown route
    assert odd(om, n, 2, 2) == pdg.PD_EINVAL                # batched route solves all blocks
    assert odd(om, n, 0, 0, pdg.make_opts(start="user")) == pdg.PD_EINVAL
    assert L.pd_odd_workspace_bytes(1, 0, 0, 0, ctypes.byref(o)) == 0
    assert L.pd_odd_workspace_bytes(om, n, 0, 3, ctypes.byref(o)) == 0
    big = pdg.make_opts(krylov=40)
    assert odd(om, n, 0, 2, big) == pdg.PD_ERANGE           # krylov above the batched limit
    info = pdg.TruncInfo()
    for args in ((0, 0, 10, 100), (om, om + 1, 10, 100), (om, n, 0, 100), (om, n, 10, 0), (om, n, 10, 2 ** 31)):
        w, nn, lim, bins = args
        assert L.pd_trunc_select(w, nn, pdg._hp(eps), pdg._hp(V), lim, bins, None, 0, ctypes.byref(info),
                                 None) == pdg.PD_EINVAL, args
    assert L.pd_trunc_select_bytes(om, n, 0) == 0 and L.pd_trunc_select_bytes(70, 3, 10) == 0
    assert L.pd_lanczos_eigs(None, pdg._hp(eps), pdg._hp(V), 2, ctypes.byref(o), None, 0, None, None, None, None,
                             None, None) == pdg.PD_EINVAL
    so = pdg.ScfOpts(max_iter=10, tol=1e-8, mixing=0.5, reuse_psi=1)
    assert L.pd_scf_ground(None, pdg._hp(eps), pdg._hp(V), pdg._hp(V), ctypes.byref(so), ctypes.byref(o), None, 0,
                           None, None, ctypes.byref(E), None, None, None) == pdg.PD_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits 2
    before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sigma_launch_shape_fits_its_limit_for_every_space():
    """Every space with a product kernel (Omega <= 62, min(n, Omega - n) <=
    20), in both precisions and both rank widths: the workgroup pd_sigma
    launches asks for no more LDS than the kernel runs under, within the
    160 KB of a CU less the static LDS.  (FP64 at Omega=35, n=17 once chose
    512 threads at 162,864 bytes against a 162,816-byte limit.)"""
    usable = 160 * 1024 - 1024
    count = 0
    for om in range(1, 63):
        for n in range(om + 1):
            if min(n, om - n) > 20:
                continue
            for dt in ("f64", "f32"):
                t, lds, lim = pdg.sigma_launch_shape(om, n, dt)
                assert t in (256, 512), (om, n, dt)
                assert lds <= lim <= usable, (om, n, dt, t, lds, lim)
                count += 1
    assert count > 2500
    assert pdg.sigma_launch_shape(35, 17, "f64")[0] == 256
    assert pdg.sigma_launch_shape(32, 16, "f64")[0] == 512


def test_sigma_launch_shape_errors():
    L = pdg.load()
    t, a, b = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
    assert L.pd_sigma_launch_shape(63, 2, 0, ctypes.byref(t), ctypes.byref(a), ctypes.byref(b)) == 1   # PD_EINVAL
    assert L.pd_sigma_launch_shape(20, 21, 0, ctypes.byref(t), ctypes.byref(a), ctypes.byref(b)) == 1
    assert L.pd_sigma_launch_shape(20, 10, 7, ctypes.byref(t), ctypes.byref(a), ctypes.byref(b)) == 1
    assert L.pd_sigma_launch_shape(20, 10, 0, None, ctypes.byref(a), ctypes.byref(b)) == 1
    assert L.pd_sigma_launch_shape(62, 21, 0, ctypes.byref(t), ctypes.byref(a), ctypes.byref(b)) == 2  # PD_ERANGE


def test_bench_kernel_hash_ignores_comments_and_layout():
    """The counter summaries are matched to the product kernel by a hash of
    its code: comments and whitespace do not enter it, string literals and
    every token of code do."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    a = "int f(int x) {  // first\n  return x + 1; /* two\n lines */ }\n"
    b = "int f(int x) {\n\n    return x + 1;   }  // another\n"
    assert bench.code_tokens(a) == bench.code_tokens(b) == "int f(int x) { return x + 1; }"
    assert bench.code_tokens("s = \"a // b\"; c = '/'; // x") == "s = \"a // b\"; c = '/';"
    assert bench.code_tokens(a.replace("x + 1", "x + 2")) != bench.code_tokens(a)
    src = open(os.path.join(ROOT, "paper_2001_01978_amd", "csrc", "sigma_impl.h")).read()
    assert bench.code_tokens(src) == bench.code_tokens(re.sub(r"//[^\n]*", "", src))
    assert len(bench.kernel_source_hash()) == 16
