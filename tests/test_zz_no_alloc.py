"""GPU: the allocation-free ground-state entry point (pd_lanczos_ground_static,
whose workspace is the library's static device array) against the entry point
with a caller workspace (pd_lanczos_ground), on two calls in a row, the second
with a smaller problem, and its size limit."""
import math

import numpy as np
import pytest

from paper_2001_01978_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_01978_amd import pairdiag
    pairdiag.load()
    return pairdiag


def _compare(pdg, om, n, seed, precision):
    _, _, eps, V = inputs.c5_instance(om, n, seed=seed)
    b = pdg.Basis(om, n, store_states=False)
    kw = dict(krylov=16, tol=1e-10, start="random", seed=seed, precision=precision)
    assert pdg.workspace_bytes(b, **{k: kw[k] for k in ("krylov", "precision")}) <= pdg.STATIC_SCRATCH_BYTES
    ref = pdg.lanczos_ground(b, eps, V, **kw)
    got = pdg.lanczos_ground_static(b, eps, V, **kw)
    assert ref.converged and got.converged
    # the same algorithm on the same start: E0 to the FP64 bar, and the state
    assert abs(got.E0 - ref.E0) <= 1e-10 * abs(ref.E0)
    np.testing.assert_allclose(got.occ, ref.occ, atol=1e-8)
    assert float((got.psi - ref.psi).abs().max()) <= 1e-8
    assert got.iterations == ref.iterations
    assert got.sigma_seconds_f64 == 0.0 and got.sigma_seconds_f32 == 0.0
    return got


def test_static_matches_workspace_entry_point_two_calls(pdg, oracle_mod):
    # first call: 705,432 states (FP64, 16 vectors: 96 MB of the array)
    a = _compare(pdg, 22, 11, 3, "f64")
    # second call, smaller: 48,620 states; also checked against dense diagonalisation
    bsm = _compare(pdg, 18, 9, 4, "f64")
    _, _, eps, V = inputs.c5_instance(18, 9, seed=4)
    e_dense = oracle_mod.dense_ground(18, 9, eps, V)[0] if math.comb(18, 9) <= 12870 else None
    if e_dense is not None:
        assert abs(bsm.E0 - e_dense) <= 1e-10 * abs(e_dense)
    assert a.E0 != bsm.E0


def test_static_mixed_precision_and_small_after_large(pdg, oracle_mod):
    _compare(pdg, 24, 12, 5, "f32")          # 2.7e6 states, mixed precision, 16 vectors
    _, _, eps, V = inputs.c5_instance(14, 7, seed=6)
    b = pdg.Basis(14, 7, store_states=False)
    got = pdg.lanczos_ground_static(b, eps, V, krylov=16, tol=1e-10, start="random", seed=6)
    e0 = oracle_mod.dense_ground(14, 7, eps, V)[0]
    assert got.converged and abs(got.E0 - e0) <= 1e-10 * abs(e0)


def test_static_rejects_too_large(pdg):
    om, n = 26, 13                     # 1.04e7 states: FP64 with 16 vectors needs 1.5 GB
    _, _, eps, V = inputs.c5_instance(om, n, seed=0)
    b = pdg.Basis(om, n, store_states=False)
    with pytest.raises(pdg.PairDiagError) as ei:
        pdg.lanczos_ground_static(b, eps, V, krylov=16, tol=1e-10, start="random", want_psi=False)
    assert ei.value.status == pdg.PD_ERANGE
