"""GPU checks of the warm-start pieces: BF16 matrix-core layers and their
gradients against the FP64 oracle network, Adam, the product-state expansion
against the oracle, and a trained network that saves Lanczos products."""
import math

import numpy as np
import pytest

from paper_2001_01978_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2001_01978_amd import pairdiag, warm
    pairdiag.load()
    return torch, pairdiag, warm


def _bf16(a):
    """Round to BF16 (nearest even) and back, as the kernels stage operands."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("omega,batch,hidden", [(8, 37, 40), (24, 256, 256), (13, 100, 70)])
def test_forward_matches_oracle(mods, oracle_mod, omega, batch, hidden):
    torch, pdg, warm = mods
    net = warm.WarmNet(omega, hidden=hidden, seed=omega)
    # non-zero biases so their path is exercised
    p = net.params.cpu().numpy()
    p += np.random.default_rng(1).normal(0, 0.05, p.size).astype(np.float32)
    net.params = torch.tensor(p, device="cuda")
    X = np.random.default_rng(2).normal(size=(batch, warm.n_features(omega))).astype(np.float32)
    logits, z1 = net.forward_first_layer(torch.tensor(X, device="cuda"))
    got = logits.cpu().numpy().astype(np.float64)
    want, _ = oracle_mod.mlp_forward(net.param_arrays(), X.astype(np.float64))
    # three BF16 layers (operands rounded to 8-bit mantissas) against FP64:
    # every logit within 1e-2 of the largest one
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < 1e-2, err
    # The first layer's rounding model, element by element: operands rounded to
    # BF16 (their products are exact in FP32), sums accumulated in FP32.  With
    # K = in terms, any FP32 summation order stays within (K + 1) 2^-24 of the
    # sum of magnitudes; the FP64 sum of the rounded operands is the reference.
    W1, b1 = [np.asarray(a, np.float64) for a in net.param_arrays()[:2]]
    ref = _bf16(X) @ _bf16(W1) + b1
    mag = np.abs(_bf16(X)) @ np.abs(_bf16(W1)) + np.abs(b1)
    K = X.shape[1]
    z1 = z1.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(z1 - ref) <= (K + 1) * 2.0 ** -24 * mag), np.abs(z1 - ref).max()
    assert np.abs(z1 - ref).max() <= 1e-5 * np.abs(ref).max()


def test_gradients_match_oracle(mods, oracle_mod):
    torch, pdg, warm = mods
    omega, batch = 10, 64
    net = warm.WarmNet(omega, hidden=48, seed=3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(batch, warm.n_features(omega))).astype(np.float32)
    T = rng.uniform(0, 1, (batch, omega)).astype(np.float32)
    g, loss = net.gradients(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"))
    params = net.param_arrays()
    out, cache = oracle_mod.mlp_forward(params, X.astype(np.float64))
    l64, dout = oracle_mod.mlp_loss(out, T)
    want = np.concatenate([a.reshape(-1) for a in oracle_mod.mlp_backward(params, cache, dout)])
    got = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - l64) <= 1e-2 * abs(l64)
    # element by element, per parameter block (W1, b1, W2, b2, W3, b3): within
    # 1e-2 of the block's largest FP64 gradient
    o = 0
    for name, a in zip(["W1", "b1", "W2", "b2", "W3", "b3"], params):
        w = want[o:o + a.size]
        e = np.abs(got[o:o + a.size] - w).max() / np.abs(w).max()
        assert e < 1e-2, (name, e)
        o += a.size


def test_adam_matches_formula(mods):
    torch, pdg, warm = mods
    net = warm.WarmNet(6, hidden=8, seed=0)
    p0 = net.params.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0.copy()
    for step in range(1, 4):
        g = rng.normal(size=p0.size).astype(np.float32)
        net.adam(torch.tensor(g, device="cuda"), lr=1e-2)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        p -= 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    assert np.allclose(net.params.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("om,n", [(10, 4), (14, 7), (16, 8)])
def test_warm_expansion_vs_oracle(mods, oracle_mod, om, n):
    torch, pdg, warm = mods
    lo = np.random.default_rng(om).normal(0, 2, om).astype(np.float32)
    b = pdg.Basis(om, n, store_states=False)
    x0 = b.warm_start(torch.tensor(lo)).cpu().numpy()
    assert np.all(x0 > 0) and x0.max() <= 1.0 + 1e-15
    want = oracle_mod.pbcs_vector(om, n, lo.astype(np.float64))
    assert np.allclose(x0 / np.linalg.norm(x0), want, rtol=1e-12, atol=1e-15)


def test_constant_logits_give_degenerate_shell_ground_state(mods):
    torch, pdg, warm = mods
    om, n, g = 12, 5, 0.4
    eps = np.full(om, 0.75)
    V = np.full((om, om), -g)
    b = pdg.Basis(om, n, store_states=False)
    x0 = b.warm_start(torch.full((om,), 0.3))
    r = pdg.lanczos_ground(b, eps, V, x0=x0, krylov=10, tol=1e-12)
    assert r.iterations == 1 and r.converged
    assert math.isclose(r.E0, 2 * n * 0.75 - g * n * (om - n + 1), rel_tol=1e-14)


def test_features_canonical_order(mods):
    torch, pdg, warm = mods
    om, n, eps, V = inputs.family3_instance(5, omega=12, n=5)
    perm = np.random.default_rng(0).permutation(om)
    x1, p1 = warm.features(om, eps, V)
    x2, p2 = warm.features(om, eps[perm], V[np.ix_(perm, perm)])
    assert np.array_equal(x1, x2)
    assert np.array_equal(perm[p2], p1)


def test_trained_network_saves_products(mods):
    """Train on 512 GPU-labelled Omega=14 instances; on held-out instances the
    warm start needs fewer products than the random start, same E0."""
    torch, pdg, warm = mods
    om, n = 14, 7
    train = [inputs.family3_instance(s, omega=om, n=n) for s in range(512)]
    X, T, _ = warm.labels(train, tol=1e-8, krylov=16)
    net = warm.WarmNet(om, hidden=128, seed=1)
    hist = net.train(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"), epochs=120, batch=128, lr=2e-3)
    assert hist[-1] < 0.3 * hist[0]
    b = pdg.Basis(om, n, store_states=False)
    its_w, its_r = [], []
    for s in range(10 ** 6, 10 ** 6 + 16):
        _, _, eps, V = inputs.family3_instance(s, omega=om, n=n)
        rw = warm.solve(b, eps, V, net, krylov=12, tol=1e-10, want_psi=False)
        rr = warm.solve(b, eps, V, None, krylov=12, tol=1e-10, want_psi=False, seed=s)
        assert rw.converged and rr.converged
        assert abs(rw.E0 - rr.E0) <= 1e-10 * abs(rr.E0)
        its_w.append(rw.iterations)
        its_r.append(rr.iterations)
    assert np.mean(its_w) < np.mean(its_r), (np.mean(its_w), np.mean(its_r))
