"""Learned warm start: a small network predicts the ground-state occupations
of a pairing instance; their pair amplitudes give a number-projected product
start vector for the Lanczos iteration.

Every computation runs in libpairdiag.so (BF16 matrix-core layers, loss,
backward, Adam, start-vector expansion, Lanczos); this module builds input
features, batches, and drives training.

Features.  The Hamiltonian is invariant under a relabelling of the orbits
(the same permutation applied to eps and to both indices of V gives the same
spectrum and permuted occupations), so instances are put in a canonical
order first: orbits sorted by eps.  The input is then (eps_sorted / omega,
(G_sorted upper triangle incl. diagonal - 0.35) / 0.15) with G = -V: omega +
omega(omega+1)/2 numbers (24 + 300 = 324 at omega = 24).  The outputs are
one logit per sorted orbit, mapped back to the caller's orbit order.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import pairdiag as pdg

G_CENTER, G_SCALE = 0.35, 0.15


def n_features(omega: int) -> int:
    return omega + omega * (omega + 1) // 2


def features(omega: int, eps, V):
    """(x, perm): canonical features and the sorting permutation of the orbits."""
    eps = np.asarray(eps, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    perm = np.argsort(eps, kind="stable")
    es = eps[perm]
    G = -V[np.ix_(perm, perm)]
    iu = np.triu_indices(omega)
    x = np.concatenate([es / omega, (G[iu] - G_CENTER) / G_SCALE])
    return x.astype(np.float32), perm


def unsort(values_sorted, perm):
    out = np.empty_like(values_sorted)
    out[perm] = values_sorted
    return out


class WarmNet:
    """in -> hidden -> hidden -> omega network on libpairdiag's kernels."""

    def __init__(self, omega: int, hidden: int = 256, seed: int = 0, device="cuda"):
        import torch
        self.omega = omega
        self.shape = pdg.MlpShape(n_features(omega), hidden, hidden, omega)
        self.device = device
        L = pdg.load()
        self.nparams = int(L.pd_mlp_param_count(ctypes.byref(self.shape)))
        rng = np.random.default_rng(seed)
        parts = []
        for a, b in [(self.shape.inp, hidden), (hidden, hidden), (hidden, omega)]:
            lim = math.sqrt(6.0 / (a + b))          # Glorot uniform
            parts += [rng.uniform(-lim, lim, a * b), np.zeros(b)]
        flat = np.concatenate(parts).astype(np.float32)
        assert flat.size == self.nparams
        self.params = torch.tensor(flat, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    # ---------------------------------------------------------------- (de)serialisation
    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), omega=self.omega, hidden=self.shape.h1)

    @classmethod
    def load(cls, path, device="cuda"):
        import torch
        d = np.load(path, allow_pickle=False)
        net = cls(int(d["omega"]), int(d["hidden"]), device=device)
        net.params = torch.tensor(d["params"], device=device)
        return net

    def param_arrays(self):
        """[W1, b1, W2, b2, W3, b3] as float64 numpy arrays (W as in x out)."""
        p = self.params.cpu().numpy().astype(np.float64)
        s = self.shape
        out, o = [], 0
        for a, b in [(s.inp, s.h1), (s.h1, s.h2), (s.h2, s.out)]:
            out.append(p[o:o + a * b].reshape(a, b))
            o += a * b
            out.append(p[o:o + b])
            o += b
        return out

    # ---------------------------------------------------------------- kernels
    def _work(self, batch):
        nb = pdg.load().pd_mlp_workspace_bytes(ctypes.byref(self.shape), batch)
        return pdg.device_buffer(nb, self.device), nb

    def forward(self, X):
        """X: (B, in) float32 device tensor -> logits (B, omega)."""
        import torch
        B = X.shape[0]
        (buf, off), nb = self._work(B)
        out = torch.empty(B, self.omega, dtype=torch.float32, device=self.device)
        pdg._check(pdg.load().pd_mlp_forward(ctypes.byref(self.shape), pdg._dptr(self.params), pdg._dptr(X), B,
                                             ctypes.c_void_p(buf.data_ptr() + off), nb, pdg._dptr(out),
                                             pdg._stream(None)))
        return out

    def forward_first_layer(self, X):
        """Logits, and the first layer's pre-activations Z1 = X W1 + b1 (B x h1)
        that pd_mlp_forward leaves at the start of its workspace."""
        import torch
        B = X.shape[0]
        (buf, off), nb = self._work(B)
        out = torch.empty(B, self.omega, dtype=torch.float32, device=self.device)
        pdg._check(pdg.load().pd_mlp_forward(ctypes.byref(self.shape), pdg._dptr(self.params), pdg._dptr(X), B,
                                             ctypes.c_void_p(buf.data_ptr() + off), nb, pdg._dptr(out),
                                             pdg._stream(None)))
        z1 = buf[off: off + 4 * B * self.shape.h1].view(torch.float32).reshape(B, self.shape.h1).clone()
        return out, z1

    def gradients(self, X, T):
        """(grads, loss) of the mean squared error of sigmoid(logits) against T."""
        import torch
        B = X.shape[0]
        (buf, off), nb = self._work(B)
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        pdg._check(pdg.load().pd_mlp_backward(ctypes.byref(self.shape), pdg._dptr(self.params), pdg._dptr(X),
                                              pdg._dptr(T), B, ctypes.c_void_p(buf.data_ptr() + off), nb,
                                              pdg._dptr(g), pdg._dptr(loss), pdg._stream(None)))
        return g, loss

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        pdg._check(pdg.load().pd_mlp_adam(self.nparams, pdg._dptr(self.params), pdg._dptr(g), pdg._dptr(self.m),
                                          pdg._dptr(self.v), self.step, lr, b1, b2, eps, pdg._stream(None)))

    def train(self, X, T, epochs=200, batch=256, lr=1e-3, seed=0, log=None):
        """Minibatch Adam over (X, T) (device tensors); returns the loss history per epoch."""
        import torch
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        hist = []
        for ep in range(epochs):
            idx = torch.tensor(rng.permutation(n), device=self.device)
            tot = 0.0
            nb = 0
            for s in range(0, n - batch + 1, batch):
                sel = idx[s:s + batch]
                g, loss = self.gradients(X[sel].contiguous(), T[sel].contiguous())
                self.adam(g, lr=lr)
                tot += float(loss.item())
                nb += 1
            hist.append(tot / max(nb, 1))
            if log and (ep % 20 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {hist[-1]:.3e}")
        return hist

    # ---------------------------------------------------------------- use
    def logits(self, omega, eps, V):
        import torch
        x, perm = features(omega, eps, V)
        lo = self.forward(torch.tensor(x[None, :], device=self.device))[0].cpu().numpy()
        return unsort(lo, perm)


def solve(basis: pdg.Basis, eps, V, net: WarmNet | None, fallback=True, **kw):
    """Ground state from the warm start (with the RANDOM fallback), or from the
    RANDOM start when net is None."""
    import torch
    if net is None:
        return pdg.lanczos_ground(basis, eps, V, start="random", **kw)
    lo = net.logits(basis.omega, eps, V)
    x0 = basis.warm_start(torch.tensor(lo, dtype=torch.float32))
    return pdg.lanczos_ground(basis, eps, V, x0=x0, fallback=fallback, **kw)


def labels(instances, tol=1e-8, krylov=20):
    """Half occupations <N_i>/2 (canonical orbit order) from the batched GPU solver."""
    r = pdg.lanczos_ground_batched(instances, krylov=krylov, tol=tol)
    X, T = [], []
    for (om, n, eps, V), occ in zip(instances, r.occ):
        x, perm = features(om, eps, V)
        X.append(x)
        T.append((occ[perm] / 2.0).astype(np.float32))
    return np.stack(X), np.stack(T), r


def labels_single(instances, tol=1e-4, krylov=16, precision="f32", log=None):
    """Half occupations from the single-instance solver (for spaces beyond the
    batched kernel), canonical orbit order."""
    X, T = [], []
    basis = None
    for q, (om, n, eps, V) in enumerate(instances):
        if basis is None or (basis.omega, basis.n) != (om, n):
            basis = pdg.Basis(om, n, store_states=False)
        r = pdg.lanczos_ground(basis, eps, V, krylov=krylov, tol=tol, start="hf", precision=precision,
                               want_psi=False)
        x, perm = features(om, eps, V)
        X.append(x)
        T.append((r.occ[perm] / 2.0).astype(np.float32))
        if log:
            log(f"label {q + 1}/{len(instances)}: products {r.iterations}, rho {r.residual:.1e}, {r.seconds:.1f} s")
    return np.stack(X), np.stack(T)


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
