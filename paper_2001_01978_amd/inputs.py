"""Seeded synthetic instances for the pairing Hamiltonian (shared by the GPU
path's tests/bench and by the oracle's tests).

This module holds random-number generation and instance recipes only; none of
the method's arithmetic lives here.  The coupling returned is the paper's V of
Eq. hamiltonian2 (V_ij = -G_ij, G > 0 attractive), so every instance below has
V_ij < 0.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used counter-style: draw k of stream `seed` is
mix(seed + (k + 1) * 0x9E3779B97F4A7C15), and a uniform double in [0, 1) is
(draw >> 11) * 2^-53.

Per-instance draw order: (omega, n when random), then the omega eps draws,
then u_ij for i <= j in row-major order (mirrored to j < i).

The paper's own workloads use eps_i = i (integers from 1) and constant G
(Sec. 5); the random families widen that to orbit-dependent couplings.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of SplitMix64 stream `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from draws start .. start+count-1."""
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, start, count) - 1.0


class _Stream:
    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def take(self, count: int) -> np.ndarray:
        u = uniform01(self.seed, self.pos, count)
        self.pos += count
        return u


def _sym_from_upper(omega: int, upper: np.ndarray) -> np.ndarray:
    m = np.zeros((omega, omega))
    iu = np.triu_indices(omega)
    m[iu] = upper
    m = m + np.triu(m, 1).T
    return m


def random_coupling(stream: _Stream, omega: int, g0: float, spread: float) -> np.ndarray:
    """G_ij = g0 * (1 + spread * u_ij), u uniform [-1, 1), symmetric; returns V = -G."""
    u = 2.0 * stream.take(omega * (omega + 1) // 2) - 1.0
    g = _sym_from_upper(omega, g0 * (1.0 + spread * u))
    return -g


def equal_spacing(omega: int, g: float, float_g: bool = False):
    """Paper workload: eps_i = i (i = 1..omega), constant V_ij = -g.

    float_g=True rounds g to IEEE single first, which is how the paper's
    Fortran literal entered its runs (it reproduces the paper's tables)."""
    gg = float(np.float32(g)) if float_g else float(g)
    eps = np.arange(1, omega + 1, dtype=np.float64)
    V = np.full((omega, omega), -gg)
    return eps, V


def c1_instance(seed: int):
    """Omega=16, n=8: eps = 10*sort(U[0,1)^16), G_ij = 0.3(1 + 0.2u)."""
    st = _Stream(seed)
    eps = 10.0 * np.sort(st.take(16))
    V = random_coupling(st, 16, 0.3, 0.2)
    return 16, 8, eps, V


def c2b_instance(seed: int):
    """Omega=28, n=14: eps ~ U[0,14), G_ij = 0.4(1 + 0.3u)."""
    st = _Stream(seed)
    eps = 14.0 * st.take(28)
    V = random_coupling(st, 28, 0.4, 0.3)
    return 28, 14, eps, V


def c2a_instance():
    """Omega=28, n=14: eps_i = i, constant G = 0.4 (Richardson-checkable)."""
    eps, V = equal_spacing(28, 0.4)
    return 28, 14, eps, V


def family3_instance(seed: int, omega: int | None = None, n: int | None = None):
    """Batched family: omega ~ U{10..24}, n ~ U{ceil(omega/4)..floor(omega/2)},
    eps ~ U[0, omega), G0 ~ U[0.1, 0.6), G_ij = G0(1 + 0.2u).
    Fixing omega (and n) skips those draws (used for the warm-start family)."""
    st = _Stream(seed)
    if omega is None:
        omega = 10 + int(st.take(1)[0] * 15)
    if n is None:
        lo, hi = math.ceil(omega / 4), omega // 2
        n = lo + int(st.take(1)[0] * (hi - lo + 1))
    eps = omega * st.take(omega)
    g0 = 0.1 + 0.5 * st.take(1)[0]
    V = random_coupling(st, omega, g0, 0.2)
    return omega, n, eps, V


def c5_instance(omega: int, n: int, seed: int = 0):
    """Large family: eps ~ U[0, omega), G_ij = 0.3(1 + 0.2u)."""
    st = _Stream(seed)
    eps = omega * st.take(omega)
    V = random_coupling(st, omega, 0.3, 0.2)
    return omega, n, eps, V


def random_vector(seed: int, dim: int) -> np.ndarray:
    """The RANDOM Lanczos start: x_k = 2*u_k - 1 with u_k draw k of stream seed."""
    return uniform_pm1(seed, 0, dim)


def dyadic_vector(seed: int, dim: int, bits: int = 8) -> np.ndarray:
    """Integers in [-2^bits, 2^bits) as doubles: products and sums stay exact."""
    u = uniform01(seed, 0, dim)
    return np.floor(u * 2.0 ** (bits + 1)) - 2.0 ** bits


def dyadic_instance(omega: int, n: int, seed: int):
    """eps and V on a coarse dyadic grid (multiples of 1/8 within +-4), so every
    sigma product and partial sum is exact in FP64 and the result is order-free."""
    st = _Stream(seed)
    eps = np.floor(st.take(omega) * 32.0) / 8.0
    upper = -np.floor(st.take(omega * (omega + 1) // 2) * 32.0) / 8.0
    V = _sym_from_upper(omega, upper)
    return omega, n, eps, V
