"""Thin Python binding of libpairdiag.so (include/pairdiag.h).

Argument marshalling only: device memory comes from torch tensors, streams
from torch.cuda, and every computation runs in the HIP library.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpairdiag.so")

PD_OK, PD_EINVAL, PD_ERANGE, PD_ENOMEM, PD_EDEVICE, PD_ENOCONV = range(6)
PD_F64, PD_F32 = 0, 1
PD_TRUNC_BITMAP, PD_TRUNC_BSEARCH = 0, 1
START = {"e1": 0, "hf": 1, "random": 2, "user": 3}


class PairDiagError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_STATUS = {0: "PD_OK", 1: "PD_EINVAL", 2: "PD_ERANGE", 3: "PD_ENOMEM", 4: "PD_EDEVICE", 5: "PD_ENOCONV"}


class LanczosOpts(ctypes.Structure):
    _fields_ = [("krylov", ctypes.c_int), ("tol", ctypes.c_double), ("max_restarts", ctypes.c_int),
                ("mode", ctypes.c_int), ("start", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("fallback", ctypes.c_int), ("precision", ctypes.c_int), ("verbose", ctypes.c_int)]


class LanczosInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("iterations_f32", ctypes.c_int), ("restarts", ctypes.c_int),
                ("converged", ctypes.c_int), ("residual", ctypes.c_double), ("monopole_min", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sigma_seconds_f64", ctypes.c_double),
                ("sigma_seconds_f32", ctypes.c_double), ("fallback_used", ctypes.c_int),
                ("reorth_second_passes", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("grid", ctypes.c_int), ("tuned", ctypes.c_int), ("teams", ctypes.c_int),
                ("team_size", ctypes.c_int), ("large", ctypes.c_int), ("converged", ctypes.c_int),
                ("total_iterations", ctypes.c_longlong), ("tune_seconds", ctypes.c_double),
                ("kernel_seconds", ctypes.c_double), ("seconds", ctypes.c_double)]


class TruncInfo(ctypes.Structure):
    _fields_ = [("full_dim", ctypes.c_int64), ("limit", ctypes.c_int64), ("kept", ctypes.c_int64),
                ("bins", ctypes.c_int64), ("cut_bin", ctypes.c_int64), ("dmin", ctypes.c_double),
                ("dmax", ctypes.c_double), ("scale", ctypes.c_double), ("cutoff", ctypes.c_double)]


class ScfOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("tol", ctypes.c_double), ("mixing", ctypes.c_double),
                ("reuse_psi", ctypes.c_int)]


class ScfInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("products", ctypes.c_int),
                ("products_first", ctypes.c_int), ("lanczos_converged", ctypes.c_int), ("change", ctypes.c_double),
                ("last_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class MlpShape(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_int), ("h1", ctypes.c_int), ("h2", ctypes.c_int), ("out", ctypes.c_int)]


# name -> (restype, argtypes); the full exported surface of include/pairdiag.h
P, I, I64, U64, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "pd_version": (ctypes.c_char_p, []),
    "pd_status_str": (ctypes.c_char_p, [I]),
    "pd_last_error": (ctypes.c_char_p, []),
    "pd_basis_bytes": (SZ, [I, I, I]),
    "pd_dimension": (I64, [I, I]),
    "pd_basis_create": (I, [I, I, I, P, SZ, P, ctypes.POINTER(P)]),
    "pd_basis_destroy": (None, [P]),
    "pd_basis_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I64)]),
    "pd_basis_states": (P, [P]),
    "pd_basis_rank": (I, [P, P, I64, P, P]),
    "pd_basis_unrank": (I, [P, P, I64, P, P]),
    "pd_sigma": (I, [P, P, P, I, P, P, P]),
    "pd_trunc_select_bytes": (SZ, [I, I, I64]),
    "pd_trunc_select": (I, [I, I, P, P, I64, I64, P, SZ, ctypes.POINTER(TruncInfo), P]),
    "pd_basis_truncated_bytes": (SZ, [I, I, ctypes.POINTER(TruncInfo)]),
    "pd_basis_create_truncated": (I, [I, I, P, P, ctypes.POINTER(TruncInfo), I, P, SZ, P, ctypes.POINTER(P)]),
    "pd_basis_kept_ranks": (I, [P, P, P]),
    "pd_basis_truncation": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I64)]),
    "pd_lanczos_default_opts": (None, [ctypes.POINTER(LanczosOpts)]),
    "pd_lanczos_workspace_bytes": (SZ, [P, ctypes.POINTER(LanczosOpts)]),
    "pd_lanczos_ground": (I, [P, P, P, ctypes.POINTER(LanczosOpts), P, SZ, P, ctypes.POINTER(D), P, P,
                              ctypes.POINTER(LanczosInfo), P]),
    "pd_lanczos_eigs_workspace_bytes": (SZ, [P, I, ctypes.POINTER(LanczosOpts)]),
    "pd_lanczos_eigs": (I, [P, P, P, I, ctypes.POINTER(LanczosOpts), P, SZ, P, P, P, P, ctypes.POINTER(LanczosInfo),
                            P]),
    "pd_scf_workspace_bytes": (SZ, [P, ctypes.POINTER(LanczosOpts)]),
    "pd_scf_ground": (I, [P, P, P, P, ctypes.POINTER(ScfOpts), ctypes.POINTER(LanczosOpts), P, SZ, P, P,
                          ctypes.POINTER(D), P, ctypes.POINTER(ScfInfo), P]),
    "pd_occupations_workspace_bytes": (SZ, [P]),
    "pd_occupations": (I, [P, P, P, SZ, P, P]),
    "pd_tridiag_lowest": (I, [I, P, P, ctypes.POINTER(D), P]),
    "pd_warm_start": (I, [P, P, P, P]),
    "pd_mlp_param_count": (SZ, [ctypes.POINTER(MlpShape)]),
    "pd_mlp_workspace_bytes": (SZ, [ctypes.POINTER(MlpShape), I]),
    "pd_mlp_forward": (I, [ctypes.POINTER(MlpShape), P, P, I, P, SZ, P, P]),
    "pd_mlp_backward": (I, [ctypes.POINTER(MlpShape), P, P, P, I, P, SZ, P, P, P]),
    "pd_mlp_adam": (I, [I64, P, P, P, P, I, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, ctypes.c_float, P]),
    "pd_odd_workspace_bytes": (SZ, [I, I, I, I, ctypes.POINTER(LanczosOpts)]),
    "pd_lanczos_ground_odd": (I, [I, I, P, P, I, I, ctypes.POINTER(LanczosOpts), P, SZ, ctypes.POINTER(D),
                                  ctypes.POINTER(I), P, P, ctypes.POINTER(LanczosInfo), P]),
    "pd_batched_workspace_bytes": (SZ, [I, P, P, ctypes.POINTER(LanczosOpts)]),
    "pd_lanczos_ground_batched": (I, [I, P, P, P, P, ctypes.POINTER(LanczosOpts), I, P, SZ, P, P,
                                      ctypes.POINTER(LanczosInfo), ctypes.POINTER(BatchInfo), P]),
    "pd_lanczos_ground_static": (I, [P, P, P, ctypes.POINTER(LanczosOpts), P, ctypes.POINTER(D), P, P,
                                     ctypes.POINTER(LanczosInfo), P]),
    "pd_stream_probe_bytes": (I64, [I, I64]),
    "pd_sigma_launch_shape": (I, [I, I, I, ctypes.POINTER(I), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "pd_stream_probe": (I, [I, P, P, P, I64, P]),
}

_lib = None


def load():
    """Loads libpairdiag.so (raises if it was not built).

    torch is imported first: the library's HIP runtime dependency
    (libamdhip64.so.7) then resolves to the runtime torch already loaded, so
    the process holds one HIP runtime that both use."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see docstring)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2001_01978_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(status: int, allow=()):
    if status != PD_OK and status not in allow:
        raise PairDiagError(status, load().pd_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _host_f64(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _hp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def device_buffer(nbytes: int, device="cuda"):
    """Caller-owned device memory for the library (256-byte aligned)."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, off


PROBE = {"read": 0, "copy": 1, "triad": 2, "write": 3}
PD_PROBE_NONTEMPORAL = 16


def stream_probe(kind: str, a, b, c, nontemporal=False, stream=None) -> int:
    """One launch of the library's streaming kernel `kind` over float32 device
    tensors of equal length (pd_stream_probe); returns the bytes it moves.
    a is unused by 'write', b is used by 'triad' only (None allowed)."""
    L = load()
    k = PROBE[kind] | (PD_PROBE_NONTEMPORAL if nontemporal else 0)
    n = c.numel()
    _check(L.pd_stream_probe(k, _dptr(a) if a is not None else None, _dptr(b) if b is not None else None, _dptr(c),
                             n, _stream(stream)))
    return int(L.pd_stream_probe_bytes(k, n))


def sigma_launch_shape(omega: int, n: int, dtype="f64"):
    """(threads per workgroup, dynamic LDS bytes, LDS limit bytes) of pd_sigma
    on the space (omega, n) (pd_sigma_launch_shape; host only)."""
    L = load()
    t, lds, lim = I(), I64(), I64()
    dt = PD_F32 if dtype in ("f32", PD_F32) else PD_F64
    _check(L.pd_sigma_launch_shape(omega, n, dt, ctypes.byref(t), ctypes.byref(lds), ctypes.byref(lim)))
    return int(t.value), int(lds.value), int(lim.value)


def dimension(omega: int, n: int) -> int:
    return int(load().pd_dimension(omega, n))


def tridiag_lowest(alpha, beta):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    m = a.size
    y = np.empty(m)
    th = ctypes.c_double()
    rc = load().pd_tridiag_lowest(m, _hp(a), _hp(b) if b.size else None, ctypes.byref(th), _hp(y))
    if rc != 0:
        raise PairDiagError(PD_EINVAL, "tridiag_lowest failed")
    return th.value, y


def trunc_select(omega: int, n: int, eps, V, limit: int, bins: int = 10**8, device="cuda", stream=None) -> TruncInfo:
    """The truncation cut of Sec. 3.5 (pd_trunc_select)."""
    L = load()
    eps = _host_f64(eps, (omega,))
    V = _host_f64(V, (omega, omega))
    nb = L.pd_trunc_select_bytes(omega, n, bins)
    if nb == 0:
        raise PairDiagError(PD_EINVAL, f"invalid space omega={omega} n={n} or bins={bins}")
    buf, off = device_buffer(nb, device)
    info = TruncInfo()
    _check(L.pd_trunc_select(omega, n, _hp(eps), _hp(V), limit, bins, ctypes.c_void_p(buf.data_ptr() + off), nb,
                             ctypes.byref(info), _stream(stream)))
    del buf
    return info


class Basis:
    """Handle for the space of n pairs on omega orbits (pd_basis_create), or
    for a truncated part of it (Basis.truncated)."""

    truncated_space = False
    trunc_info = None

    @classmethod
    def truncated(cls, omega: int, n: int, eps, V, limit: int, bins: int = 10**8, index="bitmap", device="cuda",
                  stream=None, info: TruncInfo | None = None) -> "Basis":
        """The kept states of Sec. 3.5's truncation (pd_trunc_select +
        pd_basis_create_truncated).  index: 'bitmap' or 'bsearch'."""
        L = load()
        if info is None:
            info = trunc_select(omega, n, eps, V, limit, bins, device, stream)
        eps = _host_f64(eps, (omega,))
        V = _host_f64(V, (omega, omega))
        nbytes = L.pd_basis_truncated_bytes(omega, n, ctypes.byref(info))
        if nbytes == 0:
            raise PairDiagError(PD_EINVAL, "bad truncation info")
        self = cls.__new__(cls)
        self._buf, self._off = device_buffer(nbytes, device)
        h = ctypes.c_void_p()
        mode = {"bitmap": PD_TRUNC_BITMAP, "bsearch": PD_TRUNC_BSEARCH}[index]
        _check(L.pd_basis_create_truncated(omega, n, _hp(eps), _hp(V), ctypes.byref(info), mode,
                                           ctypes.c_void_p(self._buf.data_ptr() + self._off), nbytes,
                                           _stream(stream), ctypes.byref(h)))
        self._h = h
        self.omega, self.n = omega, n
        self.dim = int(info.kept)
        self.full_dim = int(info.full_dim)
        self.store_states = False
        self.device = device
        self.truncated_space = True
        self.trunc_info = info
        return self

    def kept_ranks(self, stream=None):
        """Full-space ranks of the kept states (device int64, ascending)."""
        torch = _torch()
        out = torch.empty(self.dim, dtype=torch.int64, device=self._buf.device)
        _check(load().pd_basis_kept_ranks(self._h, _dptr(out), _stream(stream)))
        return out

    def __init__(self, omega: int, n: int, store_states: bool = True, device="cuda", stream=None):
        L = load()
        nbytes = L.pd_basis_bytes(omega, n, int(store_states))
        if nbytes == 0:
            raise PairDiagError(PD_EINVAL, f"invalid space omega={omega} n={n}")
        self._buf, self._off = device_buffer(nbytes, device)
        h = ctypes.c_void_p()
        _check(L.pd_basis_create(omega, n, int(store_states), ctypes.c_void_p(self._buf.data_ptr() + self._off),
                                 nbytes, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.omega, self.n = omega, n
        self.dim = dimension(omega, n)
        self.store_states = store_states
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().pd_basis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def states(self):
        """Device view (int64 bit patterns) of the stored ascending state array."""
        if not self.store_states:
            raise RuntimeError("basis was created without stored states")
        torch = _torch()
        ptr = load().pd_basis_states(self._h)
        offset = ptr - self._buf.data_ptr()
        return self._buf[offset: offset + self.dim * 8].view(torch.int64)

    def rank(self, states, stream=None):
        torch = _torch()
        states = states.contiguous()
        out = torch.empty(states.numel(), dtype=torch.int64, device=states.device)
        _check(load().pd_basis_rank(self._h, _dptr(states), states.numel(), _dptr(out), _stream(stream)))
        return out

    def unrank(self, ranks, stream=None):
        torch = _torch()
        ranks = ranks.contiguous().to(torch.int64)
        out = torch.empty(ranks.numel(), dtype=torch.int64, device=ranks.device)
        _check(load().pd_basis_unrank(self._h, _dptr(ranks), ranks.numel(), _dptr(out), _stream(stream)))
        return out

    def sigma(self, eps, V, x, y=None, stream=None):
        """y = H x (pd_sigma); dtype from x (float64 or float32)."""
        torch = _torch()
        eps = _host_f64(eps, (self.omega,))
        V = _host_f64(V, (self.omega, self.omega))
        if x.dtype == torch.float64:
            dt = PD_F64
        elif x.dtype == torch.float32:
            dt = PD_F32
        else:
            raise TypeError("x must be float64 or float32")
        if x.numel() != self.dim or not x.is_contiguous():
            raise ValueError("x must be a contiguous vector of length dim")
        if y is None:
            y = torch.empty_like(x)
        _check(load().pd_sigma(self._h, _hp(eps), _hp(V), dt, _dptr(x), _dptr(y), _stream(stream)))
        return y

    def warm_start(self, logits, x0=None, stream=None):
        """Number-projected product start vector from per-orbit logits (pd_warm_start)."""
        torch = _torch()
        logits = logits.to(device=self._buf.device, dtype=torch.float32).contiguous()
        if logits.numel() != self.omega:
            raise ValueError("one logit per orbit")
        if x0 is None:
            x0 = torch.empty(self.dim, dtype=torch.float64, device=self._buf.device)
        _check(load().pd_warm_start(self._h, _dptr(logits), _dptr(x0), _stream(stream)))
        return x0

    def occupations(self, psi, stream=None):
        L = load()
        nb = L.pd_occupations_workspace_bytes(self._h)
        buf, off = device_buffer(nb, psi.device)
        occ = np.empty(self.omega)
        _check(L.pd_occupations(self._h, _dptr(psi), ctypes.c_void_p(buf.data_ptr() + off), nb, _hp(occ),
                                _stream(stream)))
        return occ


@dataclass
class GroundState:
    E0: float
    psi: object
    occ: np.ndarray
    iterations: int
    iterations_f32: int
    restarts: int
    converged: bool
    residual: float
    monopole_min: float
    seconds: float
    sigma_seconds_f64: float
    sigma_seconds_f32: float
    fallback_used: bool
    status: int
    reorth_second_passes: int = 0


def make_opts(krylov=50, tol=1e-10, max_restarts=1000, mode=0, start="e1", seed=0, precision="f64",
              verbose=False, fallback=False) -> LanczosOpts:
    o = LanczosOpts()
    load().pd_lanczos_default_opts(ctypes.byref(o))
    o.krylov, o.tol, o.max_restarts, o.mode = krylov, tol, max_restarts, mode
    o.start = START[start] if isinstance(start, str) else int(start)
    o.seed = seed
    o.precision = {"f32": PD_F32, "mixed": PD_F32, PD_F32: PD_F32, "f32_f64cols": 2, 2: 2}.get(precision, PD_F64)
    o.verbose = int(verbose)
    o.fallback = int(fallback)
    return o


def workspace_bytes(basis: Basis, **kw) -> int:
    o = make_opts(**kw)
    return int(load().pd_lanczos_workspace_bytes(basis.handle, ctypes.byref(o)))


def lanczos_ground(basis: Basis, eps, V, x0=None, want_psi=True, workspace=None, stream=None, **kw) -> GroundState:
    """Ground state by restarted Lanczos (pd_lanczos_ground)."""
    torch = _torch()
    L = load()
    if x0 is not None:
        kw["start"] = "user"
    o = make_opts(**kw)
    eps = _host_f64(eps, (basis.omega,))
    V = _host_f64(V, (basis.omega, basis.omega))
    nb = L.pd_lanczos_workspace_bytes(basis.handle, ctypes.byref(o))
    if nb == 0:
        raise PairDiagError(PD_EINVAL, "bad options")
    if workspace is None:
        buf, off = device_buffer(nb, basis.device)
    else:
        buf, off = workspace
    psi = torch.empty(basis.dim, dtype=torch.float64, device=basis.device) if want_psi else None
    occ = np.empty(basis.omega)
    e0 = ctypes.c_double()
    info = LanczosInfo()
    st = L.pd_lanczos_ground(basis.handle, _hp(eps), _hp(V), ctypes.byref(o),
                             ctypes.c_void_p(buf.data_ptr() + off), nb,
                             _dptr(x0) if x0 is not None else None, ctypes.byref(e0),
                             _dptr(psi) if psi is not None else None, _hp(occ), ctypes.byref(info),
                             _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    return GroundState(E0=e0.value, psi=psi, occ=occ, iterations=info.iterations,
                       iterations_f32=info.iterations_f32, restarts=info.restarts, converged=bool(info.converged),
                       residual=info.residual, monopole_min=info.monopole_min, seconds=info.seconds,
                       sigma_seconds_f64=info.sigma_seconds_f64, sigma_seconds_f32=info.sigma_seconds_f32,
                       fallback_used=bool(info.fallback_used), status=st,
                       reorth_second_passes=info.reorth_second_passes)


STATIC_SCRATCH_BYTES = 256 << 20


def lanczos_ground_static(basis: Basis, eps, V, x0=None, want_psi=True, stream=None, **kw) -> GroundState:
    """Ground state by restarted Lanczos in the library's static workspace
    (pd_lanczos_ground_static: no workspace argument, no allocation)."""
    torch = _torch()
    L = load()
    if x0 is not None:
        kw["start"] = "user"
    o = make_opts(**kw)
    eps = _host_f64(eps, (basis.omega,))
    V = _host_f64(V, (basis.omega, basis.omega))
    psi = torch.empty(basis.dim, dtype=torch.float64, device=basis.device) if want_psi else None
    occ = np.empty(basis.omega)
    e0 = ctypes.c_double()
    info = LanczosInfo()
    st = L.pd_lanczos_ground_static(basis.handle, _hp(eps), _hp(V), ctypes.byref(o),
                                    _dptr(x0) if x0 is not None else None, ctypes.byref(e0),
                                    _dptr(psi) if psi is not None else None, _hp(occ), ctypes.byref(info),
                                    _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    return GroundState(E0=e0.value, psi=psi, occ=occ, iterations=info.iterations,
                       iterations_f32=info.iterations_f32, restarts=info.restarts, converged=bool(info.converged),
                       residual=info.residual, monopole_min=info.monopole_min, seconds=info.seconds,
                       sigma_seconds_f64=info.sigma_seconds_f64, sigma_seconds_f32=info.sigma_seconds_f32,
                       fallback_used=bool(info.fallback_used), status=st,
                       reorth_second_passes=info.reorth_second_passes)


@dataclass
class Eigenpairs:
    E: np.ndarray
    psi: object
    occ: np.ndarray
    residuals: np.ndarray
    iterations: int
    iterations_f32: int
    restarts: int
    converged: bool
    seconds: float
    status: int


def lanczos_eigs(basis: Basis, eps, V, nev: int, want_psi=True, workspace=None, stream=None, **kw) -> Eigenpairs:
    """The nev lowest eigenpairs by thick-restart Lanczos (pd_lanczos_eigs)."""
    torch = _torch()
    L = load()
    kw.setdefault("start", "random")
    o = make_opts(**kw)
    eps = _host_f64(eps, (basis.omega,))
    V = _host_f64(V, (basis.omega, basis.omega))
    nb = L.pd_lanczos_eigs_workspace_bytes(basis.handle, nev, ctypes.byref(o))
    if nb == 0:
        raise PairDiagError(PD_EINVAL, "bad options")
    if workspace is None:
        buf, off = device_buffer(nb, basis.device)
    else:
        buf, off = workspace
    psi = torch.empty((nev, basis.dim), dtype=torch.float64, device=basis.device) if want_psi else None
    E = np.empty(nev)
    occ = np.empty((nev, basis.omega))
    res = np.empty(nev)
    info = LanczosInfo()
    st = L.pd_lanczos_eigs(basis.handle, _hp(eps), _hp(V), nev, ctypes.byref(o),
                           ctypes.c_void_p(buf.data_ptr() + off), nb, _hp(E),
                           _dptr(psi) if psi is not None else None, _hp(occ), _hp(res), ctypes.byref(info),
                           _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    return Eigenpairs(E=E, psi=psi, occ=occ, residuals=res, iterations=info.iterations,
                      iterations_f32=info.iterations_f32, restarts=info.restarts,
                      converged=bool(info.converged), seconds=info.seconds, status=st)


@dataclass
class ScfResult:
    eps: np.ndarray
    occ: np.ndarray
    E0: float
    psi: object
    info: dict
    status: int


def scf_ground(basis: Basis, eps0, W, V, mixing=0.5, tol=1e-10, max_iter=200, reuse_psi=True, want_psi=False,
               lanczos_tol=1e-12, workspace=None, stream=None, **kw) -> ScfResult:
    """Ground state inside a self-consistent loop with the mean field eps0 + W <N>/2 (pd_scf_ground).
    tol: on the field change; lanczos_tol: of every solve."""
    torch = _torch()
    L = load()
    o = make_opts(tol=lanczos_tol, **kw)
    so = ScfOpts(max_iter=max_iter, tol=tol, mixing=mixing, reuse_psi=int(reuse_psi))
    om = basis.omega
    eps0 = _host_f64(eps0, (om,))
    W = _host_f64(W, (om, om))
    V = _host_f64(V, (om, om))
    nb = L.pd_scf_workspace_bytes(basis.handle, ctypes.byref(o))
    if nb == 0:
        raise PairDiagError(PD_EINVAL, "bad options")
    if workspace is None:
        buf, off = device_buffer(nb, basis.device)
    else:
        buf, off = workspace
    psi = torch.empty(basis.dim, dtype=torch.float64, device=basis.device) if want_psi else None
    eps = np.empty(om)
    occ = np.empty(om)
    e0 = ctypes.c_double()
    info = ScfInfo()
    st = L.pd_scf_ground(basis.handle, _hp(eps0), _hp(W), _hp(V), ctypes.byref(so), ctypes.byref(o),
                         ctypes.c_void_p(buf.data_ptr() + off), nb, _hp(eps), _hp(occ), ctypes.byref(e0),
                         _dptr(psi) if psi is not None else None, ctypes.byref(info), _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    return ScfResult(eps=eps, occ=occ, E0=e0.value, psi=psi, info={k: getattr(info, k) for k, _ in ScfInfo._fields_},
                     status=st)


@dataclass
class BatchResult:
    E0: np.ndarray
    occ: list
    iterations: np.ndarray
    restarts: np.ndarray
    converged: np.ndarray
    residual: np.ndarray
    seconds: np.ndarray
    info: dict
    status: int


def _pack_batch(instances):
    om = np.array([int(i[0]) for i in instances], dtype=np.int32)
    n = np.array([int(i[1]) for i in instances], dtype=np.int32)
    eps = np.concatenate([np.ascontiguousarray(i[2], dtype=np.float64).reshape(-1) for i in instances])
    V = np.concatenate([np.ascontiguousarray(i[3], dtype=np.float64).reshape(-1) for i in instances])
    return om, n, eps, V


def batched_workspace_bytes(instances, krylov=20, **kw) -> int:
    om, n, _, _ = _pack_batch(instances)
    o = make_opts(krylov=krylov, **kw)
    return int(load().pd_batched_workspace_bytes(len(om), _hp(om), _hp(n), ctypes.byref(o)))


def lanczos_ground_batched(instances, krylov=20, tol=1e-10, max_restarts=1000, seed=0, block=0,
                           workspace=None, device="cuda", stream=None) -> BatchResult:
    """Ground states of many (omega, n, eps, V) instances in one persistent launch
    (pd_lanczos_ground_batched)."""
    L = load()
    om, n, eps, V = _pack_batch(instances)
    count = len(om)
    o = make_opts(krylov=krylov, tol=tol, max_restarts=max_restarts, seed=seed)
    nb = L.pd_batched_workspace_bytes(count, _hp(om), _hp(n), ctypes.byref(o))
    if nb == 0:
        raise PairDiagError(PD_EINVAL, L.pd_last_error().decode())
    if workspace is None:
        buf, off = device_buffer(nb, device)
    else:
        buf, off = workspace
    E0 = np.empty(count)
    occ = np.empty(int(om.sum()))
    infos = (LanczosInfo * count)()
    bi = BatchInfo()
    st = L.pd_lanczos_ground_batched(count, _hp(om), _hp(n), _hp(eps), _hp(V), ctypes.byref(o), block,
                                     ctypes.c_void_p(buf.data_ptr() + off), nb, _hp(E0), _hp(occ), infos,
                                     ctypes.byref(bi), _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    splits = np.cumsum(om)[:-1]
    return BatchResult(E0=E0, occ=np.split(occ, splits),
                       iterations=np.array([f.iterations for f in infos]),
                       restarts=np.array([f.restarts for f in infos]),
                       converged=np.array([bool(f.converged) for f in infos]),
                       residual=np.array([f.residual for f in infos]),
                       seconds=np.array([f.seconds for f in infos]),
                       info={k: getattr(bi, k) for k, _ in BatchInfo._fields_}, status=st)


ODD_ROUTE = {"auto": 0, "sequential": 1, "batched": 2}


@dataclass
class OddGroundState:
    E: float
    block: int
    E_blocks: np.ndarray
    occ: np.ndarray
    iterations: int
    iterations_f32: int
    restarts: int
    converged: bool
    residual: float
    monopole_min: float
    seconds: float
    reorth_second_passes: int
    status: int


def odd_workspace_bytes(omega: int, n: int, block=0, route="auto", **kw) -> int:
    o = make_opts(**kw)
    return int(load().pd_odd_workspace_bytes(omega, n, block, ODD_ROUTE[route], ctypes.byref(o)))


def lanczos_ground_odd(omega: int, n: int, eps, V, block=0, route="auto", workspace=None, device="cuda",
                       stream=None, **kw) -> OddGroundState:
    """Odd system of 2n+1 particles, blocking approximation (pd_lanczos_ground_odd).
    block: 1..omega solves that block, 0 all of them (the lowest is returned)."""
    L = load()
    o = make_opts(**kw)
    eps = _host_f64(eps, (omega,))
    V = _host_f64(V, (omega, omega))
    r = ODD_ROUTE[route]
    nb = L.pd_odd_workspace_bytes(omega, n, block, r, ctypes.byref(o))
    if nb == 0:
        raise PairDiagError(PD_EINVAL, L.pd_last_error().decode())
    if workspace is None:
        buf, off = device_buffer(nb, device)
    else:
        buf, off = workspace
    E = ctypes.c_double()
    b = ctypes.c_int()
    Eb = np.empty(omega)
    occ = np.empty(omega)
    info = LanczosInfo()
    st = L.pd_lanczos_ground_odd(omega, n, _hp(eps), _hp(V), block, r, ctypes.byref(o),
                                 ctypes.c_void_p(buf.data_ptr() + off), nb, ctypes.byref(E), ctypes.byref(b),
                                 _hp(Eb), _hp(occ), ctypes.byref(info), _stream(stream))
    _check(st, allow=(PD_ENOCONV,))
    return OddGroundState(E=E.value, block=b.value, E_blocks=Eb, occ=occ, iterations=info.iterations,
                          iterations_f32=info.iterations_f32, restarts=info.restarts,
                          converged=bool(info.converged), residual=info.residual,
                          monopole_min=info.monopole_min, seconds=info.seconds,
                          reorth_second_passes=info.reorth_second_passes, status=st)
