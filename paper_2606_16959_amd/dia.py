"""Binding of the general DIA-operator calls (``hs_dia_*``, ``hs_spme``,
``hs_estimate_timesteps``): the paper's single-propagator pipeline
(Alg. 2 SpME, the Section 3.1 step search, Alg. 3).  Argument marshalling
only; every step runs in libhamsim.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib, _marshal_terms, _state_args, _stream_ptr, dtype_code, HS_C128


class DiaOperator:
    """Owning wrapper of an ``hs_dia`` handle."""

    def __init__(self, handle):
        self._h = handle
        N, nd, dt = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
        _lib.check(_lib.load().hs_dia_info(self._h, N, nd, dt))
        self.N, self.n_diags, self.dtype_code = N.value, nd.value, dt.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.load().hs_dia_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def offsets(self) -> list:
        out = (ctypes.c_longlong * max(1, self.n_diags))()
        _lib.check(_lib.load().hs_dia_offsets(self._h, out, self.n_diags))
        return list(out)[: self.n_diags]

    def diagonal(self, j: int, start: int = 0, count=None, stream=None) -> np.ndarray:
        d = self.offsets[j]
        if count is None:
            count = self.N - abs(d) - start
        out = np.empty(count, dtype=np.complex128 if self.dtype_code == HS_C128 else np.complex64)
        _lib.check(_lib.load().hs_dia_copy_diagonal(self._h, j, int(start), int(count), out.ctypes.data,
                                                    _stream_ptr(stream)))
        return out

    def to_dict(self) -> dict:
        return {d: self.diagonal(j) for j, d in enumerate(self.offsets)}

    def maxabs(self, stream=None) -> float:
        v = ctypes.c_double()
        _lib.check(_lib.load().hs_dia_maxabs(self._h, _stream_ptr(stream), v))
        return v.value

    def __matmul__(self, other: "DiaOperator") -> "DiaOperator":
        return spgemm(self, other)

    def to_c64(self, stream=None) -> "DiaOperator":
        h = ctypes.c_void_p()
        _lib.check(_lib.load().hs_dia_to_c64(self._h, _stream_ptr(stream), ctypes.byref(h)))
        return DiaOperator(h)


def from_pauli(strings, coeffs, n, stream=None) -> DiaOperator:
    arr, ri, _keep = _marshal_terms(strings, coeffs, n)
    h = ctypes.c_void_p()
    _lib.check(_lib.load().hs_dia_from_pauli(n, len(ri), arr, ri.ctypes.data, _stream_ptr(stream),
                                             ctypes.byref(h)))
    return DiaOperator(h)


def from_dict(diags: dict, N: int, stream=None) -> DiaOperator:
    """Operator from {offset: complex128 array of N - |d| entries}."""
    offs = sorted(diags)
    arrs = [np.ascontiguousarray(np.asarray(diags[d], dtype=np.complex128)) for d in offs]
    for d, a in zip(offs, arrs):
        if a.size != N - abs(d):
            raise ValueError("diagonal length must be N - |d|")
    coff = (ctypes.c_longlong * len(offs))(*offs)
    ptrs = (ctypes.c_void_p * len(offs))(*[a.ctypes.data for a in arrs])
    h = ctypes.c_void_p()
    _lib.check(_lib.load().hs_dia_from_host(N, len(offs), coff, ptrs, _stream_ptr(stream), ctypes.byref(h)))
    return DiaOperator(h)


def spgemm(A: DiaOperator, B: DiaOperator, stream=None) -> DiaOperator:
    h = ctypes.c_void_p()
    _lib.check(_lib.load().hs_dia_spgemm(A.handle, B.handle, _stream_ptr(stream), ctypes.byref(h)))
    return DiaOperator(h)


def spme(H: DiaOperator, dt: float, tol: float = 1e-6, max_iter: int = 30, squarings: int = -1,
         stream=None):
    """(U, n_terms) with U ~ exp(-i H dt) by the truncated Taylor series with
    scaling and squaring (`squarings` -1: the library's rule; 0: none)."""
    h = ctypes.c_void_p()
    k = ctypes.c_int()
    _lib.check(_lib.load().hs_spme(H.handle, float(dt), float(tol), int(max_iter), int(squarings),
                                   _stream_ptr(stream), ctypes.byref(h), ctypes.byref(k)))
    return DiaOperator(h), k.value


def estimate_timesteps(H: DiaOperator, t: float, budget: int, tol: float = 1e-6, max_iter: int = 30,
                       stream=None) -> int:
    r = ctypes.c_int()
    _lib.check(_lib.load().hs_estimate_timesteps(H.handle, float(t), int(budget), float(tol), int(max_iter),
                                                 _stream_ptr(stream), ctypes.byref(r)))
    return r.value


def evolve(U: DiaOperator, psi, steps: int, stream=None):
    """psi <- U^steps psi (Alg. 3's loop), psi a device tensor [N] or [B, N]."""
    batch, N, code = _state_args(psi, U.N)
    if code != U.dtype_code:
        raise ValueError("state dtype differs from the operator's dtype")
    _lib.check(_lib.load().hs_dia_evolve(U.handle, ctypes.c_void_p(psi.data_ptr()), batch, int(steps),
                                         _stream_ptr(stream)))
    return psi


def simulate(strings, coeffs, n, t, psi, budget=None, steps=None, tol=1e-6, max_iter=30, dtype="c128",
             stream=None):
    """Alg. 3 end to end: steps = EstimateTimesteps(H, t, budget) unless given,
    U = SpME(H, t / steps), psi <- U^steps psi.  Returns (steps, n_terms, n_diags)."""
    H = from_pauli(strings, coeffs, n, stream=stream)
    if steps is None:
        steps = estimate_timesteps(H, t, budget, tol, max_iter, stream=stream)
    U, K = spme(H, t / steps, tol, max_iter, stream=stream)
    if dtype_code(dtype) != HS_C128:
        U64 = U.to_c64(stream=stream)
        U.close()
        U = U64
    evolve(U, psi, steps, stream=stream)
    nd = U.n_diags
    U.close()
    H.close()
    return steps, K, nd


def norm_bound(A: DiaOperator, stream=None) -> float:
    """nu(A): the sum of the per-diagonal largest entry moduli."""
    v = ctypes.c_double()
    _lib.check(_lib.load().hs_dia_norm_bound(A.handle, _stream_ptr(stream), ctypes.byref(v)))
    return v.value


def taylor_terms(H: DiaOperator, dt: float, tol: float = 1e-6, max_terms: int = 64, stream=None) -> int:
    """Smallest K with (|dt| nu(H))^(K+1) / (K+1)! < tol."""
    k = ctypes.c_int()
    _lib.check(_lib.load().hs_taylor_terms(H.handle, float(dt), float(tol), int(max_terms),
                                           _stream_ptr(stream), ctypes.byref(k)))
    return k.value


def taylor_evolve(H: DiaOperator, psi, dt: float, K: int, steps: int, stream=None):
    """psi <- p_K(-i dt H)^steps psi: the Taylor expansion fused into the state
    update by Horner's rule (no propagator is formed)."""
    batch, N, code = _state_args(psi, H.N)
    if code != H.dtype_code:
        raise ValueError("state dtype differs from the operator's dtype")
    _lib.check(_lib.load().hs_taylor_evolve(H.handle, ctypes.c_void_p(psi.data_ptr()), batch, float(dt),
                                            int(K), int(steps), _stream_ptr(stream)))
    return psi


def taylor_steps(H: DiaOperator, t: float, theta: float = 1.0, stream=None) -> int:
    """Smallest r with |t / r| nu(H) <= theta."""
    r = ctypes.c_int()
    _lib.check(_lib.load().hs_taylor_steps(H.handle, float(t), float(theta), _stream_ptr(stream),
                                           ctypes.byref(r)))
    return r.value


def taylor_simulate(strings, coeffs, n, t, psi, steps=None, tol=1e-6, theta=1.0, dtype="c128", stream=None):
    """H from Pauli strings, then r steps of the fused Taylor update with
    dt = t / r.  r defaults to the smallest with |dt| nu(H) <= theta.
    Returns (steps, K)."""
    H = from_pauli(strings, coeffs, n, stream=stream)
    if steps is None:
        steps = taylor_steps(H, t, theta, stream=stream)
    K = taylor_terms(H, t / steps, tol, stream=stream)
    if dtype_code(dtype) != HS_C128:
        H64 = H.to_c64(stream=stream)
        H.close()
        H = H64
    taylor_evolve(H, psi, t / steps, K, steps, stream=stream)
    H.close()
    return steps, K
