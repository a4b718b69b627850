"""MI355X (gfx950) library for diagonal-budgeted Trotterized Hamiltonian
simulation -- thin Python binding of the C ABI in ``include/hamsim.h``.

Every step of the computation runs in the HIP kernels of ``libhamsim.so``;
this module only marshals arguments.  PyTorch supplies device memory and
streams: states are ``torch`` tensors of dtype complex64 or complex128 on a
ROCm device, shaped ``[N]`` or ``[B, N]``.

    f = build_factors(strings, coeffs, n, t, steps, budget, dtype="c64")
    evolve(f, psi, steps)          # psi <- (U_F ... U_1)^steps psi, in place
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (HS_C64, HS_C128, HS_MERGE_DIAG, HS_NO_FUSE, HS_ORDER2, HS_ORDER4,  # noqa: F401
                   HS_RENORM, HamsimError)

__all__ = ["Factors", "plan", "build_factors", "evolve", "norm2", "fidelity", "fidelity_noalloc", "dia_spmv",
           "HamsimError", "dtype_code"]


def dtype_code(dtype) -> int:
    s = str(dtype)
    if s in ("c64", "complex64", "torch.complex64", "<class 'numpy.complex64'>") or dtype is np.complex64:
        return HS_C64
    if s in ("c128", "complex128", "torch.complex128", "<class 'numpy.complex128'>") or dtype is np.complex128:
        return HS_C128
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream_ptr(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _marshal_terms(strings, coeffs, n):
    strings = list(strings)
    enc = [s.encode("ascii") for s in strings]
    arr = (ctypes.c_char_p * len(enc))(*enc)
    c = np.asarray(coeffs)
    ri = np.zeros((len(strings), 2), dtype=np.float64)
    ri[:, 0] = np.real(c)
    ri[:, 1] = np.imag(c) if np.iscomplexobj(c) else 0.0
    return arr, ri, enc


class Factors:
    """Owning wrapper of an ``hs_factors`` handle."""

    def __init__(self, handle, built: bool):
        self._h = handle
        self.built = built
        lib = _lib.load()
        n, nf, nt, nd, dt_code = (ctypes.c_int() for _ in range(5))
        dt = ctypes.c_double()
        steps = ctypes.c_int()
        _lib.check(lib.hs_factors_info(self._h, n, nf, nt, nd, dt_code, dt, steps))
        self.n, self.n_factors, self.n_terms = n.value, nf.value, nt.value
        self.n_diag_terms, self.dtype_code = nd.value, dt_code.value
        self.dt, self.steps = dt.value, steps.value
        self.N = 1 << self.n

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.load().hs_free_factors(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> dict:
        lib = _lib.load()
        diag = (ctypes.c_int * max(1, self.n_diag_terms))()
        _lib.check(lib.hs_diag_terms(self._h, diag, self.n_diag_terms))
        out = {"diag_terms": list(diag)[: self.n_diag_terms], "factors": []}
        for k in range(self.n_factors):
            hd, ng, nd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            sm, nb = ctypes.c_ulonglong(), ctypes.c_size_t()
            _lib.check(lib.hs_factor_info(self._h, k, hd, ng, nd, sm, nb))
            terms = (ctypes.c_int * max(1, ng.value))()
            _lib.check(lib.hs_factor_terms(self._h, k, terms, ng.value))
            offs = (ctypes.c_longlong * nd.value)()
            _lib.check(lib.hs_factor_offsets(self._h, k, offs, nd.value))
            h = ctypes.c_double()
            _lib.check(lib.hs_factor_step(self._h, k, h))
            ps, pc = ctypes.c_int(), ctypes.c_int()
            _lib.check(lib.hs_factor_storage(self._h, k, ps, pc))
            out["factors"].append({"has_diag": bool(hd.value), "terms": list(terms)[: ng.value],
                                   "offsets": list(offs), "support_mask": sm.value,
                                   "bytes": nb.value, "dt": h.value,
                                   "storage": (ps.value, pc.value)})
        ln = ctypes.c_int()
        _lib.check(lib.hs_step_sequence(self._h, None, 0, ln))
        seq = (ctypes.c_int * max(1, ln.value))()
        _lib.check(lib.hs_step_sequence(self._h, seq, ln.value, ln))
        out["sequence"] = list(seq)[: ln.value]
        j = ctypes.c_int()
        _lib.check(lib.hs_step_joint(self._h, j))
        out["joint"] = j.value
        return out

    def copy_diagonal(self, k: int, j: int, offset: int, start: int = 0, count=None,
                      stream=None) -> np.ndarray:
        """Entries [start, start+count) of diagonal j of factor k (host copy)."""
        if count is None:
            count = self.N - abs(int(offset)) - start
        out = np.empty(count, dtype=np.complex128 if self.dtype_code == HS_C128 else np.complex64)
        _lib.check(_lib.load().hs_factor_copy_diagonal(self._h, k, j, int(start), int(count),
                                                       out.ctypes.data, _stream_ptr(stream)))
        return out

    def step_launches(self, batch: int = 1, fuse: bool = True, part: int = 0) -> list:
        """[(first, n_factors)] of the launches of one Trotter step: positions
        in the part's factor sequence (:meth:`part_sequence`)."""
        lib = _lib.load()
        n = ctypes.c_int()
        flags = 0 if fuse else HS_NO_FUSE
        _lib.check(lib.hs_step_launches(self._h, batch, flags, part, n, None, None, 0))
        first = (ctypes.c_int * max(1, n.value))()
        cnt = (ctypes.c_int * max(1, n.value))()
        _lib.check(lib.hs_step_launches(self._h, batch, flags, part, n, first, cnt, n.value))
        return [(first[i], cnt[i]) for i in range(n.value)]

    def part_sequence(self, part: int = 0, desc: dict | None = None) -> list:
        """Factor indices one step applies: part 0 a lone step, 1/2/3 the
        first/middle/last step of several (differ only with a joint factor)."""
        d = desc or self.describe()
        seq, j = d["sequence"], d["joint"]
        if j < 0 or part == 0:
            return list(seq)
        if part == 1:
            return seq[:-1] + [j]
        if part == 2:
            return seq[1:-1] + [j]
        return seq[1:]

    def footprint(self, batch: int = 1, dtype=None) -> int:
        """Device bytes an evolution of `batch` states needs (the handle's
        dtype, or `dtype`: a planned handle has none yet)."""
        b = ctypes.c_size_t()
        if dtype is None:
            _lib.check(_lib.load().hs_footprint(self._h, batch, b))
        else:
            _lib.check(_lib.load().hs_footprint_dtype(self._h, batch, dtype_code(dtype), b))
        return b.value

    def check_closure(self, stream=None) -> bool:
        v = ctypes.c_int()
        _lib.check(_lib.load().hs_check(self._h, _stream_ptr(stream), v))
        return v.value == 0


def _build_flags(merge_diag, order):
    flags = HS_MERGE_DIAG if merge_diag else 0
    if order == 2:
        flags |= HS_ORDER2
    elif order == 4:
        flags |= HS_ORDER4
    elif order != 1:
        raise ValueError("order must be 1, 2 or 4")
    return flags


def plan(strings, coeffs, n, t, steps, budget, merge_diag=True, order=1) -> Factors:
    """Host-only grouping and diagonal sets (no device memory)."""
    lib = _lib.load()
    arr, ri, _keep = _marshal_terms(strings, coeffs, n)
    h = ctypes.c_void_p()
    _lib.check(lib.hs_plan(n, len(ri), arr, ri.ctypes.data, float(t), int(steps), int(budget),
                           _build_flags(merge_diag, order), ctypes.byref(h)))
    return Factors(h, built=False)


def build_factors(strings, coeffs, n, t, steps, budget, dtype="c64", merge_diag=True,
                  stream=None, order=1) -> Factors:
    """Group, plan and build the factors (order 1: Eq. 4; 2: symmetric; 4: Suzuki)."""
    lib = _lib.load()
    arr, ri, _keep = _marshal_terms(strings, coeffs, n)
    h = ctypes.c_void_p()
    _lib.check(lib.hs_build_factors(n, len(ri), arr, ri.ctypes.data, float(t), int(steps),
                                    int(budget), dtype_code(dtype), _build_flags(merge_diag, order),
                                    _stream_ptr(stream), ctypes.byref(h)))
    return Factors(h, built=True)


def _state_args(psi, N=None):
    if not getattr(psi, "is_cuda", False):
        raise ValueError("state must be a tensor in device memory (a host tensor would fault the GPU)")
    import torch
    if psi.device.index != torch.cuda.current_device():
        raise ValueError(f"state lives on {psi.device}, the current device is cuda:{torch.cuda.current_device()}")
    if not psi.is_contiguous():
        raise ValueError("state must be contiguous")
    batch = 1 if psi.dim() == 1 else psi.shape[0]
    n_amp = psi.shape[-1]
    if N is not None and n_amp != N:
        raise ValueError(f"state has {n_amp} amplitudes, expected {N}")
    return batch, n_amp, dtype_code(psi.dtype)


def evolve(f: Factors, psi, steps: int, renorm: bool = False, fuse: bool = True, stream=None):
    """psi <- (U_F ... U_1)^steps psi in place (enqueued on the stream)."""
    batch, _, code = _state_args(psi, f.N)
    if code != f.dtype_code:
        raise ValueError("state dtype differs from the factors' dtype")
    flags = (HS_RENORM if renorm else 0) | (0 if fuse else HS_NO_FUSE)
    _lib.check(_lib.load().hs_evolve(f.handle, ctypes.c_void_p(psi.data_ptr()), batch, int(steps),
                                     _stream_ptr(stream), flags))
    return psi


def norm2(psi, stream=None) -> np.ndarray:
    batch, N, code = _state_args(psi)
    out = np.zeros(batch, dtype=np.float64)
    _lib.check(_lib.load().hs_norm2(ctypes.c_void_p(psi.data_ptr()), batch, N, code,
                                    _stream_ptr(stream), out.ctypes.data))
    return out


def fidelity(phi, psi, stream=None) -> np.ndarray:
    """[B, 5]: Re<phi|psi>, Im<phi|psi>, <phi|phi>, <psi|psi>, fidelity."""
    batch, N, cp = _state_args(phi)
    b2, N2, cq = _state_args(psi)
    if (batch, N) != (b2, N2):
        raise ValueError("shape mismatch")
    out = np.zeros((batch, 5), dtype=np.float64)
    _lib.check(_lib.load().hs_fidelity(ctypes.c_void_p(phi.data_ptr()), cp,
                                       ctypes.c_void_p(psi.data_ptr()), cq, batch, N,
                                       _stream_ptr(stream), out.ctypes.data))
    return out


def fidelity_noalloc(phi, psi, out, stream=None):
    """fidelity() into a device float64 tensor out [B, 5], enqueued on the
    stream without allocating or synchronising (B <= 8; see hs_fidelity_noalloc)."""
    batch, N, cp = _state_args(phi)
    b2, N2, cq = _state_args(psi)
    if (batch, N) != (b2, N2):
        raise ValueError("shape mismatch")
    import torch
    if (not out.is_cuda or out.dtype != torch.float64 or not out.is_contiguous()
            or out.numel() != batch * 5 or out.device != phi.device):
        raise ValueError("out must be a contiguous float64 device tensor of batch * 5 entries")
    _lib.check(_lib.load().hs_fidelity_noalloc(ctypes.c_void_p(phi.data_ptr()), cp,
                                               ctypes.c_void_p(psi.data_ptr()), cq, batch, N,
                                               _stream_ptr(stream), ctypes.c_void_p(out.data_ptr())))
    return out


def dia_spmv(offsets, diags, x, y=None, stream=None):
    """y = A x for A given by ascending ``offsets`` and device ``diags``."""
    import torch
    batch, N, code = _state_args(x)
    if y is None:
        y = torch.empty_like(x)
    offs = (ctypes.c_longlong * len(offsets))(*[int(d) for d in offsets])
    ptrs = (ctypes.c_void_p * len(diags))(*[d.data_ptr() for d in diags])
    for d, v in zip(offsets, diags):
        if v.numel() != N - abs(int(d)) or dtype_code(v.dtype) != code:
            raise ValueError("diagonal length or dtype mismatch")
        if not v.is_cuda or v.device != x.device:
            raise ValueError("diagonals must be device tensors on the state's device")
    if not y.is_cuda or y.device != x.device:
        raise ValueError("y must be a device tensor on x's device")
    _lib.check(_lib.load().hs_dia_spmv(len(offsets), offs, ptrs, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), batch, N, code,
                                       _stream_ptr(stream)))
    return y
