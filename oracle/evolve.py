"""Trotterized evolution in FP64: ctypes front-end of ``evolve.c`` plus a
NumPy twin for small cases (test infrastructure only).

Paper: Eq. 4 (product of factor exponentials, repeated r times), Eq. 2
(each factor exponentiated exactly), Section 3.4 (a diagonal operator is
exponentiated elementwise); the future-work section's higher-order products
(second-order symmetric and fourth-order Suzuki).  First-order step order: D
first, then the groups in their creation order; inside a group each member's
rotation cos(c h) I - i sin(c h) P (members commute, so the order is
immaterial).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .factors import Partition, diag_phase
from .pauli import apply_pauli

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile evolve.c with gcc (-O2, OpenMP) into oracle/_build/."""
    os.makedirs(_BUILD, exist_ok=True)
    src = os.path.join(_HERE, "evolve.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_evolve.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, P,
                                      ctypes.c_int, P, ctypes.c_int, P, P,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int]
        lib.oracle_evolve.restype = ctypes.c_int
        lib.oracle_evolve_seq.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, P,
                                          ctypes.c_int, P, ctypes.c_int, P, P,
                                          ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int]
        lib.oracle_evolve_seq.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return _load().oracle_max_threads()


SUZUKI_P = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))


def product_sequence(partition: Partition, dt: float, order: int = 1) -> list:
    """One step of a product formula as [(group index or -1 for D, h)].

    Factors F_1..F_L are D (when present) then the groups in order.
    order 1: F_1(dt) ... F_L(dt)                      (Eq. 4)
    order 2: F_1(dt/2) .. F_{L-1}(dt/2) F_L(dt) F_{L-1}(dt/2) .. F_1(dt/2)
             (the symmetric second-order product)
    order 4: S2(p dt) S2(p dt) S2((1-4p) dt) S2(p dt) S2(p dt),
             p = 1/(4 - 4^(1/3)) (Suzuki's fourth-order recursion)
    """
    F = ([-1] if partition.diag else []) + list(range(len(partition.groups)))
    if order == 1:
        return [(g, dt) for g in F]

    def s2(h):
        if len(F) == 1:
            return [(F[0], h)]
        return [(g, h / 2) for g in F[:-1]] + [(F[-1], h)] + [(g, h / 2) for g in reversed(F[:-1])]
    if order == 2:
        return s2(dt)
    if order == 4:
        p = SUZUKI_P
        return s2(p * dt) + s2(p * dt) + s2((1 - 4 * p) * dt) + s2(p * dt) + s2(p * dt)
    raise ValueError(f"order {order} not supported")


def merge_adjacent(seq: list) -> list:
    """Combine neighbouring entries of the same factor: exp(-i a G) exp(-i b G)
    = exp(-i (a + b) G) exactly, since G commutes with itself.  Time steps add
    left to right."""
    out = []
    for g, h in seq:
        if out and out[-1][0] == g:
            out[-1] = (g, out[-1][1] + h)
        else:
            out.append((g, h))
    return out


def evolve(terms, partition: Partition, psi: np.ndarray, n: int, dt: float, steps: int,
           threads: int = 0, order: int = 1) -> np.ndarray:
    """Return psi_r for a [N] or [B, N] state (a new complex128 array)."""
    lib = _load()
    out = np.ascontiguousarray(np.array(psi, dtype=np.complex128, copy=True))
    batch = 1 if out.ndim == 1 else out.shape[0]
    assert out.shape[-1] == 1 << n
    xm = np.array([t.xmask for t in terms], dtype=np.uint64)
    zm = np.array([t.zmask for t in terms], dtype=np.uint64)
    ny = np.array([t.ny for t in terms], dtype=np.int32)
    cf = np.array([t.coeff for t in terms], dtype=np.float64)
    di = np.array(partition.diag, dtype=np.int32)
    gp = np.zeros(len(partition.groups) + 1, dtype=np.int32)
    for j, g in enumerate(partition.groups):
        gp[j + 1] = gp[j] + len(g)
    gi = np.array([k for g in partition.groups for k in g], dtype=np.int32)
    if gi.size == 0:
        gi = np.zeros(1, dtype=np.int32)
    if di.size == 0:
        di = np.zeros(1, dtype=np.int32)
        nd = 0
    else:
        nd = len(partition.diag)
    seq = product_sequence(partition, dt, order)
    sg = np.array([g for g, _ in seq] or [0], dtype=np.int32)
    sd = np.array([h for _, h in seq] or [0.0], dtype=np.float64)
    rc = lib.oracle_evolve_seq(n, batch, out.ctypes.data, len(terms), xm.ctypes.data, zm.ctypes.data,
                               ny.ctypes.data, cf.ctypes.data, nd, di.ctypes.data,
                               len(partition.groups), gp.ctypes.data, gi.ctypes.data,
                               len(seq), sg.ctypes.data, sd.ctypes.data, int(steps), int(threads))
    if rc != 0:
        raise MemoryError("oracle_evolve failed")
    return out


def evolve_np(terms, partition: Partition, psi: np.ndarray, n: int, dt: float,
              steps: int, order: int = 1) -> np.ndarray:
    """NumPy twin of :func:`evolve` (vectorised, small n)."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    seq = product_sequence(partition, dt, order)
    for _ in range(steps):
        for g, h in seq:
            if g < 0:
                out = out * diag_phase(terms, partition.diag, n, h)
                continue
            for k in partition.groups[g]:
                th = terms[k].coeff * h
                out = np.cos(th) * out - 1j * np.sin(th) * apply_pauli(terms[k], out)
    return out
