"""Norm and state fidelity in FP64 (test infrastructure only).

Paper: Section 4.3, "State Fidelity" -- the fidelity between the computed
state and a reference solution; the formula is not printed.  Reading: for
possibly unnormalised states, F = |<phi|psi>|^2 / (<phi|phi> <psi|psi>),
with the norm drift | ||psi|| - 1 | reported separately.
"""
from __future__ import annotations

import numpy as np


def norm2(psi: np.ndarray) -> np.ndarray:
    p = np.asarray(psi, dtype=np.complex128)
    return np.sum(p.real * p.real + p.imag * p.imag, axis=-1)


def inner(phi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """<phi|psi> = sum conj(phi) psi along the last axis."""
    a = np.asarray(phi, dtype=np.complex128)
    b = np.asarray(psi, dtype=np.complex128)
    return np.sum(np.conj(a) * b, axis=-1)


def fidelity(phi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    ov = inner(phi, psi)
    return (ov.real ** 2 + ov.imag ** 2) / (norm2(phi) * norm2(psi))
