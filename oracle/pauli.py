"""Pauli strings: parsing, dense matrices and action on state vectors.

Paper: Section 4.3 (HamLib supplies each Hamiltonian as Pauli strings with
coefficients).  The paper does not state the string convention; the reading
used here is: character k of a string acts on qubit k, which is bit k of the
basis index (least-significant first).

For a string with X-part mask m and Z-part mask z (a Y sets both bits) and
ny = number of Y characters, using Y = i X Z on each qubit,

    P |x> = i^ny (-1)^{popcount(x & z)} |x XOR m>,

so  P[y, x] = i^ny (-1)^{popcount(x & z)} when y = x XOR m, else 0.
The tests pin this against Kronecker products of the 2x2 Pauli matrices.
"""
from __future__ import annotations

import numpy as np

SIGMA = {
    "I": np.array([[1, 0], [0, 1]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


class Term:
    """One Pauli term c * P with its bit masks."""

    __slots__ = ("string", "coeff", "xmask", "zmask", "ny")

    def __init__(self, string: str, coeff: float):
        self.string = string
        self.coeff = float(coeff)
        x = z = 0
        ny = 0
        for k, ch in enumerate(string):
            if ch == "X":
                x |= 1 << k
            elif ch == "Z":
                z |= 1 << k
            elif ch == "Y":
                x |= 1 << k
                z |= 1 << k
                ny += 1
            elif ch != "I":
                raise ValueError(f"bad Pauli character {ch!r} in {string!r}")
        self.xmask, self.zmask, self.ny = x, z, ny

    @property
    def is_diagonal(self) -> bool:
        return self.xmask == 0

    @property
    def support(self) -> int:
        return self.xmask | self.zmask

    def __repr__(self):
        return f"Term({self.string!r}, {self.coeff})"


def parse_terms(strings, coeffs, n: int):
    """Parse strings of length ``n``; complex coefficients must be real.

    A coefficient whose imaginary part exceeds 1e-12 * max|c| makes the sum
    non-Hermitian and is rejected (the paper requires Hermitian H, Eq. 1).
    """
    coeffs = np.asarray(coeffs)
    if np.iscomplexobj(coeffs):
        scale = max(1e-300, float(np.max(np.abs(coeffs)))) if coeffs.size else 1.0
        if np.any(np.abs(coeffs.imag) > 1e-12 * scale):
            raise ValueError("non-Hermitian: complex coefficient")
        coeffs = coeffs.real
    terms = []
    for s, c in zip(strings, coeffs):
        if len(s) != n:
            raise ValueError(f"string {s!r} has length {len(s)} != {n}")
        terms.append(Term(s, float(c)))
    return terms


def popcount(v) -> int:
    return bin(int(v)).count("1")


def popcount_array(a: np.ndarray) -> np.ndarray:
    """Bit count of each element of a non-negative int64 array."""
    a = a.astype(np.uint64)
    c = np.zeros(a.shape, dtype=np.int64)
    while np.any(a):
        c += (a & np.uint64(1)).astype(np.int64)
        a = a >> np.uint64(1)
    return c


def dense_pauli(string: str) -> np.ndarray:
    """Kronecker product of 2x2 Pauli matrices, qubit 0 = least-significant."""
    M = np.array([[1.0 + 0j]])
    for ch in reversed(string):          # highest qubit is the left factor
        M = np.kron(M, SIGMA[ch])
    return M


def dense_hamiltonian(terms, n: int) -> np.ndarray:
    N = 1 << n
    H = np.zeros((N, N), dtype=np.complex128)
    for t in terms:
        H += t.coeff * dense_pauli(t.string)
    return H


def dense_propagator(Hd: np.ndarray, t: float) -> np.ndarray:
    """exp(-i H t) of a dense Hermitian matrix by its eigendecomposition
    H = V diag(w) V^dagger (numpy.linalg.eigh): V diag(exp(-i w t)) V^dagger.
    The exact propagator of Eq. 2 that a Trotter product approximates (for
    small n: the matrix is 2^n x 2^n)."""
    w, V = np.linalg.eigh(Hd)
    return (V * np.exp(-1j * t * w)) @ V.conj().T


def apply_pauli(term: Term, psi: np.ndarray) -> np.ndarray:
    """Return P psi for a state (or a [.., N] batch) using the mask form."""
    N = psi.shape[-1]
    y = np.arange(N, dtype=np.int64)
    src = y ^ term.xmask
    sign = 1.0 - 2.0 * (popcount_array(src & term.zmask) & 1)
    phase = (1j) ** term.ny
    return phase * sign * psi[..., src]


def commute(a: Term, b: Term) -> bool:
    """Pauli strings commute iff the symplectic product is even."""
    return (popcount(a.xmask & b.zmask) + popcount(a.zmask & b.xmask)) % 2 == 0


def hamiltonian_offsets(terms, n: int, tol: float = 0.0):
    """Offsets d = col - row of the diagonals of H that hold a nonzero entry.

    Computed exactly from the Pauli structure: entry (y, y ^ m) collects
    every term with X-mask m; a diagonal is active when some entry on it is
    nonzero after summing the terms that share an X-mask.
    """
    N = 1 << n
    by_mask: dict = {}
    for t in terms:
        by_mask.setdefault(t.xmask, []).append(t)
    y = np.arange(N, dtype=np.int64)
    offs = set()
    nnz = 0
    for m, ts in by_mask.items():
        col = y ^ m
        val = np.zeros(N, dtype=np.complex128)
        for t in ts:
            sign = 1.0 - 2.0 * (popcount_array(col & t.zmask) & 1)
            val += t.coeff * (1j) ** t.ny * sign
        nz = np.abs(val) > tol
        nnz += int(np.count_nonzero(nz))
        offs.update(np.unique(col[nz] - y[nz]).tolist())
    return sorted(offs), nnz
