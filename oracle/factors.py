"""Grouping of Pauli terms into diagonal-budgeted Trotter factors (FP64).

Paper: Eq. 4 (first-order Trotter product over H = sum_j H_j, Section 2.1),
Eq. 5 (diagonal budget num_diags(e^{-i H dt}) <= D_max, Section 3.1), the
exact O(N) exponential of a diagonal operator (Section 3.3 "SpME",
Section 3.4), and the structural dry run that fixes a factor's diagonal set
before any storage is allocated (Section 3.2).

Readings where the paper is silent (each is listed in the design notes):

* Factors are *commuting* groups of Pauli terms; the budget bounds each
  factor's own exponential (the paper applies Eq. 5 to the whole H, whose
  single-slice exponential cannot meet small budgets when factors are split).
* All Z-only terms (including the identity) form the diagonal factor D with
  D[x] = exp(-i dt E(x)), E(x) = sum_k c_k (-1)^{popcount(x & z_k)}.
* Off-diagonal terms are grouped first-fit in input order: a term joins the
  first existing group all of whose members it commutes with and whose
  exponential then still has <= budget diagonals; otherwise it opens a new
  group.  A single term whose own exponential exceeds the budget is an error.
  A group may act on at most 10 qubits (its local unitary is a dense
  2^k x 2^k matrix); a term that would push a group past that limit skips it.
* ``num_diags`` counts numerically nonzero diagonals: offsets
  spr(b) - spr(a) over local-unitary entries |L[a, b]| > 1e-15, where spr
  spreads local bits onto the support's qubit positions.  Entries at or below
  the threshold are treated as exactly zero.
* A step applies D first, then the groups in creation order.  Merging D into
  the first group (U_1 D) changes no number.
* Because the members of a group commute and each Pauli squares to I, the
  group exponential is exactly prod_k (cos(c_k dt) I - i sin(c_k dt) P_k);
  the product is formed in member order.
"""
from __future__ import annotations

import numpy as np

from .pauli import commute, parse_terms, popcount_array

TAU = 1e-15
MAX_SUPPORT = 10


def support_bits(terms) -> list:
    s = 0
    for t in terms:
        s |= t.support
    return [q for q in range(64) if (s >> q) & 1]


def _pext(v: int, bits) -> int:
    out = 0
    for j, q in enumerate(bits):
        out |= ((v >> q) & 1) << j
    return out


def _spread(a: int, bits) -> int:
    out = 0
    for j, q in enumerate(bits):
        out |= ((a >> j) & 1) << q
    return out


def local_unitary(terms, dt: float):
    """Return (support, L) with L = prod_k exp(-i c_k dt P_k) on the support.

    Row/column index a is the support-local basis index (bit j = qubit
    support[j]).  The k-th member is applied k-th (it multiplies from the
    left).  Each factor is cos(th) I - i sin(th) P restricted to the support.
    """
    bits = support_bits(terms)
    k = len(bits)
    if k > MAX_SUPPORT:
        raise ValueError(f"group support of {k} qubits exceeds {MAX_SUPPORT}")
    K = 1 << k
    L = np.eye(K, dtype=np.complex128)
    y = np.arange(K, dtype=np.int64)
    for t in terms:
        m = _pext(t.xmask, bits)
        z = _pext(t.zmask, bits)
        th = t.coeff * dt
        src = y ^ m
        sign = 1.0 - 2.0 * (popcount_array(src & z) & 1)
        pl = ((1j) ** t.ny) * sign            # (P L)[y,:] = pl[y] * L[y^m,:]
        L = np.cos(th) * L - 1j * np.sin(th) * (pl[:, None] * L[src, :])
    return bits, L


def local_offsets(bits, L, tau: float = TAU) -> list:
    """Sorted offsets spr(b) - spr(a) over entries |L[a, b]| > tau."""
    a_idx, b_idx = np.nonzero(np.abs(L) > tau)
    spr = np.array([_spread(a, bits) for a in range(L.shape[0])], dtype=np.int64)
    return sorted(set((spr[b_idx] - spr[a_idx]).tolist()))


def num_diags(terms, dt: float) -> int:
    bits, L = local_unitary(terms, dt)
    return len(local_offsets(bits, L))


class Partition:
    """Diagonal terms and ordered off-diagonal groups (term indices)."""

    def __init__(self, diag, groups):
        self.diag = list(diag)
        self.groups = [list(g) for g in groups]

    def factor_list(self, merge_diag: bool = True):
        """Factors in application order as (has_diag, group_terms) pairs."""
        out = []
        if self.diag and (not merge_diag or not self.groups):
            out.append((True, []))
            for g in self.groups:
                out.append((False, g))
        else:
            for j, g in enumerate(self.groups):
                out.append((bool(self.diag) and j == 0, g))
        return out

    def __eq__(self, other):
        return self.diag == other.diag and self.groups == other.groups

    def __repr__(self):
        return f"Partition(diag={self.diag}, groups={self.groups})"


class BudgetError(ValueError):
    pass


def first_fit(terms, budget: int, dt: float) -> Partition:
    """First-fit grouping of ``terms`` (list of Term) under ``budget``."""
    diag, groups = [], []
    for i, t in enumerate(terms):
        if t.is_diagonal:
            diag.append(i)
            continue
        placed = False
        for g in groups:
            if not all(commute(t, terms[j]) for j in g):
                continue
            if len(support_bits([terms[j] for j in g] + [t])) > MAX_SUPPORT:
                continue
            if num_diags([terms[j] for j in g] + [t], dt) <= budget:
                g.append(i)
                placed = True
                break
        if not placed:
            if num_diags([t], dt) > budget:
                raise BudgetError(f"term {i} ({t.string}) alone exceeds budget {budget}")
            groups.append([i])
    return Partition(diag, groups)


def partition_from_strings(strings, coeffs, n, budget, t, steps) -> Partition:
    terms = parse_terms(strings, coeffs, n)
    return first_fit(terms, budget, t / steps)


def energies(terms, idx, n: int) -> np.ndarray:
    """E(x) = sum_{k in idx} c_k (-1)^{popcount(x & z_k)} for all x (FP64)."""
    x = np.arange(1 << n, dtype=np.int64)
    E = np.zeros(1 << n, dtype=np.float64)
    for k in idx:
        t = terms[k]
        E += t.coeff * (1.0 - 2.0 * (popcount_array(x & t.zmask) & 1))
    return E


def diag_phase(terms, idx, n: int, dt: float) -> np.ndarray:
    ph = -dt * energies(terms, idx, n)
    return np.cos(ph) + 1j * np.sin(ph)


def factor_offsets(terms, factor, dt: float) -> list:
    has_diag, g = factor
    if not g:
        return [0]
    bits, L = local_unitary([terms[j] for j in g], dt)
    return local_offsets(bits, L)


def factor_entries(terms, partition: Partition, factor, n: int, dt: float,
                   rows: np.ndarray, d: int) -> np.ndarray:
    """U_f[r, r + d] for each r in ``rows`` (rows with r + d outside [0, N)
    must not be passed).  U_f = G (L on the support, identity elsewhere),
    times D on the right when the factor carries the diagonal terms."""
    has_diag, g = factor
    rows = np.asarray(rows, dtype=np.int64)
    cols = rows + d
    if g:
        bits, L = local_unitary([terms[j] for j in g], dt)
        L = np.where(np.abs(L) > TAU, L, 0.0)
        smask = 0
        for q in bits:
            smask |= 1 << q
        same = ((rows ^ cols) & ~smask) == 0
        a = np.array([_pext(int(r), bits) for r in rows], dtype=np.int64)
        b = np.array([_pext(int(c), bits) for c in cols], dtype=np.int64)
        val = np.where(same, L[a, b], 0.0)
    else:
        val = np.where(rows == cols, 1.0 + 0j, 0.0 + 0j)
    if has_diag:
        x = cols
        E = np.zeros(len(cols), dtype=np.float64)
        for k in partition.diag:
            t = terms[k]
            E += t.coeff * (1.0 - 2.0 * (popcount_array(x & t.zmask) & 1))
        ph = -dt * E
        val = val * (np.cos(ph) + 1j * np.sin(ph))
    return val


def factor_dense(terms, partition: Partition, factor, n: int, dt: float) -> np.ndarray:
    """Dense N x N matrix of one factor (small n only): L placed on every
    orbit of the support (identity on the other qubits), then D applied on
    the right when the factor carries the diagonal terms."""
    N = 1 << n
    has_diag, g = factor
    if g:
        bits, L = local_unitary([terms[j] for j in g], dt)
        L = np.where(np.abs(L) > TAU, L, 0.0)
        smask = 0
        for q in bits:
            smask |= 1 << q
        base = np.arange(N, dtype=np.int64)
        base = base[(base & smask) == 0]
        U = np.zeros((N, N), dtype=np.complex128)
        K = L.shape[0]
        for a in range(K):
            ra = base | _spread(a, bits)
            for b in range(K):
                U[ra, base | _spread(b, bits)] = L[a, b]
    else:
        U = np.eye(N, dtype=np.complex128)
    if has_diag:
        U = U * diag_phase(terms, partition.diag, n, dt)[None, :]
    return U
