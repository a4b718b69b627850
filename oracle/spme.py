"""Sparse matrix exponential by truncated Taylor series, the diagonal-budget
step search and the single-propagator simulation loop, in FP64 (test
infrastructure only).

Paper: Alg. 2 (SpME: X = -i A t; U = T = I; T <- T X / i; stop when the norm
of T falls below the tolerance, 1e-6 as printed; otherwise U += T) in the
scaling-and-squaring form the SpME subsection says is used in practice (the
series is summed for X / 2^s, then the result is squared s times by sparse
products), Alg. 3
(n = EstimateTimesteps(A, T, D_max); dt = T / n; U = SpME(A, dt); n times
x <- U x), the EstimateTimesteps flowchart of Section 3.1 and Eq. 5
(smallest r with num_diags(e^{-i H t / r}) <= D_max), the structural dry run
of Section 3.2 (the output diagonal set is known from the offsets alone).

Readings where the paper is silent:

* ``T.norm()`` is the largest entry modulus of T.
* num_diags of the propagator is its structural diagonal count: the union of
  the offset sets of the kept Taylor terms, where term k's offsets are the
  k-fold sums of H's (numerically nonzero) offsets, clipped to (-N, N).
* A diagonal H takes the exact elementwise exponential (Section 3.3), K = 0.
* Scaling-and-squaring: the paper fixes no rule for s.  Reading: s is the
  smallest s >= 0 with |dt| * nu(H) / 2^s <= 1/2, where nu(H) is the sum over
  H's diagonals (ascending offset) of each diagonal's largest entry modulus,
  an upper bound of ||H||_1, ||H||_inf and ||H||_2 (the classical Taylor
  scaling target of Moler and Van Loan, "Nineteen dubious ways", method 3).
  Squaring doubles the structural offset set each time: S <- S + S.  An
  explicit s (0 = plain Alg. 2) may be passed instead.
* num_diags of the propagator counts the offsets after squaring.
* EstimateTimesteps: a diagonal H needs r = 1; otherwise l = 1; if the
  budget holds at l, r = l; else u = 2 l, l <- u while the budget fails at u
  (doubling), then binary search on (l_prev, u] for the smallest feasible r.
* max_iterations defaults to 30.

The Taylor sum is formed with a library sparse matrix product
(scipy.sparse, CSR) in the order T_k = T_{k-1} X / k.

Pin status: SpME is pinned against scipy.linalg.expm within the Taylor
remainder, and the simulation loop against exp(-iHt) psi.  The step search
(estimate_timesteps) is parity unpinned: its predicate, the structural
diagonal count of the propagator, has no reference outside this module (the
tests check that the searched r is the smallest r by brute force over the
same predicate and that the predicate is monotone over the tested range),
and the step counts the paper prints (r = 1120 for a 10-qubit TFIM,
r = 71-107 for 10-qubit Heisenberg models) depend on a budget the paper does
not state, so they cannot be reproduced.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .pauli import parse_terms, popcount_array

DEFAULT_TOL = 1e-6
DEFAULT_MAX_ITER = 30


def hamiltonian_csr(terms, n: int) -> sp.csr_matrix:
    """H as a sparse matrix from the Pauli action H[y, y^m] += c i^ny (-1)^{popcount((y^m)&z)}."""
    N = 1 << n
    rows, cols, vals = [], [], []
    y = np.arange(N, dtype=np.int64)
    for t in terms:
        col = y ^ t.xmask
        sign = 1.0 - 2.0 * (popcount_array(col & t.zmask) & 1)
        rows.append(y)
        cols.append(col)
        vals.append(t.coeff * (1j) ** t.ny * sign)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N), dtype=np.complex128)
    H.sum_duplicates()
    H.eliminate_zeros()
    return H


def offsets_of(M) -> list:
    """Offsets (col - row) of the diagonals holding a nonzero entry."""
    C = sp.coo_matrix(M)
    nz = C.data != 0
    return sorted(set((C.col[nz] - C.row[nz]).tolist()))


def sumset(a, b, N) -> list:
    return sorted({x + y for x in a for y in b if -N < x + y < N})


def modulus(z: np.ndarray) -> np.ndarray:
    """|z| as sqrt(re^2 + im^2)."""
    return np.sqrt(z.real * z.real + z.imag * z.imag)


def norm_bound(H: sp.csr_matrix) -> float:
    """nu(H) = sum over diagonals (ascending offset) of max |H[r, r+d]|."""
    C = sp.coo_matrix(H)
    off = C.col.astype(np.int64) - C.row.astype(np.int64)
    mags = modulus(C.data)
    total = 0.0
    for d in sorted(set(off.tolist())):
        total += float(mags[off == d].max())
    return total


def squarings(H: sp.csr_matrix, dt: float) -> int:
    """Smallest s >= 0 with |dt| nu(H) / 2^s <= 1/2."""
    x, s = abs(dt) * norm_bound(H), 0
    while x > 0.5 * 2.0 ** s:
        s += 1
    return s


def spme(H: sp.csr_matrix, dt: float, tol: float = DEFAULT_TOL, max_iter: int = DEFAULT_MAX_ITER,
         n_squarings: int | None = None):
    """Truncated Taylor series of exp(-i H dt) with scaling and squaring
    (`n_squarings` None: the rule above; 0: plain Alg. 2).

    Returns (U, K, offsets): U as CSR, K = number of Taylor terms added after
    the identity, and the structural offset set of U."""
    N = H.shape[0]
    offX = offsets_of(H)
    if offX in ([], [0]):
        # diagonal H: the exponential is exact and elementwise (Section 3.3)
        d = H.diagonal()
        return sp.diags(np.cos(-dt * d.real) + 1j * np.sin(-dt * d.real), format="csr"), 0, [0]
    s = squarings(H, dt) if n_squarings is None else int(n_squarings)
    dt = dt / 2.0 ** s
    X = (H * (-1j * dt)).tocsr()
    U = sp.identity(N, dtype=np.complex128, format="csr")
    T = sp.identity(N, dtype=np.complex128, format="csr")
    offT = [0]
    offU = {0}
    K = 0
    for i in range(1, max_iter + 1):
        T = (T @ X) / i
        offT = sumset(offT, offX, N)
        norm = float(np.max(modulus(T.data))) if T.nnz else 0.0
        if norm < tol:
            break
        U = U + T
        offU.update(offT)
        K = i
    offs = sorted(offU)
    for _ in range(s):
        U = U @ U
        offs = sumset(offs, offs, N)
    return U.tocsr(), K, offs


def num_diags(H, t, r, tol=DEFAULT_TOL, max_iter=DEFAULT_MAX_ITER) -> int:
    return len(spme(H, t / r, tol, max_iter)[2])


def estimate_timesteps(H, t, budget, tol=DEFAULT_TOL, max_iter=DEFAULT_MAX_ITER, r_max=1 << 24):
    """Smallest r with num_diags(SpME(H, t/r)) <= budget (flowchart of Section 3.1).
    Parity unpinned (see the module docstring)."""
    if offsets_of(H) in ([], [0]):
        return 1

    def ok(r):
        return num_diags(H, t, r, tol, max_iter) <= budget

    lo = 1
    if ok(lo):
        return lo
    u = 2 * lo
    while not ok(u):
        lo = u
        u *= 2
        if u > r_max:
            raise ValueError("no feasible step count below r_max")
    # smallest feasible in (lo, u]
    while u - lo > 1:
        mid = (lo + u) // 2
        if ok(mid):
            u = mid
        else:
            lo = mid
    return u


def simulate(H, psi0: np.ndarray, t: float, r: int, tol=DEFAULT_TOL, max_iter=DEFAULT_MAX_ITER,
             n_squarings: int | None = None):
    """Alg. 3 with a given r: U = SpME(H, t/r); r times psi <- U psi."""
    U, K, offs = spme(H, t / r, tol, max_iter, n_squarings)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(r):
        psi = (U @ psi.T).T if psi.ndim == 2 else U @ psi
    return psi, K, offs


def hamiltonian_from_strings(strings, coeffs, n):
    return hamiltonian_csr(parse_terms(strings, coeffs, n), n)
