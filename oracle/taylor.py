"""The Taylor expansion of exp(-i H dt) applied to states without forming the
propagator, in FP64 (test infrastructure only).

Paper: the future-work section (fuse the Taylor expansion into the
state-vector update, removing the intermediate matrix); the series itself is
the one of Alg. 2, T_k = T_{k-1} X / k with X = -i H dt.

One step maps x to  sum_{k=0..K} v_k,  v_0 = x,  v_k = (-i dt / k) H v_{k-1},
summed term by term (the plain definition; the library evaluates the same
polynomial by Horner's rule).  H is a scipy.sparse matrix.

Readings where the paper is silent (it gives no algorithm for this update):

* K is fixed before the step from the norm bound nu(H) (the sum of the
  per-diagonal largest entry moduli, which bounds ||H||_2): the smallest
  K >= 1 with (|dt| nu)^(K+1) / (K+1)! < tol, so the first dropped term of
  the operator series is below tol in 2-norm; tol = 1e-6 as in Alg. 2.  A
  state-dependent stop would need a reduction and a host round trip per term.
* The step count is the smallest r with |t / r| nu <= theta (theta = 1 by
  default); the diagonal budget does not apply, since no propagator is built.
"""
from __future__ import annotations

import math

import numpy as np

from .spme import norm_bound

DEFAULT_TOL = 1e-6


def taylor_terms(H, dt: float, tol: float = DEFAULT_TOL, max_terms: int = 64) -> int:
    """Smallest K >= 1 with (|dt| nu(H))^(K+1) / (K+1)! < tol."""
    x = abs(dt) * norm_bound(H)
    b = x                                   # x^k / k! for k = 1
    for k in range(1, max_terms + 1):
        b = b * x / (k + 1)
        if b < tol:
            return k
    raise ValueError("max_terms Taylor terms do not reach the tolerance")


def taylor_steps(H, t: float, theta: float = 1.0) -> int:
    """Smallest r >= 1 with |t / r| nu(H) <= theta."""
    nu = norm_bound(H)
    r = 1
    while abs(t / r) * nu > theta:
        r += 1
    return r


def taylor_step(H, psi: np.ndarray, dt: float, K: int) -> np.ndarray:
    """sum_{k=0..K} (-i dt H)^k psi / k! for psi [N] or [B, N]."""
    x = np.array(psi, dtype=np.complex128, copy=True)
    cols = x.T                               # [N] or [N, B]
    y = cols.copy()
    v = cols
    for k in range(1, K + 1):
        v = (H @ v) * (-1j * dt / k)
        y = y + v
    return np.ascontiguousarray(y.T)


def taylor_evolve(H, psi: np.ndarray, dt: float, K: int, steps: int) -> np.ndarray:
    out = np.array(psi, dtype=np.complex128, copy=True)
    for _ in range(steps):
        out = taylor_step(H, out, dt, K)
    return out


def remainder_bound(x: float, K: int) -> float:
    """sum_{k > K} x^k / k!  (>= ||exp(X) - p_K(X)||_2 when ||X||_2 <= x)."""
    return sum(x ** k / math.factorial(k) for k in range(K + 1, K + 80))


def _apply_rows(terms, rows: np.ndarray, values_at) -> np.ndarray:
    """(H v)[rows] from the Pauli action H[y, y^m] += c i^ny (-1)^{popcount((y^m) & z)},
    where values_at(idx) returns v[idx]."""
    from .pauli import popcount_array
    out = np.zeros(len(rows), dtype=np.complex128)
    for t in terms:
        col = rows ^ np.int64(t.xmask)
        sign = 1.0 - 2.0 * (popcount_array(col & np.int64(t.zmask)) & 1)
        out += t.coeff * (1j) ** t.ny * sign * values_at(col)
    return out


def step_rows(terms, x: np.ndarray, rows, dt: float, K: int) -> np.ndarray:
    """Entries `rows` of one step sum_{k<=K} (-i dt H)^k x / k! for a state
    too large to multiply whole: (X^k x / k!)[idx] is formed from
    (X^(k-1) x / (k-1)!) at the rows that idx couples to, recursively (cost
    grows as (#terms)^K per sampled row)."""
    rows = np.asarray(rows, dtype=np.int64)

    def v(k, idx):
        if k == 0:
            return np.asarray(x[idx], dtype=np.complex128)
        return (-1j * dt / k) * _apply_rows(terms, idx, lambda c: v(k - 1, c))

    return sum(v(k, rows) for k in range(K + 1))
