"""Seeded Pauli-sum Hamiltonians of the four families the paper evaluates.

The paper loads HamLib instances (TFIM, Heisenberg, MaxCut, TSP; Section 4,
"Benchmarks") which are not available here.  These generators are synthetic
stand-ins with the same structure: the same families, qubit ranges and
diagonal counts (2n+1 for a 1-D TFIM, 2*bonds+1 for a Heisenberg chain, one
diagonal for MaxCut/TSP cost functions; Table "tab:benchmarks").

Every generator returns a :class:`Hamiltonian`: ``n`` qubits and an ordered
list of ``(pauli_string, real_coefficient)`` terms.  Term order is part of
the input (the factor grouping is first-fit in this order).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations

import numpy as np


@dataclass
class Hamiltonian:
    n: int
    terms: list = field(default_factory=list)   # [(str, float)]
    name: str = ""

    @property
    def strings(self):
        return [s for s, _ in self.terms]

    @property
    def coeffs(self):
        return np.array([c for _, c in self.terms], dtype=np.float64)

    def add(self, ops: dict, coeff: float):
        """Append the term prod_{q: P} P_q (``ops`` maps qubit -> 'X'|'Y'|'Z')."""
        s = ["I"] * self.n
        for q, p in ops.items():
            s[q] = p
        self.terms.append(("".join(s), float(coeff)))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tfim_1d(n: int, J: float = 1.0, h: float = 1.0, periodic: bool = False) -> Hamiltonian:
    """H = -J sum Z_i Z_{i+1} - h sum X_i; bonds first, then fields."""
    H = Hamiltonian(n, name=f"tfim1d_n{n}")
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((n - 1, 0))
    for i, j in bonds:
        H.add({i: "Z", j: "Z"}, -J)
    for q in range(n):
        H.add({q: "X"}, -h)
    return H


def tfim_2d(rows: int, cols: int, J: float = 1.0, h: float = 1.0,
            n_total: int | None = None) -> Hamiltonian:
    """Open rows x cols lattice, site (r, c) -> qubit cols*r + c.

    Bonds: all horizontal ones row-major, then all vertical ones row-major,
    each ``-J Z Z``; then ``-h X_q`` for every lattice site.  Qubits at or
    above rows*cols (an idle ancilla when ``n_total`` is larger) carry no term.
    """
    n_sites = rows * cols
    n = n_sites if n_total is None else n_total
    H = Hamiltonian(n, name=f"tfim2d_{rows}x{cols}_n{n}")
    for r in range(rows):
        for c in range(cols - 1):
            H.add({cols * r + c: "Z", cols * r + c + 1: "Z"}, -J)
    for r in range(rows - 1):
        for c in range(cols):
            H.add({cols * r + c: "Z", cols * (r + 1) + c: "Z"}, -J)
    for q in range(n_sites):
        H.add({q: "X"}, -h)
    return H


def heisenberg_1d(n: int, J: float = 1.0, fields=None, periodic: bool = False) -> Hamiltonian:
    """H = J sum (XX + YY + ZZ) on chain bonds + sum h_i Z_i.

    Per bond the order is XX, YY, ZZ; the field terms follow all bonds.
    """
    H = Hamiltonian(n, name=f"heis1d_n{n}")
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((n - 1, 0))
    for i, j in bonds:
        for p in "XYZ":
            H.add({i: p, j: p}, J)
    if fields is not None:
        for q, hq in enumerate(fields):
            H.add({q: "Z"}, float(hq))
    return H


def random_regular_graph(n: int, degree: int, rng) -> list:
    """Uniform random pairing of ``degree*n`` stubs, rejecting self-loops and
    repeated edges and retrying.  Returns sorted edges (i < j)."""
    if (n * degree) % 2:
        raise ValueError("n*degree must be even")
    stubs = np.repeat(np.arange(n), degree)
    for _ in range(100000):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        edges = {tuple(sorted((int(a), int(b)))) for a, b in pairs}
        if len(edges) != len(pairs):
            continue
        return sorted(edges)
    raise RuntimeError("could not draw a simple regular graph")


def maxcut(n: int, edges, weights, mixer: float = 0.0) -> Hamiltonian:
    """H_C = sum_w w (I - Z_i Z_j)/2, plus ``mixer * sum X_q`` when nonzero.

    Term order: the constant (identity) term, the ZZ terms in edge order,
    then the X mixer terms in qubit order.
    """
    H = Hamiltonian(n, name=f"maxcut_n{n}")
    H.add({}, 0.5 * float(np.sum(weights)))
    for (i, j), w in zip(edges, weights):
        H.add({i: "Z", j: "Z"}, -0.5 * float(w))
    if mixer != 0.0:
        for q in range(n):
            H.add({q: "X"}, mixer)
    return H


def _poly_to_z_terms(n: int, poly: dict) -> Hamiltonian:
    """Expand a polynomial in binary variables x_q = (1 - Z_q)/2.

    ``poly`` maps frozenset(qubits) -> coefficient of prod_{q in set} x_q.
    Returns the equivalent sum of Z strings, ordered by their bit mask.
    """
    acc: dict = {}
    for mono, c in poly.items():
        qs = sorted(mono)
        scale = c / (2 ** len(qs))
        for k in range(len(qs) + 1):
            for sub in combinations(qs, k):
                mask = 0
                for q in sub:
                    mask |= 1 << q
                acc[mask] = acc.get(mask, 0.0) + scale * (-1) ** k
    H = Hamiltonian(n)
    for mask in sorted(acc):
        c = acc[mask]
        if abs(c) < 1e-12:
            continue
        H.add({q: "Z" for q in range(n) if (mask >> q) & 1}, c)
    return H


def tsp_onehot(dist, penalty: float = 20.0) -> Hamiltonian:
    """One-hot TSP cost on ``m*m`` qubits (x_{c,p} on qubit m*c + p).

    Cost = A sum_c (1 - sum_p x_{c,p})^2 + A sum_p (1 - sum_c x_{c,p})^2
           + sum_p sum_{u != v} d_uv x_{u,p} x_{v,(p+1) mod m}
    (the usual Ising TSP formulation), expanded into Z strings.  Diagonal only.
    """
    dist = np.asarray(dist, dtype=np.float64)
    m = dist.shape[0]
    n = m * m
    poly: dict = {}

    def addp(qs, c):
        key = frozenset(qs)
        poly[key] = poly.get(key, 0.0) + c

    def one_hot_penalty(group):
        # A (1 - sum x)^2 = A (1 - sum x + 2 sum_{i<j} x_i x_j)   (x^2 = x)
        addp((), penalty)
        for q in group:
            addp((q,), -penalty)
        for a, b in combinations(group, 2):
            addp((a, b), 2.0 * penalty)

    for c in range(m):
        one_hot_penalty([m * c + p for p in range(m)])
    for p in range(m):
        one_hot_penalty([m * c + p for c in range(m)])
    for p in range(m):
        for u in range(m):
            for v in range(m):
                if u != v:
                    addp((m * u + p, m * v + (p + 1) % m), dist[u, v])
    H = _poly_to_z_terms(n, poly)
    H.name = f"tsp{m}_n{n}"
    return H


# The four fixed workloads, by what they are (seeds are fixed per workload).
WORKLOADS = ("tfim_chain_n8", "heisenberg_chain_n20", "tfim_5x5_ancilla_n26", "maxcut_3reg_n24")


def workload_hamiltonian(name: str) -> Hamiltonian:
    """The Hamiltonian of a named workload:
    tfim_chain_n8          open TFIM chain, J = h = 1
    heisenberg_chain_n20   open Heisenberg chain, J = 1, fields U[-1, 1] (seed 2)
    tfim_5x5_ancilla_n26   5x5 open TFIM lattice, J = 1, h = 3.04, plus an idle qubit
    maxcut_3reg_n24        weighted MaxCut on a random 3-regular graph (seed 4),
                           weights U[1, 10], transverse mixer 0.7"""
    if name == "tfim_chain_n8":
        return tfim_1d(8, J=1.0, h=1.0)
    if name == "heisenberg_chain_n20":
        rng = _rng(2)
        return heisenberg_1d(20, J=1.0, fields=rng.uniform(-1.0, 1.0, 20))
    if name == "tfim_5x5_ancilla_n26":
        return tfim_2d(5, 5, J=1.0, h=3.04, n_total=26)
    if name == "maxcut_3reg_n24":
        rng = _rng(4)
        edges = random_regular_graph(24, 3, rng)
        w = rng.uniform(1.0, 10.0, len(edges))
        return maxcut(24, edges, w, mixer=0.7)
    raise ValueError(name)


# (t, steps, budget, dtypes, batch) of each named workload
WORKLOAD_RUN = {
    "tfim_chain_n8": dict(t=1.0, steps=10, budget=8, dtypes=("c128",), batch=1),
    "heisenberg_chain_n20": dict(t=2.0, steps=100, budget=16, dtypes=("c128", "c64"), batch=1),
    "tfim_5x5_ancilla_n26": dict(t=1.0, steps=50, budget=16, dtypes=("c64",), batch=1),
    "maxcut_3reg_n24": dict(t=1.0, steps=200, budget=16, dtypes=("c64",), batch=8),
}
