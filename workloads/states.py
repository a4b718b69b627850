"""Seeded initial state vectors (complex, length 2^n, unit norm).

Random-phase states draw u ~ U[0,1) from PCG64(seed) in index order and set
psi[x] = exp(2 pi i u_x) / sqrt(N).  Generation is chunked so that large
states (n = 26: 2^26 amplitudes) do not need a second full-size temporary;
the chunked stream equals the unchunked one (one 64-bit draw per double).
"""
from __future__ import annotations

import numpy as np

_CHUNK = 1 << 22


def _alloc(n: int, dtype):
    return np.zeros(1 << n, dtype=dtype)


def zero_state(n: int, dtype=np.complex128) -> np.ndarray:
    psi = _alloc(n, dtype)
    psi[0] = 1.0
    return psi


def neel_state(n: int, dtype=np.complex128) -> np.ndarray:
    """Basis state with qubit q set iff q is odd (index sum_{q odd} 2^q)."""
    psi = _alloc(n, dtype)
    idx = sum(1 << q for q in range(1, n, 2))
    psi[idx] = 1.0
    return psi


def uniform_state(n: int, dtype=np.complex128) -> np.ndarray:
    N = 1 << n
    return np.full(N, 1.0 / np.sqrt(N), dtype=dtype)


def random_phase_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    N = 1 << n
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(N, dtype=dtype)
    amp = 1.0 / np.sqrt(N)
    for lo in range(0, N, _CHUNK):
        hi = min(N, lo + _CHUNK)
        phi = (2.0 * np.pi) * rng.random(hi - lo)
        out[lo:hi] = amp * (np.cos(phi) + 1j * np.sin(phi))
    return out


def workload_states(name: str, dtype=np.complex128) -> np.ndarray:
    """Initial states of a named workload as a [batch, N] array: |0..0> for
    the n = 8 chain, the Neel state for the n = 20 chain, a random-phase state
    (seed 3) at n = 26, and at n = 24 the uniform state plus seven
    random-phase states (seeds 401..407)."""
    if name == "tfim_chain_n8":
        return zero_state(8, dtype)[None, :]
    if name == "heisenberg_chain_n20":
        return neel_state(20, dtype)[None, :]
    if name == "tfim_5x5_ancilla_n26":
        return random_phase_state(26, 3, dtype)[None, :]
    if name == "maxcut_3reg_n24":
        out = np.empty((8, 1 << 24), dtype=dtype)
        out[0] = uniform_state(24, dtype)
        for b in range(1, 8):
            out[b] = random_phase_state(24, 4 * 100 + b, dtype)
        return out
    raise ValueError(name)
