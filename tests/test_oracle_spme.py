"""Pins of the oracle's truncated-Taylor SpME, step search and Alg. 3 loop.

Pins: scipy.linalg.expm with the Taylor remainder bound, the exact diagonal
case, dense nonzero patterns against the structural offset sets, brute-force
minimality of the step count, and convergence of the simulated state to the
exact e^{-iHt} psi as the tolerance tightens.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import dia as odia, pauli, spme
from workloads import hamiltonians as wh


def _H(Hw):
    return spme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, Hw.n)


def test_hamiltonian_csr_is_dense_sum():
    Hw = wh.heisenberg_1d(5, 1.0, fields=np.linspace(-1, 1, 5))
    terms = pauli.parse_terms(Hw.strings, Hw.coeffs, 5)
    assert np.allclose(_H(Hw).toarray(), pauli.dense_hamiltonian(terms, 5), atol=1e-15)
    # XX + YY cancellation leaves 2 * bonds + 1 diagonals
    assert len(spme.offsets_of(_H(Hw))) == 2 * 4 + 1


@pytest.mark.parametrize("dt", [1e-3, 0.02, 0.2])
def test_taylor_is_expm_within_the_remainder(dt):
    Hw = wh.tfim_1d(6, 1.0, 1.0)
    H = _H(Hw)
    U, K, offs = spme.spme(H, dt)
    ref = sl.expm(-1j * dt * H.toarray())
    norm_x = dt * np.abs(Hw.coeffs).sum()          # >= ||X||_2
    tail = sum(norm_x ** k / math.factorial(k) for k in range(K + 1, K + 40))
    assert np.abs(U.toarray() - ref).max() <= tail + 1e-15
    # the first dropped term was below the tolerance
    assert K >= 1
    # structural offsets contain every nonzero diagonal of U
    assert set(odia.dense_to_dia(np.where(np.abs(U.toarray()) > 0, 1, 0)).keys()) <= set(offs)


def test_first_order_offsets_are_hamiltonian_offsets():
    Hw = wh.tfim_1d(7, 1.0, 1.0)
    H = _H(Hw)
    # small dt: T_1 ~ 1e-5 is kept, T_2 ~ 1e-10 is below the tolerance, so
    # U = I + X and its diagonals are those of H (2n+1)
    U, K, offs = spme.spme(H, 1e-5)
    assert K == 1 and offs == spme.offsets_of(H) and len(offs) == 15


def test_diagonal_hamiltonian_is_exact():
    Hw = wh.tsp_onehot(np.array([[0, 2.0], [2, 0]]), 3.0)
    H = _H(wh.Hamiltonian(4, Hw.terms))
    U, K, offs = spme.spme(H, 0.37)
    assert K == 0 and offs == [0]
    assert np.allclose(U.toarray(), sl.expm(-0.37j * H.toarray()), atol=1e-15)
    assert spme.estimate_timesteps(H, 1.0, 1) == 1


@pytest.mark.parametrize("budget", [9, 17, 40])
def test_step_search_is_minimal(budget):
    Hw = wh.tfim_1d(4, 1.0, 1.0)
    H = _H(Hw)
    t = 1.0
    r = spme.estimate_timesteps(H, t, budget)
    assert spme.num_diags(H, t, r) <= budget
    # brute force: no smaller r meets the budget
    for q in range(1, r):
        assert spme.num_diags(H, t, q) > budget
    # the predicate is monotone on this range
    flags = [spme.num_diags(H, t, q) <= budget for q in range(1, 2 * r + 2)]
    assert flags == sorted(flags)


def test_simulation_converges_to_exact_evolution():
    Hw = wh.heisenberg_1d(5, 1.0, fields=np.linspace(-1, 1, 5))
    H = _H(Hw)
    rng = np.random.default_rng(0)
    psi0 = rng.normal(size=32) + 1j * rng.normal(size=32)
    psi0 /= np.linalg.norm(psi0)
    exact = sl.expm(-1j * 1.0 * H.toarray()) @ psi0
    errs = []
    for tol in (1e-4, 1e-6, 1e-9):
        psi, K, _ = spme.simulate(H, psi0, 1.0, 20, tol=tol)
        errs.append(np.linalg.norm(psi - exact))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8
