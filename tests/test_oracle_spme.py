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


@pytest.mark.parametrize("dt", [1e-3, 0.02, 0.2, 1.5])
@pytest.mark.parametrize("squared", [False, True])
def test_taylor_is_expm_within_the_remainder(dt, squared):
    Hw = wh.tfim_1d(6, 1.0, 1.0)
    H = _H(Hw)
    s = spme.squarings(H, dt) if squared else 0
    U, K, offs = spme.spme(H, dt, n_squarings=None if squared else 0)
    ref = sl.expm(-1j * dt * H.toarray())
    norm_y = dt * np.abs(Hw.coeffs).sum() / 2 ** s       # >= ||X / 2^s||_2
    tail = sum(norm_y ** k / math.factorial(k) for k in range(K + 1, K + 60))
    # ||A^m - B^m|| <= m (1 + tail)^(m-1) tail for ||B|| = 1, ||A - B|| <= tail
    m = 2 ** s
    assert np.linalg.norm(U.toarray() - ref, 2) <= m * (1 + tail) ** (m - 1) * tail + 1e-13
    assert K >= 1
    # structural offsets contain every nonzero diagonal of U
    assert set(odia.dense_to_dia(np.where(np.abs(U.toarray()) > 0, 1, 0)).keys()) <= set(offs)
    if squared and dt == 1.5:
        assert s >= 4 and len(offs) > 2 * 6 + 1


def test_norm_bound_and_squaring_count():
    """nu(H) is the sum of per-diagonal maxima (brute force over the dense
    matrix) and bounds the 1-, inf- and 2-norms; s is the smallest count that
    brings |dt| nu / 2^s to 1/2 or below."""
    rng = np.random.default_rng(8)
    for Hw in (wh.tfim_1d(5, 1.0, 0.7), wh.heisenberg_1d(5, 1.0, fields=np.linspace(-1, 1, 5)),
               wh.Hamiltonian(4, [("".join(rng.choice(list("IXYZ"), 4)), c) for c in rng.normal(size=9)])):
        H = _H(Hw)
        A = H.toarray()
        N = A.shape[0]
        brute = sum(np.abs(np.diagonal(A, d)).max() for d in range(-N + 1, N) if np.abs(np.diagonal(A, d)).max() > 0)
        nu = spme.norm_bound(H)
        assert abs(nu - brute) <= 1e-13 * brute
        assert nu >= max(np.linalg.norm(A, 1), np.linalg.norm(A, np.inf), np.linalg.norm(A, 2)) - 1e-12
        for dt in (1e-4, 0.01, 0.3, 2.0, -0.7):
            s = spme.squarings(H, dt)
            assert abs(dt) * nu / 2 ** s <= 0.5
            assert s == 0 or abs(dt) * nu / 2 ** (s - 1) > 0.5


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
    # plain Alg. 2 and the scaled-and-squared form (s = 2 here); squaring
    # multiplies the truncation error by up to 2^s
    for n_sq, floor in ((0, 1e-8), (None, 1e-7)):
        errs = []
        for tol in (1e-4, 1e-6, 1e-9):
            psi, K, _ = spme.simulate(H, psi0, 1.0, 20, tol=tol, n_squarings=n_sq)
            errs.append(np.linalg.norm(psi - exact))
        assert errs[0] > errs[1] > errs[2] and errs[2] < floor, (n_sq, errs)
    assert spme.squarings(H, 1.0 / 20) == 2
