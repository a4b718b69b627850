"""Pins of the oracle's fused Taylor update (the future-work section's
state-vector form of Alg. 2's series).

Pins: the dense matrix polynomial sum X^k / k! (NumPy matrix powers), the
oracle's own SpME propagator with the same number of terms (a different code
path: sparse matrix products), scipy.linalg.expm within the Taylor remainder,
the K = 1 closed form, minimality of K and of the step count, and
convergence as the tolerance tightens.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import pauli, spme, taylor
from workloads import hamiltonians as wh


def _H(Hw):
    return spme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, Hw.n)


def _state(n, seed, batch=None):
    rng = np.random.default_rng(seed)
    shape = (1 << n,) if batch is None else (batch, 1 << n)
    psi = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return psi / np.linalg.norm(psi, axis=-1, keepdims=True)


@pytest.mark.parametrize("K", [1, 2, 5, 9])
def test_step_is_the_matrix_polynomial(K):
    Hw = wh.heisenberg_1d(5, 1.0, fields=np.linspace(-1, 1, 5))
    H = _H(Hw)
    dt = 0.13
    X = -1j * dt * H.toarray()
    P = sum(np.linalg.matrix_power(X, k) / math.factorial(k) for k in range(K + 1))
    psi = _state(5, 1, batch=3)
    got = taylor.taylor_step(H, psi, dt, K)
    assert np.abs(got - (P @ psi.T).T).max() < 1e-13
    if K == 1:
        assert np.abs(got - (psi - 1j * dt * (H @ psi.T).T)).max() < 1e-15


def test_step_equals_the_spme_propagator_with_the_same_terms():
    Hw = wh.tfim_1d(6, 1.0, 0.8)
    H = _H(Hw)
    dt = 0.05
    U, K, _ = spme.spme(H, dt, n_squarings=0)
    assert K >= 3
    psi = _state(6, 2)
    assert np.abs(taylor.taylor_step(H, psi, dt, K) - U @ psi).max() < 1e-14


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-10])
def test_evolution_is_expm_within_the_remainder(tol):
    Hw = wh.tfim_1d(6, 1.0, 1.0)
    H = _H(Hw)
    t = 1.0
    r = taylor.taylor_steps(H, t)
    dt = t / r
    K = taylor.taylor_terms(H, dt, tol)
    psi = _state(6, 3)
    got = taylor.taylor_evolve(H, psi, dt, K, r)
    exact = sl.expm(-1j * t * H.toarray()) @ psi
    x = abs(dt) * spme.norm_bound(H)
    tail = taylor.remainder_bound(x, K)
    # ||p^r - e^{rX}|| <= r (1 + tail)^(r-1) tail, ||e^X||_2 = 1
    assert np.linalg.norm(got - exact) <= r * (1 + tail) ** (r - 1) * tail + 1e-13
    # the first dropped term's bound is below tol, and K is minimal
    assert x ** (K + 1) / math.factorial(K + 1) < tol
    assert K == 1 or x ** K / math.factorial(K) >= tol


def test_step_count_is_minimal():
    for Hw, t, theta in ((wh.tfim_1d(5, 1.0, 1.0), 1.0, 1.0), (wh.heisenberg_1d(4, 1.0), 2.5, 0.5),
                         (wh.tfim_1d(4, 1.0, 0.3), -0.7, 2.0)):
        H = _H(Hw)
        nu = spme.norm_bound(H)
        r = taylor.taylor_steps(H, t, theta)
        assert abs(t / r) * nu <= theta
        assert r == 1 or abs(t / (r - 1)) * nu > theta


def test_tightening_the_tolerance_converges():
    Hw = wh.heisenberg_1d(5, 1.0, fields=np.linspace(-1, 1, 5))
    H = _H(Hw)
    t, r = 1.0, 4                      # |dt| nu = 5.25: long series
    psi = _state(5, 4)
    exact = sl.expm(-1j * t * H.toarray()) @ psi
    errs = []
    for tol in (1e-1, 1e-2, 1e-3, 1e-4):
        K = taylor.taylor_terms(H, t / r, tol)
        errs.append(np.linalg.norm(taylor.taylor_evolve(H, psi, t / r, K, r) - exact))
    assert all(a > b for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-12, errs


@pytest.mark.parametrize("K", [1, 2, 3])
def test_sampled_rows_equal_the_whole_step(K):
    """The row-sampled form (used at sizes the whole step cannot take) equals
    the sparse-product step on every row."""
    Hw = wh.heisenberg_1d(6, 1.0, fields=np.linspace(-1, 1, 6))
    terms = pauli.parse_terms(Hw.strings, Hw.coeffs, 6)
    psi = _state(6, 5)
    whole = taylor.taylor_step(_H(Hw), psi, 0.07, K)
    rows = np.arange(64)
    assert np.abs(taylor.step_rows(terms, psi, rows, 0.07, K) - whole).max() < 1e-15
