"""Pins of the oracle's factor grouping, local unitaries and factor matrices.

Pins: dense matrix exponentials from SciPy (a library routine independent of
the oracle's rotation products), brute-force diagonal counts of global
matrices, the Heisenberg-bond closed form, and partitions worked out by hand
from the first-fit rule for the four named workloads.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import dia, factors, pauli
from workloads import workload_hamiltonian
from workloads import hamiltonians as wh


def _terms(strings, coeffs, n):
    return pauli.parse_terms(strings, coeffs, n)


def _global_count(strings, coeffs, n, dt, tol=1e-12):
    """Diagonal count of expm(-i dt H_g) on the full n-qubit space."""
    terms = _terms(strings, coeffs, n)
    U = sl.expm(-1j * dt * pauli.dense_hamiltonian(terms, n))
    return len(dia.dense_to_dia(np.where(np.abs(U) > tol, U, 0)))


@pytest.mark.parametrize("strings,expect", [
    (["XXIIII"], 5),                     # one XX term: offsets 0, +-1, +-3
    (["XIIIII", "IXIIII"], 7),           # {X_q, X_q+1}
    (["IXIIII", "IIXIII", "IIIXII"], 15),  # three adjacent X
    (["XIIIII", "IIXIII"], 9),           # {X_q, X_q+2}
    (["XXIIII", "YYIIII"], 3),           # Heisenberg bond XX+YY: cancels +-3
    (["XXIIII", "YYIIII", "IIXXII", "IIYYII"], 9),
])
def test_group_diagonal_counts(strings, expect):
    n = len(strings[0])
    # equal couplings (as in an XXX chain) so that XX and YY cancel where they should
    coeffs = np.full(len(strings), 0.9)
    dt = 0.05
    assert factors.num_diags(_terms(strings, coeffs, n), dt) == expect
    assert _global_count(strings, coeffs, n, dt) == expect


def test_local_unitary_is_expm_of_group():
    rng = np.random.default_rng(11)
    n = 4
    # a commuting group with Y and Z content
    strings = ["XXII", "YYII", "ZZII", "IIXZ"]
    coeffs = rng.uniform(-1, 1, 4)
    terms = _terms(strings, coeffs, n)
    bits, L = factors.local_unitary(terms, 0.3)
    assert bits == [0, 1, 2, 3]
    Hg = pauli.dense_hamiltonian(terms, n)
    assert np.allclose(L, sl.expm(-0.3j * Hg), atol=1e-14)


def test_local_unitary_on_sparse_support():
    # support {1, 3} of a 5-qubit system: L is 4x4 on local bits (q1, q3)
    terms = _terms(["IXIXI", "IZIZI"], [0.4, -0.9], 5)
    bits, L = factors.local_unitary(terms, 0.2)
    assert bits == [1, 3]
    loc = _terms(["XX", "ZZ"], [0.4, -0.9], 2)
    assert np.allclose(L, sl.expm(-0.2j * pauli.dense_hamiltonian(loc, 2)), atol=1e-14)


def test_heisenberg_bond_closed_form():
    # exp(-i t (XX+YY+ZZ)): e^{-it} on |00>,|11>; on span{|01>,|10>}
    # e^{it}(cos 2t I - i sin 2t X)
    t = 0.37
    terms = _terms(["XX", "YY", "ZZ"], [1.0, 1.0, 1.0], 2)
    part = factors.first_fit(terms, 16, t)
    assert part.diag == [2] and part.groups == [[0, 1]]
    U = np.eye(4, dtype=complex)
    for f in part.factor_list():
        U = factors.factor_dense(terms, part, f, 2, t) @ U
    ref = np.zeros((4, 4), dtype=complex)
    ref[0, 0] = ref[3, 3] = np.exp(-1j * t)
    blk = np.exp(1j * t) * np.array([[np.cos(2 * t), -1j * np.sin(2 * t)],
                                      [-1j * np.sin(2 * t), np.cos(2 * t)]])
    ref[1:3, 1:3] = blk
    assert np.allclose(U, ref, atol=1e-15)


@pytest.mark.parametrize("cfg", list(wh.WORKLOADS))
def test_workload_partitions_by_hand(cfg):
    H = workload_hamiltonian(cfg)
    run = wh.WORKLOAD_RUN[cfg]
    terms = _terms(H.strings, H.coeffs, H.n)
    part = factors.first_fit(terms, run["budget"], run["t"] / run["steps"])
    kinds = [pauli.Term(s, 1).is_diagonal for s in H.strings]
    assert part.diag == [i for i, k in enumerate(kinds) if k]
    if cfg == "tfim_chain_n8":
        # ZZ bonds 0..6 then X_0..X_7 at indices 7..14; budget 8 -> pairs
        assert part.groups == [[7, 8], [9, 10], [11, 12], [13, 14]]
    elif cfg == "heisenberg_chain_n20":
        # per bond i: XX at 3i, YY at 3i+1; bonds {0,2},{1,3},{4,6},...,{16,18},{17}
        pairs = []
        for base in range(0, 16, 4):
            pairs += [[base, base + 2], [base + 1, base + 3]]
        pairs += [[16, 18], [17]]
        assert part.groups == [[3 * b + o for b in p for o in (0, 1)] for p in pairs]
    elif cfg == "tfim_5x5_ancilla_n26":
        # 40 ZZ bonds, then X_q at 40 + q; groups of three consecutive X
        assert part.groups == [[40 + q for q in range(s, min(s + 3, 25))] for s in range(0, 25, 3)]
    else:
        # identity + 36 ZZ terms, then X_q at 37 + q
        assert part.groups == [[37 + q for q in range(s, s + 3)] for s in range(0, 24, 3)]
    fl = part.factor_list()
    counts = [len(factors.factor_offsets(terms, f, run["t"] / run["steps"])) for f in fl]
    expect = {"tfim_chain_n8": [7] * 4, "heisenberg_chain_n20": [9] * 9 + [3],
              "tfim_5x5_ancilla_n26": [15] * 8 + [3], "maxcut_3reg_n24": [15] * 8}[cfg]
    assert counts == expect
    assert fl[0][0] is True            # the diagonal factor rides on the first group


def test_budget_error_and_reading_of_single_term():
    terms = _terms(["XXX"], [1.0], 3)       # 2^3 + 1 = 9 diagonals
    assert factors.num_diags(terms, 0.1) == 9
    with pytest.raises(factors.BudgetError):
        factors.first_fit(terms, 8, 0.1)
    assert factors.first_fit(terms, 9, 0.1).groups == [[0]]


def test_noncommuting_terms_never_share_a_group():
    H = wh.heisenberg_1d(6, 1.0, fields=None)
    terms = _terms(H.strings, H.coeffs, 6)
    part = factors.first_fit(terms, 64, 0.1)
    for g in part.groups:
        for a in g:
            for b in g:
                assert pauli.commute(terms[a], terms[b])
    allidx = sorted(part.diag + [k for g in part.groups for k in g])
    assert allidx == list(range(len(terms)))


@pytest.mark.parametrize("cfg", ["tfim_chain_n8"])
def test_factor_dense_is_expm_of_factor_hamiltonian(cfg):
    H = workload_hamiltonian(cfg)
    run = wh.WORKLOAD_RUN[cfg]
    dt = run["t"] / run["steps"]
    terms = _terms(H.strings, H.coeffs, H.n)
    part = factors.first_fit(terms, run["budget"], dt)
    HD = pauli.dense_hamiltonian([terms[k] for k in part.diag], H.n)
    for has_diag, g in part.factor_list():
        Hg = pauli.dense_hamiltonian([terms[k] for k in g], H.n)
        ref = sl.expm(-1j * dt * Hg)
        if has_diag:                    # D is applied first: U_1 D
            ref = ref @ sl.expm(-1j * dt * HD)
        U = factors.factor_dense(terms, part, (has_diag, g), H.n, dt)
        assert np.allclose(U, ref, atol=1e-14)
        # its DIA offsets are exactly the planned offsets
        offs = sorted(dia.dense_to_dia(U).keys())
        assert offs == factors.factor_offsets(terms, (has_diag, g), dt)


def test_factor_entries_match_dense_on_every_diagonal():
    H = wh.heisenberg_1d(6, 1.0, fields=np.linspace(-0.5, 0.7, 6))
    terms = _terms(H.strings, H.coeffs, 6)
    dt = 0.07
    part = factors.first_fit(terms, 16, dt)
    for f in part.factor_list():
        U = factors.factor_dense(terms, part, f, 6, dt)
        for d in factors.factor_offsets(terms, f, dt):
            r = np.arange(max(0, -d), min(64, 64 - d))
            assert np.array_equal(factors.factor_entries(terms, part, f, 6, dt, r, d), U[r, r + d])
