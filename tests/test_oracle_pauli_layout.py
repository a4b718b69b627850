"""Pins of the oracle's Pauli algebra and DIA layout (CPU only).

Pins: textbook 2x2 Pauli matrices and Kronecker products; the paper's worked
layout example (Section 2.3 table, panel g); the quick-start SpMV (Appendix);
diagonal counts and sparsity printed in Table 'tab:benchmarks'; the storage
arithmetic of Section 3.2 ('Storage implications').
"""
import json
import os

import numpy as np
import pytest

from oracle import dia, pauli
from workloads import hamiltonians as wh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Pauli algebra

def test_single_qubit_matrices_are_textbook():
    X = pauli.dense_pauli("X")
    Y = pauli.dense_pauli("Y")
    Z = pauli.dense_pauli("Z")
    assert np.array_equal(X, [[0, 1], [1, 0]])
    assert np.array_equal(Y, [[0, -1j], [1j, 0]])
    assert np.array_equal(Z, [[1, 0], [0, -1]])
    # Y = i X Z, and the Pauli group relations
    assert np.allclose(Y, 1j * X @ Z)
    assert np.allclose(X @ Y, 1j * Z)


def test_character_k_acts_on_bit_k():
    # X on qubit 0 maps |0> to |1> (index 1); X on qubit 2 maps |0> to |4>
    e0 = np.zeros(8)
    e0[0] = 1
    assert np.argmax(np.abs(pauli.dense_pauli("XII") @ e0)) == 1
    assert np.argmax(np.abs(pauli.dense_pauli("IIX") @ e0)) == 4
    # Z on qubit 1 gives -1 exactly on indices with bit 1 set
    d = np.diag(pauli.dense_pauli("IZI")).real
    assert np.array_equal(d, [1 - 2 * ((x >> 1) & 1) for x in range(8)])


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_mask_action_matches_kron(n):
    rng = np.random.default_rng(10 + n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    for _ in range(20):
        s = "".join(rng.choice(list("IXYZ"), size=n))
        t = pauli.Term(s, 1.0)
        assert np.allclose(pauli.apply_pauli(t, psi), pauli.dense_pauli(s) @ psi, atol=1e-14)


def test_commutation_rule_matches_matrices():
    rng = np.random.default_rng(3)
    for _ in range(200):
        a = "".join(rng.choice(list("IXYZ"), size=3))
        b = "".join(rng.choice(list("IXYZ"), size=3))
        A, B = pauli.dense_pauli(a), pauli.dense_pauli(b)
        comm = np.allclose(A @ B, B @ A)
        assert pauli.commute(pauli.Term(a, 1), pauli.Term(b, 1)) == comm


def test_complex_coefficient_rejected():
    with pytest.raises(ValueError):
        pauli.parse_terms(["XX"], np.array([1.0 + 1e-3j]), 2)
    ts = pauli.parse_terms(["XX"], np.array([1.0 + 1e-15j]), 2)
    assert ts[0].coeff == 1.0
    with pytest.raises(ValueError):
        pauli.parse_terms(["XQ"], [1.0], 2)


# ---------------------------------------------------------------- DIA layout

def test_worked_layout_example():
    g = _gold("layout_4x4.json")
    sym = {s: float(i + 1) for i, s in enumerate("abcdef")}
    sym["0"] = 0.0
    A = np.array([[sym[e] for e in row] for row in g["dense"]])
    D = dia.dense_to_dia(A)
    assert sorted(D) == sorted(g["off"])
    # concatenating the diagonals in the printed order reproduces Val
    val = np.concatenate([D[d] for d in g["off"]]).real
    assert np.array_equal(val, [sym[s] for s in g["val"]])
    # lengths N - |d|
    assert [len(D[d]) for d in g["off"]] == [4, 1, 1]
    assert np.array_equal(dia.dia_to_dense(D, 4).real, A)


def test_quickstart_spmv_and_pauli_form():
    g = _gold("quickstart.json")
    H = np.array(g["H"], dtype=np.complex128)
    psi = np.array(g["psi"], dtype=np.complex128)
    D = dia.dense_to_dia(H)
    assert sorted(D) == [-1, 0, 1]
    assert np.array_equal(dia.dia_spmv(D, psi), np.array(g["y"], dtype=np.complex128))
    pf = g["pauli_form"]
    terms = pauli.parse_terms(pf["terms"], pf["coeffs"], 2)
    assert np.array_equal(pauli.dense_hamiltonian(terms, 2), H)
    offs, nnz = pauli.hamiltonian_offsets(terms, 2)
    assert offs == [-1, 0, 1] and nnz == 6


@pytest.mark.parametrize("N", [1, 5, 16, 37])
def test_dia_spmv_is_dense_matvec(N):
    rng = np.random.default_rng(N)
    A = np.zeros((N, N), dtype=np.complex128)
    for d in rng.choice(np.arange(-(N - 1), N), size=min(2 * N - 1, 6), replace=False):
        for i in range(N - abs(d)):
            r, c = (i, i + d) if d >= 0 else (i - d, i)
            A[r, c] = rng.normal() + 1j * rng.normal()
    x = rng.normal(size=(3, N)) + 1j * rng.normal(size=(3, N))
    D = dia.dense_to_dia(A)
    assert np.allclose(dia.dia_spmv(D, x), x @ A.T, atol=1e-13)
    assert np.array_equal(dia.dia_to_dense(D, N), A)


def test_storage_arithmetic_far_diagonals():
    # A 2^16 operator: a diagonal at offset +-2^15 holds 2^15 complex128
    # entries = 512 KiB; a padded DIA row would hold 2^16 (another 512 KiB).
    N = 1 << 16
    assert dia.dia_nbytes([1 << 15], N, 16) == 512 * 1024
    assert dia.dia_nbytes([-(1 << 15)], N, 16) == 512 * 1024
    assert N * 16 - dia.dia_nbytes([1 << 15], N, 16) == 512 * 1024
    # Table-sized operators: 16 diagonals whose offsets reach +-2^15 stay
    # within 16 * 2^16 * 16 B = 16 MiB, never more.
    offs = [0] + [s * (1 << k) for k in range(8, 16) for s in (1, -1)][:15]
    assert dia.dia_nbytes(offs, N, 16) <= 16 * N * 16


# ---------------------------------------------------------------- Table pins

def _sparsity(nnz, n):
    return 100.0 * (1.0 - nnz / float(1 << (2 * n)))


def test_benchmark_table_tfim():
    for row in _gold("benchmark_table.json")["tfim"]:
        n = row["n"]
        H = wh.tfim_1d(n, 1.0, 1.0, periodic=row.get("periodic", False))
        offs, nnz = pauli.hamiltonian_offsets(pauli.parse_terms(H.strings, H.coeffs, n), n)
        assert len(offs) == row["diagonals"] == 2 * n + 1
        if "sparsity" in row:
            assert round(_sparsity(nnz, n), 4) == row["sparsity"]


def test_benchmark_table_heisenberg():
    for row in _gold("benchmark_table.json")["heisenberg"]:
        n = row["n"]
        H = wh.heisenberg_1d(n, 1.0, fields=None, periodic=row.get("periodic", False))
        terms = pauli.parse_terms(H.strings, H.coeffs, n)
        offs, nnz = pauli.hamiltonian_offsets(terms, n)
        assert len(offs) == row["diagonals"]
        if "sparsity" in row:
            assert round(_sparsity(nnz, n), 4) == row["sparsity"]


def test_benchmark_table_diagonal_only():
    rows = {r["label"]: r for r in _gold("benchmark_table.json")["diagonal_only"]}
    rng = np.random.default_rng(0)
    d = rng.uniform(1, 10, (4, 4))
    d = np.triu(d, 1) + np.triu(d, 1).T
    H = wh.tsp_onehot(d, 20.0)
    offs, nnz = pauli.hamiltonian_offsets(pauli.parse_terms(H.strings, H.coeffs, 16), 16)
    assert len(offs) == rows["TSP-5"]["diagonals"]
    assert round(_sparsity(nnz, 16), 4) == rows["TSP-5"]["sparsity"]
    edges = wh.random_regular_graph(10, 3, np.random.Generator(np.random.PCG64(1)))
    H = wh.maxcut(10, edges, np.ones(len(edges)))
    offs, _ = pauli.hamiltonian_offsets(pauli.parse_terms(H.strings, H.coeffs, 10), 10)
    assert len(offs) == rows["MAXCUT-1"]["diagonals"]


def test_hamiltonian_offsets_match_dense():
    rng = np.random.default_rng(5)
    for _ in range(10):
        n = 4
        strings = ["".join(rng.choice(list("IXYZ"), size=n)) for _ in range(6)]
        terms = pauli.parse_terms(strings, rng.normal(size=6), n)
        H = pauli.dense_hamiltonian(terms, n)
        offs, nnz = pauli.hamiltonian_offsets(terms, n, tol=1e-12)
        assert offs == sorted(dia.dense_to_dia(np.where(np.abs(H) > 1e-12, H, 0)).keys())
        assert nnz == int(np.count_nonzero(np.abs(H) > 1e-12))
