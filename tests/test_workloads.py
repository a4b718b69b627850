"""Input generators: determinism, shapes and the structure each family must have."""
import numpy as np

from workloads import workload_hamiltonian, hamiltonians as wh, states as ws


def test_states_are_unit_and_seeded():
    for psi in (ws.zero_state(5), ws.neel_state(6), ws.uniform_state(7), ws.random_phase_state(9, 3)):
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    assert np.argmax(np.abs(ws.neel_state(20))) == 0xAAAAA
    a = ws.random_phase_state(12, 42)
    b = ws.random_phase_state(12, 42)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, ws.random_phase_state(12, 43))
    assert np.allclose(np.abs(a), 1 / 64.0)


def test_random_phase_chunking_is_invisible(monkeypatch):
    ref = ws.random_phase_state(14, 7)
    monkeypatch.setattr(ws, "_CHUNK", 1000)
    assert np.array_equal(ws.random_phase_state(14, 7), ref)
    c64 = ws.random_phase_state(14, 7, np.complex64)
    assert np.array_equal(c64, ref.astype(np.complex64))


def test_workload_shapes():
    sizes = {"tfim_chain_n8": (8, 15), "heisenberg_chain_n20": (20, 77), "tfim_5x5_ancilla_n26": (26, 65),
             "maxcut_3reg_n24": (24, 61)}
    for k, (n, nt) in sizes.items():
        H = workload_hamiltonian(k)
        assert H.n == n and len(H.terms) == nt
        assert all(len(s) == n for s in H.strings)
    H3 = workload_hamiltonian("tfim_5x5_ancilla_n26")
    assert all(s[25] == "I" for s in H3.strings)          # idle ancilla
    assert sum(1 for s in H3.strings if "X" in s) == 25
    assert all(c == -3.04 for s, c in H3.terms if "X" in s)


def test_regular_graph_is_simple_and_regular():
    rng = np.random.Generator(np.random.PCG64(4))
    edges = wh.random_regular_graph(24, 3, rng)
    assert len(edges) == 36
    deg = np.zeros(24, int)
    for i, j in edges:
        assert i < j
        deg[i] += 1
        deg[j] += 1
    assert np.all(deg == 3)


def test_tsp_is_diagonal_and_penalises_invalid_tours():
    d = np.array([[0, 1, 2, 3], [1, 0, 4, 5], [2, 4, 0, 6], [3, 5, 6, 0]], float)
    H = wh.tsp_onehot(d, 20.0)
    assert H.n == 16 and all(set(s) <= {"I", "Z"} for s in H.strings)

    def energy(x):
        e = 0.0
        for s, c in H.terms:
            sgn = 1
            for q, ch in enumerate(s):
                if ch == "Z" and (x >> q) & 1:
                    sgn = -sgn
            e += c * sgn
        return e
    # the tour 0->1->2->3 (city c at position c): qubit 4c + p set iff p == c
    tour = sum(1 << (4 * c + c) for c in range(4))
    assert abs(energy(tour) - (1 + 4 + 6 + 3)) < 1e-9
    assert energy(0) >= 20.0 - 1e-9
