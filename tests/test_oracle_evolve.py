"""Pins of the oracle's Trotterized evolution (CPU only).

Pins: products of SciPy matrix exponentials of the factor Hamiltonians
(n <= 8), the exact e^{-iHt} for commuting Hamiltonians, two closed forms
(MaxCut cost phases; TFIM with J = 0), first-order error scaling (global
error ~ 1/r, one-step error ~ dt^2) under the commutator bound of Childs et
al. (PRX 11, 011020, 2021), and norm conservation.  A few planted mistakes
in copies of the oracle confirm that the pins catch them.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle.evolve as oev
from oracle import factors, metrics, pauli
from workloads import workload_hamiltonian, hamiltonians as wh, states as ws


def _setup(H, budget, dt):
    terms = pauli.parse_terms(H.strings, H.coeffs, H.n)
    return terms, factors.first_fit(terms, budget, dt)


def _expm_product(terms, part, n, dt, r, psi0):
    """(U_m ... U_1 D)^r psi0 with every factor from scipy.linalg.expm."""
    step = np.eye(1 << n, dtype=np.complex128)
    if part.diag:
        step = sl.expm(-1j * dt * pauli.dense_hamiltonian([terms[k] for k in part.diag], n)) @ step
    for g in part.groups:
        step = sl.expm(-1j * dt * pauli.dense_hamiltonian([terms[k] for k in g], n)) @ step
    return np.linalg.matrix_power(step, r) @ psi0


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def _heis(n=6):
    return wh.heisenberg_1d(n, 1.0, fields=np.linspace(-0.8, 0.6, n))


def test_c_oracle_matches_numpy_twin(oracle_lib):
    rng = np.random.default_rng(1)
    n = 6
    strings = ["".join(rng.choice(list("IXYZ"), size=n)) for _ in range(14)]
    H = wh.Hamiltonian(n, list(zip(strings, rng.normal(size=14))))
    terms, part = _setup(H, 64, 0.05)
    psi = np.stack([_rand_state(n, 2), _rand_state(n, 3)])
    a = oev.evolve(terms, part, psi, n, 0.05, 5)
    b = oev.evolve_np(terms, part, psi, n, 0.05, 5)
    assert np.abs(a - b).max() < 1e-14


@pytest.mark.parametrize("which", ["tfim8", "heis", "random"])
def test_trotter_product_equals_expm_product(oracle_lib, which):
    if which == "tfim8":
        H, budget, dt, r = workload_hamiltonian("tfim_chain_n8"), 8, 0.1, 10
    elif which == "heis":
        H, budget, dt, r = _heis(6), 16, 0.13, 7
    else:
        rng = np.random.default_rng(7)
        strings = ["".join(rng.choice(list("IXYZ"), size=5)) for _ in range(12)]
        H, budget, dt, r = wh.Hamiltonian(5, list(zip(strings, rng.normal(size=12)))), 32, 0.09, 6
    terms, part = _setup(H, budget, dt)
    psi0 = _rand_state(H.n, 5)
    got = oev.evolve(terms, part, psi0, H.n, dt, r)
    ref = _expm_product(terms, part, H.n, dt, r, psi0)
    assert np.abs(got - ref).max() < 1e-12


def _cut_value(n, edges, w):
    x = np.arange(1 << n)
    cut = np.zeros(1 << n)
    for (i, j), wij in zip(edges, w):
        cut += wij * (((x >> i) & 1) != ((x >> j) & 1))
    return cut


@pytest.mark.parametrize("r", [1, 3, 10])
def test_maxcut_cost_phases_closed_form(oracle_lib, r):
    # H_C|x> = cut(x)|x>: from the uniform state psi_t[x] = e^{-i t cut(x)}/sqrt(N)
    n = 10
    rng = np.random.Generator(np.random.PCG64(9))
    edges = wh.random_regular_graph(n, 3, rng)
    w = rng.uniform(1, 10, len(edges))
    H = wh.maxcut(n, edges, w)
    t = 0.7
    terms, part = _setup(H, 16, t / r)
    assert part.groups == []
    got = oev.evolve(terms, part, ws.uniform_state(n), n, t / r, r)
    ref = np.exp(-1j * t * _cut_value(n, edges, w)) / np.sqrt(1 << n)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("r", [1, 4])
def test_tfim_without_coupling_closed_form(oracle_lib, r):
    # H = -h sum X from |0..0>: amplitude cos(ht)^(n-|x|) (i sin(ht))^|x|
    n, h, t = 9, 1.3, 0.8
    H = wh.tfim_1d(n, J=0.0, h=h)
    H.terms = [(s, c) for s, c in H.terms if "X" in s]
    terms, part = _setup(H, 16, t / r)
    got = oev.evolve(terms, part, ws.zero_state(n), n, t / r, r)
    w = np.array([bin(x).count("1") for x in range(1 << n)])
    ref = np.cos(h * t) ** (n - w) * (1j * np.sin(h * t)) ** w
    assert np.abs(got - ref).max() < 1e-13


def test_commuting_hamiltonian_is_exact_for_any_r(oracle_lib):
    n, t = 8, 1.1
    H = wh.tsp_onehot(np.array([[0, 2.0], [2.0, 0]]), 3.0)   # 4 qubits, diagonal
    H.n = 4
    psi0 = _rand_state(4, 8)
    exact = sl.expm(-1j * t * pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, 4), 4)) @ psi0
    for r in (1, 2, 9):
        terms, part = _setup(H, 16, t / r)
        assert np.abs(oev.evolve(terms, part, psi0, 4, t / r, r) - exact).max() < 1e-13
    # an off-diagonal but commuting family (X-type strings only), split over
    # several factors by a tight budget: still exact for any r
    H2 = wh.Hamiltonian(n, [("X" * 2 + "I" * (n - 2), 0.3), ("I" * 2 + "XX" + "I" * (n - 4), -0.4),
                            ("XIXIIIII", 0.2)])
    psi0 = _rand_state(n, 4)
    exact = sl.expm(-1j * t * pauli.dense_hamiltonian(pauli.parse_terms(H2.strings, H2.coeffs, n), n)) @ psi0
    for r in (1, 5):
        terms, part = _setup(H2, 5, t / r)
        assert len(part.groups) >= 2
        assert np.abs(oev.evolve(terms, part, psi0, n, t / r, r) - exact).max() < 1e-13


def _commutator_bound(terms, part, n, t, r):
    mats = []
    if part.diag:
        mats.append(pauli.dense_hamiltonian([terms[k] for k in part.diag], n))
    for g in part.groups:
        mats.append(pauli.dense_hamiltonian([terms[k] for k in g], n))
    s = 0.0
    for j in range(len(mats)):
        for k in range(j + 1, len(mats)):
            s += np.linalg.norm(mats[k] @ mats[j] - mats[j] @ mats[k], 2)
    return t * t / (2 * r) * s


@pytest.mark.parametrize("name", ["tfim", "heis"])
def test_first_order_error_scaling_and_bound(oracle_lib, name):
    n, t = 8, 1.0
    H = wh.tfim_1d(n, 1.0, 1.0) if name == "tfim" else _heis(n)
    Hd = pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, n), n)
    psi0 = _rand_state(n, 12)
    exact = sl.expm(-1j * t * Hd) @ psi0
    errs = []
    for r in (16, 32, 64, 128):
        terms, part = _setup(H, 16, t / r)
        got = oev.evolve(terms, part, psi0, n, t / r, r)
        e = np.linalg.norm(got - exact)
        assert e <= _commutator_bound(terms, part, n, t, r)
        errs.append(e)
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.8 < q < 2.2 for q in ratios), ratios
    assert abs(ratios[-1] - 2.0) < 0.05
    # one-step (local) error falls like dt^2
    loc = []
    for dt in (0.04, 0.02, 0.01):
        terms, part = _setup(H, 16, dt)
        one = oev.evolve(terms, part, psi0, n, dt, 1)
        loc.append(np.linalg.norm(one - sl.expm(-1j * dt * Hd) @ psi0))
    assert 3.6 < loc[0] / loc[1] < 4.4 and 3.6 < loc[1] / loc[2] < 4.4


def test_norm_is_conserved(oracle_lib):
    H = wh.heisenberg_1d(16, 1.0, fields=np.linspace(-1, 1, 16))
    terms, part = _setup(H, 16, 0.02)
    psi = oev.evolve(terms, part, ws.neel_state(16), 16, 0.02, 60)
    assert abs(metrics.norm2(psi) - 1.0) < 1e-12
    assert metrics.fidelity(psi, psi) == pytest.approx(1.0, abs=1e-15)


def test_batch_equals_single_states(oracle_lib):
    H = _heis(7)
    terms, part = _setup(H, 16, 0.1)
    psi = np.stack([_rand_state(7, s) for s in range(3)])
    both = oev.evolve(terms, part, psi, 7, 0.1, 4)
    for b in range(3):
        assert np.array_equal(both[b], oev.evolve(terms, part, psi[b], 7, 0.1, 4))


def test_fidelity_definition():
    rng = np.random.default_rng(0)
    a = rng.normal(size=16) + 1j * rng.normal(size=16)
    assert metrics.fidelity(a, 3.0 * np.exp(0.4j) * a) == pytest.approx(1.0, abs=1e-15)
    e0, e1 = np.eye(2)[0].astype(complex), np.eye(2)[1].astype(complex)
    assert metrics.fidelity(e0, e1) == 0.0
    plus = (e0 + e1) / np.sqrt(2)
    assert metrics.fidelity(e0, plus) == pytest.approx(0.5, abs=1e-15)


# ------------------------------------------------- planted mistakes are caught

def _pin_holds(terms, part, n, dt, r, psi0, evolve_fn):
    return np.abs(evolve_fn(terms, part, psi0, n, dt, r) - _expm_product(terms, part, n, dt, r, psi0)).max() < 1e-12


@pytest.mark.parametrize("mutant", ["drop_y_phase", "sign_of_rotation", "diag_last", "drop_a_term"])
def test_planted_mistakes_fail_the_pins(monkeypatch, mutant):
    H = _heis(5)
    dt, r = 0.11, 3
    terms, part = _setup(H, 16, dt)
    psi0 = _rand_state(5, 1)
    assert _pin_holds(terms, part, 5, dt, r, psi0, oev.evolve_np)
    if mutant == "drop_y_phase":
        real_apply = pauli.apply_pauli

        def no_phase(term, psi):
            return real_apply(term, psi) / (1j) ** term.ny
        monkeypatch.setattr(oev, "apply_pauli", no_phase)
        fn = oev.evolve_np
    elif mutant == "sign_of_rotation":
        def fn(terms, part, psi0, n, dt, r):
            return oev.evolve_np(terms, part, psi0, n, -dt, r)
    elif mutant == "diag_last":
        def fn(terms, part, psi0, n, dt, r):
            out = psi0
            D = factors.diag_phase(terms, part.diag, n, dt)
            for _ in range(r):
                out = oev.evolve_np(terms, factors.Partition([], part.groups), out, n, dt, 1) * D
            return out
    else:
        def fn(terms, part, psi0, n, dt, r):
            return oev.evolve_np(terms, factors.Partition(part.diag, [g[:-1] or g for g in part.groups]),
                                 psi0, n, dt, r)
    assert not _pin_holds(terms, part, 5, dt, r, psi0, fn)


# ------------------------------------------------- higher-order products

def _expm_sequence(terms, part, n, dt, r, psi0, order):
    step = np.eye(1 << n, dtype=np.complex128)
    for g, h in oev.product_sequence(part, dt, order):
        idx = part.diag if g < 0 else part.groups[g]
        step = sl.expm(-1j * h * pauli.dense_hamiltonian([terms[k] for k in idx], n)) @ step
    return np.linalg.matrix_power(step, r) @ psi0


def test_product_sequences_are_symmetric():
    part = factors.Partition([0, 1], [[2], [3, 4], [5]])
    s2 = oev.product_sequence(part, 0.1, 2)
    assert [g for g, _ in s2] == [-1, 0, 1, 2, 1, 0, -1]
    assert [h for _, h in s2] == [0.05, 0.05, 0.05, 0.1, 0.05, 0.05, 0.05]
    s4 = oev.product_sequence(part, 0.1, 4)
    assert len(s4) == 5 * len(s2)
    p = oev.SUZUKI_P
    assert abs(4 * p + (1 - 4 * p) - 1.0) < 1e-15
    # the total time each factor receives per step is dt
    for seq in (s2, s4):
        for g in (-1, 0, 1, 2):
            assert abs(sum(h for q, h in seq if q == g) - 0.1) < 1e-15


@pytest.mark.parametrize("order", [2, 4])
def test_merged_neighbours_give_the_same_product(order):
    """Combining same-generator neighbours, within a step and where steps
    meet, leaves S(dt)^r unchanged (exp(aG) exp(bG) = exp((a+b)G))."""
    H = _heis(4)
    dt, r = 0.23, 3
    terms, part = _setup(H, 16, dt)
    one = oev.product_sequence(part, dt, order)
    whole = oev.merge_adjacent(one * r)
    L = len(part.groups) + (1 if part.diag else 0)
    assert L >= 2
    # S4 meets itself four times inside a step; every step boundary joins once
    inner = 4 if order == 4 else 0
    assert len(oev.merge_adjacent(one)) == len(one) - inner
    assert len(whole) == r * (len(one) - inner) - (r - 1)
    assert all(a[0] != b[0] for a, b in zip(whole, whole[1:]))
    # the total time of every factor is preserved
    for g in [-1] + list(range(len(part.groups))):
        assert abs(sum(h for q, h in whole if q == g) - r * dt) < 1e-14
    psi0 = _rand_state(4, 5)
    ref = _expm_sequence(terms, part, 4, dt, r, psi0, order)
    U = np.eye(16, dtype=np.complex128)
    for g, h in whole:
        idx = part.diag if g < 0 else part.groups[g]
        U = sl.expm(-1j * h * pauli.dense_hamiltonian([terms[k] for k in idx], 4)) @ U
    assert np.abs(U @ psi0 - ref).max() < 1e-13


@pytest.mark.parametrize("order", [2, 4])
def test_higher_order_equals_expm_products_and_numpy_twin(oracle_lib, order):
    H = _heis(5)
    dt, r = 0.17, 3
    terms, part = _setup(H, 16, dt)
    psi0 = _rand_state(5, 3)
    got = oev.evolve(terms, part, psi0, 5, dt, r, order=order)
    assert np.abs(got - _expm_sequence(terms, part, 5, dt, r, psi0, order)).max() < 1e-12
    assert np.abs(got - oev.evolve_np(terms, part, psi0, 5, dt, r, order=order)).max() < 1e-13


@pytest.mark.parametrize("order,ratio,rs", [(2, 4.0, (8, 16, 32, 64)), (4, 16.0, (4, 8, 16, 32))])
def test_higher_order_error_scaling(oracle_lib, order, ratio, rs):
    n, t = 7, 1.0
    H = wh.tfim_1d(n, 1.0, 1.0)
    Hd = pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, n), n)
    psi0 = _rand_state(n, 21)
    exact = sl.expm(-1j * t * Hd) @ psi0
    errs = []
    for r in rs:
        terms, part = _setup(H, 8, t / r)
        errs.append(np.linalg.norm(oev.evolve(terms, part, psi0, n, t / r, r, order=order) - exact))
    q = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert abs(q[-1] - ratio) < 0.1 * ratio, q
    # and far below the first-order error at the same r
    terms, part = _setup(H, 8, t / rs[-1])
    e1 = np.linalg.norm(oev.evolve(terms, part, psi0, n, t / rs[-1], rs[-1]) - exact)
    assert errs[-1] < e1 / 10


# ------------------------------------------------------------------ exact e^{-iHt} by eigendecomposition (n = 10)

def test_eigh_propagator_is_unitary_and_agrees_with_expm():
    """The eigendecomposition reference against an independent routine
    (scipy's Pade scaling-and-squaring) and unitarity."""
    n = 6
    H = wh.heisenberg_1d(n, 1.0, fields=np.linspace(-0.8, 0.6, n))
    Hd = pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, n), n)
    U = pauli.dense_propagator(Hd, 0.7)
    assert np.abs(U - sl.expm(-0.7j * Hd)).max() < 1e-12
    assert np.abs(U.conj().T @ U - np.eye(1 << n)).max() < 1e-12


def test_commuting_hamiltonian_matches_eigh_propagator_n10(oracle_lib):
    """Disjoint Heisenberg bonds with equal Z fields on both qubits of a bond:
    every term commutes with D's fields and with the other bonds, so the
    Trotter product is exact for any r (Eq. 4 with commuting H_j equals Eq. 2)."""
    n, t = 10, 0.9
    terms_s = []
    for b in range(n // 2):
        i = 2 * b
        for p in "XYZ":
            s = ["I"] * n
            s[i] = s[i + 1] = p
            terms_s.append(("".join(s), 0.7 + 0.1 * b))
        hb = -0.5 + 0.3 * b
        for q in (i, i + 1):
            s = ["I"] * n
            s[q] = "Z"
            terms_s.append(("".join(s), hb))
    H = wh.Hamiltonian(n, terms_s)
    Hd = pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, n), n)
    psi0 = _rand_state(n, 21)
    exact = pauli.dense_propagator(Hd, t) @ psi0
    for r in (1, 3, 8):
        terms, part = _setup(H, 16, t / r)
        assert len(part.groups) >= 2
        assert np.abs(oev.evolve(terms, part, psi0, n, t / r, r) - exact).max() < 1e-12


@pytest.mark.parametrize("name", ["tfim", "heis"])
def test_first_order_converges_to_eigh_propagator_n10(oracle_lib, name):
    """n = 10: the oracle's product against exp(-iHt) from the dense
    eigendecomposition: global error ratio 2 per doubling of r (first order)."""
    n, t = 10, 1.0
    H = wh.tfim_1d(n, 1.0, 1.0) if name == "tfim" else _heis(n)
    Hd = pauli.dense_hamiltonian(pauli.parse_terms(H.strings, H.coeffs, n), n)
    psi0 = _rand_state(n, 31)
    exact = pauli.dense_propagator(Hd, t) @ psi0
    errs = []
    for r in (32, 64, 128, 256):
        terms, part = _setup(H, 16, t / r)
        errs.append(np.linalg.norm(oev.evolve(terms, part, psi0, n, t / r, r) - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.85 < q < 2.15 for q in ratios), ratios
    assert errs[-1] < 0.05
