"""GPU parity of the single-propagator pipeline (Alg. 2 SpME from SpGEMM, the
Section 3.1 step search, Alg. 3) against the oracle (scipy.sparse products
with the same stopping rule) and dense algebra."""
import numpy as np
import pytest

from gpu_common import fid, hs_gpu, note
from oracle import dia as odia, pauli as opauli, spme as ospme
from workloads import hamiltonians as wh, states as ws

pytestmark = pytest.mark.gpu


def _dia():
    hs, torch = hs_gpu()
    import paper_2606_16959_amd.dia as hd
    return hd, torch


def _csr_to_dia(M):
    A = M.toarray()
    return odia.dense_to_dia(A)


@pytest.mark.parametrize("which", ["tfim", "heis", "random"])
def test_hamiltonian_diagonals_from_pauli(which):
    hd, torch = _dia()
    if which == "tfim":
        Hw = wh.tfim_1d(8, 1.0, 0.7, periodic=True)
    elif which == "heis":
        Hw = wh.heisenberg_1d(8, 1.0, fields=np.linspace(-1, 1, 8))
    else:
        rng = np.random.default_rng(3)
        strings = ["".join(rng.choice(list("IXYZ"), size=7)) for _ in range(15)]
        Hw = wh.Hamiltonian(7, list(zip(strings, rng.normal(size=15))))
    note(f"dia_from_pauli {which}")
    H = hd.from_pauli(Hw.strings, Hw.coeffs, Hw.n)
    ref = _csr_to_dia(ospme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, Hw.n))
    assert H.offsets == sorted(ref)
    got = H.to_dict()
    for d, v in ref.items():
        assert np.abs(got[d] - v).max() <= 1e-14 * max(1.0, np.abs(v).max())
    if which == "heis":
        assert H.n_diags == 2 * 7 + 1          # XX + YY cancel on +-3 * 2^i
    H.close()


@pytest.mark.parametrize("N,kind", [(1 << 10, "near"), (1 << 12, "far"), (64, "all")])
def test_spgemm_matches_dense_product(N, kind):
    hd, torch = _dia()
    rng = np.random.default_rng(N)
    if kind == "near":
        oa, ob = [-3, -1, 0, 2, 5], [-2, 0, 1, 7]
    elif kind == "far":
        oa, ob = [-(N - 1), -N // 2, 0, 17, N - 3], [-(N // 2), -1, 0, N // 2, N - 1]
    else:
        oa = list(range(-(N - 1), N, 3))
        ob = list(range(-(N - 2), N, 5))

    def rand(offs):
        return {d: rng.normal(size=N - abs(d)) + 1j * rng.normal(size=N - abs(d)) for d in offs}
    Da, Db = rand(oa), rand(ob)
    note(f"spgemm N={N} {kind}")
    A, B = hd.from_dict(Da, N), hd.from_dict(Db, N)
    C = hd.spgemm(A, B)
    ref = odia.dia_to_dense(Da, N) @ odia.dia_to_dense(Db, N)
    got = odia.dia_to_dense(C.to_dict(), N)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # structural offsets: every a + b inside (-N, N)
    assert C.offsets == sorted({a + b for a in oa for b in ob if -N < a + b < N})
    for X in (A, B, C):
        X.close()


@pytest.mark.parametrize("squarings", [-1, 0, 2])
@pytest.mark.parametrize("which,dt", [("tfim", 0.02), ("tfim", 0.3), ("heis", 0.05), ("tsp", 0.5),
                                      ("heis", 0.8)])
def test_spme_matches_oracle(which, dt, squarings):
    hd, torch = _dia()
    if which == "tfim":
        Hw = wh.tfim_1d(8, 1.0, 1.0)
    elif which == "heis":
        Hw = wh.heisenberg_1d(7, 1.0, fields=np.linspace(-0.5, 0.5, 7))
    else:
        rng = np.random.default_rng(1)
        d = rng.uniform(1, 10, (3, 3))
        d = np.triu(d, 1) + np.triu(d, 1).T
        Hw = wh.tsp_onehot(d, 20.0)            # 9 qubits, diagonal
    note(f"spme {which} dt={dt} squarings={squarings}")
    H = hd.from_pauli(Hw.strings, Hw.coeffs, Hw.n)
    U, K = hd.spme(H, dt, squarings=squarings)
    Href = ospme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, Hw.n)
    Uref, Kref, offs = ospme.spme(Href, dt, n_squarings=None if squarings < 0 else squarings)
    assert K == Kref
    assert U.offsets == offs
    N = 1 << Hw.n
    got = odia.dia_to_dense(U.to_dict(), N)
    # the unscaled series at |dt| nu ~ 16 (Heisenberg, dt = 0.8, s = 0) runs
    # to K = 30 and still agrees within the same bar (measured 2e-13)
    assert np.abs(got - Uref.toarray()).max() <= 1e-12
    U.close()
    H.close()


@pytest.mark.parametrize("which,n,budget,t", [("tfim", 5, 11, 1.0), ("tfim", 5, 40, 1.0), ("tfim", 6, 13, 0.5),
                                               ("tfim", 4, 9, 2.0), ("tfim", 8, 200, 0.5), ("heis", 9, 60, 1.0),
                                               ("heis", 8, 400, 0.3)])
def test_step_search_matches_oracle(which, n, budget, t):
    """The search shares powers of H across probes; the oracle recomputes
    each probe's Taylor chain (Alg. 2) from scratch.  The last two cases keep
    two and four terms, so powers up to H^4 are stored."""
    hd, torch = _dia()
    Hw = wh.tfim_1d(n, 1.0, 1.0) if which == "tfim" else wh.heisenberg_1d(n, 1.0, fields=np.linspace(-1, 1, n))
    note(f"estimate_timesteps {which} n={n} budget={budget}")
    H = hd.from_pauli(Hw.strings, Hw.coeffs, n)
    r = hd.estimate_timesteps(H, t, budget)
    assert r == ospme.estimate_timesteps(ospme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, n), t, budget)
    H.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_single_propagator_simulation_matches_oracle(dtype):
    hd, torch = _dia()
    Hw = wh.heisenberg_1d(8, 1.0, fields=np.linspace(-1, 1, 8))
    rng = np.random.default_rng(4)
    psi0 = rng.normal(size=(2, 256)) + 1j * rng.normal(size=(2, 256))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    npd = np.complex128 if dtype == "c128" else np.complex64
    psi = torch.from_numpy(psi0.astype(npd)).cuda()
    note(f"simulate heis n=8 {dtype}")
    steps, K, nd = hd.simulate(Hw.strings, Hw.coeffs, 8, 1.0, psi, budget=40, dtype=dtype)
    Href = ospme.hamiltonian_from_strings(Hw.strings, Hw.coeffs, 8)
    assert steps == ospme.estimate_timesteps(Href, 1.0, 40)
    ref, Kref, offs = ospme.simulate(Href, psi0.astype(npd).astype(np.complex128), 1.0, steps)
    assert K == Kref and nd == len(offs) <= 40
    got = psi.cpu().numpy().astype(np.complex128)
    F = fid(got, ref)
    assert np.all(F >= (1 - 1e-12 if dtype == "c128" else 1 - 1e-6)), F
    if dtype == "c128":
        assert np.abs(got - ref).max() <= 1e-11


def test_diagonal_hamiltonian_single_step_is_exact():
    hd, torch = _dia()
    Hw = wh.maxcut(10, wh.random_regular_graph(10, 3, np.random.Generator(np.random.PCG64(2))),
                   np.linspace(1, 3, 15))
    note("simulate diagonal maxcut n=10")
    psi0 = np.full(1024, 1 / 32.0, dtype=np.complex128)
    psi = torch.from_numpy(psi0.copy()).cuda()
    steps, K, nd = hd.simulate(Hw.strings, Hw.coeffs, 10, 0.8, psi, budget=1)
    assert steps == 1 and K == 0 and nd == 1
    terms = opauli.parse_terms(Hw.strings, Hw.coeffs, 10)
    E = np.real(np.diag(opauli.dense_hamiltonian(terms, 10)))
    assert np.abs(psi.cpu().numpy() - np.exp(-0.8j * E) * psi0).max() <= 1e-14


def test_single_propagator_full_size_sampled_rows():
    """The bench's n = 24 chain (budget 2n + 1): the searched r keeps K = 1,
    so U x = x - i dt H x, the first-order Taylor step, which the oracle
    evaluates on sampled rows (ends, tile edges, random) from the Pauli
    action.  One complex64 SpMV of the open-tile Alg. 3 loop."""
    hd, torch = _dia()
    from oracle import taylor as otay
    n = 24
    Hw = wh.tfim_1d(n, 1.0, 1.0)
    note("single propagator n=24 c64 (full size, sampled rows)")
    H = hd.from_pauli(Hw.strings, Hw.coeffs, n)
    r = hd.estimate_timesteps(H, 1.0, 2 * n + 1)
    U, K = hd.spme(H, 1.0 / r)
    assert K == 1 and U.n_diags == 2 * n + 1
    U64 = U.to_c64()
    U.close()
    H.close()
    x0 = ws.random_phase_state(n, 7, np.complex64)
    psi = torch.from_numpy(x0.copy()).cuda()
    hd.evolve(U64, psi, 1)
    got = psi.cpu().numpy()
    U64.close()
    N = 1 << n
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([np.arange(64), N - 1 - np.arange(64), 8192 * np.arange(1, 64) - 1,
                                     8192 * np.arange(1, 64), rng.integers(0, N, 2048)]))
    terms = opauli.parse_terms(Hw.strings, Hw.coeffs, n)
    ref = otay.step_rows(terms, x0.astype(np.complex128), rows, 1.0 / r, 1)
    assert np.abs(got[rows].astype(np.complex128) - ref).max() <= 2.0 ** -20 * np.abs(x0).max() * 4



@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_ragged_operator_pipeline(dtype):
    """An operator of N = 777 rows (not a power of two, odd): a random
    Hermitian DIA matrix through SpME (with squaring), the Alg. 3 loop and the
    fused Taylor update, against the oracle's sparse products."""
    hd, torch = _dia()
    from oracle import taylor as otay
    import scipy.sparse as sp
    N = 777
    rng = np.random.default_rng(777)
    D = {0: rng.normal(size=N) + 0j}
    for d in (1, 2, 37, 400):
        v = 0.3 * (rng.normal(size=N - d) + 1j * rng.normal(size=N - d))
        D[d], D[-d] = v, np.conj(v)
    note(f"ragged operator N=777 {dtype}")
    H = hd.from_dict(D, N)
    Href = sp.csr_matrix(odia.dia_to_dense(D, N))
    dt = 0.07
    U, K = hd.spme(H, dt)
    Uref, Kref, offs = ospme.spme(Href, dt)
    assert K == Kref and U.offsets == offs
    assert np.abs(odia.dia_to_dense(U.to_dict(), N) - Uref.toarray()).max() <= 1e-12
    npd = np.complex128 if dtype == "c128" else np.complex64
    psi0 = (rng.normal(size=(3, N)) + 1j * rng.normal(size=(3, N)))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    tol = 1e-12 if dtype == "c128" else 2e-6
    # Alg. 3 loop: psi <- U^5 psi
    Ud = U if dtype == "c128" else U.to_c64()
    psi = torch.from_numpy(psi0.astype(npd)).cuda()
    hd.evolve(Ud, psi, 5)
    ref = psi0.astype(npd).astype(np.complex128)
    for _ in range(5):
        ref = (Uref @ ref.T).T
    assert np.abs(psi.cpu().numpy() - ref).max() <= tol
    # fused Taylor update: p_K(-i dt H)^4 psi
    Hd = H if dtype == "c128" else H.to_c64()
    K2 = hd.taylor_terms(H, dt)
    assert K2 == otay.taylor_terms(Href, dt)
    psi = torch.from_numpy(psi0.astype(npd)).cuda()
    hd.taylor_evolve(Hd, psi, dt, K2, 4)
    ref = otay.taylor_evolve(Href, psi0.astype(npd).astype(np.complex128), dt, K2, 4)
    assert np.abs(psi.cpu().numpy() - ref).max() <= tol
    for X in {id(v): v for v in (H, U, Ud, Hd)}.values():
        X.close()
