"""Whole evolutions of small states in one launch (one workgroup per state,
the state in LDS, every factor of every step): the same values as one launch
per fused run and step (the tile path, selected with HAMSIM_WHOLE_MAX_ROWS=0),
and the FP64 oracle (Eq. 4 repeated r times, the loop of Alg. 3).  The cap
is raised to the kernel's capacity (8192 / 4096 rows) so that every case
runs it."""
import numpy as np
import pytest

from gpu_common import env, fid, hs_gpu, note, oracle_run
from workloads import hamiltonians as wh, workload_hamiltonian, states as ws

pytestmark = pytest.mark.gpu


def _ham(kind, n):
    if kind == "tfim":
        return wh.tfim_1d(n, 1.0, 0.8)
    if kind == "heis":
        return wh.heisenberg_1d(n, 1.0, fields=np.linspace(-0.9, 0.7, n))
    rng = np.random.Generator(np.random.PCG64(n))
    m = n - (n % 2)
    edges = wh.random_regular_graph(m, 3, rng)
    H = wh.maxcut(m, edges, rng.uniform(1.0, 10.0, len(edges)), mixer=0.7)
    H.n = m
    return H


CASES = [("tfim", 2, "c128", 1, 1, 3), ("tfim", 3, "c64", 1, 3, 1), ("heis", 5, "c128", 2, 2, 7),
         ("tfim", 7, "c64", 4, 1, 5), ("heis", 8, "c64", 1, 9, 20), ("maxcut", 10, "c64", 1, 4, 13),
         ("heis", 10, "c128", 2, 3, 6), ("tfim", 11, "c128", 1, 2, 9), ("heis", 12, "c128", 1, 1, 4),
         ("tfim", 12, "c64", 4, 2, 3), ("heis", 13, "c64", 1, 5, 11), ("maxcut", 13, "c64", 2, 8, 2)]


@pytest.mark.parametrize("kind,n,dtype,order,batch,steps", CASES)
def test_whole_evolution_equals_launch_per_run(kind, n, dtype, order, batch, steps):
    hs, torch = hs_gpu()
    H = _ham(kind, n)
    n = H.n
    npd = np.complex128 if dtype == "c128" else np.complex64
    rng = np.random.default_rng(n * 31 + batch)
    psi0 = rng.normal(size=(batch, 1 << n)) + 1j * rng.normal(size=(batch, 1 << n))
    psi0 = (psi0 / np.linalg.norm(psi0, axis=1, keepdims=True)).astype(npd)
    note(f"whole evolution {kind} n={n} {dtype} order={order} batch={batch} steps={steps}")
    f = hs.build_factors(H.strings, H.coeffs, n, 0.9, steps, 16, dtype=dtype, order=order,
                         merge_diag=order == 1)
    a = torch.from_numpy(psi0.copy()).cuda()
    with env(HAMSIM_WHOLE_MAX_ROWS=8192):
        hs.evolve(f, a, steps)
    b = torch.from_numpy(psi0.copy()).cuda()
    with env(HAMSIM_WHOLE_MAX_ROWS=0):
        hs.evolve(f, b, steps)
    got = a.cpu().numpy()
    assert np.array_equal(got, b.cpu().numpy())
    f.close()
    ref = oracle_run(H, 16, 0.9, steps, psi0.astype(np.complex128))
    if order == 1:      # the oracle's product is first order; orders 2 and 4 are pinned elsewhere
        if dtype == "c128":
            assert np.abs(got - ref).max() <= 1e-12
        else:
            assert np.all(fid(got.astype(np.complex128), ref) >= 1 - 1e-6)


def test_whole_evolution_split_calls_and_tfim_chain_n8():
    """First order: evolve(7) + evolve(13) == evolve(20) bit for bit, and the
    n = 8 chain of 10 steps (complex128) against the oracle within 1e-12."""
    hs, torch = hs_gpu()
    H = workload_hamiltonian("heisenberg_chain_n20")
    H10 = wh.heisenberg_1d(10, 1.0, fields=np.linspace(-1, 1, 10))
    f = hs.build_factors(H10.strings, H10.coeffs, 10, 2.0, 20, 16, dtype="c64")
    psi0 = ws.neel_state(10, np.complex64)[None]
    note("whole evolution split calls n=10")
    a = torch.from_numpy(psi0.copy()).cuda()
    hs.evolve(f, a, 20)
    b = torch.from_numpy(psi0.copy()).cuda()
    hs.evolve(f, b, 7)
    hs.evolve(f, b, 13)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    f.close()
    del H
    H8 = workload_hamiltonian("tfim_chain_n8")
    f = hs.build_factors(H8.strings, H8.coeffs, 8, 1.0, 10, 8, dtype="c128")
    p = torch.from_numpy(ws.zero_state(8)[None].copy()).cuda()
    hs.evolve(f, p, 10)
    ref = oracle_run(H8, 8, 1.0, 10, ws.zero_state(8))
    assert np.abs(p.cpu().numpy()[0] - ref).max() <= 1e-12
    f.close()


def test_whole_evolution_leaves_renormalised_runs_on_the_tile_path():
    """HS_RENORM takes the launch per run and step (its FP64 norm per step):
    a renormalised evolution of a small state equals the same evolution with
    the whole-evolution kernel disabled, bit for bit."""
    hs, torch = hs_gpu()
    H = wh.tfim_1d(9, 1.0, 1.1)
    f = hs.build_factors(H.strings, H.coeffs, 9, 1.0, 12, 16, dtype="c64")
    psi0 = (ws.random_phase_state(9, 4, np.complex64) * 2.5)[None]
    note("whole evolution: renormalised run n=9")
    a = torch.from_numpy(psi0.copy()).cuda()
    hs.evolve(f, a, 12, renorm=True)
    b = torch.from_numpy(psi0.copy()).cuda()
    with env(HAMSIM_WHOLE_MAX_ROWS=0):
        hs.evolve(f, b, 12, renorm=True)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    f.close()
