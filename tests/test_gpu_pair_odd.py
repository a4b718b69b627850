"""The pair kernel's odd-offset path gives the row kernel's bits.

In a contiguous tile a factor that flips qubit 0 has odd offsets, so the
partners of a thread's two rows start at an odd LDS entry and the pair's
coefficients at an odd diagonal entry.  Such closed complex64 launches run
in the pair kernel too (8-byte aligned 16-byte loads, clamped at the ends
of each diagonal and of the tile), with HAMSIM_PAIR_LDS 1 (the default) and
2, at every batch size.  Every setting must give the same
bits: 2 and 1 against 0 (every launch row by row).  Small states (tile =
whole state, whole-state evolution switched off) put many row pairs at the
clamps.
"""
import numpy as np
import pytest

from gpu_common import env, hs_gpu, note
from workloads import hamiltonians as wh
from workloads import states as ws

pytestmark = pytest.mark.gpu


def _random_ham(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 13))
    nt = int(rng.integers(2, 14))
    terms = []
    for _ in range(nt):
        k = int(rng.integers(1, 4))
        qs = rng.choice(n, size=min(k, n), replace=False)
        s = ["I"] * n
        for q in qs:
            s[q] = str(rng.choice(list("XYZ")))
        if rng.integers(0, 2):            # qubit 0 flipped in about half the terms
            s[0] = str(rng.choice(list("XY")))
        terms.append(("".join(s), float(np.round(rng.normal(), 3))))
    # a term flipping k qubits alone needs up to 3^k diagonals
    flips = max(sum(ch in "XY" for ch in s) for s, _ in terms)
    budget = max(int(rng.choice([4, 8, 16, 32])), 3 ** flips)
    return wh.Hamiltonian(n, terms), budget, int(rng.integers(1, 9)), \
        int(rng.choice([1, 1, 2, 4])), bool(rng.integers(0, 2))


def _named(name):
    rng = np.random.default_rng(9)
    if name == "tfim_n14":
        return wh.tfim_1d(14, 1.0, 0.9)
    if name == "tfim_n5":
        return wh.tfim_1d(5, 1.0, 1.3, periodic=True)
    if name == "heisenberg_n16":
        return wh.heisenberg_1d(16, 1.0, rng.uniform(-1, 1, 16))
    if name == "maxcut_n18":
        edges = wh.random_regular_graph(18, 3, rng)
        return wh.maxcut(18, edges, rng.uniform(1, 10, len(edges)), mixer=0.7)
    raise KeyError(name)


def _run_settings(hs, torch, H, budget, batch, order, renorm, steps=(2, 3), settings=("0", "1", "2")):
    f = hs.build_factors(H.strings, H.coeffs, H.n, 1.0, 10, budget, dtype="c64", order=order)
    psi0 = torch.from_numpy(np.stack([ws.random_phase_state(H.n, 40 + b, np.complex64)
                                      for b in range(batch)])).cuda()
    outs = {}
    with env(HAMSIM_WHOLE_MAX_ROWS=0):
        for k in settings:
            with env(HAMSIM_PAIR_LDS=k):
                p = psi0.clone()
                for s in steps:
                    hs.evolve(f, p, s, renorm=renorm)
                torch.cuda.synchronize()
            outs[k] = p.cpu().numpy()
            del p
    closed = f.check_closure()
    f.close()
    return outs, closed


def _assert_same(outs):
    ref = outs["0"]
    for k, v in outs.items():
        assert np.array_equal(ref.view(np.uint8), v.view(np.uint8)), k


@pytest.mark.parametrize("name,budget,batch,order,renorm", [
    ("tfim_n14", 16, 1, 1, False), ("tfim_n14", 16, 3, 2, True), ("tfim_n14", 8, 8, 4, False),
    ("tfim_n5", 16, 2, 1, False), ("tfim_n5", 4, 8, 2, True),
    ("heisenberg_n16", 16, 5, 1, True), ("heisenberg_n16", 32, 8, 1, False),
    ("maxcut_n18", 16, 8, 1, False), ("maxcut_n18", 16, 2, 2, False), ("maxcut_n18", 16, 13, 1, True)])
def test_odd_pairs_same_bits(name, budget, batch, order, renorm):
    hs, torch = hs_gpu()
    H = _named(name)
    note(f"odd pairs: {name} budget={budget} batch={batch} order={order} renorm={renorm}")
    outs, closed = _run_settings(hs, torch, H, budget, batch, order, renorm)
    assert closed
    _assert_same(outs)


@pytest.mark.parametrize("seed", range(24))
def test_odd_pairs_random_small_hamiltonians(seed):
    hs, torch = hs_gpu()
    H, budget, batch, order, renorm = _random_ham(seed)
    note(f"odd pairs: random seed={seed} n={H.n} budget={budget} batch={batch} order={order}")
    outs, closed = _run_settings(hs, torch, H, budget, batch, order, renorm)
    assert closed
    _assert_same(outs)


def test_odd_pairs_full_size_maxcut_n24_eight_states():
    hs, torch = hs_gpu()
    from workloads import workload_hamiltonian
    H = workload_hamiltonian("maxcut_3reg_n24")
    note("odd pairs: maxcut_3reg_n24 8 states, 2 steps, settings 1 and 2")
    f = hs.build_factors(H.strings, H.coeffs, 24, 1.0, 200, 16, dtype="c64")
    psi0 = torch.from_numpy(ws.workload_states("maxcut_3reg_n24", np.complex64)).cuda()
    outs = {}
    for k in ("1", "2"):
        with env(HAMSIM_PAIR_LDS=k):
            p = psi0.clone()
            hs.evolve(f, p, 2)
            torch.cuda.synchronize()
        outs[k] = p.cpu().numpy()
        del p
    assert f.check_closure()
    assert np.array_equal(outs["1"].view(np.uint8), outs["2"].view(np.uint8))
    f.close()
