"""Seeded random Pauli Hamiltonians through the whole Trotter path against
the oracle: random sizes (n = 4..16, so tiles are contiguous, strided or open
for long-range couplings), supports of up to four qubits anywhere, budgets,
product orders, merging, batches (across the 8-state chunking) and both
dtypes."""
import numpy as np
import pytest

from gpu_common import fid, hs_gpu, note, oracle_threads
from oracle import evolve as oev, factors as ofac, pauli as opauli
from workloads import hamiltonians as wh

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(4, 17))
    nt = int(rng.integers(2, 16))
    strings = []
    for _ in range(nt):
        k = int(rng.integers(1, 5))
        qs = rng.choice(n, size=min(k, n), replace=False)
        s = ["I"] * n
        for q in qs:
            s[q] = str(rng.choice(list("XYZ")))
        strings.append("".join(s))
    coeffs = np.round(rng.normal(size=nt), 3)
    return dict(n=n, strings=strings, coeffs=coeffs,
                budget=int(rng.choice([8, 16, 32, 81])), order=int(rng.choice([1, 1, 2, 4])),
                merge=bool(rng.integers(0, 2)), steps=int(rng.integers(1, 9)), batch=int(rng.integers(1, 11)),
                t=float(rng.uniform(0.1, 1.5)), dtype=str(rng.choice(["c128", "c64"])))


@pytest.mark.parametrize("seed", range(24))
def test_random_hamiltonian_matches_oracle(seed):
    hs, torch = hs_gpu()
    c = _case(seed)
    H = wh.Hamiltonian(c["n"], list(zip(c["strings"], c["coeffs"])))
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    dt = c["t"] / c["steps"]
    try:
        part = ofac.first_fit(terms, c["budget"], dt)
    except ofac.BudgetError:
        with pytest.raises(hs.HamsimError):
            hs.plan(H.strings, H.coeffs, H.n, c["t"], c["steps"], c["budget"], order=c["order"])
        return
    note(f"random seed={seed} n={c['n']} terms={len(terms)} budget={c['budget']} order={c['order']} "
         f"merge={c['merge']} steps={c['steps']} batch={c['batch']} {c['dtype']}")
    npd = np.complex128 if c["dtype"] == "c128" else np.complex64
    rng = np.random.default_rng(seed)
    psi0 = rng.normal(size=(c["batch"], 1 << c["n"])) + 1j * rng.normal(size=(c["batch"], 1 << c["n"]))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    psi0 = psi0.astype(npd)
    merge = c["merge"] and c["order"] == 1
    f = hs.build_factors(H.strings, H.coeffs, H.n, c["t"], c["steps"], c["budget"], dtype=c["dtype"],
                         merge_diag=merge, order=c["order"])
    p = torch.from_numpy(psi0.copy()).cuda()
    hs.evolve(f, p, c["steps"])
    got = p.cpu().numpy().astype(np.complex128)
    assert f.check_closure()
    f.close()
    ref = oev.evolve(terms, part, psi0.astype(np.complex128), H.n, dt, c["steps"], order=c["order"],
                     threads=oracle_threads())
    if c["dtype"] == "c128":
        assert np.abs(got - ref).max() <= 1e-11
    else:
        assert np.all(fid(got, ref) >= 1 - 1e-6)
