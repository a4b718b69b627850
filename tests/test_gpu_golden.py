"""The paper's two worked examples through the GPU library: the 4x4 layout
example (Section 2.3 format table) and the quick-start SpMV (Appendix), plus
the closed-form evolution of the quick-start Hamiltonian (a Heisenberg bond
XX + YY + ZZ, whose terms commute, so one factor is exact)."""
import json
import os

import numpy as np
import pytest

from gpu_common import hs_gpu, note

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_layout_example_spmv():
    hs, torch = hs_gpu()
    g = _load("layout_4x4.json")
    sym = {k: float(i + 1) for i, k in enumerate("abcdef")}        # a..f -> 1..6
    dense = np.array([[sym.get(v, 0.0) if v != "0" else 0.0 for v in row] for row in g["dense"]])
    vals = [sym[v] for v in g["val"]]
    # val lists diagonal 0 (4 entries), then -3 and +3 (1 entry each)
    diags = {0: np.array(vals[:4]), -3: np.array(vals[4:5]), 3: np.array(vals[5:6])}
    offs = sorted(diags)
    note("golden layout example through hs_dia_spmv")
    x = np.array([[1, 2, 3, 4], [0.5, -1, 2, -3]], dtype=np.complex128) + 1j * np.array([[0, 1, 0, -1], [1, 0, 0, 1]])
    y = hs.dia_spmv(offs, [torch.from_numpy(diags[d].astype(np.complex128)).cuda() for d in offs],
                    torch.from_numpy(x).cuda())
    assert np.abs(y.cpu().numpy() - (dense @ x.T).T).max() <= 1e-14


def test_quickstart_hamiltonian_spmv_and_closed_form():
    hs, torch = hs_gpu()
    import paper_2606_16959_amd.dia as hd
    g = _load("quickstart.json")
    Hp = np.array(g["H"], dtype=np.complex128)
    pf = g["pauli_form"]
    note("golden quick-start through from_pauli, dia_evolve and the Trotter path")
    H = hd.from_pauli(pf["terms"], pf["coeffs"], 2)
    assert H.offsets == [-1, 0, 1]                        # XX + YY cancel on the +-3 diagonals
    D = H.to_dict()
    for d in (-1, 0, 1):
        assert np.abs(D[d] - np.diagonal(Hp, d)).max() <= 1e-15
    # the printed SpMV: y = H psi
    diag_t = [torch.from_numpy(D[d]).cuda() for d in (-1, 0, 1)]
    y = hs.dia_spmv([-1, 0, 1], diag_t, torch.from_numpy(np.array(g["psi"], dtype=np.complex128)).cuda())
    assert np.array_equal(y.cpu().numpy(), np.array(g["y"], dtype=np.complex128))
    H.close()
    # exp(-i t H): e^{-it} on |00>, |11>; on span{|01>, |10>} e^{it}(cos 2t I - i sin 2t X)
    t = 0.7
    c, s = np.cos(2 * t), np.sin(2 * t)
    U = np.zeros((4, 4), dtype=np.complex128)
    U[0, 0] = U[3, 3] = np.exp(-1j * t)
    U[1, 1] = U[2, 2] = np.exp(1j * t) * c
    U[1, 2] = U[2, 1] = np.exp(1j * t) * (-1j * s)
    rng = np.random.default_rng(2)
    psi0 = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    for steps in (1, 5):
        f = hs.build_factors(pf["terms"], pf["coeffs"], 2, t, steps, 16, dtype="c128")
        p = torch.from_numpy(psi0.copy()).cuda()
        hs.evolve(f, p, steps)
        assert np.abs(p.cpu().numpy() - (U @ psi0.T).T).max() <= 1e-14, steps
        f.close()
