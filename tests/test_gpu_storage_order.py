"""Diagonals stored in level-major chunk order give the same results.

Factors applied by strided tiles whose levels lie far apart may be stored
with their entries permuted inside each diagonal (hs_factor_storage; still
exactly N - |d| entries per diagonal, Eq. 6).  The kernels read the same
coefficients in the same order either way, so every evolution must equal
the natural-order build of the same Hamiltonian bit for bit, and the
diagonal copies must come back in natural order.  HAMSIM_PERM_MIN_BYTES=1
stores every eligible strided factor permuted (even at small n, where the
default leaves them in natural order); 0 stores none.
"""
import numpy as np
import pytest

from gpu_common import env, hs_gpu, note
from workloads import hamiltonians as wh
from workloads import states as ws

pytestmark = pytest.mark.gpu


def _ham(name):
    rng = np.random.default_rng(7)
    if name == "tfim2d_4x5":
        return wh.tfim_2d(4, 5, 1.0, 1.7)
    if name == "heisenberg_n18":
        return wh.heisenberg_1d(18, 1.0, rng.uniform(-1, 1, 18))
    if name == "maxcut_n20":
        edges = wh.random_regular_graph(20, 3, rng)
        return wh.maxcut(20, edges, rng.uniform(1, 10, len(edges)), mixer=0.7)
    if name == "tfim_n13":
        return wh.tfim_1d(13, 1.0, 0.9)
    raise KeyError(name)


def _build(hs, H, steps, dtype, order, perm, chunk=0, budget=16):
    """chunk: bytes per storage chunk, 0 = the library's choice (four row windows)."""
    with env(HAMSIM_PERM_MIN_BYTES=1 if perm else 0, HAMSIM_PERM_CHUNK_BYTES=chunk):
        return hs.build_factors(H.strings, H.coeffs, H.n, 1.0, steps, budget, dtype=dtype, order=order)


def _states(torch, n, batch, dtype, seed):
    npd = np.complex128 if dtype == "c128" else np.complex64
    psi = np.stack([ws.random_phase_state(n, seed + b, npd) for b in range(batch)])
    return torch.from_numpy(psi).cuda()


CASES = [
    # (Hamiltonian, dtype, batch, order, renorm, chunk bytes, pair-form knob)
    ("tfim2d_4x5", "c64", 1, 1, False, 0, "1"),
    ("tfim2d_4x5", "c64", 1, 1, False, 256, "2"),
    ("tfim2d_4x5", "c64", 3, 2, True, 16, "1"),
    ("tfim2d_4x5", "c128", 1, 1, False, 256, "1"),
    ("tfim2d_4x5", "c128", 2, 4, False, 4096, "1"),
    ("heisenberg_n18", "c64", 8, 1, False, 0, "1"),
    ("heisenberg_n18", "c64", 5, 1, True, 4096, "0"),
    ("heisenberg_n18", "c128", 3, 2, False, 16, "1"),
    ("maxcut_n20", "c64", 8, 1, False, 0, "1"),
    ("maxcut_n20", "c64", 2, 1, False, 256, "2"),
    ("maxcut_n20", "c128", 1, 1, True, 0, "1"),
]


@pytest.mark.parametrize("name,dtype,batch,order,renorm,chunk,pairs", CASES)
def test_permuted_storage_evolves_bit_identically(name, dtype, batch, order, renorm, chunk, pairs):
    hs, torch = hs_gpu()
    H = _ham(name)
    steps = 5
    note(f"storage order: {name} {dtype} batch={batch} order={order} renorm={renorm} chunk={chunk} pairs={pairs}")
    fn = _build(hs, H, steps, dtype, order, perm=False)
    fp = _build(hs, H, steps, dtype, order, perm=True, chunk=chunk)
    dn, dp = fn.describe(), fp.describe()
    assert all(f["storage"] == (0, 0) for f in dn["factors"])
    permuted = [k for k, f in enumerate(dp["factors"]) if f["storage"][0] > 0]
    assert permuted, "some strided factor should be stored permuted"
    esz = 16 if dtype == "c128" else 8
    for k in permuted:
        s, c = dp["factors"][k]["storage"]
        assert 1 <= c <= s
        if chunk:
            assert (1 << c) == min(1 << s, max(2, chunk // esz))
        assert all(abs(d) % (1 << s) == 0 for d in dp["factors"][k]["offsets"])
    psi0 = _states(torch, H.n, batch, dtype, 11)
    outs = []
    for f in (fn, fp):
        with env(HAMSIM_PAIR_LDS=pairs):
            p = psi0.clone()
            hs.evolve(f, p, 3, renorm=renorm)
            hs.evolve(f, p, 2, renorm=renorm)
            torch.cuda.synchronize()
        outs.append(p.cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))
    # one launch per factor: a factor runs alone, in the tile its own flips
    # need (contiguous when they fit one), whatever order it is stored in
    unfused = []
    for f in (fn, fp):
        p = psi0.clone()
        hs.evolve(f, p, 3, renorm=renorm, fuse=False)
        torch.cuda.synchronize()
        unfused.append(p.cpu().numpy())
    assert np.array_equal(unfused[0].view(np.uint8), unfused[1].view(np.uint8))
    assert fp.check_closure() and fn.check_closure()
    fn.close()
    fp.close()


@pytest.mark.parametrize("dtype,chunk", [("c64", 0), ("c64", 16), ("c128", 0), ("c128", 4096)])
def test_permuted_diagonals_copy_back_in_natural_order(dtype, chunk):
    hs, torch = hs_gpu()
    H = _ham("tfim2d_4x5")
    note(f"storage order: diagonal copies {dtype} chunk={chunk}")
    fn = _build(hs, H, 4, dtype, 1, perm=False)
    fp = _build(hs, H, 4, dtype, 1, perm=True, chunk=chunk)
    dp = fp.describe()
    rng = np.random.default_rng(3)
    checked = 0
    for k, fac in enumerate(dp["factors"]):
        if fac["storage"][0] == 0:
            continue
        for j, d in enumerate(fac["offsets"]):
            a = fn.copy_diagonal(k, j, d)
            b = fp.copy_diagonal(k, j, d)
            assert a.shape == (fn.N - abs(d),)
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
            for _ in range(3):
                start = int(rng.integers(0, a.size))
                count = int(rng.integers(0, a.size - start + 1))
                sub = fp.copy_diagonal(k, j, d, start=start, count=count)
                assert np.array_equal(sub.view(np.uint8), a[start:start + count].view(np.uint8))
            checked += 1
    assert checked > 0
    fn.close()
    fp.close()


def test_small_state_with_permuted_storage_takes_the_tile_path():
    """A permuted factor of a small state leaves the whole-evolution kernel
    (which reads natural order) for the tile launches; results agree bit for
    bit with the natural-order handle's whole evolution."""
    hs, torch = hs_gpu()
    H = _ham("tfim_n13")
    note("storage order: n=13 whole-evolution guard")
    with env(HAMSIM_WHOLE_MAX_ROWS=8192):
        fn = _build(hs, H, 6, "c64", 1, perm=False)
        fp = _build(hs, H, 6, "c64", 1, perm=True)
        assert any(f["storage"][0] > 0 for f in fp.describe()["factors"])
        psi0 = _states(torch, 13, 2, "c64", 5)
        outs = []
        for f in (fn, fp):
            p = psi0.clone()
            hs.evolve(f, p, 6)
            torch.cuda.synchronize()
            outs.append(p.cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))
    fn.close()
    fp.close()


def test_headline_n26_default_storage_and_bitwise_steps():
    """tfim_5x5_ancilla_n26 in complex64 with the default threshold: the
    factors of the strided launch over qubits 18-24 (levels 2 MiB apart,
    windows of 64 rows) are stored permuted with chunks of four windows, the
    other launches' factors (contiguous; levels 32 KiB apart) in natural
    order, and two steps equal the natural-order build bit for bit.  With
    the threshold at 32 KiB the middle launch's factors are permuted too
    (windows of 128 rows)."""
    hs, torch = hs_gpu()
    from workloads import workload_hamiltonian
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    note("storage order: n=26 default threshold vs natural, 2 steps")
    fp = hs.build_factors(H.strings, H.coeffs, 26, 1.0, 50, 16, dtype="c64")
    dp = fp.describe()
    launches = fp.step_launches(1)
    seq = fp.part_sequence(0, dp)
    perm = {k for k, f in enumerate(dp["factors"]) if f["storage"][0] > 0}
    assert len(launches) == 3
    (f0, n0), (f1, n1), (f2, n2) = launches
    assert perm == set(seq[f2:f2 + n2])
    for k in seq[f2:f2 + n2]:
        assert dp["factors"][k]["storage"] == (18, 8)
    psi0 = _states(torch, 26, 1, "c64", 3)
    pa = psi0.clone()
    hs.evolve(fp, pa, 2)
    torch.cuda.synchronize()
    a = pa.cpu().numpy()
    del pa
    # a whole permuted diagonal (about 2^26 entries: the copy gathers it in pieces)
    kd = seq[f2]
    dd = dp["factors"][kd]["offsets"][0]
    diag_p = fp.copy_diagonal(kd, 0, dd)
    fp.close()
    with env(HAMSIM_PERM_MIN_BYTES=32 << 10):
        fm = hs.build_factors(H.strings, H.coeffs, 26, 1.0, 50, 16, dtype="c64")
    dm = fm.describe()
    for k in seq[f1:f1 + n1]:
        assert dm["factors"][k]["storage"] == (12, 9)
    for k in seq[f2:f2 + n2]:
        assert dm["factors"][k]["storage"] == (18, 8)
    pm = psi0.clone()
    hs.evolve(fm, pm, 2)
    torch.cuda.synchronize()
    assert np.array_equal(a.view(np.uint8), pm.cpu().numpy().view(np.uint8))
    del pm
    fm.close()
    with env(HAMSIM_PERM_MIN_BYTES=0):
        fn = hs.build_factors(H.strings, H.coeffs, 26, 1.0, 50, 16, dtype="c64")
    assert all(f["storage"] == (0, 0) for f in fn.describe()["factors"])
    diag_n = fn.copy_diagonal(kd, 0, dd)
    assert diag_n.shape == ((1 << 26) - abs(dd),)
    assert np.array_equal(diag_p.view(np.uint8), diag_n.view(np.uint8))
    del diag_p, diag_n
    pb = psi0.clone()
    hs.evolve(fn, pb, 2)
    torch.cuda.synchronize()
    assert np.array_equal(a.view(np.uint8), pb.cpu().numpy().view(np.uint8))
    fn.close()
