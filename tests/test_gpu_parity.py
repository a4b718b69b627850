"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerances.  complex128 runs are compared element by element within
1e-12 (well above accumulated FP64 rounding for these sizes) and by fidelity
>= 1 - 1e-12.  complex64 runs store coefficients rounded to FP32 and
accumulate in FP32: per element the error is bounded by a small multiple of
2^-24 * sum_d |c_d| |x_{r+d}| per launch, checked as 2^-20 * that sum; whole
evolutions are checked by fidelity >= 1 - 1e-6 against the oracle.
"""
import numpy as np
import pytest

from gpu_common import fid, hs_gpu, note, oracle_run, oracle_threads, tol_c64
from oracle import dia as odia, factors as ofac, metrics, pauli as opauli
from workloads import workload_hamiltonian, hamiltonians as wh, states as ws

pytestmark = pytest.mark.gpu


def _to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda()


def _heis10():
    return wh.heisenberg_1d(10, 1.0, fields=np.linspace(-0.9, 0.7, 10))


# ------------------------------------------------------------------ (a0) construction

@pytest.mark.parametrize("case,dtype,merge", [
    ("tfim8", "c128", True), ("tfim8", "c64", True), ("heis10", "c128", False), ("heis10", "c64", True),
])
def test_construction_matches_oracle_entries(case, dtype, merge):
    hs, torch = hs_gpu()
    if case == "tfim8":
        H, budget, t, steps = workload_hamiltonian("tfim_chain_n8"), 8, 1.0, 10
    else:
        H, budget, t, steps = _heis10(), 16, 0.7, 9
    note(f"construct {case} {dtype} merge={merge}")
    f = hs.build_factors(H.strings, H.coeffs, H.n, t, steps, budget, dtype=dtype, merge_diag=merge)
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, budget, t / steps)
    desc = f.describe()
    N = 1 << H.n
    for k, (fd, fo) in enumerate(zip(desc["factors"], part.factor_list(merge_diag=merge))):
        for j, d in enumerate(fd["offsets"]):
            got = f.copy_diagonal(k, j, d).astype(np.complex128)
            rows = np.arange(N - abs(d)) - min(d, 0)        # storage index i -> row i - min(d, 0)
            ref = ofac.factor_entries(terms, part, fo, H.n, t / steps, rows, d)
            # structural zeros are exact zeros
            assert np.array_equal(got == 0, ref == 0), (k, d)
            if dtype == "c128":
                assert np.abs(got - ref).max() <= 1e-15
            else:
                assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) * 1.5 + 1e-30)
    f.close()


def test_construction_sampled_at_full_size_tfim_5x5_n26():
    hs, torch = hs_gpu()
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    note("construct tfim_5x5_ancilla_n26 c64 (sampled windows)")
    f = hs.build_factors(H.strings, H.coeffs, H.n, 1.0, 50, 16, dtype="c64")
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, 16, 1.0 / 50)
    desc = f.describe()
    N = 1 << 26
    rng = np.random.default_rng(3)
    for k, (fd, fo) in enumerate(zip(desc["factors"], part.factor_list())):
        for j, d in enumerate(fd["offsets"]):
            length = N - abs(d)
            for start in [0, length - 512] + list(rng.integers(0, length - 512, 2)):
                got = f.copy_diagonal(k, j, d, start=int(start), count=512).astype(np.complex128)
                rows = np.arange(start, start + 512) - min(d, 0)
                ref = ofac.factor_entries(terms, part, fo, 26, 0.02, rows, d)
                assert np.array_equal(got == 0, ref == 0)
                assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) * 1.5 + 1e-30)
    f.close()


# ------------------------------------------------------------------ (a1) generic DIA SpMV

def _random_dia(rng, N, offsets, dtype):
    diags = []
    for d in offsets:
        v = rng.normal(size=N - abs(d)) + 1j * rng.normal(size=N - abs(d))
        v[rng.random(N - abs(d)) < 0.1] = 0.0
        diags.append(v.astype(dtype))
    return diags


@pytest.mark.parametrize("N,B,dtype,kind", [
    (2, 1, "c128", "all"), (1 << 10, 1, "c128", "near"), (1 << 14, 3, "c64", "near"),
    (1 << 16, 1, "c64", "far"), (1 << 16, 8, "c64", "far"), (1 << 15, 2, "c128", "strided"),
    (1 << 16, 1, "c64", "strided"), (1 << 13, 5, "c128", "mixed"), (1 << 12, 11, "c64", "mixed"),
    # N not a multiple of the tile (any N): the last tile is partial, odd N makes odd diagonals
    (1, 1, "c128", "all"), (3, 2, "c64", "all"), (1000, 3, "c64", "near"), (4097, 1, "c128", "far"),
    (12345, 2, "c64", "mixed"), (99999, 5, "c64", "far"),
])
def test_dia_spmv_matches_definition(N, B, dtype, kind):
    hs, torch = hs_gpu()
    rng = np.random.default_rng(N + B)
    npd = np.complex128 if dtype == "c128" else np.complex64
    if kind == "all":
        offs = list(range(-(N - 1), N))
    elif kind == "near":
        offs = sorted(set(rng.integers(-9, 10, 7).tolist()) | {0})
    elif kind == "far":            # includes |d| >= N/2 and the extreme offsets
        offs = sorted({-(N - 1), -(N // 2), -3, 0, 5, N // 2 + 7, N - 1})
    elif kind == "strided":        # multiples of 64 reaching far: strided tiles
        offs = sorted({-64 * 37, -128, 0, 64, 64 * 5, 64 * 200})
    else:
        offs = sorted(set(rng.integers(-N + 1, N, 12).tolist()))
    diags = _random_dia(rng, N, offs, npd)
    x = (rng.normal(size=(B, N)) + 1j * rng.normal(size=(B, N))).astype(npd)
    note(f"dia_spmv N={N} B={B} {dtype} {kind}")
    y = hs.dia_spmv(offs, [_to_dev(torch, v, npd) for v in diags], _to_dev(torch, x, npd))
    got = y.cpu().numpy().astype(np.complex128)
    D = {d: v.astype(np.complex128) for d, v in zip(offs, diags)}
    ref = odia.dia_spmv(D, x.astype(np.complex128))
    bound = odia.dia_spmv({d: np.abs(v) for d, v in D.items()}, np.abs(x.astype(np.complex128)))
    fac = 1e-14 if dtype == "c128" else tol_c64()
    assert np.all(np.abs(got - ref) <= fac * bound + 1e-300)


def test_dia_spmv_rejects_overlap_and_bad_offsets():
    hs, torch = hs_gpu()
    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    v = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(hs.HamsimError):
        hs.dia_spmv([0], [v], x, y=x)
    with pytest.raises(hs.HamsimError):
        hs.dia_spmv([1, 0], [v[:63], v], x)


# ------------------------------------------------------------------ (a2) evolution

def _evolve_vs_oracle(H, budget, t, steps, psi0, dtype, run_steps=None, **kw):
    hs, torch = hs_gpu()
    npd = np.complex128 if dtype == "c128" else np.complex64
    psi0 = np.atleast_2d(psi0).astype(npd)
    f = hs.build_factors(H.strings, H.coeffs, H.n, t, steps, budget, dtype=dtype)
    psi = _to_dev(torch, psi0, npd)
    hs.evolve(f, psi, steps if run_steps is None else run_steps, **kw)
    got = psi.cpu().numpy().astype(np.complex128)
    assert f.check_closure()
    f.close()
    ref = oracle_run(H, budget, t, steps, psi0.astype(np.complex128), run_steps, threads=oracle_threads())
    return got, ref


def test_evolve_tfim_chain_n8_complex128():
    note("evolve tfim_chain_n8 c128")
    H = workload_hamiltonian("tfim_chain_n8")
    got, ref = _evolve_vs_oracle(H, 8, 1.0, 10, ws.zero_state(8), "c128")
    assert np.abs(got - ref).max() <= 1e-12
    assert fid(got, ref)[0] >= 1 - 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_evolve_heisenberg_chain_n20(dtype):
    note(f"evolve heisenberg_chain_n20 {dtype}")
    H = workload_hamiltonian("heisenberg_chain_n20")
    got, ref = _evolve_vs_oracle(H, 16, 2.0, 100, ws.neel_state(20), dtype)
    F = fid(got, ref)[0]
    if dtype == "c128":
        assert F >= 1 - 1e-12 and np.abs(got - ref).max() <= 1e-12
    else:
        assert F >= 1 - 1e-6


def test_evolve_tfim_5x5_n26_full_size_few_steps():
    note("evolve tfim_5x5_ancilla_n26 c64, 2 of 50 steps, vs oracle")
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    psi0 = ws.random_phase_state(26, 3, np.complex64)
    got, ref = _evolve_vs_oracle(H, 16, 1.0, 50, psi0, "c64", run_steps=2)
    assert fid(got, ref)[0] >= 1 - 1e-6
    bound = 2e-6 * np.abs(ref).max()
    assert np.abs(got - ref).max() <= bound


def test_five_states_on_whole_lds_tiles_match_single_state_runs():
    """Closed complex64 launches of 5 states stage 4096-row tiles in the
    whole 160 KiB LDS of a CU: a maxcut_3reg_n24 step takes 3 launches, as
    with 4 states (2048-row tiles would need 4), and each column equals its
    one-state run bit for bit (with per-step renormalisation the FP64 norm
    sums over other tiles, so the columns agree to FP32 rounding)."""
    hs, torch = hs_gpu()
    note("evolve maxcut_3reg_n24 B=5 c64 (4096-row tiles), 2 steps, columns vs one-state runs")
    H = workload_hamiltonian("maxcut_3reg_n24")
    psi0 = ws.workload_states("maxcut_3reg_n24", np.complex64)[:5]
    f = hs.build_factors(H.strings, H.coeffs, 24, 1.0, 200, 16, dtype="c64")
    assert len(f.step_launches(5)) == 3 and len(f.step_launches(4)) == 3 and len(f.step_launches(6)) == 4
    for renorm in (False, True):
        five = _to_dev(torch, psi0, np.complex64)
        hs.evolve(f, five, 2, renorm=renorm)
        got = five.cpu().numpy()
        del five
        for b in (0, 2, 4):
            one = _to_dev(torch, psi0[b:b + 1], np.complex64)
            hs.evolve(f, one, 2, renorm=renorm)
            alone = one.cpu().numpy()[0]
            if renorm:
                assert np.max(np.abs(alone - got[b])) < 1e-9, b
            else:
                assert np.array_equal(alone.view(np.uint8), got[b].view(np.uint8)), b
    assert f.check_closure()
    f.close()


def test_two_complex128_states_on_4096_row_tiles_match_single_state_runs():
    """Closed complex128 launches of 2 states stage 4096-row tiles (128 KiB,
    as one state): heisenberg_chain_n20 keeps the one-state launch count and
    each column equals its one-state run bit for bit."""
    hs, torch = hs_gpu()
    note("evolve heisenberg_chain_n20 B=2 c128 (4096-row tiles), 3 steps, columns vs one-state runs")
    H = workload_hamiltonian("heisenberg_chain_n20")
    psi0 = np.stack([ws.random_phase_state(20, 70 + b, np.complex128) for b in range(2)])
    f = hs.build_factors(H.strings, H.coeffs, 20, 2.0, 100, 16, dtype="c128")
    assert len(f.step_launches(2)) == len(f.step_launches(1))
    two = _to_dev(torch, psi0, np.complex128)
    hs.evolve(f, two, 3)
    got = two.cpu().numpy()
    for b in range(2):
        one = _to_dev(torch, psi0[b:b + 1], np.complex128)
        hs.evolve(f, one, 3)
        assert np.array_equal(one.cpu().numpy()[0].view(np.uint8), got[b].view(np.uint8)), b
    assert f.check_closure()
    f.close()


def test_evolve_maxcut_n24_full_size_batched():
    hs, torch = hs_gpu()
    note("evolve maxcut_3reg_n24 B=8 c64, 2 of 200 steps, vs oracle + column invariance")
    H = workload_hamiltonian("maxcut_3reg_n24")
    psi0 = ws.workload_states("maxcut_3reg_n24", np.complex64)
    got, ref = _evolve_vs_oracle(H, 16, 1.0, 200, psi0, "c64", run_steps=2)
    assert np.all(fid(got, ref) >= 1 - 1e-6)
    # column b of the batched run equals the single-state run, bit for bit
    f = hs.build_factors(H.strings, H.coeffs, 24, 1.0, 200, 16, dtype="c64")
    for b in (0, 5):
        one = _to_dev(torch, psi0[b:b + 1], np.complex64)
        hs.evolve(f, one, 2)
        assert np.array_equal(one.cpu().numpy()[0], got[b].astype(np.complex64))
    f.close()


def _c64_run_bound(n_factor_apps, max_diags):
    """2-norm bound of the complex64 error of a whole evolution: each factor
    application rounds every stored coefficient to FP32 and accumulates at
    most `max_diags` products in FP32 (relative error <= max_diags * 2^-24
    per application, counting the coefficient rounding), and a unitary step
    does not amplify earlier errors, so the errors add over the run."""
    return n_factor_apps * max_diags * 2.0 ** -24


def test_evolve_tfim_5x5_n26_full_length_against_oracle():
    """The whole stated run of the n = 26 2-D TFIM (50 steps, 9 factors of at
    most 15 diagonals) against the FP64 oracle of the same product (Eq. 4,
    fidelity as in Section 4.3): complex64 at fidelity >= 1 - 1e-6 and within
    the accumulated FP32 bound, complex128 within 1e-12; the two GPU paths
    also agree with each other."""
    hs, torch = hs_gpu()
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    psi0 = ws.random_phase_state(26, 3, np.complex128)
    note("full-length oracle run tfim_5x5_ancilla_n26, 50 steps (host)")
    ref = oracle_run(H, 16, 1.0, 50, psi0, threads=oracle_threads())
    got = {}
    for dtype, npd in (("c64", np.complex64), ("c128", np.complex128)):
        note(f"evolve tfim_5x5_ancilla_n26 {dtype}, all 50 steps")
        f = hs.build_factors(H.strings, H.coeffs, 26, 1.0, 50, 16, dtype=dtype)
        nf, maxd = f.n_factors, max(len(x["offsets"]) for x in f.describe()["factors"])
        p = _to_dev(torch, psi0, npd)
        hs.evolve(f, p, 50)
        got[dtype] = p.cpu().numpy().astype(np.complex128)
        f.close()
        del p
        torch.cuda.empty_cache()
    g64, g128 = got["c64"], got["c128"]
    bound = _c64_run_bound(50 * nf, maxd)
    assert np.min(fid(g64, ref)) >= 1 - 1e-6
    assert np.linalg.norm(g64 - ref) <= bound
    assert abs(np.linalg.norm(g64) - 1.0) <= bound
    assert np.abs(g128 - ref).max() <= 1e-12 and np.min(fid(g128, ref)) >= 1 - 1e-12
    assert np.min(fid(g64, g128)) >= 1 - 1e-6


def test_evolve_maxcut_n24_full_length_batched_against_oracle():
    """All 200 steps of the n = 24 MaxCut run with 8 states batched (DIA SpMM),
    states 0, 1 and 7 against the FP64 oracle; state 7 also equals its
    single-state run bit for bit after the whole run."""
    hs, torch = hs_gpu()
    H = workload_hamiltonian("maxcut_3reg_n24")
    psi0 = ws.workload_states("maxcut_3reg_n24", np.complex64)
    note("evolve maxcut_3reg_n24 B=8 c64, all 200 steps")
    f = hs.build_factors(H.strings, H.coeffs, 24, 1.0, 200, 16, dtype="c64")
    nf, maxd = f.n_factors, max(len(x["offsets"]) for x in f.describe()["factors"])
    p = _to_dev(torch, psi0, np.complex64)
    hs.evolve(f, p, 200)
    got = p.cpu().numpy()
    one = _to_dev(torch, psi0[7:8], np.complex64)
    hs.evolve(f, one, 200)
    assert np.array_equal(one.cpu().numpy()[0], got[7])
    f.close()
    del p, one
    note("full-length oracle run maxcut_3reg_n24, states 0, 1, 7, 200 steps (host)")
    cols = [0, 1, 7]
    ref = oracle_run(H, 16, 1.0, 200, psi0[cols].astype(np.complex128), threads=oracle_threads())
    g = got[cols].astype(np.complex128)
    bound = _c64_run_bound(200 * nf, maxd)
    assert np.all(fid(g, ref) >= 1 - 1e-6)
    for b in range(len(cols)):
        assert np.linalg.norm(g[b] - ref[b]) <= bound
        assert abs(np.linalg.norm(g[b]) - 1.0) <= bound


def test_fused_unfused_split_and_repeat_are_bitwise_equal():
    hs, torch = hs_gpu()
    H = workload_hamiltonian("heisenberg_chain_n20")
    note("bitwise: fused/unfused/split/repeat heisenberg_chain_n20 c64")
    f = hs.build_factors(H.strings, H.coeffs, 20, 2.0, 100, 16, dtype="c64")
    psi0 = _to_dev(torch, ws.neel_state(20, np.complex64)[None], np.complex64)
    runs = []
    for fuse in (True, False):
        p = psi0.clone()
        hs.evolve(f, p, 30, fuse=fuse)
        runs.append(p.cpu().numpy())
    p = psi0.clone()
    hs.evolve(f, p, 11)
    hs.evolve(f, p, 19)
    runs.append(p.cpu().numpy())
    p = psi0.clone()
    hs.evolve(f, p, 30)
    runs.append(p.cpu().numpy())
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    f.close()


def test_renorm_keeps_unit_norm_and_fidelity():
    hs, torch = hs_gpu()
    H = workload_hamiltonian("heisenberg_chain_n20")
    note("renorm heisenberg_chain_n20 c64")
    f = hs.build_factors(H.strings, H.coeffs, 20, 2.0, 100, 16, dtype="c64")
    psi0 = ws.neel_state(20, np.complex64)[None]
    p = _to_dev(torch, psi0, np.complex64)
    hs.evolve(f, p, 100, renorm=True)
    n2 = hs.norm2(p)[0]
    assert abs(n2 - 1.0) < 1e-6
    q = _to_dev(torch, psi0, np.complex64)
    hs.evolve(f, q, 40, renorm=True)
    hs.evolve(f, q, 60, renorm=True)
    assert np.array_equal(q.cpu().numpy(), p.cpu().numpy())
    ref = oracle_run(H, 16, 2.0, 100, psi0.astype(np.complex128), threads=oracle_threads())
    assert fid(p.cpu().numpy().astype(np.complex128), ref)[0] >= 1 - 1e-6
    f.close()


# ------------------------------------------------------------------ (a3) single diagonal

def _maxcut_cost(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = wh.random_regular_graph(n, 3, rng)
    return wh.maxcut(n, edges, rng.uniform(1.0, 10.0, len(edges)), mixer=0.0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("batch", [1, 3])
def test_diagonal_steps_in_one_pass_equal_step_by_step(dtype, batch):
    """A diagonal Hamiltonian's step is one diagonal factor; without
    renormalisation the library applies all steps in one pass.  That pass
    equals one call per step, and two calls of 11 and 26 steps, bit for bit
    (one and three states), and with renormalisation (step by step) it stays
    within rounding of it."""
    hs, torch = hs_gpu()
    H = _maxcut_cost(16, 9)
    npd = np.complex128 if dtype == "c128" else np.complex64
    note(f"diagonal steps one pass vs step by step {dtype} batch {batch}")
    f = hs.build_factors(H.strings, H.coeffs, 16, 1.0, 37, 16, dtype=dtype)
    assert f.n_factors == 1 and f.describe()["factors"][0]["offsets"] == [0]
    psi0 = np.stack([ws.random_phase_state(16, s, npd) for s in (1, 2, 3)[:batch]])
    a = _to_dev(torch, psi0, npd)
    hs.evolve(f, a, 37)
    b = _to_dev(torch, psi0, npd)
    for _ in range(37):
        hs.evolve(f, b, 1)
    c = _to_dev(torch, psi0, npd)
    hs.evolve(f, c, 11)
    hs.evolve(f, c, 26)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())
    r = _to_dev(torch, psi0, npd)
    hs.evolve(f, r, 37, renorm=True)
    tol = 1e-12 if dtype == "c128" else 2e-5
    got, ref = r.cpu().numpy().astype(np.complex128), a.cpu().numpy().astype(np.complex128)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    f.close()


def test_diagonal_only_full_size_n26_matches_closed_form_on_sampled_rows():
    """MaxCut cost (no mixer) at n = 26, complex64, 200 steps in one pass: the
    diagonal factor exp(-i dt E) of Section 3.4 applied 200 times equals
    exp(-i t E) psi0 (exact Trotterisation of a diagonal H) to FP32
    rounding, on rows at both ends and spread over the state."""
    hs, torch = hs_gpu()
    n, t, r = 26, 1.0, 200
    H = _maxcut_cost(n, 26)
    terms = opauli.parse_terms(H.strings, H.coeffs, n)
    part = ofac.first_fit(terms, 16, t)
    fac = part.factor_list(merge_diag=True)[0]
    rng = np.random.default_rng(26)
    rows = np.unique(np.concatenate([np.arange(64), (1 << n) - 1 - np.arange(64),
                                     rng.integers(0, 1 << n, 4096)]))
    note("diagonal-only maxcut cost n=26 c64, 200 steps in one pass")
    f = hs.build_factors(H.strings, H.coeffs, n, t, r, 16, dtype="c64")
    psi0 = ws.random_phase_state(n, 5, np.complex64)
    p = _to_dev(torch, psi0, np.complex64)
    hs.evolve(f, p, r)
    got = p.cpu().numpy()[rows].astype(np.complex128)
    f.close()
    exact = ofac.factor_entries(terms, part, fac, n, t, rows, 0) * psi0[rows].astype(np.complex128)
    # r complex multiplications in FP32, each within a few ulp
    assert np.abs(got - exact).max() <= r * 4 * 2.0 ** -24 * np.abs(exact).max()


def test_diagonal_only_hamiltonian_matches_closed_form():
    hs, torch = hs_gpu()
    rng = np.random.Generator(np.random.PCG64(5))
    d = rng.uniform(1, 10, (4, 4))
    d = np.triu(d, 1) + np.triu(d, 1).T
    H = wh.tsp_onehot(d, 20.0)
    note("diagonal-only TSP n=16 c64 and c128")
    terms = opauli.parse_terms(H.strings, H.coeffs, 16)
    E = ofac.energies(terms, list(range(len(terms))), 16)
    psi0 = ws.random_phase_state(16, 11)
    exact = np.exp(-1j * 1.0 * E) * psi0
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-5)):
        npd = np.complex128 if dtype == "c128" else np.complex64
        f = hs.build_factors(H.strings, H.coeffs, 16, 1.0, 20, 16, dtype=dtype)
        assert f.n_factors == 1 and f.describe()["factors"][0]["offsets"] == [0]
        p = _to_dev(torch, psi0[None], npd)
        hs.evolve(f, p, 20)
        got = p.cpu().numpy()[0].astype(np.complex128)
        assert np.abs(got - exact).max() <= tol * np.abs(exact).max()
        f.close()


# ------------------------------------------------------------------ (a5, a6) reductions

@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_norm_and_fidelity_reductions(dtype):
    hs, torch = hs_gpu()
    npd = np.complex128 if dtype == "c128" else np.complex64
    rng = np.random.default_rng(9)
    for N, B in ((1, 1), (1000, 3), (1 << 20, 2)):
        note(f"reductions N={N} B={B} {dtype}")
        a = (rng.normal(size=(B, N)) + 1j * rng.normal(size=(B, N))).astype(npd)
        b = (rng.normal(size=(B, N)) + 1j * rng.normal(size=(B, N))).astype(npd)
        da, db = _to_dev(torch, a, npd), _to_dev(torch, b, npd)
        n2 = hs.norm2(da)
        ref = metrics.norm2(a.astype(np.complex128))
        assert np.all(np.abs(n2 - ref) <= 1e-13 * ref)
        assert np.array_equal(n2, hs.norm2(da))            # deterministic
        out = hs.fidelity(da, db)
        ov = metrics.inner(a.astype(np.complex128), b.astype(np.complex128))
        assert np.all(np.abs(out[:, 0] - ov.real) <= 1e-12 * np.sqrt(ref * metrics.norm2(b)))
        assert np.all(np.abs(out[:, 1] - ov.imag) <= 1e-12 * np.sqrt(ref * metrics.norm2(b)))
        fref = metrics.fidelity(a.astype(np.complex128), b.astype(np.complex128))
        assert np.all(np.abs(out[:, 4] - fref) <= 1e-12)
    # mixed precision: complex64 against complex128
    a = (rng.normal(size=(1, 4096)) + 1j * rng.normal(size=(1, 4096)))
    out = hs.fidelity(_to_dev(torch, a, np.complex64), _to_dev(torch, a, np.complex128))
    assert out[0, 4] == pytest.approx(metrics.fidelity(a.astype(np.complex64).astype(np.complex128), a)[0], abs=1e-14)


# ------------------------------------------------------------------ degenerate cases

def test_degenerate_cases():
    hs, torch = hs_gpu()
    note("degenerate: identity-only, n=1, steps=0, odd batches")
    # identity-only Hamiltonian: a global phase e^{-i c t}
    f = hs.build_factors(["III"], [0.7], 3, 2.0, 5, 1, dtype="c128")
    p = _to_dev(torch, ws.uniform_state(3)[None], np.complex128)
    hs.evolve(f, p, 5)
    assert np.allclose(p.cpu().numpy()[0], np.exp(-1.4j) * ws.uniform_state(3), atol=1e-14)
    hs.evolve(f, p, 0)
    f.close()
    # one qubit, X field: exact rotation
    f = hs.build_factors(["X"], [0.3], 1, 1.0, 4, 3, dtype="c128")
    p = _to_dev(torch, ws.zero_state(1)[None], np.complex128)
    hs.evolve(f, p, 4)
    assert np.allclose(p.cpu().numpy()[0], [np.cos(0.3), -1j * np.sin(0.3)], atol=1e-15)
    f.close()
    # batch sizes that are not powers of two, and above the launch limit of 8
    H = _heis10()
    f = hs.build_factors(H.strings, H.coeffs, 10, 0.5, 5, 16, dtype="c64")
    states = np.stack([ws.random_phase_state(10, s, np.complex64) for s in range(11)])
    p = _to_dev(torch, states, np.complex64)
    hs.evolve(f, p, 5)
    got = p.cpu().numpy()
    for b in (0, 2, 10):
        q = _to_dev(torch, states[b:b + 1], np.complex64)
        hs.evolve(f, q, 5)
        assert np.array_equal(q.cpu().numpy()[0], got[b])
    ref = oracle_run(H, 16, 0.5, 5, states.astype(np.complex128))
    assert np.all(fid(got.astype(np.complex128), ref) >= 1 - 1e-6)
    f.close()


def test_merge_flag_does_not_change_the_result():
    hs, torch = hs_gpu()
    note("merge on/off tfim_chain_n8 c128")
    H = workload_hamiltonian("tfim_chain_n8")
    outs = []
    for merge in (True, False):
        f = hs.build_factors(H.strings, H.coeffs, 8, 1.0, 10, 8, dtype="c128", merge_diag=merge)
        p = _to_dev(torch, ws.zero_state(8)[None], np.complex128)
        hs.evolve(f, p, 10)
        outs.append(p.cpu().numpy()[0])
        f.close()
    assert np.abs(outs[0] - outs[1]).max() <= 1e-13


# ------------------------------------------------------------------ higher-order products

@pytest.mark.parametrize("order", [2, 4])
def test_higher_order_products_match_oracle(order):
    hs, torch = hs_gpu()
    from oracle import evolve as oev
    note(f"order {order}: tfim_chain_n8 c128 and heisenberg_chain_n20 c64")
    H = workload_hamiltonian("tfim_chain_n8")
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, 8, 0.1)
    f = hs.build_factors(H.strings, H.coeffs, 8, 1.0, 10, 8, dtype="c128", order=order)
    assert f.describe()["joint"] >= 0
    # one step (the plain sequence), two (first and last parts), ten (middle parts too)
    for r in (1, 2, 10):
        p = _to_dev(torch, ws.zero_state(8)[None], np.complex128)
        hs.evolve(f, p, r)
        ref = oev.evolve(terms, part, ws.zero_state(8), 8, 0.1, r, order=order)
        assert np.abs(p.cpu().numpy()[0] - ref).max() <= 1e-12, r
    # fused and unfused launches agree bit for bit
    q = _to_dev(torch, ws.zero_state(8)[None], np.complex128)
    hs.evolve(f, q, 10, fuse=False)
    assert np.array_equal(p.cpu().numpy(), q.cpu().numpy())
    f.close()
    H = workload_hamiltonian("heisenberg_chain_n20")
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, 16, 0.02)
    f = hs.build_factors(H.strings, H.coeffs, 20, 2.0, 100, 16, dtype="c64", order=order)
    p = _to_dev(torch, ws.neel_state(20, np.complex64)[None], np.complex64)
    hs.evolve(f, p, 20)
    ref = oev.evolve(terms, part, ws.neel_state(20), 20, 0.02, 20, order=order, threads=oracle_threads())
    assert fid(p.cpu().numpy()[0].astype(np.complex128), ref) >= 1 - 1e-6
    assert f.check_closure()
    f.close()


# ------------------------------------------------------------------ long-range factors

@pytest.mark.parametrize("n,dtype", [(16, "c128"), (20, "c64")])
def test_long_range_factor_takes_an_open_launch(n, dtype):
    """A periodic chain's closing bond X_0 X_{n-1} + Y_0 Y_{n-1} couples bits 0
    and n-1, wider than any tile held in LDS: that factor runs as an open
    launch into the scratch state.  Same oracle bar; fusion and batching stay
    bit-exact."""
    hs, torch = hs_gpu()
    H = wh.heisenberg_1d(n, 1.0, fields=np.linspace(-1, 1, n), periodic=True)
    npd = np.complex128 if dtype == "c128" else np.complex64
    note(f"periodic heisenberg n={n} {dtype} (open launch)")
    f = hs.build_factors(H.strings, H.coeffs, n, 1.0, 20, 16, dtype=dtype)
    fac = f.describe()["factors"]
    wide = [k for k, x in enumerate(fac) if x["support_mask"] & 1 and x["support_mask"] >> (n - 1) & 1]
    assert wide, "the closing bond should form a factor over qubits 0 and n-1"
    desc_bytes = sum(x["bytes"] for x in fac)
    elem = 16 if dtype == "c128" else 8
    assert f.footprint(1) >= desc_bytes + 2 * (1 << n) * elem        # state + scratch
    psi0 = np.stack([ws.neel_state(n, npd), ws.random_phase_state(n, 5, npd), ws.zero_state(n, npd)])
    p = _to_dev(torch, psi0, npd)
    hs.evolve(f, p, 6)
    terms = opauli.parse_terms(H.strings, H.coeffs, n)
    part = ofac.first_fit(terms, 16, 0.05)
    from oracle import evolve as oev
    ref = oev.evolve(terms, part, psi0.astype(np.complex128), n, 0.05, 6, threads=oracle_threads())
    got = p.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.abs(got - ref).max() <= 1e-12
    assert np.all(fid(got, ref) >= (1 - 1e-12 if dtype == "c128" else 1 - 1e-6))
    q = _to_dev(torch, psi0, npd)
    hs.evolve(f, q, 6, fuse=False)
    assert np.array_equal(p.cpu().numpy(), q.cpu().numpy())
    single = _to_dev(torch, psi0[1:2], npd)
    hs.evolve(f, single, 6)
    assert np.array_equal(single.cpu().numpy()[0], p.cpu().numpy()[1])
    assert f.check_closure()
    f.close()


@pytest.mark.parametrize("n,hi,batch,dtype", [(11, 10, 1, "c64"), (11, 10, 6, "c128"), (20, 11, 8, "c64")])
def test_hull_filling_the_tile_levels(n, hi, batch, dtype):
    """A factor coupling bits 1 and `hi` whose hull [1, hi+1) has exactly as
    many levels as the tile has rows would leave one row per level (W = 1),
    and a thread's row pair would not be adjacent: such a factor takes a
    bigger tile for one state at a time or an open launch.  n = 11 (1024-row
    tiles): open launch; n = 20 with 8 complex64 states (2048-row tiles): one
    state per launch on 4096 rows.  Oracle bar, closure flag clear."""
    hs, torch = hs_gpu()
    s = ["I"] * n
    s[1], s[hi] = "X", "Y"
    H = wh.Hamiltonian(n, [("".join(s), 0.8)] + [(("I" * q) + "Z" + "I" * (n - q - 1), 0.3 + 0.1 * q)
                                                 for q in range(n)] + [("X" + "I" * (n - 1), -0.6)])
    npd = np.complex128 if dtype == "c128" else np.complex64
    note(f"hull filling the tile n={n} bits 1..{hi} batch={batch} {dtype}")
    f = hs.build_factors(H.strings, H.coeffs, n, 0.6, 4, 8, dtype=dtype, merge_diag=False)
    rng = np.random.default_rng(n + batch)
    psi0 = rng.normal(size=(batch, 1 << n)) + 1j * rng.normal(size=(batch, 1 << n))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    p = _to_dev(torch, psi0, npd)
    hs.evolve(f, p, 4)
    assert f.check_closure()
    terms = opauli.parse_terms(H.strings, H.coeffs, n)
    part = ofac.first_fit(terms, 8, 0.15)
    from oracle import evolve as oev
    ref = oev.evolve(terms, part, psi0.astype(np.complex128), n, 0.15, 4, threads=oracle_threads())
    got = p.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.abs(got - ref).max() <= 1e-12
    assert np.all(fid(got, ref) >= (1 - 1e-12 if dtype == "c128" else 1 - 1e-6))
    f.close()


@pytest.mark.parametrize("order", [2, 4])
def test_higher_order_full_size_tfim_5x5_n26(order):
    """The n = 26 workload with the bench's launch plan, 3 steps (first,
    middle and last step lists, joint factors included), against the
    oracle's unmerged product on the full state."""
    hs, torch = hs_gpu()
    from oracle import evolve as oev
    note(f"order {order}: tfim_5x5_ancilla_n26 c64, 3 of 50 steps, vs oracle")
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    psi0 = ws.random_phase_state(26, 3, np.complex64)
    f = hs.build_factors(H.strings, H.coeffs, 26, 1.0, 50, 16, dtype="c64", order=order)
    desc = f.describe()
    applications = sum(len(f.part_sequence(q, desc)) for q in (1, 2, 3))
    p = _to_dev(torch, psi0[None], np.complex64)
    hs.evolve(f, p, 3)
    got = p.cpu().numpy()[0].astype(np.complex128)
    f.close()
    del p
    terms = opauli.parse_terms(H.strings, H.coeffs, 26)
    part = ofac.first_fit(terms, 16, 0.02)
    ref = oev.evolve(terms, part, psi0.astype(np.complex128), 26, 0.02, 3, order=order,
                     threads=oracle_threads())
    assert fid(got, ref) >= 1 - 1e-6
    # each complex64 factor application (unitary, <= 15 diagonals, FP32
    # accumulation, coefficients rounded once) adds at most a few 2^-24 of
    # the row scale; the errors add over the applications
    assert np.abs(got - ref).max() <= applications * 2.0 ** -22 * np.abs(ref).max()


@pytest.mark.parametrize("cfg,steps", [("heisenberg_chain_n20", 100), ("maxcut_3reg_n24", 5)])
def test_complex64_matches_the_complex128_path(cfg, steps):
    """The complex64 path against the plain complex128 GPU path on the same
    inputs (the n = 20 chain: the whole run; n = 24 MaxCut: 8 batched states)."""
    hs, torch = hs_gpu()
    H = workload_hamiltonian(cfg)
    run = wh.WORKLOAD_RUN[cfg]
    psi0 = np.ascontiguousarray(ws.workload_states(cfg, np.complex128))
    note(f"{cfg}: complex64 vs complex128, {steps} steps")
    out = {}
    for dtype, npd in (("c128", np.complex128), ("c64", np.complex64)):
        f = hs.build_factors(H.strings, H.coeffs, H.n, run["t"], run["steps"], run["budget"], dtype=dtype)
        p = _to_dev(torch, psi0, npd)
        hs.evolve(f, p, steps)
        out[dtype] = p.cpu().numpy().astype(np.complex128)
        f.close()
        del p
    assert np.all(fid(out["c64"], out["c128"]) >= 1 - 1e-6)


def test_streamed_and_cached_stores_give_the_same_bits():
    """Launches whose states reach 128 MiB write them with non-temporal
    stores (a kernel instantiation of its own); smaller ones keep plain
    stores.  At n = 23 (complex64) one state is 64 MiB and two are 128 MiB:
    the pair evolved together must equal each state evolved alone, bit for
    bit, and match the oracle."""
    hs, torch = hs_gpu()
    n = 23
    H = wh.tfim_1d(n, 1.0, 0.8)
    note("n=23 complex64: 2 states (streamed stores) vs 1 state (plain stores)")
    f = hs.build_factors(H.strings, H.coeffs, n, 0.3, 3, 8, dtype="c64")
    psi0 = np.stack([ws.random_phase_state(n, 41, np.complex64), ws.random_phase_state(n, 42, np.complex64)])
    pair = _to_dev(torch, psi0, np.complex64)
    hs.evolve(f, pair, 3)
    for b in range(2):
        one = _to_dev(torch, psi0[b:b + 1], np.complex64)
        hs.evolve(f, one, 3)
        assert np.array_equal(one.cpu().numpy()[0], pair.cpu().numpy()[b])
    assert f.check_closure()
    f.close()
    terms = opauli.parse_terms(H.strings, H.coeffs, n)
    part = ofac.first_fit(terms, 8, 0.1)
    from oracle import evolve as oev
    ref = oev.evolve(terms, part, psi0.astype(np.complex128), n, 0.1, 3, threads=oracle_threads())
    assert np.all(fid(pair.cpu().numpy().astype(np.complex128), ref) >= 1 - 1e-6)


@pytest.mark.parametrize("batch,renorm", [(1, False), (3, True)])
def test_maximum_size_n30_sampled_rows(batch, renorm):
    """n = 30, the largest state the library accepts (8 GiB complex64 per
    state): one step of H = 0.8 Z0 Z1 - 0.45 Z15 + 0.6 X29 (D merged into the
    X29 factor: offsets 0 and +-2^29, a strided tile over bit 29), checked on
    sampled rows against the oracle's factor entries applied to the input
    rows they couple to.  Three states with renormalisation also take the
    fused per-tile norm over 2^30 rows per state."""
    hs, torch = hs_gpu()
    n, N = 30, 1 << 30
    strings = ["ZZ" + "I" * 28, "I" * 15 + "Z" + "I" * 14, "I" * 29 + "X"]
    coeffs = [0.8, -0.45, 0.6]
    note(f"maximum size n=30 c64 batch={batch} renorm={renorm}, one step (sampled rows)")
    f = hs.build_factors(strings, coeffs, n, 0.3, 1, 8, dtype="c64")
    desc = f.describe()
    assert len(desc["factors"]) == 1 and desc["factors"][0]["offsets"] == [-(1 << 29), 0, 1 << 29]
    # structured-phase inputs built on the device: e^{2 pi i frac(r g_b)} / sqrt(N)
    psi = torch.empty(batch, N, dtype=torch.complex64, device="cuda")
    amp, chunk = 1.0 / np.sqrt(N), 1 << 26
    gs = [0.6180339887498949 * (b + 1) % 1.0 for b in range(batch)]
    for b, g in enumerate(gs):
        for lo in range(0, N, chunk):
            r = torch.arange(lo, lo + chunk, dtype=torch.float64, device="cuda")
            phi = 2.0 * np.pi * torch.frac(r * g)
            psi[b, lo:lo + chunk] = torch.polar(torch.full_like(phi, amp), phi).to(torch.complex64)
            del r, phi
    rng = np.random.default_rng(30)
    rows = np.unique(np.concatenate([np.arange(64), N - 1 - np.arange(64), (1 << 29) + np.arange(-64, 64),
                                     8192 * np.arange(1, 64) - 1, rng.integers(0, N, 4096)])).astype(np.int64)
    need = np.unique(np.concatenate([rows, rows - (1 << 29), rows + (1 << 29)]))
    need = need[(need >= 0) & (need < N)]
    need_dev, rows_dev = torch.from_numpy(need).cuda(), torch.from_numpy(rows).cuda()
    x_at = [dict(zip(need.tolist(), psi[b][need_dev].cpu().numpy().astype(np.complex128).tolist()))
            for b in range(batch)]
    hs.evolve(f, psi, 1, renorm=renorm)
    got = [psi[b][rows_dev].cpu().numpy().astype(np.complex128) for b in range(batch)]
    norms = hs.norm2(psi) if renorm else None
    f.close()
    del psi
    terms = opauli.parse_terms(strings, coeffs, n)
    part = ofac.first_fit(terms, 8, 0.3)
    fac = part.factor_list(merge_diag=True)[0]
    vals = {}
    for d in (-(1 << 29), 0, 1 << 29):
        ok = (rows + d >= 0) & (rows + d < N)
        vals[d] = (ok, ofac.factor_entries(terms, part, fac, n, 0.3, rows[ok], d))
    for b in range(batch):
        ref = np.zeros(len(rows), dtype=np.complex128)
        for d, (ok, v) in vals.items():
            ref[ok] += v * np.array([x_at[b][int(c)] for c in rows[ok] + d])
        # the inputs have unit norm up to complex64 rounding, so renormalising
        # moves the result by far less than the bound
        assert np.abs(got[b] - ref).max() <= 2.0 ** -20 * amp * 4
    if renorm:
        assert np.all(np.abs(np.asarray(norms) - 1.0) <= 1e-6)


@pytest.mark.parametrize("order,ratio,rs", [(1, 2.0, (16, 32, 64)), (2, 4.0, (8, 16, 32)), (4, 16.0, (4, 8, 16))])
def test_error_scaling_on_the_gpu(order, ratio, rs):
    """complex128 GPU evolutions against exp(-iHt) from the dense
    eigendecomposition (n = 7): the global error falls by 2^order per
    doubling of r."""
    hs, torch = hs_gpu()
    n, t = 7, 1.0
    H = wh.tfim_1d(n, 1.0, 1.0)
    Hd = opauli.dense_hamiltonian(opauli.parse_terms(H.strings, H.coeffs, n), n)
    rng = np.random.default_rng(order)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    exact = opauli.dense_propagator(Hd, t) @ psi0
    note(f"error scaling order {order} r={rs}")
    errs = []
    for r in rs:
        f = hs.build_factors(H.strings, H.coeffs, n, t, r, 8, dtype="c128", order=order)
        p = _to_dev(torch, psi0[None], np.complex128)
        hs.evolve(f, p, r)
        errs.append(np.linalg.norm(p.cpu().numpy()[0] - exact))
        f.close()
    q = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert abs(q[-1] - ratio) < 0.15 * ratio, (errs, q)
