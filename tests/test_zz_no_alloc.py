"""The entry point that allocates nothing (hs_fidelity_noalloc) against
hs_fidelity, through the C ABI: the same kernels with their partial sums in
the library's static device scratch instead of a per-call allocation, so the
values must be the same bits.  Two calls in a row, the second with fewer
states and a shorter state, so that it runs over the first call's leftovers
in the scratch."""
import numpy as np
import pytest

from gpu_common import hs_gpu, note

pytestmark = pytest.mark.gpu


def _states(torch, batch, n, dtype, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(batch, 1 << n)) + 1j * rng.normal(size=(batch, 1 << n))
    npd = np.complex128 if dtype == "c128" else np.complex64
    return torch.from_numpy(np.ascontiguousarray(a.astype(npd))).cuda()


def test_fidelity_noalloc_equals_fidelity_on_two_calls_second_smaller():
    hs, torch = hs_gpu()
    for call, (batch, n, dp, dq) in enumerate([(7, 18, "c64", "c128"), (3, 11, "c128", "c64")]):
        note(f"no-alloc fidelity call {call}: batch {batch}, n {n}, {dp} x {dq}")
        phi = _states(torch, batch, n, dp, 10 + call)
        psi = _states(torch, batch, n, dq, 20 + call)
        ref = hs.fidelity(phi, psi)
        out = torch.full((batch, 5), float("nan"), dtype=torch.float64, device="cuda")
        hs.fidelity_noalloc(phi, psi, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (call, got, ref)


def test_fidelity_noalloc_rejects_more_states_than_the_scratch_holds():
    hs, torch = hs_gpu()
    phi = _states(torch, 9, 6, "c64", 1)
    out = torch.zeros((9, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(hs.HamsimError, match="batch must be 1..8"):
        hs.fidelity_noalloc(phi, phi, out)
