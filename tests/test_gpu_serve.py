"""Served loop on the GPU: each job's result is the same alone and in the mix
(bit for bit: same kernels, same launch shapes), results match the oracle,
admission respects a tight HBM budget, and a failing job stays isolated."""
import numpy as np
import pytest

from gpu_common import fid, hs_gpu, note, oracle_run
from workloads.serve_stream import job_stream

pytestmark = pytest.mark.gpu


def _jobs(k=10, n_max=14, keep=True, seed=5):
    from paper_2606_16959_amd.serve import Job
    out = []
    for spec in job_stream(n_jobs=k, rate=200.0, seed=seed, n_min=10, n_max=n_max):
        H = spec.hamiltonian()
        out.append((spec, Job(spec.job_id, H.strings, H.coeffs, H.n, spec.t, spec.steps, spec.batch,
                                spec.state_seed, arrival=spec.arrival, keep_result=keep,
                                tag=spec.family)))
    return out


def test_alone_equals_mixed_bitwise_and_matches_oracle():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Server
    pairs = _jobs(10)
    jobs = [j for _, j in pairs]
    note("serve: 10 jobs mixed on 4 slots")
    mixed, st = Server(slots=4).run(jobs)
    assert st["completed"] == 10, [r.error for r in mixed]
    assert st["peak_active"] >= 2
    note("serve: the same jobs one at a time")
    for j, rm in zip(jobs, mixed):
        alone, _ = Server(slots=1).run([j], realtime=False)
        ra = alone[0]
        assert ra.status == "ok"
        assert np.array_equal(ra.psi0, rm.psi0)
        assert np.array_equal(ra.psi, rm.psi), j.job_id
    note("serve: oracle check of the mixed results")
    for (spec, j), r in zip(pairs, mixed):
        ref = oracle_run(spec.hamiltonian(), j.budget, j.t, j.steps, r.psi0.astype(np.complex128))
        assert np.all(fid(r.psi.astype(np.complex128), ref) >= 1 - 1e-6), (spec.family, spec.n)
        assert np.all(np.abs(r.norm2 - 1.0) < 1e-4)
    note("serve: the served complex64 results against the plain complex128 path")
    for j, r in list(zip(jobs, mixed))[:4]:
        f = hs.build_factors(j.strings, j.coeffs, j.n, j.t, j.steps, j.budget, dtype="c128")
        p = torch.from_numpy(r.psi0.astype(np.complex128)).cuda()
        hs.evolve(f, p, j.steps)
        f.close()
        assert np.all(fid(r.psi.astype(np.complex128), p.cpu().numpy()) >= 1 - 1e-6), j.job_id


def test_tight_budget_serialises_but_completes():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Server
    jobs = [j for _, j in _jobs(8, n_max=16, keep=False, seed=7)]
    s = Server(slots=4)
    fps = [s.footprint(j) for j in jobs]
    s.hbm_budget = max(fps) + min(fps)          # at most two jobs' worth
    note("serve: tight HBM budget")
    res, st = s.run(jobs)
    assert st["completed"] == 8
    assert st["peak_hbm_bytes"] <= s.hbm_budget


def test_failing_job_is_isolated():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Job, Server
    jobs = [j for _, j in _jobs(3, keep=False)]
    bad = Job(99, ["XXX"], np.array([1.0]), 3, 1.0, 5, 1, 0, budget=4, arrival=0.0)   # over budget
    note("serve: one failing job among good ones")
    res, st = Server(slots=2).run(jobs + [bad])
    status = {r.job_id: r.status for r in res}
    assert status[99] in ("error", "rejected")
    assert all(status[j.job_id] == "ok" for j in jobs)


def test_running_job_is_cancelled_at_a_chunk_boundary():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Server
    jobs = [j for _, j in _jobs(3, keep=False)]
    target = jobs[1]
    target.steps, target.chunk_steps = 40, 5

    class CancelAfterFirstChunk(Server):
        def _evolve_chunk(self, f, psi, steps, job, stream):
            super()._evolve_chunk(f, psi, steps, job, stream)
            if job.job_id == target.job_id:
                self.cancel(job.job_id)
    note("serve: cancel a running job after its first chunk")
    res, st = CancelAfterFirstChunk(slots=2).run(jobs)
    by = {r.job_id: r for r in res}
    assert by[target.job_id].status == "cancelled" and by[target.job_id].steps_done == 5
    assert all(by[j.job_id].status == "ok" for j in jobs if j is not target)


def test_injected_fault_after_k_steps_leaves_other_jobs_bitwise_unchanged():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Server
    pairs = _jobs(4, n_max=13)
    jobs = [j for _, j in pairs]
    for j in jobs:
        j.chunk_steps = 7
    victim = jobs[2].job_id

    class FaultAfterK(Server):
        victim_steps = 0                    # only the victim's worker thread touches it

        def _evolve_chunk(self, f, psi, steps, job, stream):
            if job.job_id == victim and self.victim_steps >= 14:
                raise RuntimeError("injected fault")
            super()._evolve_chunk(f, psi, steps, job, stream)
            if job.job_id == victim:
                self.victim_steps += steps
    note("serve: injected fault in one job after 14 steps")
    res, st = FaultAfterK(slots=4).run(jobs)
    by = {r.job_id: r for r in res}
    assert by[victim].status == "error" and "injected fault" in by[victim].error
    assert by[victim].steps_done == 14
    note("serve: the other jobs alone")
    for j in jobs:
        if j.job_id == victim:
            continue
        alone, _ = Server(slots=1).run([j], realtime=False)
        assert by[j.job_id].status == "ok"
        assert np.array_equal(alone[0].psi, by[j.job_id].psi), j.job_id


def test_footprint_uses_the_jobs_dtype():
    hs, torch = hs_gpu()
    from paper_2606_16959_amd.serve import Server
    from workloads import hamiltonians as wh
    # a coupling range of 13 bits: closed in a complex64 tile of 8192 rows,
    # open (scratch state) in complex128, whose tiles hold 4096 rows; n = 21
    # keeps 256 full-size tiles, so the planner does not shrink them
    n = 21
    strings = ["X" + "I" * 11 + "X" + "I" * (n - 13), "Z" * n]
    from paper_2606_16959_amd.serve import Job
    j64 = Job(0, strings, np.array([0.3, 0.2]), n, 1.0, 4, 2, 0, budget=16, dtype="c64")
    j128 = Job(1, strings, np.array([0.3, 0.2]), n, 1.0, 4, 2, 0, budget=16, dtype="c128")
    s = Server(slots=1)
    fp64, fp128 = s.footprint(j64), s.footprint(j128)
    for j, fp in ((j64, fp64), (j128, fp128)):
        f = hs.build_factors(j.strings, j.coeffs, n, 1.0, 4, 16, dtype=j.dtype)
        assert fp == f.footprint(j.batch)
        f.close()
    assert fp128 - 2 * fp64 > (1 << n) * 16      # the complex128 scratch state
