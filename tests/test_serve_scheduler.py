"""Admission logic of the served loop, exercised on the CPU with a test double
in place of the GPU job runner (same scheduler code, fake job execution)."""
import threading
import time

import numpy as np
import pytest

from paper_2606_16959_amd.serve import Job, Server, summarize


class FakeServer(Server):
    """Runs jobs by sleeping; footprint = declared size; records concurrency."""

    def __init__(self, sizes, durations, **kw):
        super().__init__(**kw)
        self.sizes, self.durations = sizes, durations
        self.lock = threading.Lock()
        self.live = {}
        self.max_used = 0
        self.order = []

    def footprint(self, job):
        return self.sizes[job.job_id]

    def _run_job(self, job, res, t0):
        with self.lock:
            self.live[job.job_id] = self.sizes[job.job_id]
            self.max_used = max(self.max_used, sum(self.live.values()))
            self.order.append(job.job_id)
        res.start = time.perf_counter() - t0
        time.sleep(self.durations[job.job_id])
        res.end = time.perf_counter() - t0
        with self.lock:
            del self.live[job.job_id]
        return res


def _jobs(k, gap=0.0):
    return [Job(j, ["X"], np.array([1.0]), 1, 1.0, 1, 1, 0, arrival=j * gap) for j in range(k)]


def test_fifo_when_everything_fits():
    s = FakeServer({j: 1 for j in range(8)}, {j: 0.01 for j in range(8)}, slots=2, hbm_budget=10)
    res, st = s.run(_jobs(8, 0.001))
    assert st["completed"] == 8 and s.order == list(range(8))
    assert all(r.admit >= r.arrival - 1e-9 and r.end >= r.admit for r in res)
    assert st["peak_active"] <= 2


def test_hbm_budget_is_never_exceeded():
    rng = np.random.default_rng(0)
    sizes = {j: int(rng.integers(1, 7)) for j in range(30)}
    s = FakeServer(sizes, {j: 0.005 for j in range(30)}, slots=4, hbm_budget=8)
    res, st = s.run(_jobs(30, 0.0005))
    assert st["completed"] == 30
    assert s.max_used <= 8 and st["peak_hbm_bytes"] <= 8


def test_bypass_is_bounded_and_big_job_finishes():
    # job 1 needs the whole budget while small jobs keep arriving
    sizes = {j: 1 for j in range(20)}
    sizes[1] = 10
    durations = {j: 0.02 for j in range(20)}
    s = FakeServer(sizes, durations, slots=3, hbm_budget=10, bypass_limit=3)
    res, st = s.run(_jobs(20, 0.002))
    assert st["completed"] == 20
    r1 = res[1]
    assert r1.bypassed <= 3
    # once its bypass budget is spent, job 1 starts before every job that was behind it
    later = [r for r in res if r.job_id > 1 and r.admit > r1.admit]
    assert len(later) >= 20 - 2 - 3 - 1


def test_oversize_job_is_rejected_others_complete():
    sizes = {0: 1, 1: 99, 2: 1}
    s = FakeServer(sizes, {j: 0.001 for j in range(3)}, slots=2, hbm_budget=10)
    res, st = s.run(_jobs(3))
    assert [r.status for r in res] == ["ok", "rejected", "ok"]
    assert st["completed"] == 2 and st["failed"] == 1


def test_summary_fields():
    s = FakeServer({j: 1 for j in range(5)}, {j: 0.002 for j in range(5)}, slots=2, hbm_budget=4)
    res, st = s.run(_jobs(5, 0.001))
    for key in ("latency_ms", "queue_wait_ms", "service_ms", "throughput_jobs_s", "device_busy_frac"):
        assert key in st
    assert st["latency_ms"]["p99"] >= st["latency_ms"]["p50"] > 0
    assert summarize([])["completed"] == 0


def test_queued_job_is_cancelled_others_complete(tmp_path):
    # one slot: job 0 runs while 1..4 wait; cancelling 2 removes it from the queue
    sizes = {j: 1 for j in range(5)}
    s = FakeServer(sizes, {j: 0.05 for j in range(5)}, slots=1, hbm_budget=10)
    s.cancel(2)
    path = tmp_path / "jobs.jsonl"
    res, st = s.run(_jobs(5), jsonl=str(path))
    status = {r.job_id: r.status for r in res}
    assert status == {0: "ok", 1: "ok", 2: "cancelled", 3: "ok", 4: "ok"}
    assert 2 not in s.order
    assert st["completed"] == 4 and st["cancelled"] == 1
    # the cancellation ended with its run: the same id runs in the next one
    res, st = s.run(_jobs(5), realtime=False)
    assert all(r.status == "ok" for r in res) and st["completed"] == 5


def test_jsonl_has_one_record_per_job_with_final_status(tmp_path):
    import json
    sizes = {0: 1, 1: 99, 2: 1, 3: 2}
    s = FakeServer(sizes, {j: 0.002 for j in range(4)}, slots=2, hbm_budget=10)
    s.cancel(3)
    path = tmp_path / "jobs.jsonl"
    res, st = s.run(_jobs(4, 0.001), jsonl=str(path))
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert sorted(r["job_id"] for r in recs) == [0, 1, 2, 3]
    by = {r["job_id"]: r for r in recs}
    assert by[0]["status"] == "ok" and by[2]["status"] == "ok"
    assert by[1]["status"] == "rejected" and by[3]["status"] == "cancelled"
    for r in (by[0], by[2]):
        assert r["latency_ms"] >= r["service_ms"] >= 0 and r["queue_wait_ms"] >= 0
        assert r["footprint_bytes"] == sizes[r["job_id"]]


def test_invalid_job_fails_alone():
    class Bad(FakeServer):
        def footprint(self, job):
            if job.job_id == 1:
                raise ValueError("bad Hamiltonian")
            return super().footprint(job)
    s = Bad({j: 1 for j in range(3)}, {j: 0.001 for j in range(3)}, slots=2, hbm_budget=10)
    res, st = s.run(_jobs(3))
    assert [r.status for r in res] == ["ok", "error", "ok"]
    assert "bad Hamiltonian" in res[1].error
