"""Served request loop: continuous batching of Hamiltonian-simulation jobs on
one GPU.

A job is a Pauli-sum Hamiltonian, a time t, a step count, a diagonal budget
and B initial states.  The scheduler admits jobs in arrival order while two
conditions hold: the job's device footprint (its stored factor diagonals,
its states and the library workspace, from ``hs_footprint_dtype`` for the
job's dtype) fits the free part of the HBM budget, and a stream slot is
free.  A job that does not fit may be passed by later, smaller jobs at most
``bypass_limit`` times; after that nothing else is admitted until it fits.
Footprints are planned on the host when a job arrives, outside the lock that
admission and job completion share.  Each slot is a worker thread with its
own HIP stream, so the kernels of different jobs overlap on the device;
factors and states stay resident until the job completes, and all B initial
states of a job go through one batched DIA SpMM launch per factor.

Latency is arrival -> completion of the job's last kernel (host clock after
its completion event).  Queue wait (arrival -> admission) and service time
(admission -> completion) are reported separately.  The device busy
fraction is the union of the jobs' evolution intervals on the device
timeline (HIP events recorded on each job's stream around its evolution)
over the host makespan.

A job can be cancelled (:meth:`Server.cancel`): a queued job leaves the
queue, a running one stops at the next chunk boundary (``Job.chunk_steps``
steps per enqueue; by default the whole evolution is one call).  A job that
fails (a library error, an invalid Hamiltonian) ends with status "error"
and frees its slot and memory; other jobs are unaffected.  With ``jsonl``
set, one JSON record per job is appended to that file when the job reaches
its final state.
"""
from __future__ import annotations

import json
import math
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import build_factors, evolve, norm2, plan


@dataclass
class Job:
    job_id: int
    strings: list
    coeffs: np.ndarray
    n: int
    t: float
    steps: int
    batch: int
    state_seed: int
    budget: int = 16
    dtype: str = "c64"
    arrival: float = 0.0            # seconds after the stream starts
    keep_result: bool = False       # copy initial and final states to the host
    renorm: bool = False
    tag: str = ""
    chunk_steps: int | None = None  # steps per evolve call (cancellation granularity); None = all


@dataclass
class JobResult:
    job_id: int
    status: str = "ok"              # ok | error | rejected | cancelled
    error: str = ""
    arrival: float = 0.0
    admit: float = math.nan
    start: float = math.nan         # evolution enqueued (after build and state setup)
    end: float = math.nan           # completion event observed
    footprint: int = 0
    n: int = 0
    batch: int = 0
    steps: int = 0
    steps_done: int = 0
    bypassed: int = 0
    dev_start_ms: float = math.nan  # evolution interval on the device timeline (ms after the run began)
    dev_end_ms: float = math.nan
    norm2: np.ndarray = None
    psi0: np.ndarray = None
    psi: np.ndarray = None
    tag: str = ""

    @property
    def latency(self):
        return self.end - self.arrival

    @property
    def queue_wait(self):
        return self.admit - self.arrival

    @property
    def service(self):
        return self.end - self.admit

    def record(self) -> dict:
        """The job's JSONL record (times in seconds after the run began)."""
        def num(v):
            return None if v is None or (isinstance(v, float) and math.isnan(v)) else v
        return {"job_id": self.job_id, "tag": self.tag, "status": self.status, "error": self.error,
                "n": self.n, "batch": self.batch, "steps": self.steps, "steps_done": self.steps_done,
                "footprint_bytes": self.footprint, "bypassed": self.bypassed,
                "arrival_s": num(self.arrival), "admit_s": num(self.admit), "start_s": num(self.start),
                "end_s": num(self.end), "latency_ms": num(self.latency * 1e3),
                "queue_wait_ms": num(self.queue_wait * 1e3), "service_ms": num(self.service * 1e3),
                "device_evolve_ms": num(self.dev_end_ms - self.dev_start_ms),
                "norm2": None if self.norm2 is None else [float(v) for v in self.norm2]}


class JobCancelled(Exception):
    pass


def initial_states(torch, n: int, batch: int, seed: int, dtype: str):
    """Random-phase states exp(2 pi i u)/sqrt(N), u ~ U[0,1) from torch's
    device generator seeded with ``seed`` (an input, not part of the method)."""
    N = 1 << n
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    real = torch.float32 if dtype == "c64" else torch.float64
    u = torch.rand((batch, N), generator=g, device="cuda", dtype=real)
    mag = torch.full_like(u, 1.0 / math.sqrt(N))
    return torch.polar(mag, u * (2.0 * math.pi)).contiguous()


class Server:
    def __init__(self, slots: int = 4, hbm_budget: int | None = None, bypass_limit: int = 8):
        import torch
        self.torch = torch
        self.slots = slots
        if hbm_budget is None:
            if not torch.cuda.is_available():
                raise RuntimeError("the server needs a GPU (or an explicit HBM budget)")
            free, _total = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.85)
        self.hbm_budget = int(hbm_budget)
        self.bypass_limit = bypass_limit
        self._local = threading.local()
        self._cancel = set()
        self._cancel_lock = threading.Lock()
        self._ref = None                  # device-timeline origin of the current run

    # ------------------------------------------------------------- one job
    def _stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream()
            self._local.stream = s
        return s

    def cancel(self, job_id: int):
        """Cancel a queued or running job of the current or next run (running:
        at its next chunk boundary); the request is dropped when that run ends."""
        with self._cancel_lock:
            self._cancel.add(job_id)

    def _cancelled(self, job_id: int) -> bool:
        with self._cancel_lock:
            return job_id in self._cancel

    def _evolve_chunk(self, f, psi, steps: int, job: Job, stream):
        """Enqueue `steps` Trotter steps of the job (one library call)."""
        evolve(f, psi, steps, renorm=job.renorm, stream=stream)

    def _run_job(self, job: Job, res: JobResult, t0: float):
        torch = self.torch
        s = self._stream()
        f = None
        try:
            with torch.cuda.stream(s):
                f = build_factors(job.strings, job.coeffs, job.n, job.t, job.steps, job.budget,
                                  dtype=job.dtype, stream=s)
                psi = initial_states(torch, job.n, job.batch, job.state_seed, job.dtype)
                if job.keep_result:
                    res.psi0 = psi.cpu().numpy()
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(s)
                res.start = time.perf_counter() - t0
                chunk = job.chunk_steps or job.steps
                done = 0
                while done < job.steps:
                    if self._cancelled(job.job_id):
                        raise JobCancelled()
                    k = min(chunk, job.steps - done)
                    self._evolve_chunk(f, psi, k, job, s)
                    done += k
                    res.steps_done = done
                    if done < job.steps:       # let a cancellation take effect at the boundary
                        s.synchronize()
                ev1 = torch.cuda.Event(enable_timing=True)
                ev1.record(s)
                ev1.synchronize()
                res.end = time.perf_counter() - t0
                if self._ref is not None:
                    res.dev_start_ms = self._ref.elapsed_time(ev0)
                    res.dev_end_ms = self._ref.elapsed_time(ev1)
                res.norm2 = norm2(psi, stream=s)
                if job.keep_result:
                    res.psi = psi.cpu().numpy()
                del psi
                s.synchronize()
        except JobCancelled:
            res.status, res.error = "cancelled", f"cancelled after {res.steps_done} of {job.steps} steps"
            s.synchronize()
            res.end = time.perf_counter() - t0
        except Exception as e:  # isolate the failure to this job
            res.status, res.error = "error", f"{type(e).__name__}: {e}"
            try:
                s.synchronize()
            except Exception:
                pass
            res.end = time.perf_counter() - t0
        finally:
            if f is not None:
                f.close()
        return res

    # ------------------------------------------------------------- stream
    def footprint(self, job: Job) -> int:
        """Device bytes of the job (host planning only, for the job's dtype)."""
        p = plan(job.strings, job.coeffs, job.n, job.t, job.steps, job.budget)
        try:
            return p.footprint(job.batch, dtype=job.dtype)
        finally:
            p.close()

    def run(self, jobs, realtime: bool = True, on_done=None, jsonl: str | None = None):
        """Serve ``jobs`` (sorted by arrival).  Returns (results, stats)."""
        torch = self.torch
        jobs = sorted(jobs, key=lambda j: j.arrival)
        results = {j.job_id: JobResult(j.job_id, arrival=j.arrival, n=j.n, batch=j.batch,
                                       steps=j.steps, tag=j.tag) for j in jobs}
        cond = threading.Condition()
        pending = deque()
        active = {}
        used = 0
        done = 0
        bypassed = {}
        fp_cache = {}                   # main thread only
        peak = {"used": 0, "active": 0}
        out_lock = threading.Lock()
        out_fh = open(jsonl, "a") if jsonl else None
        ex = ThreadPoolExecutor(max_workers=self.slots)
        if torch.cuda.is_available():
            self._ref = torch.cuda.Event(enable_timing=True)
            self._ref.record()
        else:
            self._ref = None
        t0 = time.perf_counter()
        if not realtime:
            t0 -= jobs[-1].arrival + 1.0 if jobs else 0.0
        idx = 0

        def final(res):
            if out_fh is not None:
                with out_lock:
                    out_fh.write(json.dumps(res.record()) + "\n")
                    out_fh.flush()
            if on_done:
                on_done(res)

        def finish(job_id, fp):
            nonlocal used, done
            with cond:
                used -= fp
                active.pop(job_id, None)
                done += 1
                cond.notify_all()
            final(results[job_id])

        def admit(job, fp):
            nonlocal used
            used += fp
            res = results[job.job_id]
            res.admit = time.perf_counter() - t0
            res.footprint = fp
            res.bypassed = bypassed.get(job.job_id, 0)
            active[job.job_id] = None          # before submit: the callback may run at once
            peak["used"] = max(peak["used"], used)
            peak["active"] = max(peak["active"], len(active))
            fut = ex.submit(self._run_job, job, res, t0)
            fut.add_done_callback(lambda _f, jid=job.job_id, fpp=fp: finish(jid, fpp))

        def drop(job, status, error):
            """Final state without running (called with the lock held)."""
            nonlocal done
            r = results[job.job_id]
            r.status, r.error = status, error
            r.admit = r.end = time.perf_counter() - t0
            done += 1
            return r

        while True:
            # arrivals and their footprints: host planning, outside the lock
            now = time.perf_counter() - t0
            arrived = []
            while idx < len(jobs) and jobs[idx].arrival <= now:
                j = jobs[idx]
                idx += 1
                try:
                    fp_cache[j.job_id] = self.footprint(j)
                except Exception as e:      # invalid job: fails alone
                    fp_cache[j.job_id] = -1
                    results[j.job_id].error = f"{type(e).__name__}: {e}"
                arrived.append(j)
            finals = []
            with cond:
                pending.extend(arrived)
                if self._cancel:
                    keep = deque()
                    for j in pending:
                        if self._cancelled(j.job_id):
                            finals.append(drop(j, "cancelled", "cancelled while queued"))
                        else:
                            keep.append(j)
                    pending = keep
                # admission in arrival order, with bounded bypass of a blocked head
                while pending and len(active) < self.slots:
                    head = pending[0]
                    fp = fp_cache[head.job_id]
                    if fp < 0 or fp > self.hbm_budget:
                        pending.popleft()
                        if fp < 0:
                            finals.append(drop(head, "error", results[head.job_id].error))
                        else:
                            finals.append(drop(head, "rejected", "footprint exceeds the HBM budget"))
                        continue
                    if used + fp <= self.hbm_budget:
                        admit(pending.popleft(), fp)
                        continue
                    if bypassed.get(head.job_id, 0) >= self.bypass_limit:
                        break
                    picked = None
                    for k in range(1, len(pending)):
                        cfp = fp_cache[pending[k].job_id]
                        if 0 <= cfp <= self.hbm_budget and used + cfp <= self.hbm_budget:
                            picked = k
                            break
                    if picked is None:
                        break
                    cand = pending[picked]
                    del pending[picked]
                    bypassed[head.job_id] = bypassed.get(head.job_id, 0) + 1
                    admit(cand, fp_cache[cand.job_id])
                if done == len(jobs):
                    break
                wait = None
                if idx < len(jobs):
                    wait = max(0.0, jobs[idx].arrival - (time.perf_counter() - t0))
                if not finals:
                    cond.wait(timeout=wait if wait is not None else 0.5)
            for r in finals:
                final(r)
        for r in finals:
            final(r)
        ex.shutdown(wait=True)
        if out_fh is not None:
            out_fh.close()
        with self._cancel_lock:             # a cancellation ends with its run
            self._cancel.difference_update(results.keys())
        out = [results[j.job_id] for j in jobs]
        stats = summarize(out)
        stats.update(peak_hbm_bytes=peak["used"], peak_active=peak["active"], slots=self.slots,
                     hbm_budget=self.hbm_budget)
        return out, stats


def _intervals_union(iv):
    iv = sorted(iv)
    total, cur_s, cur_e = 0.0, None, None
    for s, e in iv:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                total += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        total += cur_e - cur_s
    return total


def summarize(results) -> dict:
    ok = [r for r in results if r.status == "ok"]
    counts = {s: sum(1 for r in results if r.status == s) for s in ("error", "rejected", "cancelled")}
    if not ok:
        return {"completed": 0, "failed": len(results), **counts}
    lat = np.array([r.latency for r in ok]) * 1e3
    qw = np.array([r.queue_wait for r in ok]) * 1e3
    sv = np.array([r.service for r in ok]) * 1e3
    first = min(r.arrival for r in ok)
    last = max(r.end for r in ok)
    span = max(1e-9, last - first)
    dev = [(r.dev_start_ms, r.dev_end_ms) for r in ok if not math.isnan(r.dev_start_ms)]
    return {
        "completed": len(ok), "failed": len(results) - len(ok), **counts,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "mean": float(lat.mean())},
        "queue_wait_ms": {"p50": float(np.percentile(qw, 50)), "p99": float(np.percentile(qw, 99))},
        "service_ms": {"p50": float(np.percentile(sv, 50)), "p99": float(np.percentile(sv, 99))},
        "makespan_s": float(span),
        "throughput_jobs_s": float(len(ok) / span),
        # union of the jobs' evolution intervals on the device timeline / host makespan
        "device_busy_frac": float(_intervals_union(dev) * 1e-3 / span) if dev else None,
        "max_bypassed": int(max(r.bypassed for r in ok)),
    }
