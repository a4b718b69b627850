"""Served request loop: continuous batching of Hamiltonian-simulation jobs on
one GPU.

A job is a Pauli-sum Hamiltonian, a time t, a step count, a diagonal budget
and B initial states.  The scheduler admits jobs in arrival order while two
conditions hold: the job's device footprint (its stored factor diagonals,
its states and the library workspace, from ``hs_footprint``) fits the free
part of the HBM budget, and a stream slot is free.  A job that does not fit
may be passed by later, smaller jobs at most ``bypass_limit`` times; after
that nothing else is admitted until it fits.  Each slot is a worker thread
with its own HIP stream, so the kernels of different jobs overlap on the
device; factors and states stay resident until the job completes, and all B
initial states of a job go through one batched DIA SpMM launch per factor.

Latency is arrival -> completion of the job's last kernel (host clock after
its completion event).  Queue wait (arrival -> admission) and service time
(admission -> completion) are reported separately.
"""
from __future__ import annotations

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


@dataclass
class JobResult:
    job_id: int
    status: str = "ok"
    error: str = ""
    arrival: float = 0.0
    admit: float = math.nan
    start: float = math.nan         # evolution enqueued (after build and state setup)
    end: float = math.nan           # completion event observed
    footprint: int = 0
    n: int = 0
    batch: int = 0
    steps: int = 0
    bypassed: int = 0
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

    # ------------------------------------------------------------- one job
    def _stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream()
            self._local.stream = s
        return s

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
                res.start = time.perf_counter() - t0
                evolve(f, psi, job.steps, renorm=job.renorm, stream=s)
                ev = torch.cuda.Event()
                ev.record(s)
                ev.synchronize()
                res.end = time.perf_counter() - t0
                res.norm2 = norm2(psi, stream=s)
                if job.keep_result:
                    res.psi = psi.cpu().numpy()
                del psi
                s.synchronize()
        except Exception as e:  # isolate the failure to this job
            res.status, res.error = "error", f"{type(e).__name__}: {e}"
            res.end = time.perf_counter() - t0
        finally:
            if f is not None:
                f.close()
        return res

    # ------------------------------------------------------------- stream
    def footprint(self, job: Job) -> int:
        p = plan(job.strings, job.coeffs, job.n, job.t, job.steps, job.budget)
        fp = p.footprint(job.batch)
        p.close()
        if job.dtype == "c128":
            fp = 2 * fp
        return fp

    def run(self, jobs, realtime: bool = True, on_done=None):
        """Serve ``jobs`` (sorted by arrival).  Returns (results, stats)."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        results = {j.job_id: JobResult(j.job_id, arrival=j.arrival, n=j.n, batch=j.batch,
                                       steps=j.steps, tag=j.tag) for j in jobs}
        cond = threading.Condition()
        pending = deque()
        active = {}
        used = 0
        done = 0
        bypassed = {}
        fp_cache = {}
        peak = {"used": 0, "active": 0}
        ex = ThreadPoolExecutor(max_workers=self.slots)
        t0 = time.perf_counter()
        if not realtime:
            t0 -= jobs[-1].arrival + 1.0 if jobs else 0.0
        idx = 0

        def finish(job_id, fp):
            nonlocal used, done
            with cond:
                used -= fp
                active.pop(job_id, None)
                done += 1
                cond.notify_all()
            if on_done:
                on_done(results[job_id])

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

        while True:
            with cond:
                now = time.perf_counter() - t0
                while idx < len(jobs) and jobs[idx].arrival <= now:
                    pending.append(jobs[idx])
                    idx += 1
                # admission in arrival order, with bounded bypass of a blocked head
                while pending and len(active) < self.slots:
                    head = pending[0]
                    fp = fp_cache.get(head.job_id)
                    if fp is None:
                        try:
                            fp = fp_cache[head.job_id] = self.footprint(head)
                        except Exception as e:      # invalid job: fails alone
                            fp = fp_cache[head.job_id] = -1
                            results[head.job_id].error = f"{type(e).__name__}: {e}"
                    if fp < 0 or fp > self.hbm_budget:
                        pending.popleft()
                        r = results[head.job_id]
                        if fp < 0:
                            r.status = "error"
                        else:
                            r.status, r.error = "rejected", "footprint exceeds the HBM budget"
                        r.admit = r.end = time.perf_counter() - t0
                        done += 1
                        continue
                    if used + fp <= self.hbm_budget:
                        admit(pending.popleft(), fp)
                        continue
                    if bypassed.get(head.job_id, 0) >= self.bypass_limit:
                        break
                    picked = None
                    for k in range(1, len(pending)):
                        cand = pending[k]
                        cfp = fp_cache.get(cand.job_id)
                        if cfp is None:
                            try:
                                cfp = fp_cache[cand.job_id] = self.footprint(cand)
                            except Exception as e:
                                cfp = fp_cache[cand.job_id] = -1
                                results[cand.job_id].error = f"{type(e).__name__}: {e}"
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
                cond.wait(timeout=wait if wait is not None else 0.5)
        ex.shutdown(wait=True)
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
    if not ok:
        return {"completed": 0, "failed": len(results)}
    lat = np.array([r.latency for r in ok]) * 1e3
    qw = np.array([r.queue_wait for r in ok]) * 1e3
    sv = np.array([r.service for r in ok]) * 1e3
    first = min(r.arrival for r in ok)
    last = max(r.end for r in ok)
    busy = _intervals_union([(r.start, r.end) for r in ok])
    return {
        "completed": len(ok), "failed": len(results) - len(ok),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "mean": float(lat.mean())},
        "queue_wait_ms": {"p50": float(np.percentile(qw, 50)), "p99": float(np.percentile(qw, 99))},
        "service_ms": {"p50": float(np.percentile(sv, 50)), "p99": float(np.percentile(sv, 99))},
        "makespan_s": float(last - first),
        "throughput_jobs_s": float(len(ok) / max(1e-9, last - first)),
        "gpu_busy_frac": float(busy / max(1e-9, last - first)),
        "max_bypassed": int(max(r.bypassed for r in ok)),
    }
