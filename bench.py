#!/usr/bin/env python3
"""Benchmark: Trotter-step GB/s of the DIA hot path on one MI355X.

Workload (default): 2-D transverse-field Ising model on a 5x5 open lattice
plus one idle ancilla (n = 26), J = 1, h = 3.04, random-phase initial state
(seed 3), t = 1.0 over 50 first-order Trotter steps (dt = 0.02), complex64
state (512 MiB), diagonal budget 16 -> 9 factors (8 x 15 diagonals + 1 x 3).

One timed "step" is one whole Trotter step: every factor applied once to
the resident state (the fused launch plan hs_evolve uses).  Inputs are in
HBM before timing starts.  value = algorithmic bytes of the step / step time,
where a launch's algorithmic bytes are every stored coefficient of its
factors read once plus the state read once and written once:
    sum_{factors f} sum_{d in D_f} (N - |d|) * 8  +  2 * B * N * 8.

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits: the library runs on a
single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Trotter-step state GB/s vs HBM peak at n=26; p50/p99 served-solve latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = {
    "workload": "tfim2d_5x5_plus_idle_ancilla",
    "n_qubits": 26, "J": 1.0, "h": 3.04, "t": 1.0, "trotter_steps": 50, "dt": 0.02,
    "budget": 16, "state": "random_phase_seed3", "batch": 1, "dtype": "complex64",
}
# sources that decide the tile kernel's code and launch plan
KERNEL_SRC = [os.path.join(ROOT, "paper_2606_16959_amd", "csrc", f)
              for f in ("kernels.hip", "hs_internal.h", "tile_plan.h", "api.hip", "storage_order.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dia_tile_tfim2d_n26.json")
OUT_DIR = os.path.join(ROOT, "profiles")      # where summaries are written (--out-dir)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _code_only(src: str) -> str:
    """The source with comments removed and white space collapsed, so that
    the hash below changes with the code, not with its comments."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_hash() -> str:
    """Hash of the kernel and launch-planning code (not its comments): the
    stored traffic counters are reported only while it matches."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def launch_bytes(desc, launches, N, batch, elem, seq=None):
    """Algorithmic bytes of each launch of one step (`seq`: the factor
    sequence the launch positions index; the lone step by default)."""
    out = []
    if seq is None:
        seq = desc.get("sequence") or list(range(len(desc["factors"])))
    for first, cnt in launches:
        facs = [desc["factors"][k] for k in seq[first:first + cnt]]
        coef = sum((N - abs(d)) * elem for f in facs for d in f["offsets"])
        out.append(coef + 2 * batch * N * elem)
    return out


def measured_traffic(per_launch_bytes, n_launches):
    """Average HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source and launch plan; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    per = t.get("bytes_per_launch_scaled") or []
    if t.get("kernel_sha") != kernel_hash() or len(per) != n_launches:
        return None
    return int(sum(per) / len(per))


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """Device-to-device copy GB/s (read + write), the achievable reference."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(H, psi0_c64, budget, t, steps_total, sample_steps, step_bytes):
    from oracle import evolve as oev, factors as ofac, pauli as opauli
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, budget, t / steps_total)
    psi = psi0_c64.astype(np.complex128)
    threads = oev.max_threads()
    t0 = time.perf_counter()
    oev.evolve(terms, part, psi, H.n, t / steps_total, 0)          # setup only (phase table)
    t1 = time.perf_counter()
    ref = oev.evolve(terms, part, psi, H.n, t / steps_total, sample_steps)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / sample_steps
    return {
        "value": round(step_bytes / per_step / 1e9, 3), "unit": "GB/s",
        "cores": threads, "kind": "oracle",
        "sample": f"{sample_steps} Trotter steps of the same n=26 workload (its whole run when 50), full state, FP64 "
                  f"(C + OpenMP, {threads} threads); setup (phase table, {t1 - t0:.2f} s) excluded; "
                  f"value = the step's algorithmic DIA bytes / oracle step time",
        "ms_per_step": round(per_step * 1e3, 1),
    }, ref


def accuracy(got, ref):
    """Error of GPU states against reference states ([B, N] or [N])."""
    from oracle import metrics
    g = np.atleast_2d(np.asarray(got, dtype=np.complex128))
    r = np.atleast_2d(np.asarray(ref, dtype=np.complex128))
    fid = metrics.fidelity(g, r)
    return {"min_fidelity": float(np.min(fid)), "max_abs_err": float(np.abs(g - r).max()),
            "max_norm_drift": float(np.max(np.abs(np.linalg.norm(g, axis=1) - 1.0)))}


def serve_leg(torch, n_jobs, rate, slots, oracle_nmax, jsonl_dir=None):
    """Served stream (seeded Poisson arrivals of mixed-family jobs) and the
    oracle check of a 5% sample (jobs whose id hashes into the sample and
    whose n <= oracle_nmax, every n by default; state column 0, the whole run
    of the job, after the stream).  With jsonl_dir, every job's record is
    appended to serve_<jobs>jobs_<rate>per_s.jsonl there."""
    from oracle import evolve as oev, factors as ofac, metrics, pauli as opauli
    from paper_2606_16959_amd.serve import Job, Server
    from workloads.serve_stream import job_stream
    specs = job_stream(n_jobs=n_jobs, rate=rate, seed=5)
    sample = {s.job_id for s in specs
              if int(hashlib.sha256(f"5:{s.job_id}".encode()).hexdigest(), 16) % 20 == 0}
    jobs = []
    for sp in specs:
        H = sp.hamiltonian()
        jobs.append(Job(sp.job_id, H.strings, H.coeffs, H.n, sp.t, sp.steps, sp.batch, sp.state_seed,
                        arrival=sp.arrival, keep_result=sp.job_id in sample and sp.n <= oracle_nmax,
                        tag=sp.family))
    log(f"serve: {n_jobs} jobs at {rate}/s on {slots} slots")
    jsonl = None
    if jsonl_dir:
        os.makedirs(jsonl_dir, exist_ok=True)
        jsonl = os.path.join(jsonl_dir, f"serve_{n_jobs}jobs_{rate:g}per_s.jsonl")
    res, st = Server(slots=slots).run(jobs, jsonl=jsonl)
    log(f"serve: p50 {st['latency_ms']['p50']:.1f} ms p99 {st['latency_ms']['p99']:.1f} ms "
        f"{st['throughput_jobs_s']:.1f} jobs/s")
    worst, checked, t_or = 1.0, 0, time.perf_counter()
    for sp, job, r in zip(specs, jobs, res):
        if not job.keep_result or r.status != "ok":
            continue
        H = sp.hamiltonian()
        terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
        part = ofac.first_fit(terms, job.budget, job.t / job.steps)
        ref = oev.evolve(terms, part, r.psi0[0].astype(np.complex128), H.n, job.t / job.steps, job.steps)
        worst = min(worst, float(metrics.fidelity(r.psi[0].astype(np.complex128), ref)))
        checked += 1
    sampled = sum(1 for sp in specs if sp.job_id in sample and sp.n <= oracle_nmax)
    log(f"serve: oracle checked {checked} of {sampled} sampled jobs in {time.perf_counter() - t_or:.1f} s")
    st.update(jobs=n_jobs, rate_jobs_s=rate, oracle_sample=len(sample), oracle_sampled_checkable=sampled,
              oracle_checked=checked, oracle_min_fidelity=worst, oracle_nmax=oracle_nmax,
              families="tfim/heisenberg/maxcut/tsp", n_range=[10, 24])
    return st


def summarize_profiles(trace_dir, fetch_dir, write_dir, command, extra_dirs=(), bench_trace=None, bench_log=None):
    """Turn rocprofv3 CSV output of bench.py runs into the committed summaries:
    per-kernel durations (trace) and per-launch HBM bytes of the DIA tile
    kernel from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by
    what the same counter reads for the 2 GiB device copies the run makes.
    bench_trace: a kernel trace of the default bench run itself, whose first
    tile dispatches are the headline's warm-up and timed steps; their
    durations are set beside the bench line of that run (bench_log), since
    where the 65 GB of diagonals land in HBM moves the step time by a few
    percent from one process to the next."""
    import csv
    import glob

    def rows(d, pattern):
        out = []
        for fn in glob.glob(os.path.join(d, "**", pattern), recursive=True):
            with open(fn) as fh:
                out += list(csv.DictReader(fh))
        return out

    stats = rows(trace_dir, "*kernel_stats.csv")
    trace = sorted(rows(trace_dir, "*kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    tile = [r for r in trace if _step_kernel(r["Kernel_Name"])]
    os.makedirs(OUT_DIR, exist_ok=True)
    md = ["# dia_tile_kernel on tfim2d 5x5 + ancilla, n=26, complex64, budget 16", "",
          "Command (repository root, on the MI355X):", "", "```", command, "```", "",
          "## rocprofv3 --kernel-trace --stats summary", "",
          "| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in stats:
        md.append(f"| {r['Name'][:70]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    # per-launch position within a step (launches repeat each step)
    fetch = sorted(rows(fetch_dir, "*counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"]))
    write = sorted(rows(write_dir, "*counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"]))

    def copies(rs):
        return [r for r in rs if "copyBuffer" in r["Kernel_Name"]]
    wcopy = [float(r["Counter_Value"]) for r in copies(write)]
    big = max(wcopy) if wcopy else 0.0
    fcopy = [float(r["Counter_Value"]) for r in copies(fetch)]
    expected_kib = (1 << 31) / 1024.0
    f_scale = expected_kib / (sorted(fcopy)[-1] if fcopy else expected_kib)
    w_scale = expected_kib / big if big else 1.0
    ft = [float(r["Counter_Value"]) for r in fetch if _step_kernel(r["Kernel_Name"])]
    wt = [float(r["Counter_Value"]) for r in write if _step_kernel(r["Kernel_Name"])]
    nl = 3
    per = []
    for j in range(nl):
        fk = ft[j::nl]
        wk = wt[j::nl]
        per.append(int((sum(fk) / len(fk) * f_scale + sum(wk) / len(wk) * w_scale) * 1024))
    durs = [[] for _ in range(nl)]
    for i, r in enumerate(tile):
        durs[i % nl].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    reqc = {}
    for d in extra_dirs:
        rs = sorted(rows(d, "*counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"]))
        for name in {r["Counter_Name"] for r in rs}:
            reqc[name] = [float(r["Counter_Value"]) for r in rs
                          if r["Counter_Name"] == name and _step_kernel(r["Kernel_Name"])]
            cp = [float(r["Counter_Value"]) for r in rs if r["Counter_Name"] == name and "copyBuffer" in r["Kernel_Name"]]
            reqc["copy:" + name] = [max(cp)] if cp else []
    forms = [("pair" if "dia_pair_kernel" in r["Kernel_Name"] else "row") for r in tile[:nl]]
    md += ["", "## HBM traffic of the DIA tile kernel per launch position in a step", "",
           f"Copy calibration: a 2 GiB device copy reads {sorted(fcopy)[-1] if fcopy else 0:.0f} KiB "
           f"(FETCH_SIZE) and writes {big:.0f} KiB (WRITE_SIZE); scale factors {f_scale:.4f} "
           f"and {w_scale:.4f}.", ""]
    req_ok = request_bytes(reqc, 0, nl) is not None
    hdr = "| launch | kernel form | avg ms | FETCH KiB | WRITE KiB | scaled GB |"
    if req_ok:
        hdr += " request-size GB |"
    md += [hdr, "|" + "---|" * (hdr.count("|") - 1)]
    for j in range(nl):
        line = (f"| {j} | {forms[j]} | {sum(durs[j]) / max(1, len(durs[j])):.3f} | {sum(ft[j::nl]) / len(ft[j::nl]):.0f} | "
                f"{sum(wt[j::nl]) / len(wt[j::nl]):.0f} | {per[j] / 1e9:.3f} |")
        if req_ok:
            rd, wr = request_bytes(reqc, j, nl)
            line += f" {(rd + (wr or 0)) / 1e9:.3f} |"
        md.append(line)
    if req_ok:
        cr = {k[5:]: v for k, v in reqc.items() if k.startswith("copy:")}
        crd = request_bytes(cr)
        md += ["", "Request-size bytes (128 TCC_EA0_RDREQ_128B + 64 TCC_EA0_RDREQ_64B + 32 TCC_EA0_RDREQ_32B read, "
               "64 TCC_EA0_WRREQ_64B + 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B) written) need no calibration: "
               + (f"for the 2 GiB copy they give {crd[0] / 2**30:.3f} GiB read and {(crd[1] or 0) / 2**30:.3f} GiB "
                  "written. " if crd else "")
               + "FETCH_SIZE's formula counts each request that is neither a bubble nor 32 bytes as 64 bytes, so "
               "on 128-byte requests it reads half the bytes: the copy calibration's factor 2."]
    md += ["", f"Average over the {nl} launches of a step: "
           f"{float(np.mean([sum(x) / max(1, len(x)) for x in durs])):.4f} ms per launch."]
    if bench_trace:
        line = None
        if bench_log:
            with open(bench_log) as fh:
                for ln in fh:
                    if ln.startswith('{"metric"'):
                        line = json.loads(ln)
        warm, steps = (line["warmup"], line["steps"]) if line else (3, 20)
        bt = sorted((r for r in rows(bench_trace, "*kernel_trace.csv") if _step_kernel(r["Kernel_Name"])),
                    key=lambda r: int(r["Start_Timestamp"]))[warm * nl:(warm + steps) * nl]
        bd = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in bt]
        pos = [float(np.mean(bd[j::nl])) for j in range(nl)]
        md += ["", "## The bench run itself", "",
               f"Kernel trace of the default `python3 bench.py` run (rocprofv3 --kernel-trace), its {steps} timed "
               f"headline steps after {warm} warm-up steps: the first {(warm + steps) * nl} tile dispatches of the "
               "process.", "", "| launch | kernel form | avg ms | algorithmic GB | GB/s |", "|---|---|---|---|---|"]
        alg = line["roofline"]["algorithmic_bytes_per_launch"] if line else [None] * nl
        for j in range(nl):
            gbs = f"{alg[j] / (pos[j] * 1e-3) / 1e9:.0f}" if alg[j] else "-"
            gb = f"{alg[j] / 1e9:.3f}" if alg[j] else "-"
            md.append(f"| {j} | {forms[j]} | {pos[j]:.3f} | {gb} | {gbs} |")
        md += ["", f"Average launch: {float(np.mean(bd)):.4f} ms in the trace"
               + (f"; the same run's bench line (HIP events on the launch stream): {line['roofline']['avg_launch_ms']} "
                  f"ms per launch, {line['ms_per_step']} ms per step, {line['value']} GB/s = "
                  f"{line['roofline']['frac']:.4f} of 8 TB/s." if line else ".")]
    with open(os.path.join(OUT_DIR, "dia_tile_tfim2d_n26.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    with open(os.path.join(OUT_DIR, os.path.basename(TRAFFIC_FILE)), "w") as fh:
        json.dump({"kernel_sha": kernel_hash(), "bytes_per_launch_scaled": per,
                   "fetch_scale": f_scale, "write_scale": w_scale, "command": command}, fh, indent=1)
    print("\n".join(md))


SWEEP = [
    ("default", {}),
    ("no_xcd_swizzle", {"HAMSIM_XCD_SWIZZLE": "0"}),
    ("swizzle_all_launches", {"HAMSIM_XCD_SWIZZLE": "1"}),
    ("swizzle_strided_only", {"HAMSIM_XCD_SWIZZLE": "2"}),
    ("wmin512", {"HAMSIM_WMIN_BYTES": "512"}),
    ("wmin1024", {"HAMSIM_WMIN_BYTES": "1024"}),
    ("wmin2048", {"HAMSIM_WMIN_BYTES": "2048"}),
    ("fuse1", {"HAMSIM_MAX_FUSE": "1"}),
    ("fuse3", {"HAMSIM_MAX_FUSE": "3"}),
    ("pair_kernel_all", {"HAMSIM_PAIR_LDS": "2"}),
    ("pair_kernel_off", {"HAMSIM_PAIR_LDS": "0"}),
]


def sweep(torch, steps, warmup, passes=3):
    """Launch-plan variants of the same workload (environment knobs of the
    library; one handle keeps a plan per setting), timed in interleaved passes
    (median); writes a summary under profiles/."""
    import paper_2606_16959_amd as hs
    from workloads import workload_hamiltonian, states as ws
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    N = 1 << H.n
    psi0 = ws.random_phase_state(H.n, 3, np.complex64)
    f = hs.build_factors(H.strings, H.coeffs, H.n, 1.0, 50, 16, dtype="c64")
    desc = f.describe()

    def with_env(env, fn):
        saved = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            return fn()
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v

    variants = []
    for name, env in SWEEP:
        launches = with_env(env, lambda: f.step_launches(1))   # the plan for this setting
        per = launch_bytes(desc, launches, N, 1, 8)
        variants.append({"name": name, "env": env, "launches": len(launches),
                         "bytes": sum(per), "ms": []})
    psi = torch.from_numpy(psi0).cuda()
    ref = None
    for rnd in range(passes):
        for v in variants:
            psi.copy_(torch.from_numpy(psi0).cuda())

            def run():
                for _ in range(warmup):
                    hs.evolve(f, psi, 1)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(steps):
                    hs.evolve(f, psi, 1)
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / steps
            v["ms"].append(with_env(v["env"], run))
            if rnd == 0:
                out = psi.cpu().numpy()
                v["same"] = bool(ref is None or np.array_equal(out, ref))
                ref = out if ref is None else ref
        log(f"sweep pass {rnd} done")
    md = ["# Launch-plan sweep: dia_tile_kernel, tfim2d 5x5 + ancilla, n=26, complex64", "",
          "Command (repository root, on the MI355X): `python3 bench.py --sweep`", "",
          f"Per variant: {warmup} warm-up + {steps} timed steps, repeated in {passes} interleaved "
          "passes; median ms/step. Every variant's state after the first pass is compared bit for "
          "bit with the first variant's.", "",
          "| variant | environment | launches/step | GB/step | ms/step (median) | min..max | GB/s | % of 8 TB/s | same result |",
          "|---|---|---|---|---|---|---|---|---|"]
    for v in variants:
        ms = float(np.median(v["ms"]))
        gbs = v["bytes"] / ms / 1e6
        envs = " ".join(f"{k}={x}" for k, x in v["env"].items()) or "-"
        md.append(f"| {v['name']} | {envs} | {v['launches']} | {v['bytes'] / 1e9:.2f} | {ms:.3f} | "
                  f"{min(v['ms']):.3f}..{max(v['ms']):.3f} | {gbs:.1f} | {100 * gbs / HBM_PEAK_GBS:.1f} | {v['same']} |")
    f.close()
    with open(os.path.join(OUT_DIR, "sweep_launch_plan_tfim2d_n26.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


# steps checked against the oracle: the whole stated run of each workload
ACCURACY_STEPS = {"tfim_chain_n8": 10, "heisenberg_chain_n20": 100, "maxcut_3reg_n24": 200}
BACKGROUND_ORACLE = {"maxcut_3reg_n24"}    # its 8 x 200 oracle steps run beside the GPU-only legs


def other_workloads(torch, steps=10, warmup=2, pool=None):
    """The other named workloads in the same harness: per-step time
    and algorithmic GB/s (n <= 20 states stay in the 256 MB last-level cache,
    so only n = 24 and n = 26 figures are HBM-bound).  With `pool`, the
    long oracle runs are submitted there; the row's "accuracy_vs_oracle" is
    then a future, resolved by resolve_pending()."""
    import paper_2606_16959_amd as hs
    from workloads import workload_hamiltonian, states as ws
    from workloads.hamiltonians import WORKLOAD_RUN
    from oracle import evolve as oev, factors as ofac, pauli as opauli
    out = []
    oracle_refs, c128_states = {}, {}
    cases = [("tfim_chain_n8", "c128", False), ("heisenberg_chain_n20", "c128", False),
             ("heisenberg_chain_n20", "c64", False), ("maxcut_3reg_n24", "c64", False),
             ("tfim_5x5_ancilla_n26", "c64", True)]
    for cfg, dtype, renorm in cases:
        H = workload_hamiltonian(cfg)
        run = WORKLOAD_RUN[cfg]
        npd = np.complex128 if dtype == "c128" else np.complex64
        elem = 16 if dtype == "c128" else 8
        f = hs.build_factors(H.strings, H.coeffs, H.n, run["t"], run["steps"], run["budget"], dtype=dtype)
        B = run["batch"]
        launches = f.step_launches(B)
        per = launch_bytes(f.describe(), launches, 1 << H.n, B, elem)
        psi = torch.from_numpy(np.ascontiguousarray(ws.workload_states(cfg, npd))).cuda()
        for _ in range(warmup):
            hs.evolve(f, psi, 1, renorm=renorm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            hs.evolve(f, psi, 1, renorm=renorm)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        row = {"workload": cfg, "n": H.n, "batch": B, "dtype": dtype, "renorm": renorm,
               "launches_per_step": len(launches), "ms_per_step": round(ms, 4),
               "gb_per_step": round(sum(per) / 1e9, 3), "gbs": round(sum(per) / ms / 1e6, 1)}
        if H.n <= 11 and not renorm:
            # small states: the whole stated run is one call (one launch of the
            # whole-evolution kernel), timed as a run
            e0.record()
            for _ in range(5):
                hs.evolve(f, psi, run["steps"])
            e1.record()
            torch.cuda.synchronize()
            row["ms_per_run"] = round(e0.elapsed_time(e1) / 5, 4)
            row["run_steps"] = run["steps"]
        if B > 1:
            row["ms_per_state_step"] = round(ms / B, 4)
        if cfg in ACCURACY_STEPS:
            # error against the FP64 oracle over the first k steps from the
            # workload's initial states (complex64 also against complex128)
            k = ACCURACY_STEPS[cfg]
            psi0 = np.ascontiguousarray(ws.workload_states(cfg, np.complex128))
            pa = torch.from_numpy(psi0.astype(npd)).cuda()
            hs.evolve(f, pa, k)
            got = pa.cpu().numpy()
            terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
            part = ofac.first_fit(terms, run["budget"], run["t"] / run["steps"])
            job = (lambda terms=terms, part=part, psi0=psi0, n=H.n, dt=run["t"] / run["steps"], k=k, th=0:
                   oev.evolve(terms, part, psi0, n, dt, k, threads=th))
            if pool is not None and cfg in BACKGROUND_ORACLE:
                # beside the GPU legs: leave two host cores to the thread that
                # enqueues their launches (with every core busy, legs of short
                # launches measured up to 20% slower)
                fut = pool.submit(job, th=max(1, oev.max_threads() - 2))
                row["accuracy_vs_oracle"] = ("pending", fut, got, k)
            else:
                if cfg not in oracle_refs:
                    oracle_refs[cfg] = job()
                row["accuracy_vs_oracle"] = dict(accuracy(got, oracle_refs[cfg]), steps=k)
            if dtype == "c128":
                c128_states[cfg] = got
            elif cfg in c128_states:
                row["fidelity_vs_c128_gpu"] = accuracy(got, c128_states[cfg])["min_fidelity"]
            del pa
        out.append(row)
        log(f"{cfg} {dtype} B={B} renorm={renorm}: {ms:.4f} ms/step {row['gbs']} GB/s")
        f.close()
        del psi
        torch.cuda.empty_cache()
    return out


def resolve_pending(rows):
    """Wait for background oracle runs and fill in their accuracy."""
    for row in rows:
        acc = row.get("accuracy_vs_oracle")
        if isinstance(acc, tuple) and acc and acc[0] == "pending":
            _, fut, got, k = acc
            t0 = time.perf_counter()
            row["accuracy_vs_oracle"] = dict(accuracy(got, fut.result()), steps=k, states=int(got.shape[0]))
            log(f"{row['workload']} vs oracle ({k} steps, waited {time.perf_counter() - t0:.1f} s): "
                f"{row['accuracy_vs_oracle']}")
    return rows


def complex128_leg(torch, H, psi0, ref, ref_steps, state_c64, steps_total, budget, timed=10, warmup=2):
    """The plain complex128 path on the headline workload: per-step time and
    algorithmic GB/s of its own launches, and the whole run's error against
    the FP64 oracle (ref, after ref_steps steps) and against the complex64
    GPU state after the same steps."""
    import paper_2606_16959_amd as hs
    N = 1 << H.n
    f = hs.build_factors(H.strings, H.coeffs, H.n, 1.0, steps_total, budget, dtype="c128")
    launches = f.step_launches(1)
    per = launch_bytes(f.describe(), launches, N, 1, 16)
    psi = torch.from_numpy(psi0.astype(np.complex128)).cuda()
    hs.evolve(f, psi, warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(timed):
        hs.evolve(f, psi, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / timed
    k = ref_steps
    psi.copy_(torch.from_numpy(psi0.astype(np.complex128)))
    hs.evolve(f, psi, k)
    got = psi.cpu().numpy()
    f.close()
    del psi
    torch.cuda.empty_cache()
    gbs = sum(per) / ms / 1e6
    out = {"workload": "tfim2d_5x5_plus_idle_ancilla", "n": H.n, "dtype": "c128", "batch": 1,
           "launches_per_step": len(launches), "ms_per_step": round(ms, 4),
           "gb_per_step": round(sum(per) / 1e9, 3), "gbs": round(gbs, 1),
           "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
           "accuracy_vs_oracle": dict(accuracy(got, ref), steps=k),
           "fidelity_c64_vs_c128": accuracy(state_c64, got)["min_fidelity"]}
    log(f"complex128 n=26: {ms:.3f} ms/step {out['gbs']} GB/s; vs oracle {out['accuracy_vs_oracle']}; "
        f"c64 vs c128 fidelity {out['fidelity_c64_vs_c128']}")
    return out


def diagonal_leg(torch, n=26, steps=200, timed=10, seed=26):
    """Diagonal-only Hamiltonian (the MaxCut cost of a seeded 3-regular graph,
    no mixer, n = 26, complex64, t = 1): one step is the single-diagonal
    factor exp(-i dt E).  Timed step by step (one pass per step) and as the
    whole run in one pass (the library applies all steps of a diagonal step
    per entry in registers).  Algorithmic bytes per pass: the diagonal once,
    the state read and written: 3 N 8."""
    import paper_2606_16959_amd as hs
    from workloads import hamiltonians as wh, states as ws
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = wh.random_regular_graph(n, 3, rng)
    H = wh.maxcut(n, edges, rng.uniform(1.0, 10.0, len(edges)), mixer=0.0)
    N = 1 << n
    f = hs.build_factors(H.strings, H.coeffs, n, 1.0, steps, 16, dtype="c64")
    assert f.n_factors == 1
    psi = torch.from_numpy(ws.random_phase_state(n, 5, np.complex64)).cuda()
    nbytes = 3 * N * 8
    hs.evolve(f, psi, 1)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(timed):
        hs.evolve(f, psi, 1)
    e1.record()
    hs.evolve(f, psi, steps)
    e2.record()
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1) / timed
    msr = e1.elapsed_time(e2)
    f.close()
    del psi
    torch.cuda.empty_cache()
    out = {"workload": f"maxcut_cost_3reg_n{n}_no_mixer", "n": n, "dtype": "c64", "batch": 1,
           "gb_per_pass": round(nbytes / 1e9, 3),
           "one_step_per_pass": {"ms_per_step": round(ms1, 4), "gbs": round(nbytes / ms1 / 1e6, 1),
                                 "frac_of_peak": round(nbytes / ms1 / 1e6 / HBM_PEAK_GBS, 4)},
           "all_steps_one_pass": {"steps": steps, "ms": round(msr, 4), "ms_per_step": round(msr / steps, 5),
                                  "gbs": round(nbytes / msr / 1e6, 1),
                                  "frac_of_peak": round(nbytes / msr / 1e6 / HBM_PEAK_GBS, 4)}}
    log(f"diagonal n={n}: {ms1:.4f} ms/step ({out['one_step_per_pass']['gbs']} GB/s); "
        f"{steps} steps in one pass {msr:.3f} ms ({out['all_steps_one_pass']['gbs']} GB/s)")
    return out


def higher_order_leg(torch, steps=10, warmup=3):
    """The symmetric second-order and fourth-order Suzuki products on the
    n = 26 2-D TFIM (complex64, budget 16), timed as one evolution of `steps`
    steps so that steps meet in the joint factor.  Algorithmic bytes: every
    launch's coefficient diagonals plus the state read and written, summed
    over the first, middle and last steps' launch lists."""
    import paper_2606_16959_amd as hs
    from workloads import workload_hamiltonian, states as ws
    from workloads.hamiltonians import WORKLOAD_RUN
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    run = WORKLOAD_RUN["tfim_5x5_ancilla_n26"]
    N = 1 << H.n
    out = []
    for order in (2, 4):
        f = hs.build_factors(H.strings, H.coeffs, H.n, run["t"], run["steps"], run["budget"],
                             dtype="c64", order=order)
        desc = f.describe()
        parts = {p: launch_bytes(desc, f.step_launches(1, part=p), N, 1, 8, f.part_sequence(p, desc))
                 for p in (1, 2, 3)}
        nbytes = sum(parts[1]) + (steps - 2) * sum(parts[2]) + sum(parts[3])
        n_launch = len(parts[1]) + (steps - 2) * len(parts[2]) + len(parts[3])
        psi = torch.from_numpy(np.ascontiguousarray(ws.workload_states("tfim_5x5_ancilla_n26", np.complex64))).cuda()
        hs.evolve(f, psi, warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hs.evolve(f, psi, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        row = {"workload": "tfim2d_5x5_plus1_n26", "order": order, "dtype": "c64",
               "stored_factors": len(desc["factors"]),
               "factor_gb": round(sum(x["bytes"] for x in desc["factors"]) / 1e9, 2),
               "factors_per_step": len(f.part_sequence(2, desc)),
               "launches_per_step": round(n_launch / steps, 2), "ms_per_step": round(ms, 3),
               "gb_per_step": round(nbytes / steps / 1e9, 2),
               "gbs": round(nbytes / steps / ms / 1e6, 1)}
        row["frac_of_peak"] = round(row["gbs"] / HBM_PEAK_GBS, 4)
        out.append(row)
        log(f"order {order}: {ms:.3f} ms/step {row['gbs']} GB/s {row['launches_per_step']} launches/step")
        f.close()
        del psi
        torch.cuda.empty_cache()
    return out


def taylor_leg(torch, cases=None, timed_steps=3):
    """The Taylor expansion fused into the state update (complex64): H's
    diagonals once, r = smallest step count with |dt| nu(H) <= 1, K from the
    1e-6 tolerance, each step K Horner stages (one DIA SpMV of H with the
    update in its epilogue).  Algorithmic bytes per stage: every stored
    diagonal of H once, plus the state read (partners), the step's input read
    (epilogue) and the output written."""
    import paper_2606_16959_amd.dia as hd
    from workloads import workload_hamiltonian, hamiltonians as wh, states as ws
    cases = cases or [("tfim1d_n24_h1_t1", lambda: wh.tfim_1d(24, 1.0, 1.0)),
                      ("tfim2d_5x5_plus1_n26_t1", lambda: workload_hamiltonian("tfim_5x5_ancilla_n26"))]
    out = []
    for name, make in cases:
        Hw = make()
        n, N = Hw.n, 1 << Hw.n
        t0 = time.perf_counter()
        H = hd.from_pauli(Hw.strings, Hw.coeffs, n)
        nu = hd.norm_bound(H)
        r = hd.taylor_steps(H, 1.0)
        K = hd.taylor_terms(H, 1.0 / r)
        H64 = H.to_c64()
        offs = H64.offsets
        H.close()
        setup_s = time.perf_counter() - t0
        psi = torch.from_numpy(ws.random_phase_state(n, 7, np.complex64)).cuda()
        hd.taylor_evolve(H64, psi, 1.0 / r, K, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hd.taylor_evolve(H64, psi, 1.0 / r, K, timed_steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / timed_steps
        stage_bytes = sum((N - abs(d)) * 8 for d in offs) + 3 * N * 8
        row = {"workload": name, "n": n, "dtype": "c64", "nu": round(nu, 4), "steps_for_t1": r,
               "taylor_terms": K, "h_diagonals": len(offs), "setup_s": round(setup_s, 3),
               "ms_per_step": round(ms, 4), "ms_per_stage": round(ms / K, 4),
               "gb_per_stage": round(stage_bytes / 1e9, 3),
               "gbs": round(stage_bytes * K / ms / 1e6, 1),
               "full_run_s_estimate": round(ms * r / 1e3, 3),
               "dispatches": K * (1 + timed_steps)}
        row["frac_of_peak"] = round(row["gbs"] / HBM_PEAK_GBS, 4)
        out.append(row)
        log(f"taylor {name}: r={r} K={K} {ms:.3f} ms/step {row['gbs']} GB/s; t=1 in {row['full_run_s_estimate']} s")
        H64.close()
        del psi
        torch.cuda.empty_cache()
    return out


def one_workload_leg(torch, name, dtype, steps=5, warmup=2, batch=None):
    """One named workload alone (for profiling): `warmup` + `steps` Trotter
    steps of its states, then one 2 GiB device copy that calibrates the HBM
    counters.  Reports the launches of one step with their algorithmic bytes,
    so a counter summary can be set against them."""
    import paper_2606_16959_amd as hs
    from workloads import workload_hamiltonian, states as ws
    from workloads.hamiltonians import WORKLOAD_RUN
    H = workload_hamiltonian(name)
    run = WORKLOAD_RUN[name]
    npd = np.complex128 if dtype == "c128" else np.complex64
    elem = 16 if dtype == "c128" else 8
    B = batch or run["batch"]
    f = hs.build_factors(H.strings, H.coeffs, H.n, run["t"], run["steps"], run["budget"], dtype=dtype)
    launches = f.step_launches(B)
    per = launch_bytes(f.describe(), launches, 1 << H.n, B, elem)
    states = ws.workload_states(name, npd)
    psi = torch.from_numpy(np.ascontiguousarray(np.resize(states, (B, states.shape[1])))).cuda()
    hs.evolve(f, psi, warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hs.evolve(f, psi, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    f.close()
    del psi
    torch.cuda.empty_cache()
    copy_bandwidth(torch, reps=1)
    return {"workload": name, "n": H.n, "dtype": dtype, "batch": B, "warmup": warmup, "steps": steps,
            "launches_per_step": len(launches), "launch_factors": [c for _, c in launches],
            "algorithmic_bytes_per_launch": [int(b) for b in per], "ms_per_step": round(ms, 4),
            "gb_per_step": round(sum(per) / 1e9, 3), "gbs": round(sum(per) / ms / 1e6, 1),
            "frac_of_peak": round(sum(per) / ms / 1e6 / HBM_PEAK_GBS, 4)}


def _step_kernel(name):
    """The DIA tile kernel in either form (row by row, or the pair form of
    closed complex64 launches whose diagonals all pair)."""
    return "dia_tile_kernel" in name or "dia_pair_kernel" in name


def request_bytes(counters, j=None, L=1):
    """HBM bytes from the request-size counters of the L2 (TCC) to memory:
    reads 128 / 64 / 32 bytes per request by size class, writes 64 or 32.
    `counters` maps counter name -> per-dispatch values; j selects every L-th
    dispatch from position j.  Returns (read bytes, write bytes) or None."""
    def m(c):
        v = counters.get(c)
        if not v:
            return None
        v = v[j::L] if j is not None else v
        return float(np.mean(v)) if v else None
    r128, r64, r32 = m("TCC_EA0_RDREQ_128B_sum"), m("TCC_EA0_RDREQ_64B_sum"), m("TCC_EA0_RDREQ_32B_sum")
    w, w64 = m("TCC_EA0_WRREQ_sum"), m("TCC_EA0_WRREQ_64B_sum")
    if None in (r128, r64, r32):
        return None
    rd = 128 * r128 + 64 * r64 + 32 * r32
    wr = None if None in (w, w64) else 64 * w64 + 32 * (w - w64)
    return rd, wr


def _csv_rows(d, pattern):
    import csv
    import glob
    out = []
    for fn in sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True)):
        with open(fn) as fh:
            out += list(csv.DictReader(fh))
    return out


def summarize_leg_profiles(leg_output, trace_dir, counter_dirs, out_name, command):
    """Per-launch summary of the DIA tile kernel from rocprofv3 output of a
    `bench.py --leg workload` run: durations from the kernel trace, and from
    each counter run (one directory per pass) the per-dispatch counter values,
    averaged per launch position of a step.  FETCH_SIZE and WRITE_SIZE (KiB)
    are scaled by what the same counters read for the leg's 2 GiB device copy
    and set against the launch's algorithmic bytes."""
    leg = None
    with open(leg_output) as fh:
        for line in fh:
            if line.startswith('{"leg"'):
                leg = json.loads(line)["result"]
                break
    if leg is None:
        raise SystemExit(f"no leg output in {leg_output}")
    L = leg["launches_per_step"]
    alg = leg["algorithmic_bytes_per_launch"]
    trace = sorted((r for r in _csv_rows(trace_dir, "*kernel_trace.csv") if _step_kernel(r["Kernel_Name"])),
                   key=lambda r: int(r["Dispatch_Id"]))
    forms = [("pair" if "dia_pair_kernel" in r["Kernel_Name"] else "row") for r in trace[-L:]]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace]
    if len(durs) % L:
        raise SystemExit(f"{len(durs)} tile dispatches is not a multiple of {L} launches per step")
    pos_ms = [float(np.mean(durs[j::L])) for j in range(L)]
    counters = {}                      # name -> [per tile dispatch], plus the copy's value
    copy_val = {}
    for d in counter_dirs:
        rows = sorted(_csv_rows(d, "*counter_collection.csv"), key=lambda r: int(r["Dispatch_Id"]))
        for name in sorted({r["Counter_Name"] for r in rows}):
            mine = [r for r in rows if r["Counter_Name"] == name]
            counters[name] = [float(r["Counter_Value"]) for r in mine if _step_kernel(r["Kernel_Name"])]
            cp = [float(r["Counter_Value"]) for r in mine if "copyBuffer" in r["Kernel_Name"]]
            if cp:
                copy_val[name] = max(cp)
    copy_kib = (1 << 31) / 1024.0
    md = [f"# dia_tile_kernel: {leg['workload']}, n={leg['n']}, {leg['dtype']}, {leg['batch']} state(s) per launch", "",
          "Command (repository root, on the MI355X):", "", "```", command, "```", "",
          f"Leg: {leg['warmup']} warm-up + {leg['steps']} timed Trotter steps; {L} launches per step "
          f"(factors per launch {leg['launch_factors']}); {leg['ms_per_step']} ms/step from HIP events, "
          f"{leg['gb_per_step']} algorithmic GB/step, {leg['gbs']} GB/s = {100 * leg['frac_of_peak']:.1f}% of 8 TB/s.", ""]
    hdr = ["launch", "kernel form", "avg ms (trace)", "algorithmic GB", "algorithmic GB/s"]
    scaled = {}
    for cname in ("FETCH_SIZE", "WRITE_SIZE"):
        if cname in counters and copy_val.get(cname):
            scaled[cname] = copy_kib / copy_val[cname]
    if scaled:
        md += ["Copy calibration (2 GiB device copy in the same run): " +
               ", ".join(f"{c} reads {copy_val[c]:.0f} KiB, scale {s:.4f}" for c, s in scaled.items()), ""]
        hdr += ["HBM GB (scaled FETCH + WRITE)", "HBM / algorithmic"]
    other = [c for c in sorted(counters) if c not in ("FETCH_SIZE", "WRITE_SIZE")]
    req = request_bytes(counters, 0, L) is not None
    reads_only = req and request_bytes(counters, 0, L)[1] is None
    wbytes = leg["batch"] * (1 << leg["n"]) * (16 if leg["dtype"] == "c128" else 8)   # the states written once
    if req:
        hdr += (["HBM read GB (request sizes)", "read / algorithmic read"] if reads_only
                else ["HBM GB (request sizes)", "request / algorithmic"])
    hdr += other
    md += ["| " + " | ".join(hdr) + " |", "|" + "---|" * len(hdr)]
    for j in range(L):
        row = [str(j), forms[j], f"{pos_ms[j]:.4f}", f"{alg[j] / 1e9:.3f}", f"{alg[j] / pos_ms[j] / 1e6:.0f}"]
        if scaled:
            hb = sum(float(np.mean(counters[c][j::L])) * s * 1024 for c, s in scaled.items())
            row += [f"{hb / 1e9:.3f}", f"{hb / alg[j]:.3f}"]
        if req:
            rd, wr = request_bytes(counters, j, L)
            if reads_only:
                row += [f"{rd / 1e9:.3f}", f"{rd / (alg[j] - wbytes):.3f}"]
            else:
                row += [f"{(rd + wr) / 1e9:.3f}", f"{(rd + wr) / alg[j]:.3f}"]
        for c in other:
            v = counters[c][j::L]
            row.append(f"{float(np.mean(v)):.4g}" if v else "-")
        md.append("| " + " | ".join(row) + " |")
    if req:
        md += ["", "Request sizes: read bytes = 128 TCC_EA0_RDREQ_128B + 64 TCC_EA0_RDREQ_64B + 32 TCC_EA0_RDREQ_32B, "
               "write bytes = 64 TCC_EA0_WRREQ_64B + 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B), summed over the L2 "
               "channels.  FETCH_SIZE's formula counts every request that is neither a bubble nor 32 bytes as 64 "
               "bytes, so on 128-byte requests it reads half the bytes (the copy calibration's factor 2)."]
    md += ["", f"Average over the {L} launches of a step: {float(np.mean(pos_ms)):.4f} ms per launch, "
           f"{sum(alg) / len(alg) / 1e9:.3f} algorithmic GB per launch."]
    stats = _csv_rows(trace_dir, "*kernel_stats.csv")
    md += ["", "## rocprofv3 --kernel-trace --stats", "",
           "| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in stats[:6]:
        md.append(f"| {r['Name'][:95]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    os.makedirs(OUT_DIR, exist_ok=True)
    with open(os.path.join(OUT_DIR, out_name), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_diagonal_profiles(leg_output, trace_dir, fetch_dir, write_dir, command):
    """Profile summary of `bench.py --leg diagonal`: the single-diagonal
    kernel's dispatches in order (one warm-up pass, the timed one-step passes,
    then the whole run in one pass), with FETCH_SIZE / WRITE_SIZE scaled by
    the copy calibration stored with the tile kernel's traffic summary."""
    leg = None
    with open(leg_output) as fh:
        for line in fh:
            if line.startswith('{"leg"'):
                leg = json.loads(line)["result"]
    if leg is None:
        raise SystemExit(f"no diagonal leg output in {leg_output}")
    with open(TRAFFIC_FILE) as fh:
        cal = json.load(fh)

    def disp(d, cname=None):
        rs = _csv_rows(d, "*counter_collection.csv" if cname else "*kernel_trace.csv")
        rs = [r for r in rs if "diag_steps_kernel" in r["Kernel_Name"] and (not cname or r["Counter_Name"] == cname)]
        rs.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rs
    tr = disp(trace_dir)
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in tr]
    fe = [float(r["Counter_Value"]) for r in disp(fetch_dir, "FETCH_SIZE")]
    wr = [float(r["Counter_Value"]) for r in disp(write_dir, "WRITE_SIZE")]
    nb = leg["gb_per_pass"] * 1e9
    n1 = len(durs) - 1                       # the last dispatch is the whole run in one pass
    groups = [("one step per pass", slice(1, n1)), (f"all {leg['all_steps_one_pass']['steps']} steps in one pass",
                                                    slice(n1, n1 + 1))]
    md = [f"# diag_steps_kernel: {leg['workload']}, n={leg['n']}, {leg['dtype']}, one state", "",
          "Command (repository root, on the MI355X):", "", "```", command, "```", "",
          f"A step of a diagonal Hamiltonian is one diagonal factor; algorithmic bytes per pass: the diagonal once "
          f"and the state read and written, {leg['gb_per_pass']} GB.  FETCH_SIZE is scaled by "
          f"{cal['fetch_scale']:.4f} and WRITE_SIZE by {cal['write_scale']:.4f} (the copy calibration of "
          f"`{os.path.relpath(TRAFFIC_FILE, ROOT)}`).", "",
          "| dispatches | avg ms | algorithmic GB/s | % of 8 TB/s | HBM GB (scaled FETCH + WRITE) | HBM / algorithmic |",
          "|---|---|---|---|---|---|"]
    for name, sl in groups:
        d, f, w = durs[sl], fe[sl], wr[sl]
        ms = float(np.mean(d))
        hb = (float(np.mean(f)) * cal["fetch_scale"] + float(np.mean(w)) * cal["write_scale"]) * 1024
        md.append(f"| {name} ({len(d)}) | {ms:.4f} | {nb / ms / 1e6:.0f} | {100 * nb / ms / 1e6 / HBM_PEAK_GBS:.1f} | "
                  f"{hb / 1e9:.3f} | {hb / nb:.3f} |")
    steps = leg["all_steps_one_pass"]["steps"]
    ms_all = durs[n1]
    flops = 8.0 * steps * (1 << leg["n"])
    md += ["", f"The pass of {steps} steps multiplies each entry {steps} times in registers (the same "
           f"multiplications as {steps} passes, so the same bits): {flops / ms_all / 1e9:.1f} TFLOP/s of FP32 "
           f"complex products ({8 * steps} flops per entry), {100 * flops / ms_all / 1e9 / 78.6:.0f}% of the "
           "78.6 TFLOP/s of non-packed FP32 FMA (half the 157.3 TFLOP/s vector peak, which counts packed "
           "operations): it is bound by the FMA chain, not by HBM."]
    with open(os.path.join(OUT_DIR, "diag_steps_maxcut_cost_n26.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def _template_args(kernel_name):
    """Template arguments of a kernel name as printed by rocprofv3."""
    inner = kernel_name[kernel_name.index("<") + 1:kernel_name.rindex(">")]
    return [a.strip() for a in inner.split(",")]


def summarize_taylor_profiles(trace_dir, fetch_dir, write_dir, leg_output):
    """Per-stage time and HBM traffic of the fused Taylor update from a
    rocprofv3 kernel trace and FETCH_SIZE / WRITE_SIZE runs of
    `bench.py --leg taylor`, against the algorithmic bytes the leg itself
    reports (`leg_output`: a file holding the leg's JSON line, e.g. the
    profiled run's log).  The counters are scaled by the copy calibration
    stored with the tile kernel's traffic summary."""
    import csv
    import statistics
    rows = None
    with open(leg_output) as fh:
        for line in fh:
            if line.startswith('{"leg"'):
                rows = json.loads(line)["result"]
                break
    if rows is None:
        raise SystemExit(f"no taylor leg output in {leg_output}")
    for r in rows:                     # the leg runs 1 warm-up + 3 timed steps of K stages
        r.setdefault("dispatches", r["taylor_terms"] * 4)
    with open(TRAFFIC_FILE) as fh:
        cal = json.load(fh)
    f_scale, w_scale = cal["fetch_scale"], cal["write_scale"]

    def horner(name):                  # dia_tile_kernel with HORNER = true
        return name.startswith("void hs::dia_tile_kernel<") and _template_args(name)[4] == "true"

    def counters(d, cname):
        recs = [r for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv")))
                if r["Counter_Name"] == cname and horner(r["Kernel_Name"])]
        recs.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [float(r["Counter_Value"]) for r in recs]
    fetch, write = counters(fetch_dir, "FETCH_SIZE"), counters(write_dir, "WRITE_SIZE")
    trace = [r for r in csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))) if horner(r["Kernel_Name"])]
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace]
    need = sum(r["dispatches"] for r in rows)
    if not (len(fetch) == len(write) == len(durs) == need):
        raise SystemExit(f"dispatch counts differ: fetch {len(fetch)} write {len(write)} trace {len(durs)} leg {need}")
    stats = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    ksum = ", ".join(f"{r['workload']} (K = {r['taylor_terms']}, {r['h_diagonals']} diagonals of H, "
                     f"{r['dispatches']} dispatches)" for r in rows)
    leg = "python3 -u bench.py --leg taylor"
    cmd = (f"rocprofv3 --kernel-trace --stats --output-format csv -d OUT/tay_trace -o run -- {leg} > OUT/tay_trace.log; "
           f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/tay_fetch -o run -- {leg}; "
           f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/tay_write -o run -- {leg}; "
           "python3 bench.py --out-dir OUT --summarize-taylor-profiles OUT/tay_trace OUT/tay_fetch OUT/tay_write "
           "OUT/tay_trace.log")
    md = ["# Horner stage of the fused Taylor update (dia_tile_kernel, open tiles, Horner epilogue), complex64", "",
          f"Workloads: {ksum}. r = smallest step count with |dt| nu(H) <= 1, K stages per step (tolerance 1e-6), "
          "1 warm-up + 3 timed steps per workload.", "",
          "Command (repository root, on the MI355X):", "", "```", cmd, "```", "",
          "## rocprofv3 --kernel-trace --stats", "",
          "| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in stats[:6]:
        md.append(f"| {r['Name'][:95]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    md += ["", "## Per Horner stage (averages over each workload's dispatches)", "",
           f"FETCH_SIZE is scaled by {f_scale:.4f} and WRITE_SIZE by {w_scale:.4f}, the factors a 2 GiB device copy "
           f"gives (`{os.path.relpath(TRAFFIC_FILE, ROOT)}`). Algorithmic bytes: every stored diagonal of H once "
           "plus three state passes (w, the step input in the epilogue, the output).", "",
           "| workload | avg ms | FETCH KiB | WRITE KiB | scaled HBM GB | algorithmic GB | algorithmic GB/s | "
           "HBM / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    lo = 0
    for r in rows:
        hi = lo + r["dispatches"]
        fk, wk, ms = statistics.mean(fetch[lo:hi]), statistics.mean(write[lo:hi]), statistics.mean(durs[lo:hi])
        meas = (fk * f_scale + wk * w_scale) * 1024 / 1e9
        alg = r["gb_per_stage"]
        md.append(f"| {r['workload']} | {ms:.3f} | {fk:.0f} | {wk:.0f} | {meas:.3f} | {alg:.3f} | "
                  f"{alg / ms * 1e3:.0f} | {meas / alg:.3f} |")
        lo = hi
    md += ["", "The excess over the algorithmic bytes is re-reads of w by out-of-tile partner gathers: H flips "
           "every qubit, a tile is closed over 13 of them, and far partners are no longer in the XCD's L2 when "
           "they are gathered. FETCH_SIZE counts every request that leaves the L2, whether the 256 MB "
           "last-level cache or HBM serves it."]
    path = os.path.join(OUT_DIR, "dia_tile_horner_tfim_n24_n26.md")
    with open(path, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md[-6:]))


def write_serve_summary(stats, command, fname):
    md = ["# Served stream: mixed TFIM / Heisenberg / MaxCut / TSP jobs, n in [10, 24], complex64", "",
          f"Command (repository root, on the MI355X): `{command}`", "",
          "Latency = arrival -> completion event of the job's last kernel; queue wait = arrival -> "
          "admission; service = admission -> completion (factor build + state setup + evolution). "
          f"Oracle check: jobs hashed into a 5% sample with n <= {stats[0]['oracle_nmax']} (every n of the "
          "stream), state column 0, whole run, FP64 oracle.", "",
          "| jobs | rate (jobs/s) | completed | p50 ms | p99 ms | max ms | queue p50 ms | service p50 ms | "
          "service p99 ms | throughput jobs/s | device busy | peak active | oracle checked | min fidelity |",
          "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for st in stats:
        L, Q, S = st["latency_ms"], st["queue_wait_ms"], st["service_ms"]
        md.append(f"| {st['jobs']} | {st['rate_jobs_s']:g} | {st['completed']} | {L['p50']:.1f} | {L['p99']:.1f} | "
                  f"{L['max']:.1f} | {Q['p50']:.1f} | {S['p50']:.1f} | {S['p99']:.1f} | "
                  f"{st['throughput_jobs_s']:.2f} | {st['device_busy_frac'] or 0:.3f} | {st['peak_active']} | "
                  f"{st['oracle_checked']} | {st['oracle_min_fidelity']:.12f} |")
    with open(os.path.join(OUT_DIR, fname), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md), file=sys.stderr)


def single_propagator_leg(torch, n=24, budget=None, timed_steps=20):
    """The paper's own pipeline on a 1-D TFIM (h = 1, t = 1): step search
    under the diagonal budget (Section 3.1), truncated-Taylor SpME from
    SpGEMM (Alg. 2), then the Alg. 3 loop x <- U x (complex64), timed over
    `timed_steps` SpMVs.  Algorithmic bytes per SpMV: every stored diagonal of
    U once plus the state read and written."""
    import paper_2606_16959_amd.dia as hd
    from workloads import hamiltonians as wh, states as ws
    Hw = wh.tfim_1d(n, 1.0, 1.0)
    budget = budget or 2 * n + 1
    N = 1 << n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = hd.from_pauli(Hw.strings, Hw.coeffs, n)
    t1 = time.perf_counter()
    r = hd.estimate_timesteps(H, 1.0, budget)
    t2 = time.perf_counter()
    U, K = hd.spme(H, 1.0 / r)
    t3 = time.perf_counter()
    U64 = U.to_c64()
    offs = U64.offsets
    U.close()
    H.close()
    psi = torch.from_numpy(ws.random_phase_state(n, 7, np.complex64)).cuda()
    hd.evolve(U64, psi, 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hd.evolve(U64, psi, timed_steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / timed_steps
    nbytes = sum((N - abs(d)) * 8 for d in offs) + 2 * N * 8
    U64.close()
    out = {"workload": f"tfim1d_n{n}_h1_t1", "budget": budget, "steps_chosen": r, "taylor_terms": K,
           "propagator_diagonals": len(offs), "build_h_s": round(t1 - t0, 3),
           "step_search_s": round(t2 - t1, 3), "spme_s": round(t3 - t2, 3),
           "spmv_ms": round(ms, 4), "spmv_gbs": round(nbytes / ms / 1e6, 1),
           "full_run_s_estimate": round(ms * r / 1e3, 3)}
    log(f"single propagator: r={r} K={K} diags={len(offs)} spmv {ms:.3f} ms {out['spmv_gbs']} GB/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fuse", action="store_true", help="one launch per factor")
    ap.add_argument("--renorm", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=50, help="oracle sample size (0 = skip); 50 = the whole run")
    ap.add_argument("--no-copy-ref", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="served-stream size (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-oracle-nmax", type=int, default=30, help="largest n of the checked sample")
    ap.add_argument("--serve-only", action="store_true", help="only the served stream")
    ap.add_argument("--leg", choices=["taylor", "higher_order", "single_propagator", "other_workloads", "workload",
                                      "diagonal"],
                    help="run one secondary leg alone and print its JSON (for profiling)")
    ap.add_argument("--workload", default="maxcut_3reg_n24", help="named workload of --leg workload")
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"], help="dtype of --leg workload")
    ap.add_argument("--batch", type=int, default=0, help="states of --leg workload (0 = the workload's)")
    ap.add_argument("--summarize-diagonal-profiles", nargs=4, metavar=("LEG_OUTPUT", "TRACE", "FETCH", "WRITE"),
                    help="profile summary of a --leg diagonal run")
    ap.add_argument("--summarize-leg-profiles", nargs="+", metavar="DIR",
                    help="LEG_OUTPUT TRACE COUNTER_DIR... : per-launch summary of a --leg workload run")
    ap.add_argument("--summary-name", default="", help="file name under profiles/ of --summarize-leg-profiles")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--serve-sweep", default="", help="comma-separated arrival rates (jobs/s)")
    ap.add_argument("--serve-jsonl", default=None, help="directory for per-job JSONL records of served streams")
    ap.add_argument("--summarize-profiles", nargs="+", metavar="DIR",
                    help="TRACE FETCH WRITE [REQUEST_COUNTER_DIR...]: write profiles/ summaries from rocprofv3 output")
    ap.add_argument("--profile-command", default="")
    ap.add_argument("--bench-trace", default=None, help="kernel trace of the default bench run (--summarize-profiles)")
    ap.add_argument("--bench-log", default=None, help="stdout of that run (its bench line)")
    ap.add_argument("--summarize-taylor-profiles", nargs=4, metavar=("TRACE", "FETCH", "WRITE", "LEG_OUTPUT"),
                    help="write the fused Taylor update's profile summary from rocprofv3 output directories")
    ap.add_argument("--sweep", action="store_true", help="launch-plan variants (writes profiles/)")
    ap.add_argument("--out-dir", default=None, help="directory for written summaries (default profiles/)")
    args = ap.parse_args()
    if args.out_dir:
        global OUT_DIR
        OUT_DIR = os.path.abspath(args.out_dir)
        os.makedirs(OUT_DIR, exist_ok=True)
    if args.summarize_profiles:
        tr, fe, wr, *extra = args.summarize_profiles
        summarize_profiles(tr, fe, wr, args.profile_command, extra, args.bench_trace, args.bench_log)
        return
    if args.summarize_taylor_profiles:
        summarize_taylor_profiles(*args.summarize_taylor_profiles)
        return
    if args.summarize_diagonal_profiles:
        summarize_diagonal_profiles(*args.summarize_diagonal_profiles, args.profile_command)
        return
    if args.summarize_leg_profiles:
        lo, tr, *cdirs = args.summarize_leg_profiles
        summarize_leg_profiles(lo, tr, cdirs, args.summary_name or "leg_profile.md", args.profile_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2606_16959_amd as hs
    from workloads import workload_hamiltonian, states as ws

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.sweep:
        sweep(torch, args.steps, args.warmup)
        return
    if args.leg:
        legs = {"taylor": taylor_leg, "higher_order": higher_order_leg,
                "single_propagator": single_propagator_leg, "other_workloads": other_workloads,
                "workload": lambda tc: one_workload_leg(tc, args.workload, args.dtype, steps=args.steps,
                                                        warmup=args.warmup, batch=args.batch or None),
                "diagonal": diagonal_leg}
        print(json.dumps({"leg": args.leg, "result": legs[args.leg](torch)}), flush=True)
        return
    if args.serve_only:
        st = serve_leg(torch, args.serve_jobs, args.serve_rate, args.serve_slots, args.serve_oracle_nmax,
                       args.serve_jsonl)
        print(json.dumps({"metric": "served-solve latency", "serve": st}), flush=True)
        if args.out_dir:
            write_serve_summary([st], f"python3 bench.py --serve-only --serve-jobs {args.serve_jobs} "
                                      f"--serve-rate {args.serve_rate} --serve-slots {args.serve_slots}",
                                f"serve_stream_{args.serve_jobs}jobs_{int(args.serve_rate)}per_s.md")
        return
    if args.serve_sweep:
        rates = [float(r) for r in args.serve_sweep.split(",")]
        sts = [serve_leg(torch, args.serve_jobs, r, args.serve_slots, args.serve_oracle_nmax, args.serve_jsonl)
               for r in rates]
        write_serve_summary(sts, f"python3 bench.py --serve-sweep {args.serve_sweep} --serve-jobs "
                                 f"{args.serve_jobs} --serve-slots {args.serve_slots}",
                            f"serve_rate_sweep_{args.serve_jobs}jobs.md")
        return
    H = workload_hamiltonian("tfim_5x5_ancilla_n26")
    N = 1 << H.n
    budget, t, steps_total = 16, 1.0, 50

    log("building factors (FP64 construction on the GPU)")
    tb = time.perf_counter()
    f = hs.build_factors(H.strings, H.coeffs, H.n, t, steps_total, budget, dtype="c64")
    build_s = time.perf_counter() - tb
    desc = f.describe()
    launches = f.step_launches(1, fuse=not args.no_fuse)
    per_launch = launch_bytes(desc, launches, N, 1, 8)
    step_bytes = sum(per_launch)
    log(f"factors={f.n_factors} launches/step={len(launches)} bytes/step={step_bytes / 1e9:.2f} GB build={build_s:.2f}s")

    psi0 = ws.random_phase_state(H.n, 3, np.complex64)
    psi = torch.from_numpy(psi0).cuda()
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        hs.evolve(f, psi, 1, renorm=args.renorm, fuse=not args.no_fuse)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        hs.evolve(f, psi, 1, renorm=args.renorm, fuse=not args.no_fuse)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {gbs:.1f} GB/s (wall {wall:.3f}s)")
    closure_ok = f.check_closure()

    # dominant kernel: the DIA tile kernel (every launch of the step)
    avg_launch_ms = total_ms / (args.steps * len(launches))
    avg_launch_bytes = step_bytes / len(launches)
    achieved = avg_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(per_launch, len(launches)),
            "kernel": "DIA tile kernel (complex64, one state, closed tiles, all three launches in the pair form, "
                      "odd offsets of the contiguous tile included; factors of the launch over the top qubits "
                      "stored in level-major chunks)",
            "algorithmic_bytes_per_launch": [int(b) for b in per_launch],
            "avg_launch_ms": round(avg_launch_ms, 4)}

    extra = {}
    if not args.no_copy_ref:
        del psi
        torch.cuda.empty_cache()
        cb = copy_bandwidth(torch)
        extra["device_copy_gbs"] = round(cb, 1)
        extra["frac_of_copy"] = round(gbs / cb, 4)
        log(f"device copy {cb:.1f} GB/s")

    cpu = None
    ref = got64 = None
    if args.cpu_steps > 0:
        log(f"oracle sample: {args.cpu_steps} steps at n=26 on the host")
        cpu, ref = cpu_baseline(H, psi0, budget, t, steps_total, args.cpu_steps, step_bytes)
        log(f"oracle {cpu['ms_per_step']} ms/step ({cpu['cores']} threads)")
        # the same steps on the GPU from the same state: error against the oracle
        pa = torch.from_numpy(psi0.copy()).cuda()
        hs.evolve(f, pa, args.cpu_steps, renorm=args.renorm, fuse=not args.no_fuse)
        got64 = pa.cpu().numpy()
        extra["accuracy_vs_oracle"] = dict(accuracy(got64, ref), steps=args.cpu_steps)
        log(f"vs oracle after {args.cpu_steps} steps: {extra['accuracy_vs_oracle']}")
        del pa

    others = None
    if not args.no_other_workloads:
        from concurrent.futures import ThreadPoolExecutor
        f.close()
        torch.cuda.empty_cache()
        if ref is not None and not args.renorm:
            extra["complex128"] = complex128_leg(torch, H, psi0, ref, args.cpu_steps, got64, steps_total, budget)
        ref = got64 = None
        pool = ThreadPoolExecutor(max_workers=1)      # long oracle runs beside the GPU-only legs
        others = other_workloads(torch, pool=pool)
        extra["diagonal_only"] = diagonal_leg(torch)
        others.append({"higher_order": higher_order_leg(torch)})
        others.append({"taylor_fused": taylor_leg(torch)})
        others.append({"single_propagator": single_propagator_leg(torch)})
        resolve_pending(others)
        pool.shutdown()
    serve = None
    if args.serve_jobs > 0:
        f.close()
        torch.cuda.empty_cache()
        serve = serve_leg(torch, args.serve_jobs, args.serve_rate, args.serve_slots,
                          args.serve_oracle_nmax, args.serve_jsonl)

    line = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic", "config": dict(WORKLOAD, fused=not args.no_fuse, renorm=args.renorm,
                                           launches_per_step=len(launches)),
        "roofline": roof, "cpu_baseline": cpu,
        "step_ms_median": round(float(np.median(step_ms)), 4),
        "step_ms_p90": round(float(np.percentile(step_ms, 90)), 4),
        "bytes_per_step": int(step_bytes), "build_s": round(build_s, 3),
        "closure_ok": bool(closure_ok), **extra, "other_workloads": others, "serve": serve,
    }
    print(json.dumps(line), flush=True)
    f.close()


if __name__ == "__main__":
    main()
