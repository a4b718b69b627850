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

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits: this build runs on a
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
KERNEL_SRC = os.path.join(ROOT, "paper_2606_16959_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dia_tile_tfim2d_n26.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def launch_bytes(desc, launches, N, batch, elem):
    """Algorithmic bytes of each launch of one step."""
    out = []
    for first, cnt in launches:
        coef = sum((N - abs(d)) * elem for f in desc["factors"][first:first + cnt] for d in f["offsets"])
        out.append(coef + 2 * batch * N * elem)
    return out


def measured_traffic(per_launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch_scaled")


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
    oev.evolve(terms, part, psi, H.n, t / steps_total, sample_steps)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / sample_steps
    return {
        "value": round(step_bytes / per_step / 1e9, 3), "unit": "GB/s",
        "cores": threads, "kind": "oracle",
        "sample": f"{sample_steps} Trotter steps of the same n=26 workload, full state, FP64 "
                  f"(C + OpenMP, {threads} threads); setup (phase table, {t1 - t0:.2f} s) excluded; "
                  f"value = the step's algorithmic DIA bytes / oracle step time",
        "ms_per_step": round(per_step * 1e3, 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fuse", action="store_true", help="one launch per factor")
    ap.add_argument("--renorm", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8, help="oracle sample size (0 = skip)")
    ap.add_argument("--no-copy-ref", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2606_16959_amd as hs
    from workloads import config_hamiltonian, states as ws

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    H = config_hamiltonian(3)
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
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(per_launch),
            "kernel": "dia_tile_kernel<float,1,16,closed>",
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
    if args.cpu_steps > 0:
        log(f"oracle sample: {args.cpu_steps} steps at n=26 on the host")
        cpu = cpu_baseline(H, psi0, budget, t, steps_total, args.cpu_steps, step_bytes)
        log(f"oracle {cpu['ms_per_step']} ms/step ({cpu['cores']} threads)")

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
        "closure_ok": bool(closure_ok), **extra,
    }
    print(json.dumps(line), flush=True)
    f.close()


if __name__ == "__main__":
    main()
