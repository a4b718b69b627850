"""Helpers shared by the GPU tests (inputs and oracle runs on the host)."""
import contextlib
import os
import sys

import numpy as np

from oracle import evolve as oev, factors as ofac, metrics, pauli as opauli


def hs_gpu():
    """Import the library and require a GPU: GPU tests fail, never skip, without one."""
    import torch
    import paper_2606_16959_amd as hs
    from paper_2606_16959_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    _lib.load()   # raises when libhamsim.so is missing
    return hs, torch


def note(msg):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def oracle_run(H, budget, t, steps, psi0, run_steps=None, threads=0):
    terms = opauli.parse_terms(H.strings, H.coeffs, H.n)
    part = ofac.first_fit(terms, budget, t / steps)
    out = oev.evolve(terms, part, psi0, H.n, t / steps, steps if run_steps is None else run_steps,
                     threads=threads)
    return out


def fid(a, b):
    return metrics.fidelity(a, b)


def tol_c64():
    """Per-element bound factor for FP32 accumulation of complex64 data."""
    return 2.0 ** -20


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0)


@contextlib.contextmanager
def env(**kw):
    """Set library environment knobs (read by the library at every call)."""
    saved = {k: os.environ.get(k) for k in kw}
    os.environ.update({k: str(v) for k, v in kw.items()})
    try:
        yield
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
