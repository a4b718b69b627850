"""Seeded stream of Hamiltonian-simulation jobs for the served benchmark.

Jobs arrive as a Poisson process (exponential inter-arrival times).  Each
job draws its family uniformly from {TFIM-1D, Heisenberg-1D, weighted
3-regular MaxCut with an X mixer, 4-city one-hot TSP}, a qubit count n
uniform in [n_min, n_max] (TSP is always 16 qubits; MaxCut uses an even n),
a batch of 1..8 initial states and 20..200 Trotter steps; t = 1.0.  Per-job
coefficients come from PCG64 seeded with (stream seed, job id).  Initial
states are random-phase states drawn on the device from ``state_seed``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import hamiltonians as wh

FAMILIES = ("tfim", "heisenberg", "maxcut", "tsp")


@dataclass
class JobSpec:
    job_id: int
    family: str
    n: int
    batch: int
    steps: int
    t: float
    arrival: float          # seconds after the stream starts
    state_seed: int
    ham_seed: int

    def hamiltonian(self) -> wh.Hamiltonian:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.ham_seed, self.job_id])))
        if self.family == "tfim":
            return wh.tfim_1d(self.n, 1.0, float(rng.uniform(0.5, 2.0)))
        if self.family == "heisenberg":
            return wh.heisenberg_1d(self.n, 1.0, fields=rng.uniform(-1.0, 1.0, self.n))
        if self.family == "maxcut":
            edges = wh.random_regular_graph(self.n, 3, rng)
            return wh.maxcut(self.n, edges, rng.uniform(1.0, 10.0, len(edges)), mixer=0.7)
        if self.family == "tsp":
            d = rng.uniform(1.0, 10.0, (4, 4))
            d = np.triu(d, 1) + np.triu(d, 1).T
            return wh.tsp_onehot(d, 20.0)
        raise ValueError(self.family)


def job_stream(n_jobs: int = 2000, rate: float = 50.0, seed: int = 5, n_min: int = 10,
               n_max: int = 24, families=FAMILIES) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        fam = families[int(rng.integers(len(families)))]
        n = int(rng.integers(n_min, n_max + 1))
        if fam == "tsp":
            n = 16
        elif fam == "maxcut" and n % 2:
            n -= 1
        batch = int(rng.integers(1, 9))
        steps = int(rng.integers(20, 201))
        jobs.append(JobSpec(j, fam, n, batch, steps, 1.0, t, state_seed=seed * 1_000_003 + j,
                            ham_seed=seed))
    return jobs
