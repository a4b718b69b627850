"""Seeded synthetic inputs shared by the GPU path's callers and the oracle.

This package only *generates inputs*: Pauli-sum Hamiltonians as lists of
(string, coefficient) pairs and initial state vectors.  It contains none of
the method's arithmetic (no exponentials, no diagonal layout, no evolution),
so both the oracle and the library can consume its output without sharing
any computation.

Conventions (stated once, used everywhere):

* A Pauli string has one character per qubit from ``IXYZ``; character ``k``
  acts on qubit ``k``, which is bit ``k`` of the basis-state index
  (least-significant bit first).
* Every random draw comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from .hamiltonians import (  # noqa: F401
    Hamiltonian,
    tfim_1d,
    tfim_2d,
    heisenberg_1d,
    maxcut,
    random_regular_graph,
    tsp_onehot,
    WORKLOADS,
    WORKLOAD_RUN,
    workload_hamiltonian,
)
from .states import (  # noqa: F401
    zero_state,
    neel_state,
    uniform_state,
    random_phase_state,
    workload_states,
)
