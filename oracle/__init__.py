"""FP64 CPU oracle for diagonal-budgeted Trotterization -- TEST INFRASTRUCTURE.

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  It is *not* part of the product: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import, call,
link or run anything in it.  It shares no code with the GPU library (no
kernels, headers, helpers or tables), and the library never imports it.

What it computes (paper: Section 2.1, Eq. 2-4; Section 3.4; Section 3.2,
Eq. 6; Section 4.3 "State Fidelity"):

* ``pauli``   -- Pauli strings, their matrices and action on states.
* ``factors`` -- first-fit grouping of the terms into commuting factors whose
  exact exponentials fit the diagonal budget (Eq. 5 applied per factor), the
  factors' local unitaries, their DIA offset sets and matrix entries.
* ``dia``     -- the DIA layout of Eq. 6 and the SpMV it defines (Alg. 1 as a
  plain definition: y[r] = sum_d A[r, r+d] x[r+d]).
* ``evolve``  -- the Trotterized product of Eq. 4 with exactly exponentiated
  factors, applied r times, in FP64 (C with OpenMP, plus a NumPy twin for
  small cases).
* ``metrics`` -- norm and state fidelity in FP64.

Readings of points where the paper is silent are listed in each module's
docstring; every function is pinned by the CPU tests against closed forms,
dense matrix exponentials or values printed in the paper.
"""
