"""The diagonal (DIA) representation and the SpMV it defines, in FP64.

Paper: Section 3.2, Eq. 6 -- an operator is the set of (d_k, v_k) with d = 0
the main diagonal, d > 0 superdiagonals and d < 0 subdiagonals; diagonal d of
an N x N operator has exactly N - |d| entries.  The element map of the
"DiagonalTimesVector" schematic (Section 3.3) fixes which entry is stored
where: for d < 0 position i is row i - d, column i; for d >= 0 it is row i,
column i + d.  So storage index = min(row, col) and d = col - row.

The SpMV (Alg. 1) is written here as its plain definition,
y[r] = sum_d A[r, r + d] x[r + d] over the rows where r + d is in range,
one diagonal at a time with no tiling or task split.
"""
from __future__ import annotations

import numpy as np


def dense_to_dia(A: np.ndarray, keep_zero_diagonals: bool = False) -> dict:
    """{d: v_d} with v_d[i] = A[i, i+d] (d >= 0) or A[i-d, i] (d < 0).

    Only diagonals holding a nonzero entry are kept unless asked otherwise.
    """
    N = A.shape[0]
    out = {}
    for d in range(-(N - 1), N):
        if d >= 0:
            v = np.array([A[i, i + d] for i in range(N - d)])
        else:
            v = np.array([A[i - d, i] for i in range(N + d)])
        if keep_zero_diagonals or np.any(v != 0):
            out[d] = v
    return out


def dia_to_dense(dia: dict, N: int) -> np.ndarray:
    A = np.zeros((N, N), dtype=np.complex128)
    for d, v in dia.items():
        assert len(v) == N - abs(d)
        for i in range(N - abs(d)):
            if d >= 0:
                A[i, i + d] = v[i]
            else:
                A[i - d, i] = v[i]
    return A


def dia_spmv(dia: dict, x: np.ndarray) -> np.ndarray:
    """y = A x from the diagonals (x may be a [B, N] batch)."""
    N = x.shape[-1]
    y = np.zeros(x.shape, dtype=np.complex128)
    for d, v in dia.items():
        v = np.asarray(v, dtype=np.complex128)
        if d >= 0:
            # rows r = 0..N-d-1 read v_d[r] and x[r + d]
            y[..., 0:N - d] += v * x[..., d:N]
        else:
            # rows r = -d..N-1 read v_d[r + d] and x[r + d]
            y[..., -d:N] += v * x[..., 0:N + d]
    return y


def dia_nbytes(offsets, N: int, elem_bytes: int) -> int:
    """Bytes of the compact layout: sum_d (N - |d|) entries, no padding."""
    return sum((N - abs(int(d))) * elem_bytes for d in offsets)
