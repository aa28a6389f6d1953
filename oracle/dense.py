"""Dense products with the explicit point matrix (the "standard approach").

Test infrastructure: never imported by the product path.

X = Y A (Section 1: the N x t product B = Y A whose rows are y_n A) and the
adjoint dA = Y^T G, in FP64 with numpy's matmul as the one library step.  For
sizes where the N x s matrix Y does not fit, ``matmul_rows`` forms only the
requested rows of Y and ``adjoint_entries`` only the requested columns.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .points import explicit_Y


def Y_rows(inst, rows=None) -> np.ndarray:
    return explicit_Y(inst.rule, inst.N, inst.gen, inst.phi, inst.modulus, inst.shift, rows)


def matmul(inst, A=None) -> np.ndarray:
    """X = Y A for all N rows, FP64."""
    A = inst.A if A is None else A
    Y = Y_rows(inst)
    return Y @ np.asarray(A, dtype=np.float64)


def adjoint(inst, G=None) -> np.ndarray:
    """dA = Y^T G, FP64."""
    G = inst.G if G is None else G
    Y = Y_rows(inst)
    return Y.T @ np.asarray(G, dtype=np.float64)


def matmul_rows(inst, rows, A=None, chunk: int = 256) -> np.ndarray:
    """Rows X[rows, :] = Y[rows, :] A, forming Y one block of rows at a time."""
    A = np.asarray(inst.A if A is None else A, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty((len(rows), A.shape[1]), dtype=np.float64)
    for i in range(0, len(rows), chunk):
        r = rows[i:i + chunk]
        out[i:i + chunk] = Y_rows(inst, r) @ A
    return out


def adjoint_entries(inst, entries, G=None, chunk: int = 1 << 15) -> np.ndarray:
    """dA[j, k] = sum_n Y[n, j] G[n, k] for the listed (j, k), O(N) each."""
    G = np.asarray(inst.G if G is None else G, dtype=np.float64)
    js = np.array([j for j, _ in entries], dtype=np.int64)
    ks = np.array([k for _, k in entries], dtype=np.int64)
    sub = dataclasses.replace(inst, gen=np.asarray(inst.gen)[js])
    out = np.zeros(len(entries), dtype=np.float64)
    for lo in range(0, inst.N, chunk):
        rows = np.arange(lo, min(inst.N, lo + chunk))
        Yb = Y_rows(sub, rows)
        out += np.sum(Yb * G[rows][:, ks], axis=0)
    return out
