"""Dense products with the explicit point matrix (the "standard approach").

Test infrastructure: never imported by the product path.

X = Y A (Section 1: the N x t product B = Y A whose rows are y_n A) and the
adjoint dA = Y^T G, in FP64 with numpy's matmul as the one library step.  For
sizes where the N x s matrix Y does not fit, ``matmul_rows`` forms only the
requested rows of Y and ``adjoint_entries`` only the requested columns.

``epilogue`` applies the downstream step of the PDE applications to X = Y A:
the uniform case's b_{k,l} = a_{0,k,l} + Y a_{k,l} (Section 3.2, eq. (Ya)) and
the log-normal case's exp(theta) with Theta = Psi^ + Y Psi (Section 3.3,
eqs. (fastB), (eq_as)), per column c as scale[c] * f(bias[c] + X[:, c]).
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


EPI_NONE, EPI_AFFINE, EPI_EXP = 0, 1, 2


def epilogue(X, kind: int, bias=None, scale=None) -> np.ndarray:
    """scale[c] * f(bias[c] + X[:, c]) with f = identity (EPI_AFFINE) or exp
    (EPI_EXP); a missing bias is 0 and a missing scale 1; EPI_NONE returns X."""
    X = np.asarray(X, dtype=np.float64)
    if kind == EPI_NONE:
        return X.copy()
    b = 0.0 if bias is None else np.asarray(bias, dtype=np.float64)[None, :]
    z = X + b
    if kind == EPI_EXP:
        z = np.exp(z)
    elif kind != EPI_AFFINE:
        raise ValueError(f"unknown epilogue {kind}")
    return z if scale is None else z * np.asarray(scale, dtype=np.float64)[None, :]
