"""Shared helpers of the GPU parity tests (they compare the HIP path with the
CPU oracle on the same seeded inputs)."""
import sys

import numpy as np
import pytest

import oracle
import qmc_inputs as qi

TOL = {"f64": 1e-12, "f32": 1e-5}


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def plan_of(inst, dtype=None):
    import paper_1501_06286_amd as q
    return q.Plan.from_instance(inst, dtype=dtype)


def to_dev(a: np.ndarray, dtype: str):
    torch = torch_cuda()
    td = torch.float32 if dtype == "f32" else torch.float64
    return torch.from_numpy(np.ascontiguousarray(a)).to(td).cuda()


def ymax(inst) -> float:
    T = oracle.phi_residue_values(inst.rule, inst.N, inst.phi, inst.modulus, inst.shift)
    return float(np.max(np.abs(T)))


def column_errors(got: np.ndarray, ref: np.ndarray, inp: np.ndarray, inst) -> np.ndarray:
    """Per column k: max_n |got - ref| / (max|Y| * ||inp[:, k]||_1)."""
    scale = ymax(inst) * np.abs(inp).sum(axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    return np.max(np.abs(got - ref), axis=0) / scale


def assert_close(got, ref, inp, inst, dtype, what=""):
    err = column_errors(np.asarray(got, dtype=np.float64), ref, inp, inst)
    worst = float(np.max(err)) if err.size else 0.0
    assert worst <= TOL[dtype], f"{what}: normalised error {worst:.3e} > {TOL[dtype]:.0e}"
    return worst
