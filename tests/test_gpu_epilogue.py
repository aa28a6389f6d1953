"""Epilogues of the PDE applications fused into the product's writes
(Sections 3.2 and 3.3): X = scale * f(bias + Y A), f = identity or exp,
against the oracle's product with the same epilogue."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import TOL, announce, to_dev, torch_cuda, ymax

pytestmark = pytest.mark.gpu

EPS = {"f32": 2.0 ** -23, "f64": 2.0 ** -52}


def _check(got, inst, kind, bias, scale, dtype, what):
    ref0 = oracle.matmul(inst)
    ref = oracle.epilogue(ref0, kind, bias, scale)
    sc = np.ones(inst.t) if scale is None else np.abs(scale)
    dth = TOL[dtype] * ymax(inst) * np.abs(inst.A).sum(axis=0)  # allowed error of Y A per column
    if kind == oracle.EPI_EXP:
        bound = (dth[None, :] + 8 * EPS[dtype]) * np.abs(ref)
    else:
        bound = dth[None, :] * sc[None, :] + 8 * EPS[dtype] * np.abs(ref)
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    assert worst <= 1.0, f"{what}: error {worst:.3g} x the bound"


CASES = [  # (kind, N or m, s, t, tuning)
    ("lattice", 2003, 300, 7, {}),
    ("lattice", 8209, 400, 33, {"chunk_pairs": 5, "nt_store": 1}),
    ("lattice", 8209, 400, 33, {"chunk_pairs": 4, "streams": 2}),
    ("lattice", 139999, 100, 6, {"front": 2}),
    ("lattice", 65537, 300, 4, {"front": 2, "chunk_pairs": 1}),
    ("lattice", 200003, 100, 19, {"outer_q": 64}),  # the LDS back pass, ragged pair tile
    ("gf2", 12, 500, 5, {}),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("epi", ["affine", "exp"])
@pytest.mark.parametrize("rule,n,s,t,tuning", CASES)
def test_epilogue_matches_oracle(rule, n, s, t, tuning, epi, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    if rule == "lattice":
        inst = qi.small_lattice(n, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * n), dtype=dtype, seed=5)
    else:
        inst = qi.small_gf2(n, s, t, dtype=dtype, seed=5)
    # keep exp's argument moderate: scale the input so |Y A| stays O(1)
    inst.A = qi._round_to(inst.A / np.sqrt(s), dtype)
    rg = np.random.default_rng(t)
    bias = qi._round_to(rg.standard_normal(t) * 0.5, dtype)
    scale = qi._round_to(rg.uniform(0.5, 2.0, t), dtype)
    announce(f"epilogue {epi} {inst.name} {tuning} {dtype}")
    p = q.Plan.from_instance(inst)
    if tuning:
        p.set_tuning(**tuning)
    A = to_dev(inst.A, dtype)
    kind = oracle.EPI_AFFINE if epi == "affine" else oracle.EPI_EXP
    X = q.matmul(p, A, epilogue=epi, bias=to_dev(bias, dtype), scale=to_dev(scale, dtype))
    torch.cuda.synchronize()
    _check(X.cpu().numpy(), inst, kind, bias, scale, dtype, "bias and scale")
    Xb = q.matmul(p, A, epilogue=epi, bias=to_dev(bias, dtype))  # unit scale
    Xs = q.matmul(p, A, epilogue=epi, scale=to_dev(scale, dtype))  # zero bias
    torch.cuda.synchronize()
    _check(Xb.cpu().numpy(), inst, kind, bias, None, dtype, "bias only")
    _check(Xs.cpu().numpy(), inst, kind, None, scale, dtype, "scale only")


def test_epilogue_none_is_the_plain_product():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(2003, 100, 6, phi=qi.PHI_INVNORM, shift=(1, 4006), dtype="f32")
    p = q.Plan.from_instance(inst)
    A = to_dev(inst.A, "f32")
    L = q.lib()
    import ctypes
    X0 = q.matmul(p, A)
    X1 = torch.empty_like(X0)
    ws = p.workspace(6)
    rc = L.qmc_matmul_epilogue(p.handle, ctypes.c_void_p(A.data_ptr()), 6, 6,
                               ctypes.c_void_p(X1.data_ptr()), 6, 0, None, None,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    torch.cuda.synchronize()
    assert rc == 0 and torch.equal(X0, X1)


def test_epilogue_errors():
    torch = torch_cuda()
    import ctypes
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(101, 10, 4, dtype="f32")
    p = q.Plan.from_instance(inst)
    A = to_dev(inst.A, "f32")
    X = torch.empty((101, 4), device="cuda")
    ws = p.workspace(4)
    L = q.lib()
    args = lambda kind, bias: (p.handle, ctypes.c_void_p(A.data_ptr()), 4, 4,
                               ctypes.c_void_p(X.data_ptr()), 4, kind, bias, None,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert L.qmc_matmul_epilogue(*args(3, None)) == -1                       # unknown kind
    assert L.qmc_matmul_epilogue(*args(1, ctypes.c_void_p(X.data_ptr()))) == -5  # bias inside X
