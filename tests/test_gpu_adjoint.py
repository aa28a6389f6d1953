"""GPU parity of the adjoint dA = Y^T G (and the autograd wrapper)."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [(2, 3, 1), (7, 3, 2), (101, 30, 3), (257, 300, 5), (2003, 500, 4), (8209, 700, 33),
         (65537, 64, 2)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N,s,t", CASES)
def test_adjoint_lattice(N, s, t, dtype):
    torch_cuda()
    import paper_1501_06286_amd as q
    phi, shift = (qi.PHI_INVNORM, (1, 2 * N)) if N % 2 else (qi.PHI_TENT, (1, 3))
    inst = qi.small_lattice(N, s, t, phi=phi, shift=shift, dtype=dtype)
    G = qi.randn((N, t), seed=[N, s, t], dtype=dtype)
    announce(f"adjoint lattice N={N} s={s} t={t} {dtype}")
    p = plan_of(inst)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).cpu().double().numpy()
    ref = oracle.adjoint(inst, G)
    assert_close(dA, ref, G, inst, dtype, inst.name)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m,s,t", [(4, 20, 3), (10, 300, 6), (16, 64, 2)])
def test_adjoint_gf2(m, s, t, dtype):
    torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_gf2(m, s, t, dtype=dtype)
    G = qi.randn((1 << m, t), seed=[m, s, t], dtype=dtype)
    announce(f"adjoint gf2 m={m} s={s} t={t} {dtype}")
    dA = q.matmul_adjoint(plan_of(inst), to_dev(G, dtype)).cpu().double().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, inst.name)


def test_dot_product_identity():
    """<Y A, G> = <A, Y^T G> with both sides from the GPU (FP64)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 4099, 333, 6
    inst = qi.small_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N))
    G = qi.randn((N, t), seed=5)
    announce("dot-product identity")
    p = plan_of(inst)
    X = q.matmul(p, to_dev(inst.A, "f64"))
    dA = q.matmul_adjoint(p, to_dev(G, "f64"))
    lhs = float((X * to_dev(G, "f64")).sum())
    rhs = float((to_dev(inst.A, "f64") * dA).sum())
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)


def test_autograd_backward():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 1009, 50, 4
    inst = qi.small_lattice(N, s, t, phi=qi.PHI_CENTERED)
    G = qi.randn((N, t), seed=6)
    announce("autograd")
    p = plan_of(inst)
    A = to_dev(inst.A, "f64").requires_grad_(True)
    X = q.qmc_matmul(A, p)
    (X * to_dev(G, "f64")).sum().backward()
    ref = oracle.adjoint(inst, G)
    assert_close(A.grad.cpu().numpy(), ref, G, inst, "f64", "autograd")
