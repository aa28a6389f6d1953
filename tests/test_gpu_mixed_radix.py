"""GPU parity for convolution lengths M = 3 x 2^k and 5 x 2^k (the
mixed-radix outer transform).

When N - 1 is not a power of two the convolution of length L = N - 1 is
embedded in a cyclic convolution of length M >= 2L - 1.  The shortest such M
among 2^k, 3 x 2^k and 5 x 2^k is taken when the outer length M2 = M / 4096
fits one back pass; the outer DFT over w2 then has a radix-3 or radix-5
stage (register DFTs of 3 x 2^i or 5 x 2^i values, the LDS back pass for 40,
48, 80 and 96), and the FP64 spectrum a radix-3 or radix-5 pass.  Every case is compared with the CPU oracle's plain product
Y A (and Y^T G) on the same seeded inputs, to tau max|Y| ||A[:, k]||_1 with
tau = 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

# N prime, L = N - 1: (N, M2 in FP32, M2 in FP64); M = 4096 M2
LENGTHS = [(5003, 3, 3), (11003, 6, 6), (22003, 12, 12), (45007, 24, 24), (90001, 48, 48),
           (180001, 96, 128),
           (9001, 5, 5), (18013, 10, 10), (36007, 20, 20), (70001, 40, 40), (150001, 80, 128)]


def _inst(N, s, t, dtype, seed=0):
    return qi.small_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=seed)


def _check(p, inst, dtype, what):
    import paper_1501_06286_amd as q
    X = q.matmul(p, to_dev(inst.A, dtype)).double().cpu().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, f"forward {what}")
    G = qi.randn((inst.N, inst.t), seed=inst.N % 97, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, f"adjoint {what}")
    return X


@pytest.mark.parametrize("N,m2_f32,m2_f64", LENGTHS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_mixed_lengths(N, m2_f32, m2_f64, dtype):
    torch_cuda()
    inst = _inst(N, 96, 5, dtype, seed=1)
    announce(f"mixed radix N={N} {dtype}")
    p = plan_of(inst)
    info = p.info()
    m2 = m2_f32 if dtype == "f32" else m2_f64
    assert info["embedded"] == 1 and info["M1"] == 4096 and info["M2"] == m2
    assert info["M"] == 4096 * m2 and info["M"] >= 2 * (N - 1) - 1
    if m2 % 3 == 0 or m2 % 5 == 0:  # the whole outer length in one back pass
        assert (info["P2"], info["Q2"]) == (1, m2)
    _check(p, inst, dtype, f"N={N}")


@pytest.mark.parametrize("N", [11003, 90001, 9001, 70001])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_mixed_dense_front(N, dtype):
    """The dense outer front (gathers and a register DFT of 3 x 2^i or 5 x 2^i
    values)."""
    torch_cuda()
    inst = _inst(N, 200, 4, dtype, seed=2)
    announce(f"mixed radix dense front N={N} {dtype}")
    p = plan_of(inst)
    p.set_tuning(front=2)
    _check(p, inst, dtype, f"dense front N={N}")


@pytest.mark.parametrize("N,q2", [(180001, 48), (180001, 24), (180001, 12), (180001, 3),
                                  (90001, 24), (90001, 6), (45007, 12),
                                  (150001, 40), (150001, 20), (150001, 5), (70001, 10)])
def test_mixed_outer_splits(N, q2):
    """Outer radices that split M2 = P2 x Q2 with the factor 3 or 5 in Q2 (split
    pass of radix P2, back pass of radix Q2), with the sparse and the dense
    fronts."""
    torch_cuda()
    inst = _inst(N, 120, 6, "f32", seed=3)
    announce(f"mixed radix split N={N} q={q2}")
    p = plan_of(inst)
    for front in (1, 2):
        p.set_tuning(outer_q=q2, front=front)
        info = p.info()
        assert info["Q2"] == q2 and info["P2"] * q2 == info["M2"]
        _check(p, inst, "f32", f"N={N} q={q2} front={front}")


def test_mixed_outer_radix_refusals():
    torch_cuda()
    import paper_1501_06286_amd as q
    p = plan_of(_inst(180001, 20, 2, "f32"))  # M2 = 96
    for bad in (32, 16, 64, 5, 40, 7, 192, -3):  # P2 not 2^k, Q2 not dividing, bad form, > 128, < 0
        with pytest.raises(q.QMCError):
            p.set_tuning(outer_q=bad)
    assert p.info()["Q2"] == 96  # unchanged by the refused calls
    p5 = plan_of(_inst(150001, 20, 2, "f32"))  # M2 = 80
    for bad in (16, 48, 3, 6):
        with pytest.raises(q.QMCError):
            p5.set_tuning(outer_q=bad)
    p2 = plan_of(_inst(200003, 20, 2, "f32"))  # M2 = 128: a radix with a factor 3 cannot split it
    with pytest.raises(q.QMCError):
        p2.set_tuning(outer_q=48)


def test_mixed_bucket_twiddles_fall_back():
    """front = 3 needs a power-of-two M2: on M2 = 3 x 2^j (and 5 x 2^j) it runs the item
    twiddles of front = 1, with the same bits."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = _inst(22003, 300, 8, "f32", seed=4)
    announce("mixed radix front 3 fallback")
    p = plan_of(inst)
    A = to_dev(inst.A, "f32")
    p.set_tuning(front=1)
    X1 = q.matmul(p, A).clone()
    p.set_tuning(front=3)
    X3 = q.matmul(p, A)
    torch.cuda.synchronize()
    assert torch.equal(X1, X3)
    assert_close(X3.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, "f32", "front 3")


@pytest.mark.parametrize("epi", ["affine", "exp"])
def test_mixed_epilogue(epi):
    torch_cuda()
    import paper_1501_06286_amd as q
    inst = _inst(45007 if epi == "affine" else 36007, 64, 5, "f64", seed=5)
    announce(f"mixed radix epilogue {epi}")
    p = plan_of(inst)
    rg = np.random.default_rng(6)
    bias, scale = rg.standard_normal(5) * 0.1, rg.standard_normal(5)
    A = inst.A * 0.05
    sub = qi.Instance(**{**inst.__dict__, "A": A})
    X = q.matmul(p, to_dev(A, "f64"), epilogue=epi, bias=to_dev(bias, "f64"),
                 scale=to_dev(scale, "f64")).cpu().numpy()
    kind = oracle.EPI_AFFINE if epi == "affine" else oracle.EPI_EXP
    ref = oracle.epilogue(oracle.matmul(sub), kind, bias, scale)
    assert np.max(np.abs(X - ref) / (np.abs(ref) + 1.0)) < 1e-12


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_mixed_batch(dtype):
    """A batch whose products fall into several layout groups, mixed and
    power-of-two outer lengths among them."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    Ns = [5003, 11003, 22003, 45007, 90001, 180001, 9001, 18013, 36007, 70001, 150001, 200003,
          65537, 4099]
    insts = [_inst(N, 40 + 7 * k, 1 + k % 5, dtype, seed=10 + k) for k, N in enumerate(Ns)]
    announce(f"mixed radix batch {dtype}")
    plans = [plan_of(i) for i in insts]
    assert any(p.info()["M2"] % 3 == 0 for p in plans)
    Xs = q.Batch(plans, [to_dev(i.A, dtype) for i in insts]).run()
    torch.cuda.synchronize()
    for inst, X in zip(insts, Xs):
        assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, inst.name)


def test_mixed_composite_block():
    """N = 2 x 5003: the unit group is cyclic of order 5002, whose block is
    embedded in M = 3 x 4096."""
    torch_cuda()
    N, s, t = 2 * 5003, 64, 4
    inst = qi.unit_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype="f64", seed=7)
    announce(f"mixed radix composite N={N}")
    p = plan_of(inst)
    info = p.info()
    assert info["L"] == 5002 and info["M"] == 3 * 4096 and info["blocks"] >= 1
    _check(p, inst, "f64", f"composite N={N}")
