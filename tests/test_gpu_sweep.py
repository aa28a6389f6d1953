"""A seeded sweep over many small lattice rules (prime and non-prime N up to
2^18, so every layout kind appears: direct and embedded lengths, outer
lengths 2^j, 3 x 2^j and 5 x 2^j, on-chip radices 1-16, orbits summed as
blocks or directly) and polynomial lattice rules over GF(2), each product
and adjoint compared with the CPU oracle's plain Y A and Y^T G on the same
inputs, to tau max|Y| ||A[:, k]||_1 (tau = 1e-12 FP64, 1e-5 FP32)."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

PHIS = [(qi.PHI_IDENTITY, lambda N: (0, 1)), (qi.PHI_CENTERED, lambda N: (1, 3)),
        (qi.PHI_TENT, lambda N: (1, 5)), (qi.PHI_INVNORM, lambda N: (1, 2 * N))]


def _cases(count=48, long_count=24, seed=2026):
    rg = np.random.default_rng(seed)
    out = []
    for i in range(count + long_count):
        if i < count:
            # log-uniform N in [2, 2^17], about half of them prime
            N = int(np.exp(rg.uniform(np.log(2), np.log(1 << 17))))
            prime = i % 2 == 0
        else:
            # primes in [2^12, 2^18]: the long embedded lengths (2^k, 3 x 2^k, 5 x 2^k)
            N = int(np.exp(rg.uniform(np.log(1 << 12), np.log(1 << 18))))
            prime = True
        if prime:
            while not qi.is_prime(N):
                N += 1
        s = int(rg.integers(1, 160 if i < count else 64))
        t = int(rg.integers(1, 10 if i < count else 6))
        phi = int(rg.integers(0, len(PHIS)))
        dtype = "f64" if i % 3 else "f32"
        out.append((N, s, t, phi, dtype, i))
    return out


@pytest.mark.parametrize("N,s,t,phi,dtype,seed", _cases())
def test_sweep_forward_adjoint(N, s, t, phi, dtype, seed):
    torch_cuda()
    import paper_1501_06286_amd as q
    kind, shift = PHIS[phi]
    inst = qi.unit_lattice(N, s, t, phi=kind, shift=shift(N), dtype=dtype, seed=seed)
    announce(f"sweep N={N} s={s} t={t} phi={kind} {dtype}")
    p = plan_of(inst)
    X = q.matmul(p, to_dev(inst.A, dtype)).double().cpu().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, f"forward N={N}")
    G = qi.randn((N, t), seed=seed, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, f"adjoint N={N}")


def _gf2_cases(count=20, seed=2027):
    rg = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rg.integers(1, 18))
        s = int(rg.integers(1, 120))
        t = int(rg.integers(1, 8))
        phi = int(rg.integers(0, len(PHIS)))
        out.append((m, s, t, phi, "f64" if i % 2 else "f32", i))
    return out


@pytest.mark.parametrize("m,s,t,phi,dtype,seed", _gf2_cases())
def test_sweep_gf2(m, s, t, phi, dtype, seed):
    """Polynomial lattice rules over GF(2), N = 2^m, m = 1..17 (cyclic group
    of order 2^m - 1, always embedded for m >= 2)."""
    torch_cuda()
    import paper_1501_06286_amd as q
    kind, shift = PHIS[phi]
    N = 1 << m
    inst = qi.small_gf2(m, s, t, phi=kind, shift=shift(N), dtype=dtype, seed=seed)
    announce(f"sweep GF(2) m={m} s={s} t={t} phi={kind} {dtype}")
    p = plan_of(inst)
    X = q.matmul(p, to_dev(inst.A, dtype)).double().cpu().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, f"forward m={m}")
    G = qi.randn((N, t), seed=seed, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, f"adjoint m={m}")
