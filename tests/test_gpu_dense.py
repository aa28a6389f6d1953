"""The dense baseline: explicit point matrix (bit-exact against the oracle)
and the MFMA GEMM X = Y A."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rule", [qi.RULE_LATTICE, qi.RULE_POLY_GF2])
def test_explicit_points_bit_exact(rule):
    torch_cuda()
    import paper_1501_06286_amd as q
    inst = (qi.small_lattice(2003, 97, 1, phi=qi.PHI_IDENTITY) if rule == qi.RULE_LATTICE
            else qi.small_gf2(11, 97, 1, phi=qi.PHI_CENTERED))
    announce(f"explicit points rule={rule}")
    Y = q.explicit_points(plan_of(inst)).cpu().numpy()
    assert np.array_equal(Y, oracle.Y_rows(inst))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N,s,t", [(7, 3, 3), (257, 100, 129), (2003, 500, 1), (4099, 1000, 300),
                                   (1021, 77, 45), (4099, 256, 256)])
def test_dense_gemm(N, s, t, dtype):
    torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    announce(f"dense gemm N={N} s={s} t={t} {dtype}")
    p = plan_of(inst)
    Y = q.explicit_points(p)
    X = q.dense_matmul(p, Y, to_dev(inst.A, dtype)).cpu().double().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, "dense")
