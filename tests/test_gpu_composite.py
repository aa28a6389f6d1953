"""GPU parity for rank-1 lattice rules with a non-prime number of points.

Every composite N here is compared with the CPU oracle's plain product
Y A (the definition {n g_j / N + D} holds for any N; its decomposition into
orbits and unit-group blocks is pinned in test_oracle_composite.py).
Tolerance as everywhere: max_n |X - X_oracle| <= tau max|Y| ||A[:, k]||_1,
tau = 1e-12 (FP64), 1e-5 (FP32).  The cases cover cyclic unit groups (p^k,
2 p^k), two factors (2^k, p q), several (2 3 5 7 11 13), small orbits summed
directly, long blocks that need the embedded convolution and the outer split,
forward, adjoint, epilogues, launch tunings and the row-0 term.
"""
import math

import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import TOL, announce, assert_close, plan_of, to_dev, torch_cuda, ymax

pytestmark = pytest.mark.gpu

CASES = [
    (12, 5, 3), (16, 7, 4), (45, 9, 3), (64, 11, 5), (100, 13, 3), (360, 17, 4),
    (1001, 40, 5), (1024, 33, 6), (2401, 50, 3), (4096, 64, 7), (10000, 70, 4),
    (30030, 96, 3), (39366, 48, 2), (65536, 128, 6),
]


def _inst(N, s, t, phi, dtype, seed=0):
    shift = (1, 2 * N) if phi == qi.PHI_INVNORM else (0, 1)
    return qi.unit_lattice(N, s, t, phi=phi, shift=shift, dtype=dtype, seed=seed)


@pytest.mark.parametrize("N,s,t", CASES)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_composite_forward_adjoint(N, s, t, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    phi = [qi.PHI_INVNORM, qi.PHI_IDENTITY, qi.PHI_CENTERED, qi.PHI_TENT][N % 4]
    inst = _inst(N, s, t, phi, dtype, seed=N % 7)
    announce(f"composite N={N} s={s} t={t} phi={phi} {dtype}")
    p = plan_of(inst)
    info = p.info()
    assert info["L"] == sum(1 for m in range(1, N) if math.gcd(m, N) == 1) or N > 5000
    X = q.matmul(p, to_dev(inst.A, dtype)).double().cpu().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, f"forward N={N}")
    G = qi.randn((N, t), seed=N, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, f"adjoint N={N}")


def test_composite_plan_facts():
    torch_cuda()
    # 2^16: orbits 2^k, unit groups {+-1} x <5> with 5 of order 2^(k-2): blocks
    # (4 per orbit) where that order is at least 64, the others and row 0
    # summed directly
    p = plan_of(_inst(1 << 16, 32, 2, qi.PHI_INVNORM, "f32"))
    info = p.info()
    assert info["L"] == 1 << 15 and info["beta"] == 0  # U(2^16) is not cyclic
    big = [k for k in range(3, 17) if (1 << (k - 2)) >= 64]
    assert info["blocks"] == 4 * len(big)
    assert info["direct_rows"] == 1 + sum(1 << (k - 1) for k in range(1, 17) if k not in big)
    assert info["M"] == 1 << 14 and info["embedded"] == 0
    # a prime power: cyclic unit group, one block per orbit of at least 64 units
    p = plan_of(_inst(3 ** 9, 32, 2, qi.PHI_IDENTITY, "f64"))
    info = p.info()
    assert info["beta"] != 0 and info["L"] == 2 * 3 ** 8
    assert info["blocks"] == sum(1 for k in range(1, 10) if 2 * 3 ** (k - 1) >= 64)
    # highly composite: every unit group's cyclic factors are short, all direct
    p = plan_of(_inst(30030, 16, 2, qi.PHI_IDENTITY, "f64"))
    assert p.info()["blocks"] == 0 and p.info()["direct_rows"] == 30030


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_composite_large_sampled_rows(dtype):
    """N = 2^20 and N = 3^6 5^3 7 (both beyond the whole-output oracle at
    this s): rows sampled across every orbit class, the column sums, and the
    adjoint against the oracle's entries."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    for N, s, t in ((1 << 20, 200, 4), (729 * 125 * 7, 96, 3)):
        inst = _inst(N, s, t, qi.PHI_INVNORM, dtype, seed=3)
        announce(f"composite large N={N} {dtype}")
        p = plan_of(inst)
        X = q.matmul(p, to_dev(inst.A, dtype))
        rg = np.random.default_rng(N)
        rows = set(rg.choice(N, size=300, replace=False).tolist()) | {0, 1, N - 1, N // 2}
        d = 2
        while d < N:  # a row of every divisor class 2^k, 3^k, ...
            if N % d == 0:
                rows.add(d)
            d += 1 if d < 200 else d
        rows = np.array(sorted(r for r in rows if r < N))
        got = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        assert_close(got, oracle.matmul_rows(inst, rows), inst.A, inst, dtype, f"rows N={N}")
        T = oracle.phi_residue_values(qi.RULE_LATTICE, N, qi.PHI_INVNORM, 0, inst.shift)
        colsum = X.double().sum(dim=0).cpu().numpy()
        scale = ymax(inst) * np.abs(inst.A).sum(axis=0) * math.sqrt(N)
        assert np.max(np.abs(colsum - T.sum() * inst.A.sum(axis=0)) / scale) < (
            1e-10 if dtype == "f64" else 1e-5)
        ent = [(int(j), int(k)) for j, k in zip(rg.integers(0, s, 24), rg.integers(0, t, 24))]
        G = qi.randn((N, t), seed=7, dtype=dtype)
        dA = q.matmul_adjoint(p, to_dev(G, dtype))
        got = np.array([float(dA[j, k]) for j, k in ent])
        ref = oracle.adjoint_entries(inst, ent, G=G)
        sc = ymax(inst) * np.abs(G).sum(axis=0)
        err = np.abs(got - ref) / np.array([sc[k] for _, k in ent])
        assert np.max(err) <= TOL[dtype], np.max(err)


@pytest.mark.parametrize("epi", ["affine", "exp"])
def test_composite_epilogue(epi):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 4096, 40, 5
    inst = _inst(N, s, t, qi.PHI_INVNORM, "f64", seed=2)
    announce(f"composite epilogue {epi}")
    p = plan_of(inst)
    rg = np.random.default_rng(5)
    bias = rg.standard_normal(t) * 0.1
    scale = rg.standard_normal(t)
    A = inst.A * 0.05  # exp of a moderate argument
    sub = qi.Instance(**{**inst.__dict__, "A": A})
    X = q.matmul(p, to_dev(A, "f64"), epilogue=epi, bias=to_dev(bias, "f64"),
                 scale=to_dev(scale, "f64")).cpu().numpy()
    kind = oracle.EPI_AFFINE if epi == "affine" else oracle.EPI_EXP
    ref = oracle.epilogue(oracle.matmul(sub), kind, bias, scale)
    assert np.max(np.abs(X - ref) / (np.abs(ref) + 1.0)) < 1e-12


@pytest.mark.parametrize("tuning", [dict(chunk_pairs=2), dict(front=2), dict(front=1, nt_store=1),
                                    dict(chunk_pairs=1, streams=2, outer_q=16)])
def test_composite_tunings_agree(tuning):
    """Launch tunings reach every block (the results stay within tolerance
    of the oracle)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = _inst(3 * 2 ** 12, 300, 8, qi.PHI_INVNORM, "f32", seed=4)
    announce(f"composite tuning {tuning}")
    p = plan_of(inst)
    p.set_tuning(**tuning)
    X = q.matmul(p, to_dev(inst.A, "f32")).double().cpu().numpy()
    assert_close(X, oracle.matmul(inst), inst.A, inst, "f32", f"tuning {tuning}")
    G = qi.randn((inst.N, inst.t), seed=9, dtype="f32")
    dA = q.matmul_adjoint(p, to_dev(G, "f32")).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, "f32", f"adjoint tuning {tuning}")


def test_composite_dense_baseline_and_refusals():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = _inst(6000, 64, 6, qi.PHI_CENTERED, "f64", seed=1)
    p = plan_of(inst)
    A = to_dev(inst.A, "f64")
    Y = q.explicit_points(p)
    np.testing.assert_array_equal(Y.cpu().numpy(), oracle.Y_rows(inst))
    Xd = q.dense_matmul(p, Y, A).cpu().numpy()
    X = q.matmul(p, A).cpu().numpy()
    assert np.max(np.abs(X - Xd)) <= 1e-12 * np.max(np.abs(inst.A).sum(axis=0))
    with pytest.raises(q.QMCError) as e:
        p.set_row_order(q.ROWS_GROUP)
    assert e.value.code == -9
    with pytest.raises(q.QMCError) as e:
        p.tables()
    assert e.value.code == -9
    with pytest.raises(q.QMCError) as e:
        q.Batch([p], [A])
    assert e.value.code == -9
