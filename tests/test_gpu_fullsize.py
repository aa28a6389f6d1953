"""Parity at the full benchmark sizes, in the configuration bench.py times.

The Gaussian workload (N = 65537, s = t = 4096) is compared with the oracle
on every entry, in FP32 and FP64.  For the PDE field (GF(2), s = 16384,
t = 4096) and the large rule (N = 1048573, s = 65536, t = 256) the oracle
computes a row sample chosen through the plan's power table so that every
residue e1 of the on-chip transform (so every e1 tile of the back pass, with
random outer indices) appears, plus the first and last group elements; the
PDE field is also compared whole with the dense MFMA product of the explicit
Y.  Properties that hold at any size (column sums, the adjoint identity,
finite differences of a linear map) are checked on the whole output.
"""
import math

import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import TOL, announce, assert_close, plan_of, to_dev, torch_cuda, ymax

pytestmark = pytest.mark.gpu


def sample_rows(N, k, seed):
    rg = np.random.default_rng(seed)
    rows = set(rg.choice(N, size=k, replace=False).tolist())
    rows |= {0, 1, N - 1}
    return np.array(sorted(rows))


def tile_rows(p, seed):
    """Rows n = pow[e] for group indices e that take every residue
    e1 = e mod M1 once (outer index e2 drawn at random below L), plus e = 0,
    e = L - 1 and the constant row 0."""
    info = p.info()
    M1, L = info["M1"], info["L"]
    pw = p.tables()[0]
    rg = np.random.default_rng(seed)
    e1 = np.arange(min(M1, L), dtype=np.int64)
    e2 = rg.integers(0, (L - 1 - e1) // M1 + 1)
    e = np.concatenate([e1 + M1 * e2, [0, L - 1]])
    return np.unique(np.concatenate([[0], pw[e].astype(np.int64)]))


_FULL = {}


def oracle_full(inst):
    """The oracle's whole X = Y A (FP64), kept for the next test of the same
    instance (one at a time: 2 GiB at the Gaussian workload)."""
    key = (inst.name, inst.dtype)
    if key not in _FULL:
        _FULL.clear()
        announce(f"  oracle: all {inst.N} rows of {inst.name} ({inst.dtype} A)")
        _FULL[key] = oracle.matmul_rows(inst, np.arange(inst.N), chunk=1024)
    return _FULL[key]


def _check_colsums(X, inst, dtype):
    # column sums: sum_n Y[n, j] = S_phi for every j (each column runs through
    # all one-dimensional points once), so 1^T X = S_phi 1^T A
    T = oracle.phi_residue_values(inst.rule, inst.N, inst.phi, inst.modulus, inst.shift)
    S = float(np.sum(T))
    colsum = X.double().sum(dim=0).cpu().numpy()
    bound = S * inst.A.sum(axis=0)
    scale = ymax(inst) * np.abs(inst.A).sum(axis=0) * math.sqrt(inst.N)
    assert np.max(np.abs(colsum - bound) / scale) < (1e-10 if dtype == "f64" else 1e-5)


def _forward(inst, dtype, rows=None, tuning=None, autotuned=False):
    """X = Y A on the GPU against the oracle: every row when rows is None,
    else the given rows.  tuning: a fixed launch tuning; autotuned: the one
    bench.py's autotuner picks for this plan (the configuration the
    benchmark times)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    p = plan_of(inst)
    if autotuned:
        from paper_1501_06286_amd import autotune
        best, _ = autotune.tune(p, inst.t, reps=3, use_cache=False)
        announce(f"  autotuned launch {best}")
    elif tuning:
        p.set_tuning(**tuning)
    A = to_dev(inst.A, dtype)
    X = q.matmul(p, A)
    if rows is None:
        got = X.double().cpu().numpy()
        ref = oracle_full(inst)
    else:
        rows = rows(p) if callable(rows) else rows
        got = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        ref = oracle.matmul_rows(inst, rows)
    worst = assert_close(got, ref, inst.A, inst, dtype, inst.name)
    del got
    _check_colsums(X, inst, dtype)
    return p, A, X, worst


@pytest.mark.parametrize("dtype,how", [(d, h) for d in ("f32", "f64")
                                       for h in ("default", "autotuned", "chunk256_nt")])
def test_c2_gaussian_full(dtype, how):
    """Every one of the 65537 x 4096 entries against the oracle (Section 2.1,
    eq. (ZPa): the fast product equals the plain one, so every row must)."""
    inst = qi.make_c2(dtype)
    announce(f"C2 full size {dtype} {how}: whole output")
    _forward(inst, dtype, autotuned=how == "autotuned",
             tuning={"chunk_pairs": 256, "nt_store": 1} if how == "chunk256_nt" else None)


def test_c1_plain_lattice_fp64():
    """The plain-method workload as specified: N = 2003, s = 500, one column,
    phi = identity without shift, FP64; every entry at 1e-12, and the
    single column travels as the real part of one complex column pair."""
    inst = qi.make_c1()
    assert (inst.N, inst.s, inst.t, inst.phi, inst.shift, inst.dtype) == \
        (2003, 500, 1, qi.PHI_IDENTITY, (0, 1), "f64")
    announce("C1 plain lattice N=2003 s=500 t=1 FP64")
    p, A, X, worst = _forward(inst, "f64")
    assert p.info()["beta"] == 5  # the smallest primitive root of 2003
    assert worst <= 1e-12


def test_c2_matches_dense_baseline():
    """FFT path and dense MFMA GEMM agree on the whole C2 output (FP32)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.make_c2("f32")
    announce("C2 FFT vs dense")
    p = plan_of(inst)
    A = to_dev(inst.A, "f32")
    X = q.matmul(p, A)
    Y = q.explicit_points(p)
    Xd = q.dense_matmul(p, Y, A)
    scale = float(Y.abs().max()) * A.abs().sum(dim=0)
    err = float(((X - Xd).abs().max(dim=0).values / scale).max())
    assert err < 2 * TOL["f32"]


@pytest.mark.parametrize("how", ["default", "autotuned"])
def test_c3_pde_gf2_full(how):
    """Rows covering every e1 tile against the oracle, and the whole output
    against the dense MFMA product of the explicit Y (4.3 GB)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.make_c3("f32")
    announce(f"C3 full size (GF(2), m=16, s=16384, t=4096) {how}: tile rows")
    p, A, X, _ = _forward(inst, "f32", rows=lambda p: tile_rows(p, 31),
                          autotuned=how == "autotuned")
    if how != "default":
        return
    announce("C3 whole output vs the dense MFMA product")
    Y = q.explicit_points(p)
    Xd = q.dense_matmul(p, Y, A)
    scale = float(Y.abs().max()) * A.abs().sum(dim=0)
    del Y
    err = float(((X - Xd).abs().max(dim=0).values / scale).max())
    assert err < 2 * TOL["f32"], err


def test_c5_forward_adjoint_fd():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.make_c5("f32")
    announce("C5 full size forward: tile rows")
    p, A, X, _ = _forward(inst, "f32", rows=lambda p: tile_rows(p, 55))
    info = p.info()
    assert info["M2"] > 64  # exercises the split outer pass
    announce("C5 adjoint sampled entries")
    G = to_dev(inst.G, "f32")
    dA = q.matmul_adjoint(p, G)
    ent = qi.fd_entries(inst.s, inst.t)
    assert len(ent) == 32
    got = np.array([float(dA[j, k]) for j, k in ent])
    ref = oracle.adjoint_entries(inst, ent)
    scale = ymax(inst) * np.abs(inst.G).sum(axis=0)
    err = np.abs(got - ref) / np.array([scale[k] for _, k in ent])
    assert np.max(err) <= TOL["f32"], np.max(err)
    announce("C5 finite differences on all 32 seeded entries")
    # L(A) = <X(A), G> is linear in A: a central difference with the step that
    # is actually representable recovers dA up to the FP32 rounding of X
    Gd = G.double()
    Ap = A.clone()
    Xp = torch.empty_like(X)
    ws = p.workspace(inst.t, A.device)
    for (j, k) in ent:
        a0 = float(A[j, k])
        h = 16.0
        up = np.float32(a0 + h)
        dn = np.float32(a0 - h)
        Ap[j, k] = float(up)
        Lp = float((q.matmul(p, Ap, out=Xp, workspace=ws).double() * Gd).sum())
        Ap[j, k] = float(dn)
        Lm = float((q.matmul(p, Ap, out=Xp, workspace=ws).double() * Gd).sum())
        Ap[j, k] = a0
        fd = (Lp - Lm) / (float(up) - float(dn))
        assert abs(fd - float(dA[j, k])) <= 2e-3 * (abs(float(dA[j, k])) + scale[k] * 1e-3), (j, k, fd)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_split_outer_pass_lattice(dtype):
    """N = 200003 (L = 2 * 100001 not a power of two): M = 2^19, M2 = 128 > 64
    (3 x 2^17 and 5 x 2^16 < 2L - 1, so no shorter mixed length)."""
    N = 200003
    assert qi.is_prime(N)
    inst = qi.small_lattice(N, 300, 5, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    announce(f"split outer pass N={N} {dtype}")
    p, A, X, _ = _forward(inst, dtype, rows=sample_rows(N, 32, N + inst.s))
    assert p.info()["M2"] == 128
    import paper_1501_06286_amd as q
    G = qi.randn((N, inst.t), seed=11, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    assert_close(dA, oracle.adjoint(inst, G), G, inst, dtype, "split adjoint")


def test_split_outer_pass_gf2():
    """m = 19: L = 2^19 - 1, embedded in M = 2^20, M2 = 256."""
    torch_cuda()
    inst = qi.small_gf2(19, 96, 3, dtype="f64")
    announce("split outer pass GF(2) m=19")
    p, A, X, _ = _forward(inst, "f64", rows=sample_rows(inst.N, 24, inst.N + inst.s))
    assert p.info()["M2"] == 256


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_largest_supported_length(dtype):
    """The largest prime N with N - 1 not a power of two that a plan supports
    (N = 8388593: M = 2^24, outer length M2 = 4096): the split passes at
    their widest (P2 = 64) and the LDS back pass (Q2 = 64); sampled rows, the
    column sums and the adjoint (G on sampled rows) against the oracle."""
    N, q2 = 8388593, 64
    assert qi.is_prime(N)
    inst = qi.small_lattice(N, 8, 3, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=2)
    announce(f"largest length N={N} {dtype}")
    p, A, X, _ = _forward(inst, dtype, rows=sample_rows(N, 32, N + inst.s))
    info = p.info()
    assert info["M"] == 1 << 24
    assert info["Q2"] == q2 and info["P2"] == 64
    import paper_1501_06286_amd as q
    # G nonzero on 1024 sampled rows (row 0 among them), so the oracle's
    # Y^T G needs only those rows of Y
    rows = np.unique(np.concatenate([[0], sample_rows(N, 1023, 7)]))
    G = np.zeros((N, inst.t))
    G[rows] = qi.randn((len(rows), inst.t), seed=5, dtype=dtype)
    dA = q.matmul_adjoint(p, to_dev(G, dtype)).double().cpu().numpy()
    ref = oracle.Y_rows(inst, rows).T @ G[rows]
    assert_close(dA, ref, G, inst, dtype, "adjoint")
