"""Every launch tuning (sparse or dense outer front, chunks of column pairs,
one or two streams, plain or non-temporal stores) gives the same X, to the
parity bar, as the oracle."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("chunk,streams,nt,front", [
    (0, 1, 1, 1), (5, 1, 0, 1), (5, 2, 0, 1), (7, 2, 1, 1), (16, 2, 0, 1), (1, 2, 1, 1),
    (0, 1, 0, 2), (5, 1, 1, 2), (16, 1, 0, 2), (1, 1, 0, 2), (3, 2, 0, 2),
    (0, 1, 1, 3), (5, 1, 0, 3), (7, 2, 1, 3)])
def test_tuned_forward(chunk, streams, nt, front, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 8209, 400, 33  # 17 column pairs: ragged chunks
    inst = qi.small_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    announce(f"tuning chunk={chunk} streams={streams} nt={nt} front={front} {dtype}")
    p = plan_of(inst)
    p.set_tuning(chunk_pairs=chunk, streams=streams, nt_store=nt, front=front)
    assert p.get_tuning() == {"chunk_pairs": chunk, "streams": streams, "nt_store": nt,
                              "front": front, "outer_q": 0, "nt_inter": 0}
    A = to_dev(inst.A, dtype)
    X1 = q.matmul(p, A)
    X2 = q.matmul(p, A)  # back-to-back calls reuse the slots and events
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)
    assert_close(X1.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, "tuned")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("chunk", [0, 1, 5, 16])
def test_chunked_adjoint(chunk, dtype):
    """The adjoint in chunks of column pairs (chunk_pairs applies to it too;
    17 pairs: ragged chunks) matches the oracle and the unchunked adjoint."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 8209, 400, 33
    inst = qi.small_lattice(N, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=3)
    announce(f"chunked adjoint chunk={chunk} {dtype}")
    p = plan_of(inst)
    G = np.random.default_rng(8).standard_normal((N, t))
    Gd = to_dev(G, dtype)
    dA0 = q.matmul_adjoint(p, Gd)
    p.set_tuning(chunk_pairs=chunk)
    dA = q.matmul_adjoint(p, Gd)
    torch.cuda.synchronize()
    assert torch.equal(dA, dA0)
    Gr = G.astype(np.float32).astype(np.float64) if dtype == "f32" else G
    assert_close(dA.double().cpu().numpy(), oracle.adjoint(inst, Gr), Gr, inst, dtype, "adjoint")


def test_tuning_rejects_bad_values():
    torch_cuda()
    import paper_1501_06286_amd as q
    p = plan_of(qi.small_lattice(101, 5, 2))
    for bad in ({"chunk_pairs": -1}, {"streams": 3}, {"nt_store": 2}, {"front": 4},
                {"front": -1}, {"nt_inter": 3}, {"nt_inter": -1}):
        with pytest.raises(q.QMCError):
            p.set_tuning(**bad)


def test_autotune_picks_a_candidate(tmp_path, monkeypatch):
    torch_cuda()
    from paper_1501_06286_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    inst = qi.small_lattice(8209, 300, 64, phi=qi.PHI_INVNORM, shift=(1, 2 * 8209), dtype="f32")
    p = plan_of(inst)
    best, res = autotune.tune(p, 64, reps=2)
    assert best in [c for c, _ in res]
    assert p.get_tuning() == best
    best2, _ = autotune.tune(p, 64)  # from the cache
    assert best2 == best


# dense outer front on every layout kind: direct and embedded lengths, the
# split outer pass (M2 > 64), GF(2), repeated generators, odd t, one column
DENSE_CASES = [
    ("lattice", 2003, 500, 7), ("lattice", 65537, 300, 4), ("lattice", 139999, 100, 3),
    ("lattice", 557057, 64, 2), ("lattice", 101, 300, 1), ("gf2", 12, 900, 5), ("gf2", 18, 50, 2),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("kind,n,s,t", DENSE_CASES)
def test_dense_front_matches_oracle_and_sparse(kind, n, s, t, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    if kind == "lattice":
        inst = qi.small_lattice(n, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * n), dtype=dtype, seed=11)
    else:
        inst = qi.small_gf2(n, s, t, dtype=dtype, seed=11)
    announce(f"dense front {inst.name} {dtype}")
    p = plan_of(inst)
    A = to_dev(inst.A, dtype)
    p.set_tuning(front=2)
    Xd = q.matmul(p, A)
    p.set_tuning(front=1)
    Xs = q.matmul(p, A)
    torch.cuda.synchronize()
    ref = oracle.matmul(inst)
    assert_close(Xd.double().cpu().numpy(), ref, inst.A, inst, dtype, "dense front")
    assert_close(Xs.double().cpu().numpy(), ref, inst.A, inst, dtype, "sparse front")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("q,front", [(0, 1), (2, 1), (16, 1), (32, 1), (64, 1), (64, 2), (4, 2),
                                     (128, 1), (128, 2)])
def test_outer_radix(q, front, dtype):
    """Every split M2 = P2 x Q2 of the outer DFT (M = 2^19, M2 = 128) gives the
    oracle's product and adjoint; Q2 = 64 and 128 take the back pass that
    holds the outer factor in LDS (128: FP32 only, and FP32's default)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q_
    inst = qi.small_lattice(200003, 100, 5, phi=qi.PHI_INVNORM, shift=(1, 400006), dtype=dtype,
                            seed=9)
    announce(f"outer radix q={q} front={front} {dtype}")
    p = plan_of(inst)
    if q == 128 and dtype == "f64":
        with pytest.raises(q_.QMCError):
            p.set_tuning(outer_q=q, front=front)
        return
    p.set_tuning(outer_q=q, front=front)
    info = p.info()
    assert info["M2"] == 128 and info["P2"] * info["Q2"] == 128
    assert info["Q2"] == (q if q else (128 if dtype == "f32" else 32))
    A = to_dev(inst.A, dtype)
    X = q_.matmul(p, A)
    rg = np.random.default_rng(1)
    G = rg.standard_normal((inst.N, 5))
    dA = q_.matmul_adjoint(p, to_dev(G, dtype))
    torch.cuda.synchronize()
    assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, "forward")
    Gr = G.astype(np.float32).astype(np.float64) if dtype == "f32" else G
    assert_close(dA.double().cpu().numpy(), oracle.adjoint(inst, Gr), Gr, inst, dtype, "adjoint")


def test_outer_radix_rejects_bad_values():
    torch_cuda()
    import paper_1501_06286_amd as q
    p = plan_of(qi.small_lattice(200003, 20, 2))  # M2 = 128
    for bad in (3, 256, 1, -2):  # a factor 3 that M2 lacks, above 128, P2 = 128 > 64, negative
        with pytest.raises(q.QMCError):
            p.set_tuning(outer_q=bad)
    assert p.info()["Q2"] == 32  # FP64 default, unchanged by the rejected calls


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("N", [100003, 200003])
def test_default_outer_split(N, dtype):
    """The default split: one back pass over all of M2 when it fits (M2 = 64:
    both dtypes; M2 = 128: FP32), else Q2 = 32 after a split pass (FP64 at
    M2 = 128); product and adjoint match the oracle either way."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q_
    inst = qi.small_lattice(N, 70, 6, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=12)
    announce(f"default outer split N={N} {dtype}")
    p = plan_of(inst)
    info = p.info()
    M2 = info["M2"]
    assert M2 == (64 if N == 100003 else 128)
    fits = M2 <= (128 if dtype == "f32" else 64)
    assert (info["P2"], info["Q2"]) == ((1, M2) if fits else (M2 // 32, 32))
    X = q_.matmul(p, to_dev(inst.A, dtype))
    G = np.random.default_rng(13).standard_normal((N, 6))
    dA = q_.matmul_adjoint(p, to_dev(G, dtype))
    torch.cuda.synchronize()
    assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, "forward")
    Gr = G.astype(np.float32).astype(np.float64) if dtype == "f32" else G
    assert_close(dA.double().cpu().numpy(), oracle.adjoint(inst, Gr), Gr, inst, dtype, "adjoint")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("q", [64, 128])
@pytest.mark.parametrize("t", [37, 1])
def test_lds_back_tiles(q, t, dtype):
    """The LDS back pass over several and ragged tiles of 8 column pairs (t =
    37: 19 pairs) and over one column, at M2 = 128 with one split (Q2 = 64)
    and none (Q2 = 128, FP32 only), forward and adjoint."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q_
    if q == 128 and dtype == "f64":
        pytest.skip("Q2 = 128 is FP32 only (rejected for FP64 in test_outer_radix)")
    N = 200003
    inst = qi.small_lattice(N, 60, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=4)
    announce(f"lds back q={q} t={t} {dtype}")
    p = plan_of(inst)
    p.set_tuning(outer_q=q)
    X = q_.matmul(p, to_dev(inst.A, dtype))
    G = np.random.default_rng(5).standard_normal((N, t))
    dA = q_.matmul_adjoint(p, to_dev(G, dtype))
    torch.cuda.synchronize()
    assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, "forward")
    Gr = G.astype(np.float32).astype(np.float64) if dtype == "f32" else G
    assert_close(dA.double().cpu().numpy(), oracle.adjoint(inst, Gr), Gr, inst, dtype, "adjoint")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", ["gauss", "gf2", "m2_512", "m2_4096", "tiny"])
def test_bucket_twiddle_front(case, dtype):
    """The sparse front with bucket twiddles (front 3) against the oracle and
    the item-twiddle front: outer lengths with the short factors in LDS
    (M2 = 16, 32) and read from the global table (M2 = 512, 4096), and R < 16."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    if case == "gauss":
        inst = qi.small_lattice(65537, 700, 6, phi=qi.PHI_INVNORM, shift=(1, 2 * 65537),
                                dtype=dtype)
    elif case == "gf2":
        inst = qi.small_gf2(16, 900, 5, dtype=dtype)
    elif case == "m2_512":
        N = 1048573
        inst = qi.small_lattice(N, 300, 3, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    elif case == "m2_4096":
        N = 8388593
        inst = qi.small_lattice(N, 40, 2, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    else:
        inst = qi.small_lattice(1009, 50, 7, phi=qi.PHI_CENTERED, dtype=dtype)
    announce(f"bucket twiddles {case} {dtype}")
    p = plan_of(inst)
    A = to_dev(inst.A, dtype)
    p.set_tuning(front=1)
    X1 = q.matmul(p, A)
    p.set_tuning(front=3)
    X3 = q.matmul(p, A)
    torch.cuda.synchronize()
    N = inst.N
    rg = np.random.default_rng(N)
    rows = np.unique(np.concatenate([[0, 1, N - 1], rg.choice(N, size=min(N, 400), replace=False)]))
    got = X3[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert_close(got, oracle.matmul_rows(inst, rows), inst.A, inst, dtype, f"front 3 {case}")
    scale = float(np.max(np.abs(oracle.phi_residue_values(inst.rule, N, inst.phi, inst.modulus,
                                                          inst.shift))))
    d = float((X3 - X1).abs().max()) / (scale * float(np.abs(inst.A).sum(axis=0).max()))
    assert d <= (1e-12 if dtype == "f64" else 1e-5)
