"""Union of all Korobov lattice point sets (Section 2.2): the HIP path
against the oracle's explicit product, element by element."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

# K: direct (L a power of two) and embedded lengths, one and several on-chip
# sizes; s from one column of Y to more than K - 1; t odd, even, one
CASES = [
    (3, 1, 1, qi.PHI_IDENTITY, (0, 1)),
    (5, 3, 2, qi.PHI_CENTERED, (0, 1)),
    (7, 9, 3, qi.PHI_IDENTITY, (1, 3)),
    (17, 40, 5, qi.PHI_INVNORM, (0, 1)),       # no point is 0: Phi^-1 needs no shift
    (101, 64, 7, qi.PHI_INVNORM, (1, 202)),
    (257, 300, 4, qi.PHI_TENT, (0, 1)),
    (1021, 33, 2, qi.PHI_INVNORM, (1, 2042)),
    (1031, 48, 1, qi.PHI_CENTERED, (0, 1)),
]


def _union(inst, dtype):
    import paper_1501_06286_amd as q
    return q.KorobovUnion.from_instance(inst, dtype=dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("K,s,t,phi,shift", CASES)
def test_korobov_union_matches_oracle(K, s, t, phi, shift, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(K, s, t, phi=phi, shift=shift, dtype=dtype, seed=K)
    announce(f"korobov union {inst.name} phi={phi} {dtype}")
    U = _union(inst, dtype)
    info = U.info()
    assert info["N"] == (K - 1) ** 2 and info["blocks"] == K - 1 and info["L"] == K - 1
    X = q.korobov_matmul(U, to_dev(inst.A, dtype))
    torch.cuda.synchronize()
    assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, inst.name)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("t", [33, 100, 129, 250, 301])
def test_korobov_union_wide_outputs(t, dtype):
    """Many output columns: the collapse takes 2, 4 or 8 groups of 16 column
    pairs per tile (t = 33: 17 pairs, two groups, the second ragged; 301:
    151 pairs, a second tile row of two groups), element by element against
    the oracle, with colliding exponents (s > K - 1)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(31, 70, t, phi=qi.PHI_INVNORM, shift=(1, 62), dtype=dtype, seed=t)
    announce(f"korobov union wide t={t} {dtype}")
    U = _union(inst, dtype)
    X = q.korobov_matmul(U, to_dev(inst.A, dtype))
    torch.cuda.synchronize()
    assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, inst.name)


@pytest.mark.parametrize("chunk", [1, 7, 100, 0])
def test_korobov_chunks_give_the_same_bits(chunk):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(101, 50, 9, phi=qi.PHI_INVNORM, shift=(1, 202), dtype="f32", seed=1)
    announce(f"korobov chunk={chunk}")
    U = _union(inst, "f32")
    A = to_dev(inst.A, "f32")
    X0 = q.korobov_matmul(U, A)
    U.set_chunk(chunk)
    assert U.info()["chunk_blocks"] == chunk
    X1 = q.korobov_matmul(U, A, workspace=U.workspace(9))
    torch.cuda.synchronize()
    assert torch.equal(X0, X1)


def test_korobov_strided_operands():
    """Row strides beyond t on both A and X."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(61, 20, 5, phi=qi.PHI_CENTERED, dtype="f64", seed=2)
    announce("korobov strided")
    U = _union(inst, "f64")
    Abig = torch.zeros((inst.s, 8), dtype=torch.float64, device="cuda")
    Abig[:, :5] = to_dev(inst.A, "f64")
    Xbig = torch.full((inst.N, 11), 7.0, dtype=torch.float64, device="cuda")
    q.korobov_matmul(U, Abig[:, :5], out=Xbig[:, :5])
    torch.cuda.synchronize()
    assert_close(Xbig[:, :5].cpu().numpy(), oracle.matmul(inst), inst.A, inst, "f64", "strided")
    assert bool((Xbig[:, 5:] == 7.0).all())


def test_korobov_errors():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(13, 4, 2, dtype="f32")
    U = _union(inst, "f32")
    A = to_dev(inst.A, "f32")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QMCError) as e:
        q.korobov_matmul(U, A, workspace=small)
    assert e.value.code == -6
    X = torch.empty((inst.N, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(q.QMCError) as e:
        q.korobov_matmul(U, X[:inst.s], out=X)  # output overlaps the input
    assert e.value.code == -5


def test_korobov_full_size_sampled_rows():
    """The benchmark workload (K = 1021, s = 512, t = 256): every block's first
    and last row plus seeded random rows, against the oracle."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.make_korobov("f32")
    announce(f"korobov full size {inst.name}")
    U = _union(inst, "f32")
    X = q.korobov_matmul(U, to_dev(inst.A, "f32"))
    torch.cuda.synchronize()
    K = inst.modulus
    rg = np.random.default_rng(6)
    rows = np.unique(np.concatenate([np.arange(0, inst.N, K - 1), np.arange(K - 2, inst.N, K - 1),
                                     rg.integers(0, inst.N, size=512)]))
    got = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert_close(got, oracle.matmul_rows(inst, rows), inst.A, inst, "f32", "korobov full")


@pytest.mark.parametrize("epi", ["affine", "exp"])
def test_korobov_epilogue(epi):
    """The union with the per-column epilogue (Sections 3.2, 3.3) against the
    oracle's product and epilogue; no row 0 in the union, so every row goes
    through the back pass."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(31, 40, 7, phi=qi.PHI_INVNORM, shift=(1, 62), dtype="f64", seed=4)
    announce(f"korobov epilogue {epi}")
    inst.A = inst.A / np.sqrt(inst.s)
    U = q.KorobovUnion.from_instance(inst)
    rg = np.random.default_rng(9)
    bias = rg.standard_normal(inst.t) * 0.3
    scale = rg.uniform(0.5, 2.0, inst.t)
    X = q.korobov_matmul(U, to_dev(inst.A, "f64"), epilogue=epi, bias=to_dev(bias, "f64"),
                         scale=to_dev(scale, "f64"))
    torch.cuda.synchronize()
    kind = oracle.EPI_AFFINE if epi == "affine" else oracle.EPI_EXP
    ref = oracle.epilogue(oracle.matmul(inst), kind, bias, scale)
    err = np.abs(X.cpu().numpy() - ref) / np.maximum(1.0, np.abs(ref))
    assert float(err.max()) < 1e-11


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("K,s,t,chunk", [(13, 5, 3, 0), (31, 40, 7, 0), (31, 40, 7, 4),
                                         (31, 70, 1, 7), (61, 100, 16, 0)])
def test_korobov_adjoint_matches_oracle(K, s, t, chunk, dtype):
    """dA = Y^T G for the union against the oracle's explicit Y (the blocks'
    parts summed over runs of `chunk` blocks)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(K, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * K), dtype=dtype, seed=K)
    announce(f"korobov adjoint K={K} s={s} t={t} chunk={chunk} {dtype}")
    U = q.KorobovUnion.from_instance(inst)
    U.set_chunk(chunk)
    G = qi.randn((inst.N, t), seed=K + 1, dtype=dtype)
    dA = q.korobov_matmul_adjoint(U, to_dev(G, dtype))
    torch.cuda.synchronize()
    assert_close(dA.double().cpu().numpy(), oracle.adjoint(inst, G), G, inst, dtype, "adjoint")


def test_korobov_adjoint_full_size_dot_product():
    """At the full union (K = 1021, s = 512, t = 256, FP32): <Y A, G> equals
    <A, Y^T G> with both sides from the GPU."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.make_korobov("f32")
    announce("korobov adjoint full size")
    U = q.KorobovUnion.from_instance(inst)
    A = to_dev(inst.A, "f32")
    G = torch.randn((inst.N, inst.t), dtype=torch.float32, device="cuda", generator=torch.Generator(
        device="cuda").manual_seed(5))
    X = q.korobov_matmul(U, A)
    dA = q.korobov_matmul_adjoint(U, G)
    lhs = float((X.double() * G.double()).sum())
    rhs = float((A.double() * dA.double()).sum())
    scale = float(X.double().abs().sum() * G.double().abs().max())
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_korobov_autograd():
    """backward of the union's product is its adjoint: the gradient of
    <X(A), W> is Y^T W (oracle)."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_korobov(31, 40, 5, phi=qi.PHI_INVNORM, shift=(1, 62), dtype="f64", seed=8)
    announce("korobov autograd")
    U = q.KorobovUnion.from_instance(inst)
    A = to_dev(inst.A, "f64").requires_grad_(True)
    W = qi.randn((inst.N, inst.t), seed=2, dtype="f64")
    X = q.korobov_qmc_matmul(A, U)
    (X * to_dev(W, "f64")).sum().backward()
    torch.cuda.synchronize()
    assert_close(A.grad.cpu().numpy(), oracle.adjoint(inst, W), W, inst, "f64", "grad")
