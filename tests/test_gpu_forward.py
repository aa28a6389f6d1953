"""GPU parity of the forward product X = Y A against the CPU oracle.

Tolerance: max_n |X - X_oracle| <= tau max|Y| ||A[:, k]||_1 per
column k, tau = 1e-12 in FP64 and 1e-5 in FP32; the oracle reads the same
(already rounded) A.  Integer tables are compared bit for bit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import literal
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------------------
# bit-exact tables
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 3, 7, 101, 2003, 65537])
def test_lattice_tables_bit_exact(N):
    torch_cuda()
    announce(f"lattice tables N={N}")
    inst = qi.small_lattice(N, 37, 1)
    p = plan_of(inst)
    pw, lg, el, ph = p.tables()
    info = p.info()
    beta = info["beta"]
    ref_pw = np.array([pow(int(beta), e, N) for e in range(N - 1)], dtype=np.int64)
    assert np.array_equal(pw, ref_pw)
    assert lg[0] == -1 and np.array_equal(lg[pw], np.arange(N - 1))
    # beta is the smallest primitive root (brute-force check on small N)
    if N <= 2003:
        grp = literal._Lattice(N)
        assert beta == literal.primitive_element(grp)
    g = np.asarray(inst.gen, dtype=np.int64) % N
    assert np.array_equal(np.array([pow(int(beta), int(e), N) for e in el]), g)
    ref_phi = oracle.phi_residue_values(qi.RULE_LATTICE, N, qi.PHI_IDENTITY)
    assert np.array_equal(ph, ref_phi)


@pytest.mark.parametrize("m", [1, 2, 4, 8, 12])
def test_gf2_tables_bit_exact(m):
    torch_cuda()
    announce(f"gf2 tables m={m}")
    inst = qi.small_gf2(m, 19, 1, phi=qi.PHI_CENTERED)
    p = plan_of(inst)
    pw, lg, el, ph = p.tables()
    grp = literal._GF2(1 << m, inst.modulus)
    ref = literal.powers(grp, 1 if m == 1 else 2)
    assert np.array_equal(pw, np.array(ref))
    assert np.array_equal(lg[pw], np.arange((1 << m) - 1))
    assert np.array_equal(pw[el], np.asarray(inst.gen, dtype=np.int64))
    ref_phi = oracle.phi_residue_values(qi.RULE_POLY_GF2, 1 << m, qi.PHI_CENTERED, inst.modulus)
    assert np.array_equal(ph, ref_phi)


@pytest.mark.parametrize("phi,shift", [(qi.PHI_IDENTITY, (0, 1)), (qi.PHI_CENTERED, (0, 1)),
                                       (qi.PHI_TENT, (0, 1)), (qi.PHI_TENT, (3, 7)),
                                       (qi.PHI_INVNORM, (1, 2 * 4099)), (qi.PHI_INVNORM, (1, 3))])
def test_phi_table(phi, shift):
    torch_cuda()
    N = 4099
    announce(f"phi table phi={phi} shift={shift}")
    inst = qi.small_lattice(N, 5, 1, phi=phi, shift=shift)
    _, _, _, ph = plan_of(inst).tables()
    ref = oracle.phi_residue_values(qi.RULE_LATTICE, N, phi, 0, shift)
    if phi == qi.PHI_INVNORM:
        np.testing.assert_allclose(ph, ref, rtol=2e-15, atol=0)
    else:
        assert np.array_equal(ph, ref)


# ---------------------------------------------------------------------------
# forward parity on sizes the oracle finishes in seconds
# ---------------------------------------------------------------------------

LATTICE_CASES = [
    # N, s, t    (L power of two -> direct; otherwise embedded)
    (2, 3, 1), (3, 4, 2), (5, 2, 3), (7, 3, 4), (17, 40, 5), (101, 30, 7),
    (257, 300, 3), (1009, 100, 17), (2003, 500, 1), (4099, 200, 33),
    (8209, 1000, 64), (65537, 96, 3), (40009, 700, 9),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N,s,t", LATTICE_CASES)
def test_forward_lattice(N, s, t, dtype):
    torch = torch_cuda()
    phi, shift = (qi.PHI_INVNORM, (1, 2 * N)) if N % 2 else (qi.PHI_IDENTITY, (0, 1))
    if N == 2:
        phi, shift = qi.PHI_TENT, (1, 3)
    inst = qi.small_lattice(N, s, t, phi=phi, shift=shift, dtype=dtype)
    announce(f"forward lattice N={N} s={s} t={t} {dtype} phi={phi}")
    p = plan_of(inst)
    X = q_matmul(p, inst.A, dtype)
    torch.cuda.synchronize()
    ref = oracle.matmul(inst)
    assert_close(X, ref, inst.A, inst, dtype, inst.name)


GF2_CASES = [(1, 3, 2), (2, 5, 3), (4, 30, 4), (8, 300, 5), (10, 64, 33), (12, 1000, 8), (16, 40, 2)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m,s,t", GF2_CASES)
def test_forward_gf2(m, s, t, dtype):
    torch = torch_cuda()
    inst = qi.small_gf2(m, s, t, phi=qi.PHI_CENTERED, dtype=dtype)
    announce(f"forward gf2 m={m} s={s} t={t} {dtype}")
    p = plan_of(inst)
    X = q_matmul(p, inst.A, dtype)
    torch.cuda.synchronize()
    assert_close(X, oracle.matmul(inst), inst.A, inst, dtype, inst.name)


def q_matmul(plan, A, dtype):
    import paper_1501_06286_amd as q
    return q.matmul(plan, to_dev(A, dtype)).cpu().double().numpy()


def test_worked_example_regenerates_points():
    """N = 7, g = (1, 5, 3) (Example 1), A = I: X is the point matrix."""
    torch_cuda()
    announce("worked example N=7")
    inst = qi.Instance("ex1", qi.RULE_LATTICE, 7, 3, 3, np.array([1, 5, 3], dtype=np.uint64), 0,
                       qi.PHI_IDENTITY, (0, 1), "f64", np.eye(3))
    p = plan_of(inst)
    assert p.info()["beta"] == 3
    _, _, el, _ = p.tables()
    assert list(el + 1) == [1, 6, 2]  # the paper's c_j
    X = q_matmul(p, np.eye(3), "f64")
    conv = np.array([[0, 0, 0], [1, 5, 3], [2, 3, 6], [3, 1, 2], [4, 6, 5], [5, 4, 1], [6, 2, 4]])
    assert np.max(np.abs(X * 7 - conv)) < 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_identity_matrix_regenerates_Y(dtype):
    torch_cuda()
    N, s = 1031, 64
    inst = qi.small_lattice(N, s, s, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype)
    announce(f"A = I regenerates Y, N={N} {dtype}")
    X = q_matmul(plan_of(inst), np.eye(s), dtype)
    Y = oracle.Y_rows(inst)
    assert_close(X, Y, np.eye(s), inst, dtype, "A = I")


def test_determinism_bitwise():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(8209, 700, 20, phi=qi.PHI_INVNORM, shift=(1, 2 * 8209), dtype="f32")
    announce("determinism")
    p = plan_of(inst)
    A = to_dev(inst.A, "f32")
    X1 = q.matmul(p, A).clone()
    X2 = q.matmul(p, A)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)


def test_strided_inputs_and_odd_t():
    """lda > t and ldx > t (views into wider matrices), odd t."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N, s, t = 1009, 77, 5
    inst = qi.small_lattice(N, s, t, dtype="f64")
    announce("strided inputs")
    p = plan_of(inst)
    Abig = to_dev(np.concatenate([inst.A, np.full((s, 3), np.nan)], axis=1), "f64")
    Xbig = torch.full((N, t + 2), float("nan"), dtype=torch.float64, device="cuda")
    q.matmul(p, Abig[:, :t], out=Xbig[:, :t])
    torch.cuda.synchronize()
    Xb = Xbig.cpu().numpy()
    assert np.all(np.isnan(Xb[:, t:]))
    assert_close(Xb[:, :t], oracle.matmul(inst), inst.A, inst, "f64", "strided")


def test_errors_on_gpu_calls():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(101, 10, 2)
    p = plan_of(inst)
    A = to_dev(inst.A, "f64")
    with pytest.raises(q.QMCError) as e:
        q.matmul(p, A, workspace=torch.empty(8, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -6
    X = torch.empty((101, 2), dtype=torch.float64, device="cuda")
    big = torch.empty(10 ** 6, dtype=torch.float64, device="cuda")
    Aview = big[: 10 * 2].view(10, 2)
    Xview = big[10: 10 + 202].view(101, 2)
    with pytest.raises(q.QMCError) as e:
        q.matmul(p, Aview, out=Xview)
    assert e.value.code == -5


def test_empty_and_degenerate_inputs():
    """t = 0 columns is refused (QMC_ERR_ARG) before any launch; the smallest
    rules (N = 2: L = 1; N = 3) and one dimension give the oracle's product;
    A = 0 gives X = 0 exactly."""
    torch = torch_cuda()
    import ctypes
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(101, 10, 2, dtype="f64")
    p = plan_of(inst)
    A = to_dev(inst.A, "f64")
    X = torch.empty((101, 2), dtype=torch.float64, device="cuda")
    ws = p.workspace(2, "cuda")
    L = q.lib()
    rc = L.qmc_matmul(p.handle, ctypes.c_void_p(A.data_ptr()), 0, 2, ctypes.c_void_p(X.data_ptr()),
                      2, ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == -1
    for N, s, t in ((2, 1, 1), (2, 3, 2), (3, 1, 3), (5, 1, 1)):
        inst = qi.small_lattice(N, s, t, phi=qi.PHI_CENTERED, dtype="f64", seed=N + s)
        announce(f"degenerate N={N} s={s} t={t}")
        got = q.matmul(plan_of(inst), to_dev(inst.A, "f64")).cpu().numpy()
        assert_close(got, oracle.matmul(inst), inst.A, inst, "f64", f"N={N}")
    Z = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    p3 = plan_of(qi.small_lattice(101, 10, 3, dtype="f64"))
    assert torch.count_nonzero(q.matmul(p3, Z)) == 0
