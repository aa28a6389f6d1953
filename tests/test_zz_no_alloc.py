"""qmc_matmul_noalloc (the allocation-free X = Y A, workspace in the
library's static device scratch) against qmc_matmul on the same plan and
inputs: the same kernels in the same order, so the outputs must agree bit
for bit; two calls in a row, the second with fewer columns, so the second
runs on scratch that still holds the first call's contents."""
import ctypes

import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import TOL, announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

SCRATCH = 256 << 20  # QMC_NOALLOC_SCRATCH_BYTES


def _noalloc(p, A, X):
    import paper_1501_06286_amd as q
    torch = torch_cuda()
    return q.lib().qmc_matmul_noalloc(p.handle, ctypes.c_void_p(A.data_ptr()), A.shape[1],
                                      A.stride(0), ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _pair_of_calls(inst, dtype, t_small, tuning):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    p = plan_of(inst)
    p.set_tuning(**tuning)
    for t in (inst.t, t_small):
        assert p.workspace_bytes(t) <= SCRATCH
        announce(f"  noalloc {inst.name} {dtype} t={t} tuning {tuning}")
        A = to_dev(inst.A[:, :t], dtype)
        ref = q.matmul(p, A)
        X = torch.full((inst.N, t), float("nan"), dtype=A.dtype, device=A.device)
        rc = _noalloc(p, A, X)
        assert rc == 0, q.lib().qmc_strerror(rc)
        torch.cuda.synchronize()
        assert torch.equal(X, ref), "noalloc output differs from qmc_matmul"
        rows = np.array(sorted({0, 1, inst.N - 1} | set(range(2, inst.N, max(1, inst.N // 37)))))
        got = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        sub = qi.Instance(**{**inst.__dict__, "A": inst.A[:, :t], "t": t})
        assert_close(got, oracle.matmul_rows(sub, rows), sub.A, sub, dtype, "noalloc vs oracle")
    return p


def test_noalloc_sparse_front_f32():
    # the Gaussian-sampling rule at 512 columns, chunked so the workspace
    # fits the scratch; then 97 columns (odd: one half-empty pair)
    inst = qi.small_lattice(65537, 4096, 512, phi=qi.PHI_INVNORM, shift=(1, 2 * 65537),
                            dtype="f32", seed=3)
    _pair_of_calls(inst, "f32", 97, {"chunk_pairs": 64, "nt_store": 1})


def test_noalloc_two_stream_tuning_runs_on_one_stream():
    inst = qi.small_lattice(65537, 1024, 256, phi=qi.PHI_INVNORM, shift=(1, 2 * 65537),
                            dtype="f32", seed=4)
    _pair_of_calls(inst, "f32", 33, {"chunk_pairs": 32, "streams": 2})


def test_noalloc_dense_front_embedded_f64():
    # N - 1 not a power of two (embedded convolution), dense outer front, FP64
    N = 200003
    inst = qi.small_lattice(N, 300, 6, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype="f64",
                            seed=5)
    _pair_of_calls(inst, "f64", 3, {"front": 2})


def test_noalloc_gf2_f32():
    inst = qi.small_gf2(12, 200, 9, dtype="f32")
    _pair_of_calls(inst, "f32", 4, {})


def test_noalloc_non_prime_n():
    # N = 2^14: blocks of the orbits 2^k and the rows summed directly
    inst = qi.unit_lattice(1 << 14, 96, 12, phi=qi.PHI_INVNORM, shift=(1, 2 << 14),
                           dtype="f32", seed=7)
    _pair_of_calls(inst, "f32", 5, {})


def test_noalloc_rejects_what_does_not_fit():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = qi.small_lattice(65537, 64, 2, phi=qi.PHI_INVNORM, shift=(1, 2 * 65537), dtype="f32",
                            seed=6)
    p = plan_of(inst)
    t = 4096  # unchunked: the intermediate alone is 1 GiB
    assert p.workspace_bytes(t) > SCRATCH
    A = torch.zeros((inst.s, t), dtype=torch.float32, device="cuda")
    X = torch.zeros((inst.N, t), dtype=torch.float32, device="cuda")
    assert _noalloc(p, A, X) == -6  # QMC_ERR_WORKSPACE
    p.profile(True)
    assert _noalloc(p, A[:, :2], X[:, :2]) == -1  # instrumentation creates events
    p.profile(False)
    # X overlapping A: its first s rows are A
    Xo = torch.zeros((inst.N, 2), dtype=torch.float32, device="cuda")
    assert _noalloc(p, Xo[:inst.s], Xo) == -5  # QMC_ERR_ALIAS
    torch.cuda.synchronize()
    assert bool((X == 0).all())  # nothing was launched
