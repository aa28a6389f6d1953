"""Batched products: one persistent launch per pass over many plans."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

MIXED = [  # (N, s, t): direct and embedded lengths, small on-chip sizes, a split outer pass
    (2, 3, 1), (3, 5, 2), (7, 3, 3), (101, 40, 5), (257, 300, 4), (1009, 64, 7), (2003, 500, 1),
    (4099, 200, 9), (65537, 64, 2), (139999, 100, 3), (8209, 1000, 16),
]


def _instances(dtype, seed=0):
    out = []
    for k, (N, s, t) in enumerate(MIXED):
        phi, sh = (qi.PHI_INVNORM, (1, 2 * N)) if N % 2 else (qi.PHI_TENT, (1, 3))
        out.append(qi.small_lattice(N, s, t, phi=phi, shift=sh, dtype=dtype, seed=seed + k))
    out.append(qi.small_gf2(10, 77, 5, dtype=dtype, seed=seed))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_mixed(dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _instances(dtype)
    announce(f"batch mixed {dtype} ({len(insts)} products)")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, dtype) for i in insts]
    b = q.Batch(plans, As)
    Xs = b.run()
    torch.cuda.synchronize()
    for inst, X in zip(insts, Xs):
        assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, inst.name)
    # the one-shot entry point gives the same bits
    Xs2 = q.matmul_batched(plans, As)
    for X, X2 in zip(Xs, Xs2):
        assert torch.equal(X, X2)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_lds_back(dtype):
    """Products whose back pass holds the outer factor in LDS (M2 = 128 with
    Q2 = 64 after one split, or Q2 = 128 with none) batched beside
    register-back products: each matches the oracle and its single product."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    N = 200003
    insts = [qi.small_lattice(N, 100, t, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype,
                              seed=20 + t) for t in (3, 19, 1)]
    insts.append(qi.small_lattice(8209, 300, 9, phi=qi.PHI_INVNORM, shift=(1, 16418),
                                  dtype=dtype, seed=7))
    announce(f"batch lds back {dtype}")
    plans = [plan_of(i) for i in insts]
    qs = (64, 128 if dtype == "f32" else 64, 64, 0)
    for p, oq in zip(plans, qs):
        p.set_tuning(outer_q=oq)
    As = [to_dev(i.A, dtype) for i in insts]
    Xs = q.Batch(plans, As).run()
    torch.cuda.synchronize()
    for inst, p, A, X in zip(insts, plans, As, Xs):
        assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, dtype, inst.name)
        assert torch.equal(q.matmul(p, A), X)


@pytest.mark.parametrize("chunk", [0, 1, 3 << 20])
def test_batch_chunks(chunk):
    """Runs of products sized by their intermediates (0: one run per layout
    group; 1 byte: every product alone; 3 MiB: a few per run) give the same
    bits as the single products, and the workspace shrinks with the chunk."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _instances("f32", seed=11)
    announce(f"batch chunk {chunk}")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, "f32") for i in insts]
    b = q.Batch(plans, As, chunk_bytes=chunk)
    ws = b.workspace.numel()
    Xs = b.run()
    torch.cuda.synchronize()
    for p, A, X in zip(plans, As, Xs):
        assert torch.equal(q.matmul(p, A), X)
    b.set_chunk(0)
    assert b.workspace.numel() >= ws
    Xs0 = [X.clone() for X in b.run()]
    torch.cuda.synchronize()
    for X, X0 in zip(Xs, Xs0):
        assert torch.equal(X, X0)
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("epi", ["affine", "exp"])
def test_batch_epilogue(epi, dtype):
    """Per-product epilogues in a batch (Sections 3.2, 3.3) give the bits of
    qmc_matmul_epilogue on each product: register and LDS back passes, some
    products without a bias or a scale, runs of one product each."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _instances(dtype, seed=21)
    N = 200003
    insts.append(qi.small_lattice(N, 100, 19, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype,
                                  seed=22))
    announce(f"batch epilogue {epi} {dtype}")
    plans = [plan_of(i) for i in insts]
    plans[-1].set_tuning(outer_q=64)  # the LDS back pass
    for inst in insts:  # keep exp's argument moderate
        inst.A = qi._round_to(inst.A / np.sqrt(inst.s), dtype)
    As = [to_dev(i.A, dtype) for i in insts]
    rg = np.random.default_rng(3)
    biases = [None if k % 3 == 1 else to_dev(0.3 * rg.standard_normal(i.t), dtype)
              for k, i in enumerate(insts)]
    scales = [None if k % 4 == 2 else to_dev(rg.uniform(0.5, 2.0, i.t), dtype)
              for k, i in enumerate(insts)]
    b = q.Batch(plans, As, chunk_bytes=1)
    b.set_epilogue(epi, biases, scales)
    Xs = b.run()
    torch.cuda.synchronize()
    for p, A, X, bi, sc in zip(plans, As, Xs, biases, scales):
        ref = q.matmul(p, A, epilogue=epi, bias=bi, scale=sc)
        torch.cuda.synchronize()
        assert torch.equal(X, ref)
    b.set_epilogue(None)  # back to the plain products
    Xs = b.run()
    for p, A, X in zip(plans, As, Xs):
        assert torch.equal(X, q.matmul(p, A))
    b.close()


def test_batch_matches_single_products():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _instances("f32", seed=3)
    announce("batch vs single")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, "f32") for i in insts]
    Xs = q.Batch(plans, As).run()
    for p, A, X in zip(plans, As, Xs):
        assert torch.equal(q.matmul(p, A), X)


def test_batch_graph_replay():
    """Capture one batched run in a HIP graph; replay it several times with
    new inputs copied in and eager work in between; every replay matches the
    eager result."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _instances("f32", seed=5)
    announce("batch graph capture")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, "f32") for i in insts]
    b = q.Batch(plans, As)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        scale = 1.0 + rep
        for A, inst in zip(As, insts):
            A.copy_(to_dev(inst.A * scale, "f32"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        got = [X.clone() for X in b.Xs]
        ref = [q.matmul(p, A) for p, A in zip(plans, As)]
        torch.cuda.synchronize()
        for x, r in zip(got, ref):
            assert torch.equal(x, r), f"replay {rep}"
        del junk


def test_batched_config_full():
    """The 256-instance batched workload: every product checked on sampled rows."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = qi.make_c4()
    announce("C4 batched, 256 products")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, "f32") for i in insts]
    Xs = q.Batch(plans, As).run()
    torch.cuda.synchronize()
    rg = np.random.default_rng(4)
    for inst, X in zip(insts, Xs):
        rows = np.unique(np.concatenate([[0, inst.N - 1], rg.integers(0, inst.N, size=3)]))
        got = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        assert_close(got, oracle.matmul_rows(inst, rows), inst.A, inst, "f32", inst.name)


def test_batch_autotune_outer_radix():
    """The batch tuner sets an admissible outer radix per outer length, and
    the tuned batch still gives the single products' bits."""
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    from paper_1501_06286_amd import autotune
    insts = _instances("f32", seed=7)
    announce("batch outer radix tuning")
    plans = [plan_of(i) for i in insts]
    As = [to_dev(i.A, "f32") for i in insts]
    best, timings = autotune.tune_batch(plans, As, reps=1)
    for p in plans:
        m2 = p.info()["M2"]
        if m2 in best:
            assert p.get_tuning()["outer_q"] == best[m2]
    b = q.Batch(plans, As)
    (chunk, nt), res = autotune.tune_batch_chunk(b, reps=1, chunks_mib=(1, 256))
    assert (chunk, nt) in [c for c, _ in res]
    Xs = b.run()
    for p, A, X in zip(plans, As, Xs):
        assert torch.equal(q.matmul(p, A), X)


def test_batch_rejects_aliasing():
    """qmc_batch_create refuses an output X_i that overlaps another product's
    A_k or X_k, qmc_batch_set_epilogue an epilogue vector inside some X, and
    qmc_batch_run a workspace that overlaps an operand (QMC_ERR_ALIAS, before
    any launch).  Every overlapping buffer lies inside one allocation large
    enough for what the call would write, so a missed check could not write
    outside it."""
    torch = torch_cuda()
    import ctypes
    import paper_1501_06286_amd as q
    insts = [qi.small_lattice(101, 10, 3, dtype="f32", seed=1),
             qi.small_lattice(103, 12, 3, dtype="f32", seed=2)]
    announce("batch aliasing checks")
    plans = [plan_of(i) for i in insts]
    big = torch.zeros(1 << 22, dtype=torch.float32, device="cuda")
    A0 = big[0:30].view(10, 3)
    A1 = big[64:100].view(12, 3)
    A0.copy_(torch.from_numpy(insts[0].A))
    A1.copy_(torch.from_numpy(insts[1].A))
    X0 = big[1024:1024 + 303].view(101, 3)
    X1 = big[2048:2048 + 309].view(103, 3)
    for bad in ([X0, big[10:10 + 309].view(103, 3)],        # X_1 over A_0
                [X0, big[1100:1100 + 309].view(103, 3)],    # X_1 over X_0
                [big[70:70 + 303].view(101, 3), X1]):       # X_0 over A_1
        with pytest.raises(q.QMCError) as e:
            q.Batch(plans, [A0, A1], bad)
        assert e.value.code == -5
    b = q.Batch(plans, [A0, A1], [X0, X1])
    with pytest.raises(q.QMCError) as e:
        b.set_epilogue("affine", biases=[X1[0], None])
    assert e.value.code == -5
    L = q.lib()
    nb = ctypes.c_size_t()
    assert L.qmc_batch_workspace_size(b._h, ctypes.byref(nb)) == 0
    need = nb.value
    assert need < 4 * (big.numel() - 2048 - 4096)
    for start in (0, 2048):  # over A_0, over X_1
        ws = big.data_ptr() + 4 * start
        rc = L.qmc_batch_run(b._h, ctypes.c_void_p(ws), ctypes.c_size_t(need),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == -5
    torch.cuda.synchronize()
    Xs = b.run()
    torch.cuda.synchronize()
    for inst, X in zip(insts, Xs):
        assert_close(X.double().cpu().numpy(), oracle.matmul(inst), inst.A, inst, "f32", inst.name)
