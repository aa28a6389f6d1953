"""Group-order output rows (qmc_plan_set_row_order): row 0 is point 0 and row
1 + e the point of beta^e.  The values are those of the conventional product
moved to other rows (bit for bit), the lattice rows are checked against the
oracle at beta^e mod N computed here, and the adjoint reads G in the same
order."""
import numpy as np
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _insts(dtype):
    N = 8209
    return [qi.small_lattice(N, 300, 21, phi=qi.PHI_INVNORM, shift=(1, 2 * N), dtype=dtype, seed=6),
            qi.small_lattice(139999, 100, 5, phi=qi.PHI_INVNORM, shift=(1, 279998), dtype=dtype,
                             seed=7),
            qi.small_gf2(12, 200, 9, dtype=dtype, seed=6)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("which", [0, 1, 2])
@pytest.mark.parametrize("tuning", [{}, {"chunk_pairs": 3, "nt_store": 1}, {"front": 2}])
def test_group_order_forward_adjoint(which, tuning, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = _insts(dtype)[which]
    announce(f"group order {inst.name} {tuning} {dtype}")
    p = plan_of(inst)
    if tuning:
        p.set_tuning(**tuning)
    A = to_dev(inst.A, dtype)
    Xc = q.matmul(p, A)
    pw = p.tables()[0].astype(np.int64)
    perm = torch.from_numpy(np.concatenate([[0], pw])).cuda()  # group row -> conventional row
    p.set_row_order(q.ROWS_GROUP)
    Xg = q.matmul(p, A)
    torch.cuda.synchronize()
    assert torch.equal(Xg, Xc[perm])
    if inst.rule == qi.RULE_LATTICE:
        beta = p.info()["beta"]
        e = np.arange(0, inst.N - 1, max(1, (inst.N - 1) // 97))
        rows = np.array([pow(int(beta), int(k), inst.N) for k in e], dtype=np.int64)
        ref = oracle.matmul_rows(inst, rows)
        got = Xg[torch.from_numpy(1 + e).cuda()].double().cpu().numpy()
        assert_close(got, ref, inst.A, inst, dtype, "group rows")
    # the adjoint takes G in the same order: dA is unchanged
    G = qi.randn((inst.N, inst.t), seed=3, dtype=dtype)
    Gc = to_dev(G, dtype)
    p.set_row_order(q.ROWS_CONVENTIONAL)
    dAc = q.matmul_adjoint(p, Gc)
    p.set_row_order(q.ROWS_GROUP)
    dAg = q.matmul_adjoint(p, Gc[perm].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(dAg, dAc)


def test_group_order_in_a_batch_and_errors():
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    insts = _insts("f32")
    announce("group order in a batch")
    plans = [plan_of(i) for i in insts]
    plans[1].set_row_order(q.ROWS_GROUP)
    As = [to_dev(i.A, "f32") for i in insts]
    Xs = q.Batch(plans, As).run()
    for p, A, X in zip(plans, As, Xs):
        assert torch.equal(q.matmul(p, A), X)
    with pytest.raises(q.QMCError):
        plans[0].set_row_order(2)
