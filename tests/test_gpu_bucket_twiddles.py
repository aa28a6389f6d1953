"""The sparse front with bucket twiddles (tuning front = 3: an item's slot
twiddle split into W_{M2}^{e2 w2} from a table of M2 values and W_M^{e1 w2}
applied once per bucket) on every power-of-two outer length M2 = 1 .. 128 and
on-chip size R = 1 .. 16 (R = 2 and 4 hold several column pairs per
workgroup, some of them idle), direct and embedded lengths, lattice and GF(2)
rules, repeated slots (s > L), ragged chunks of column pairs, cached and
streaming stores of the intermediate: each product against the oracle and
against the item-twiddle front (front = 1)."""
import pytest

import oracle
import qmc_inputs as qi
from gpu_helpers import announce, assert_close, plan_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

# (kind, N or m, s, t, expected R, expected M2)
CASES = [
    ("lattice", 3, 40, 5, 1, 2),        # L = 2: M = 2, M1 = 1
    ("lattice", 5, 30, 3, 1, 4),        # L = 4, s > L: repeated slots
    ("lattice", 17, 100, 7, 2, 2),      # 16 transforms per workgroup, 4 pairs: 12 idle
    ("lattice", 101, 300, 9, 4, 4),     # embedded in 256
    ("lattice", 257, 200, 6, 4, 4),     # direct
    ("lattice", 1031, 500, 5, 16, 1),   # one outer frequency
    ("lattice", 16381, 300, 33, 16, 8),
    ("lattice", 65537, 400, 9, 16, 16),
    ("lattice", 50021, 700, 5, 16, 32),
    ("lattice", 200003, 100, 5, 16, 128),
    ("gf2", 12, 900, 5, 16, 2),
    ("gf2", 16, 300, 3, 16, 32),
]


def _inst(kind, n, s, t, dtype):
    if kind == "lattice":
        return qi.small_lattice(n, s, t, phi=qi.PHI_INVNORM, shift=(1, 2 * n), dtype=dtype, seed=21)
    return qi.small_gf2(n, s, t, phi=qi.PHI_CENTERED, shift=(1, 2 << n), dtype=dtype, seed=21)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("kind,n,s,t,R,M2", CASES)
def test_bucket_twiddles(kind, n, s, t, R, M2, dtype):
    torch = torch_cuda()
    import paper_1501_06286_amd as q
    inst = _inst(kind, n, s, t, dtype)
    announce(f"bucket twiddles {inst.name} {dtype}")
    p = plan_of(inst)
    info = p.info()
    assert (info["M1"], info["M2"]) == (R ** 3, M2)
    A = to_dev(inst.A, dtype)
    ref = oracle.matmul(inst)
    p.set_tuning(front=1)
    X1 = q.matmul(p, A)
    for chunk, nt_inter in ((0, 1), (2, 2)):  # all pairs, cached C; ragged chunks, streaming C
        p.set_tuning(front=3, chunk_pairs=chunk, nt_inter=nt_inter)
        X3 = q.matmul(p, A)
        torch.cuda.synchronize()
        what = f"front 3 chunk={chunk}"
        assert_close(X3.double().cpu().numpy(), ref, inst.A, inst, dtype, what)
        assert_close(X3.double().cpu().numpy(), X1.double().cpu().numpy(), inst.A, inst, dtype,
                     what + " vs front 1")
