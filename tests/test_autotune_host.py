"""Host logic of the launch tuner: the outer radices it tries (no GPU)."""
from paper_1501_06286_amd import autotune


def _default_q(M2, qmax):
    # the library's default split: all of M2 in one back pass when it fits
    return M2 if M2 <= qmax else max(32, M2 // 64)


def test_outer_radices_admissible_and_distinct():
    for qmax in (64, 128):
        for k in range(0, 13):
            M2 = 1 << k
            qs = autotune.outer_radices(M2, qmax)
            assert qs[0] == 0 and len(set(qs)) == len(qs)
            qdef = min(_default_q(M2, qmax), M2)
            for q in qs[1:]:
                assert q & (q - 1) == 0 and q <= qmax and q < M2 and M2 // q <= 64
                assert q != qdef


def test_outer_radices_keep_the_register_back_with_a_split():
    # M2 = 64 or 128 defaults to the LDS back pass with no split; the split +
    # register back pass (32) stays a candidate
    assert 32 in autotune.outer_radices(64, 128)
    assert 32 in autotune.outer_radices(128, 128)
    assert 32 in autotune.outer_radices(64, 64)
    # FP64 at M2 = 128 defaults to 32 (a split either way); 64 is the alternative
    assert autotune.outer_radices(128, 64) == [0, 16, 64]
    # short outer lengths: nothing to choose beyond 16 values per column
    assert autotune.outer_radices(32, 128) == [0, 16]
    assert autotune.outer_radices(16, 128) == [0]
    # C5-like M2 = 512: a split is needed whatever the radix
    assert autotune.outer_radices(512, 128) == [0, 16, 64, 128]
