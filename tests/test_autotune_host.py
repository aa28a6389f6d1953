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


def test_outer_radices_of_mixed_lengths():
    # M2 = 3 x 2^j: the factor 3 stays in the back pass, P2 = M2 / q a power
    # of two; the default (all of M2 up to the dtype's limit) is not repeated
    for qmax in (64, 128):
        for j in range(0, 6):
            M2 = 3 << j
            qs = autotune.outer_radices(M2, qmax)
            assert qs[0] == 0 and len(set(qs)) == len(qs)
            for q in qs[1:]:
                assert q % 3 == 0 and M2 % q == 0 and (M2 // q) & (M2 // q - 1) == 0
                assert q <= qmax and q < M2 and M2 // q <= 64
    for qmax in (64, 128):
        for j in range(0, 5):
            M2 = 5 << j
            for q in autotune.outer_radices(M2, qmax)[1:]:
                assert q % 5 == 0 and M2 % q == 0 and (M2 // q) & (M2 // q - 1) == 0
    assert autotune.outer_radices(80, 128) == [0, 10, 20, 40]
    assert autotune.outer_radices(96, 128) == [0, 12, 24, 48]
    assert autotune.outer_radices(48, 64) == [0, 12, 24]
    assert autotune.outer_radices(12, 128) == [0]


def test_bucket_twiddles_only_for_power_of_two_outer_lengths():
    fronts = lambda M2: {c["front"] for c in autotune.candidates(64, M2, 128)}
    assert fronts(64) == {1, 2, 3}
    assert fronts(96) == {1, 2}
    assert fronts(80) == {1, 2}


def test_refine_prefers_one_stream_within_two_percent(monkeypatch):
    """refine re-times the fastest few tunings and takes the least median; a
    one-stream tuning within 2% of a two-stream winner is taken instead."""
    two = {"chunk_pairs": 512, "streams": 2}
    one_close = {"chunk_pairs": 1024, "streams": 1}
    one_far = {"chunk_pairs": 256, "streams": 1}
    ms = {512: 1.000, 1024: 1.018, 256: 1.050}
    monkeypatch.setattr(autotune, "time_config", lambda plan, A, X, cfg, reps: ms[cfg["chunk_pairs"]])
    res = [(two, 1.0), (one_close, 1.0), (one_far, 1.0)]
    assert autotune.refine(None, None, None, res, reps=1) == one_close
    ms[1024] = 1.03  # beyond 2%: the two-stream tuning stays
    assert autotune.refine(None, None, None, res, reps=1) == two
    ms[256] = 0.99   # a one-stream tuning that is simply fastest
    assert autotune.refine(None, None, None, res, reps=1) == one_far
