"""Pins of the sampling oracle: closed-form enumeration of the access patterns
of Scanner Sec. 3.2 (sampling by stride, range or index list; stencil S[0,1];
slicing) and Sec. 5.1.1."""
import pytest

import synth
from oracle import sampling as S
from oracle import sampling as OS


def test_stride_every_24th_of_2400():
    rows = S.rows("stride", 2400, start=0, step=24, stop=2400)
    assert len(rows) == 100 and rows[0] == 0 and rows[-1] == 2376
    assert all(b - a == 24 for a, b in zip(rows, rows[1:]))
    prs = S.pairs("stride", 2400, start=0, step=24, stop=2400)
    assert len(prs) == 99 and prs[0] == (0, 24) and prs[-1] == (2352, 2376)


def test_stride_offsets_and_stop():
    assert S.rows("stride", 10, start=3, step=4, stop=10) == [3, 7]
    assert S.rows("stride", 10, start=0, step=1, stop=0) == []
    assert S.pairs("stride", 10, start=9, step=5, stop=10) == []


def test_gather_one_percent():
    idx = synth.gather_list(2, 2400, 0.01)
    assert len(idx) == 24 and idx == sorted(set(idx))
    prs = S.pairs("gather", 2400, idx=idx)
    assert prs == list(zip(idx, idx[1:]))


def test_range_windows_are_slices():
    # two windows: pairs never cross the boundary between them
    prs = S.pairs("range", 100, idx=[10, 14, 20, 23])
    assert prs == [(10, 11), (11, 12), (12, 13), (20, 21), (21, 22)]
    assert S.rows("range", 100, idx=[10, 14, 20, 23]) == [10, 11, 12, 13, 20, 21, 22]


def test_range_240_window_pair_count():
    (b, e), = synth.range_windows(3000, 2400, 240, 1)
    assert e - b == 240
    assert len(S.pairs("range", 2400, idx=[b, e])) == 239


@pytest.mark.parametrize("kind,kw", [
    ("stride", dict(start=0, step=0, stop=5)),
    ("stride", dict(start=0, step=1, stop=11)),
    ("gather", dict(idx=[3, 3])),
    ("gather", dict(idx=[5, 2])),
    ("gather", dict(idx=[10])),
    ("range", dict(idx=[5, 3])),
    ("range", dict(idx=[0, 5, 4, 8])),
    ("range", dict(idx=[0, 11])),
])
def test_invalid_specs_raise(kind, kw):
    with pytest.raises(S.SamplingError):
        S.slices(kind, 10, **kw)


def test_stencil_before_sampling_pairs():
    # STRIDE-24 over 2400 frames: (0, 1), (24, 25), ..., (2376, 2377)
    pb = OS.pairs_before("stride", 2400, start=0, step=24, stop=2400)
    assert len(pb) == 100 and pb[0] == (0, 1) and pb[-1] == (2376, 2377)
    assert all(b == a + 1 and a % 24 == 0 for a, b in pb)
    # a sampled last row of the table has no successor
    assert OS.pairs_before("gather", 10, idx=[2, 5, 9]) == [(2, 3), (5, 6)]
    # RANGE windows do not cut the original-neighbour pairs
    assert OS.pairs_before("range", 10, idx=[0, 2, 4, 6]) == [(0, 1), (1, 2), (4, 5), (5, 6)]
    # the after-sampling pairs of the same spec differ (low frame rate vs sparse original differences)
    assert OS.pairs("gather", 10, idx=[2, 5, 9]) == [(2, 5), (5, 9)]


def test_spacing_closed_forms():
    pos = [0, 24, 48]
    m = OS.space_map(pos, 60, "null")
    assert [t for t in range(60) if m[t] >= 0] == pos and [m[t] for t in pos] == [0, 1, 2]
    r = OS.space_map(pos, 60, "repeat")
    assert r == [0] * 24 + [1] * 24 + [2] * 12
    assert OS.space_map([3, 5], 7, "repeat") == [-1, -1, -1, 0, 0, 1, 1]
    # spacing inverts sampling: sampling the spaced sequence at the positions gives 0..K-1
    for mode in ("null", "repeat"):
        assert [OS.space_map(pos, 60, mode)[t] for t in pos] == [0, 1, 2]
    for bad in ([3, 3], [5, 2], [-1], [60]):
        with pytest.raises(OS.SamplingError):
            OS.space_map(bad, 60, "null")
