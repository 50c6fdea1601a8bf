"""Pins of the sampling oracle: closed-form enumeration of the access patterns
of Scanner Sec. 3.2 (sampling by stride, range or index list; stencil S[0,1];
slicing) and Sec. 5.1.1."""
import pytest

import synth
from oracle import sampling as S


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
