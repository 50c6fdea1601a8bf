"""Shot-boundary cue from colour-histogram differences (oracle; test
infrastructure only).

The data-mining application of Sec. 5.2.3 finds shot boundaries in films
from differences of per-frame colour histograms (the HIST output of
Sec. 5.1.2).  In Scanner's terms this is a stencil S[0,1] operation over the
histogram sequence (Sec. 3.2): it reads the histograms of sampled rows i and
i + 1 of one slice, exactly the pairs of the flow stencil.  The paper gives
neither the distance nor the decision rule; the readings below fix them.

Readings:
* Distance: the L1 distance between the two [3][16] count arrays,
  d = sum over channels c and bins b of |h2[c][b] - h1[c][b]| (an integer).
* Decision: the pair is a cut when d > threshold, for a threshold in pixel
  counts given by the caller (d ranges over [0, 6 w h]).
* Pairs are those of the sampling: consecutive sampled rows within a slice;
  no pair crosses a RANGE window.

Pins (tests): zero for identical histograms; 6 w h for two one-colour frames
whose three channels fall in different bins; symmetry; the triangle
inequality; d is even (both histograms sum to w h per channel); a brute-force
per-pixel count on tiny frames; no pair across RANGE windows; a hard cut in
a synthetic stream is the only pair over a threshold between the within-shot
and the cut distances.  Parity pinned.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def hist_l1(h1: np.ndarray, h2: np.ndarray) -> int:
    """L1 distance of two [3][16] histograms (exact integer)."""
    a = np.asarray(h1, dtype=np.int64)
    b = np.asarray(h2, dtype=np.int64)
    if a.shape != (3, 16) or b.shape != (3, 16):
        raise ValueError("histograms must be [3][16]")
    return int(np.abs(b - a).sum())


def pair_distances(hists: np.ndarray, pair_slots: Sequence[Tuple[int, int]]) -> np.ndarray:
    """d for each pair (i, j) of positions in the [M][3][16] histogram array."""
    return np.array([hist_l1(hists[i], hists[j]) for i, j in pair_slots], dtype=np.int64)


def cuts(d: np.ndarray, threshold: int) -> np.ndarray:
    """Cut flags: d > threshold."""
    return (np.asarray(d, dtype=np.int64) > int(threshold)).astype(np.uint8)


def pair_slots(slices: Sequence[Sequence[int]]) -> list:
    """Positions (i, i + 1) in the flattened row order of consecutive rows of
    each slice (the histogram array holds the rows of all slices in order)."""
    out, base = [], 0
    for s in slices:
        out.extend((base + k, base + k + 1) for k in range(len(s) - 1))
        base += len(s)
    return out
