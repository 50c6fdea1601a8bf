"""Sampling and stencil pairs (oracle; test infrastructure only).

Follows Scanner Sec. 3.2: sampling operations select a subset of a sequence's
elements by stride, range or index list; a stencil S[0,1] operation (optical
flow) needs elements i and i+1 of its input sequence; slicing inserts
boundaries that reset stencils.  Sec. 5.1.1 gives the access patterns
(every 24th frame, a sparse random index list, blocks of consecutive frames).

Readings:
* STRIDE rows are start, start+step, ... < stop.
* GATHER lists are strictly increasing in-range rows.
* Each RANGE window [begin, end) is a slice: no pair crosses two windows.
* Flow pairs join consecutive *sampled* rows (stencil after sampling); the
  last row of a slice has no successor, so a slice of M rows gives M-1 pairs.
* Stencil before sampling (Fig. e of Sec. 3.2: flow on original neighbours,
  then sampled): each sampled row s gives the pair (s, s+1) of original rows;
  a sampled last row of the table has no successor and gives no pair; RANGE
  windows do not cut these pairs (the stencil runs on the unsampled
  sequence).
* Spacing (the inverse of sampling, Sec. 3.2) of outputs placed at strictly
  increasing dense positions p_k: NULL fills map[t] = k at t = p_k and -1
  elsewhere; REPEAT fills map[t] = the last k with p_k <= t (-1 before p_0).

Pins: closed-form enumeration in tests (parity pinned).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple


class SamplingError(ValueError):
    pass


def stride_rows(n_frames: int, start: int, step: int, stop: int) -> List[int]:
    if step <= 0 or start < 0 or stop > n_frames or start > stop:
        raise SamplingError("bad stride spec")
    rows = []
    r = start
    while r < stop:
        rows.append(r)
        r += step
    return rows


def slices(kind: str, n_frames: int, start: int = 0, step: int = 1, stop: int | None = None,
           idx: Sequence[int] = ()) -> List[List[int]]:
    """Sampled rows grouped into slices (a stencil never crosses a slice boundary)."""
    if kind == "stride":
        stop = n_frames if stop is None else stop
        return [stride_rows(n_frames, start, step, stop)]
    if kind == "gather":
        rows = list(idx)
        for a, b in zip(rows, rows[1:]):
            if b <= a:
                raise SamplingError("gather list must be strictly increasing")
        if rows and (rows[0] < 0 or rows[-1] >= n_frames):
            raise SamplingError("gather row out of range")
        return [rows]
    if kind == "range":
        flat = list(idx)
        if len(flat) % 2:
            raise SamplingError("range list holds [begin, end) pairs")
        out, prev_end = [], 0
        for i in range(0, len(flat), 2):
            b, e = flat[i], flat[i + 1]
            if b < prev_end or e < b or e > n_frames or b < 0:
                raise SamplingError("ranges must be ascending, disjoint, in range")
            out.append(list(range(b, e)))
            prev_end = e
        return out
    raise SamplingError("unknown sampling kind")


def rows(kind: str, n_frames: int, **kw) -> List[int]:
    """All sampled rows, in order (the output order of HIST and convert)."""
    return [r for s in slices(kind, n_frames, **kw) for r in s]


def pairs(kind: str, n_frames: int, **kw) -> List[Tuple[int, int]]:
    """Flow pairs (r_i, r_{i+1}) of consecutive sampled rows within each slice."""
    out = []
    for s in slices(kind, n_frames, **kw):
        out.extend(zip(s, s[1:]))
    return out


def pairs_before(kind: str, n_frames: int, **kw) -> List[Tuple[int, int]]:
    """Stencil S[0,1] before sampling: (s, s+1) for every sampled row s with s+1 < n_frames."""
    return [(r, r + 1) for r in rows(kind, n_frames, **kw) if r + 1 < n_frames]


def space_map(positions: Sequence[int], n_dense: int, mode: str) -> List[int]:
    """Dense index map of outputs placed at strictly increasing positions."""
    pos = list(positions)
    for a, b in zip(pos, pos[1:]):
        if b <= a:
            raise SamplingError("positions must be strictly increasing")
    if pos and (pos[0] < 0 or pos[-1] >= n_dense):
        raise SamplingError("position out of range")
    out = [-1] * n_dense
    if mode == "null":
        for k, t in enumerate(pos):
            out[t] = k
    elif mode == "repeat":
        k = -1
        for t in range(n_dense):
            while k + 1 < len(pos) and pos[k + 1] <= t:
                k += 1
            out[t] = k
    else:
        raise SamplingError("unknown spacing mode")
    return out
